/*
 * gfx950 kernels of the FSPB dose-coefficient path.
 *
 *   k_prep      density mask (one bit per voxel) and per-grid-row extent of
 *               voxels above rho_min                          -- one wave per grid row
 *   k_raytrace  radiological-depth table of every beamlet (Sec. 2.2): Siddon
 *               crossings in FP64, compensated FP32 path sums  -- one wave per beamlet
 *   k_count     VOI members per tile of 64 grid rows (Sec. 2.1 VOI rule) and
 *               per beamlet row                                -- one wave per beamlet
 *   k_scan      exclusive scan -> CSR row pointers              -- one workgroup
 *   k_fill      Eq. 2-3 at every VOI voxel, compacted with wave ballots into
 *               ascending CSR columns                          -- one workgroup per beamlet
 *
 * The dose arithmetic is FP32; only the ray's plane-crossing parameters and
 * the per-row VOI interval are FP64.  Count and fill decide membership with
 * the same code (row_span + mask bit), so the fill writes exactly the counted
 * number of entries.
 */
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "fspb_device.h"
#include "fspb_mlp_device.h"

namespace fspb {

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ inline int mbcnt64(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <typename T>
__device__ inline T wave_incl_scan(T x)
{
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T y = __shfl_up(x, d, kWave);
        if (l >= d) x += y;
    }
    return x;
}

template <typename T>
__device__ inline T wave_sum(T x)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

/*
 * 32-bit integers: the inclusive scan by DPP, without LDS round trips.  Row
 * shifts by 1, 2, 4 and 8 lanes scan each row of 16 lanes (lanes shifted in
 * from outside the row read 0); then rows 1 and 3 add the last lane of the
 * row below (row_bcast:15) and rows 2 and 3 add lane 31 (row_bcast:31).
 * Every lane of the wave must be active.
 */
__device__ inline int wave_incl_scan(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return x;
}

/* Wave total of 32-bit integers (every lane active), the same on every lane. */
__device__ inline int wave_sum(int x) { return __builtin_amdgcn_readlane(wave_incl_scan(x), kWave - 1); }

/* ---------------------------------------------------------------- prep */

/* Mask bits and member extent of grid row `row` (= iz * ny + iy); one wave. */
__device__ void prep_row(const PlanDev &P, int row)
{
    const int lane = lane_id();
    const float *d = P.density + (size_t)row * P.nx;
    uint32_t *bits = P.bits + (size_t)row * P.wpr;
    int first = P.nx, last = -1, members = 0;
    for (int x0 = 0; x0 < P.nx; x0 += kWave) {
        const int x = x0 + lane;
        const bool m = x < P.nx && d[x] > P.rho_min;
        const uint64_t b = __ballot(m);
        const int w = (x0 >> 5) + lane;
        if (lane < 2 && w < P.wpr) bits[w] = lane ? (uint32_t)(b >> 32) : (uint32_t)b;
        if (b) {
            first = min(first, x0 + __ffsll((unsigned long long)b) - 1);
            last = x0 + 63 - __clzll((long long)b);
            members += __popcll(b);
        }
    }
    // first > last: no member voxel; kExtHoles marks a row with non-members between them
    const int holes = members != last - first + 1 && members > 0 ? kExtHoles : 0;
    if (lane == 0) P.ext[row] = make_int2(first | holes, last);
}

__global__ __launch_bounds__(kBlock) void k_prep(const PlanDev *__restrict__ plans)
{
    const PlanDev &P = plans[0];
    const int row = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (row < P.ny * P.nz) prep_row(P, row);
}

/* ------------------------------------------------------------ raytrace */

/* Compensated FP32 pair: value = s + c. */
struct cpair { float s, c; };

__device__ inline cpair cp_add(cpair a, cpair b)
{
    const float s = a.s + b.s;
    const float bb = s - a.s;
    const float e = (a.s - (s - bb)) + (b.s - bb);      // two-sum error
    return {s, (a.c + b.c) + e};
}

/*
 * Path integral of density over [tA + m step, min(tA + (m+1) step, tB)] of
 * beamlet R's axis: an incremental Siddon walk.  Crossing parameters are
 * recomputed from integer plane indices (no drift) in FP64; each segment's
 * voxel is the one holding its midpoint; rho * length is accumulated in FP32
 * with Neumaier compensation and the product's rounding error added back.
 */
__device__ cpair interval_integral(const PlanDev &P, const BeamletRec &R, int m, int n)
{
    const double t_end = (m == n - 2) ? R.tB : R.tA + (double)(m + 1) * R.step;
    double t = R.tA + (double)m * R.step;
    const int nv[3] = {P.nx, P.ny, P.nz};
    double an[3], inv_e[3], inv_sp[3];
    int pn[3], dp[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        inv_sp[k] = 1.0 / P.sp[k];
        const double e = R.e[k];
        dp[k] = 0;
        an[k] = 1e300;
        inv_e[k] = 0.0;
        if (e != 0.0) {
            inv_e[k] = 1.0 / e;
            const double c = (R.S[k] + t * e - P.lo[k]) * inv_sp[k];
            int p;
            if (e > 0.0) {
                p = (int)floor(c) + 1;
                dp[k] = 1;
            } else {
                p = (int)ceil(c) - 1;
                dp[k] = -1;
            }
            double a = (P.lo[k] + p * P.sp[k] - R.S[k]) * inv_e[k];
            if (a <= t) {
                p += dp[k];
                a = (P.lo[k] + p * P.sp[k] - R.S[k]) * inv_e[k];
            }
            pn[k] = p;
            an[k] = a;
        }
    }
    cpair acc = {0.0f, 0.0f};
    for (int it = 0; it < P.ray_iters; ++it) {
        const double tn = fmin(fmin(an[0], an[1]), fmin(an[2], t_end));
        if (tn > t) {
            const double mid = 0.5 * (t + tn);
            int idx[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                int v = (int)floor((R.S[k] + mid * R.e[k] - P.lo[k]) * inv_sp[k]);
                idx[k] = min(max(v, 0), nv[k] - 1);
            }
            const float rho = P.density[((size_t)idx[2] * P.ny + idx[1]) * P.nx + idx[0]];
            const float len = (float)(tn - t);
            const float prod = rho * len;
            const float perr = fmaf(rho, len, -prod);
            const float s = acc.s + prod;
            acc.c += (fabsf(acc.s) >= fabsf(prod)) ? ((acc.s - s) + prod) : ((prod - s) + acc.s);
            acc.c += perr;
            acc.s = s;
        }
        t = tn;
        if (t >= t_end) break;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (an[k] == tn) {
                pn[k] += dp[k];
                an[k] = (P.lo[k] + pn[k] * P.sp[k] - R.S[k]) * inv_e[k];
            }
        }
    }
    return acc;
}

/* Depth table of beamlet j; one wave, lanes over table intervals. */
/*
 * Density at S + t e by trilinear interpolation of the voxel centres, each
 * coordinate held at the first / last centre plane (FP64 position and
 * weights, eight gathers).
 */
__device__ double density_trilinear(const PlanDev &P, const BeamletRec &R, double t)
{
    const int nv[3] = {P.nx, P.ny, P.nz};
    int i0[3], st[3];
    double f[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int n = nv[k];
        double c = (R.S[k] + t * R.e[k] - P.org[k]) / P.sp[k];
        c = fmin(fmax(c, 0.0), (double)(n - 1));
        const int lo = n > 1 ? min((int)floor(c), n - 2) : 0;
        i0[k] = lo;
        st[k] = n > 1 ? 1 : 0;
        f[k] = n > 1 ? c - lo : 0.0;
    }
    const size_t sy = (size_t)P.nx, sz = (size_t)P.nx * P.ny;
    const float *base = P.density + (size_t)i0[2] * sz + (size_t)i0[1] * sy + i0[0];
    double r = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const double w = ((c & 1) ? f[0] : 1.0 - f[0]) * ((c & 2) ? f[1] : 1.0 - f[1]) *
                         ((c & 4) ? f[2] : 1.0 - f[2]);
        r += w * (double)base[((c & 4) ? st[2] * sz : 0) + ((c & 2) ? st[1] * sy : 0) + ((c & 1) ? st[0] : 0)];
    }
    return r;
}

/* Depth table from trilinear samples at the table points, trapezoid sums in
 * FP64 (one wave: lane m takes element m -> m + 1, then a wave prefix sum). */
__device__ void raytrace_trilinear(const PlanDev &P, const BeamletRec &R, float *tab)
{
    const int lane = lane_id();
    const int n = R.n_table;
    if (lane == 0) tab[0] = 0.0f;
    double carry = 0.0;
    for (int m0 = 0; m0 < n - 1; m0 += kWave) {
        const int m = m0 + lane;
        double inc = 0.0;
        if (m < n - 1) {
            const double t0 = R.tA + (double)m * R.step;
            const double t1 = (m == n - 2) ? R.tB : R.tA + (double)(m + 1) * R.step;
            inc = 0.5 * (t1 - t0) * (density_trilinear(P, R, t0) + density_trilinear(P, R, t1));
        }
        const double incl = wave_incl_scan(inc);
        if (m < n - 1) tab[m + 1] = (float)(carry + incl);
        carry += __shfl(incl, kWave - 1, kWave);
    }
}

// inlined: as a call it held k_raytrace at 196 VGPRs (two waves per SIMD), inlined it needs 90
__device__ __attribute__((always_inline)) inline void raytrace_beamlet(const PlanDev &P, int j)
{
    const int lane = lane_id();
    const BeamletRec &R = P.rec[j];
    const int n = R.n_table;
    if (n == 0) return;
    float *tab = P.tables + R.table_off;
    if (P.depth_mode == 1) {
        raytrace_trilinear(P, R, tab);
        return;
    }
    if (lane == 0) tab[0] = 0.0f;
    cpair carry = {0.0f, 0.0f};
    for (int m0 = 0; m0 < n - 1; m0 += kWave) {
        const int m = m0 + lane;
        cpair acc = {0.0f, 0.0f};
        if (m < n - 1) acc = interval_integral(P, R, m, n);
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            cpair y = {__shfl_up(acc.s, d, kWave), __shfl_up(acc.c, d, kWave)};
            if (lane >= d) acc = cp_add(y, acc);
        }
        const cpair tot = cp_add(carry, acc);
        if (m < n - 1) tab[m + 1] = tot.s + tot.c;
        const cpair last = {__shfl(acc.s, kWave - 1, kWave), __shfl(acc.c, kWave - 1, kWave)};
        carry = cp_add(carry, last);
    }
}

__global__ __launch_bounds__(kBlock) void k_raytrace(const PlanDev *__restrict__ plans)
{
    const PlanDev &P = plans[0];
    const int j = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (j < P.n_beamlets) raytrace_beamlet(P, j);
}

/* --------------------------------------------------------- VOI per row */

/* FP64 affine coefficients of t', U = (P-S).eu', V = (P-S).ev' along a grid row. */
struct RowAffine { double t0, U0, V0; };

/*
 * The FP64 quantities the VOI row interval needs: the beamlet record's block
 * from cu_sad to dx (built once per beamlet on the host, so that no division
 * is left per row): the cutoff slopes, t', U, V at column 0 of a grid row as
 * affine functions of (iy, iz), 1/c1 of the four inequalities c0 + c1 x <= 0
 * in the column x of a row (c1 is the same for every row of the beamlet; its
 * signs come with the record as bit masks), and the change of t', U, V per
 * column.
 */
struct RowGeom {
    double cu, cv;
    double t[3], u[3], v[3];
    double r1[4];
    double dx[3];
};
constexpr int kGeomWords = sizeof(RowGeom) / sizeof(double);
static_assert(offsetof(BeamletRec, dx) + 3 * sizeof(double) - offsetof(BeamletRec, cu_sad) == sizeof(RowGeom),
              "RowGeom mirrors the record's block from cu_sad to dx");

/* The block from the record, or from a copy of it. */
__device__ inline RowGeom row_geom(const double *src)
{
    RowGeom G;
    double *dst = reinterpret_cast<double *>(&G);
#pragma unroll
    for (int k = 0; k < kGeomWords; ++k) dst[k] = src[k];
    return G;
}
__device__ inline RowGeom row_geom(const BeamletRec &R) { return row_geom(&R.cu_sad); }

__device__ inline RowAffine row_affine(const RowGeom &G, int iy, int iz)
{
    const double y = (double)iy, z = (double)iz;
    RowAffine a;
    a.t0 = fma(z, G.t[2], fma(y, G.t[1], G.t[0]));
    a.U0 = fma(z, G.u[2], fma(y, G.u[1], G.u[0]));
    a.V0 = fma(z, G.v[2], fma(y, G.v[1], G.v[0]));
    return a;
}

/*
 * Columns [lo, hi] of grid row (iy, iz) whose centres satisfy
 * |U| <= (cu/SAD) t' and |V| <= (cv/SAD) t' (the VOI, which is convex, so an
 * interval), intersected with the row's extent of voxels above rho_min.
 * Solved in FP64 from the four linear inequalities.  Returns false if empty.
 */
__device__ inline bool row_span(const RowGeom &G, int c1_pos, int c1_neg, const int2 *__restrict__ ext_rows,
                                int nx, int ny, int iy, int iz, int &lo, int &hi, RowAffine &a, bool &holes)
{
    a = row_affine(G, iy, iz);
    const double c0[4] = {a.U0 - G.cu * a.t0, -a.U0 - G.cu * a.t0,
                          a.V0 - G.cv * a.t0, -a.V0 - G.cv * a.t0};
    double xlo = -1.0, xhi = (double)nx;            // already clipped to the grid
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 4; ++c) {                   // c0 + c1 x <= 0; the sign of c1 from the flags
        if (c1_pos & (1 << c)) xhi = fmin(xhi, -c0[c] * G.r1[c]);
        else if (c1_neg & (1 << c)) xlo = fmax(xlo, -c0[c] * G.r1[c]);
        else ok = ok && !(c0[c] > 0.0);
    }
    const int2 ext = ext_rows[iz * ny + iy];
    xlo = fmin(xlo, (double)nx);                    // both bounds now in [-1, nx]
    xhi = fmax(xhi, -1.0);
    lo = max((int)ceil(xlo), max(ext.x & ~kExtHoles, 0));
    hi = min((int)floor(xhi), min(ext.y, nx - 1));
    holes = (ext.x & kExtHoles) != 0;
    return ok && lo <= hi;
}

__device__ inline int popcount_range(const uint32_t *row, int lo, int hi)
{
    const int w0 = lo >> 5, w1 = hi >> 5;
    int c = 0;
    for (int w = w0; w <= w1; ++w) {
        uint32_t m = row[w];
        if (w == w0) m &= 0xffffffffu << (lo & 31);
        if (w == w1) m &= 0xffffffffu >> (31 - (hi & 31));
        c += __popc(m);
    }
    return c;
}

/* Grid-row cursor (iy, iz) of row r of a beamlet's n_iy-wide row block, stepped by a fixed count. */
struct RowCursor {
    int iy, iz;
    __device__ void step(int dy, int dz, int n_iy)
    {
        iy += dy;
        iz += dz;
        if (iy >= n_iy) {
            iy -= n_iy;
            ++iz;
        }
    }
};

/* VOI members of grid row (iy0 + c.iy, iz0 + c.iz), or 0 when r >= n_rows: lane work of count_beamlet. */
__device__ inline int count_row(const RowGeom &G, int c1_pos, int c1_neg, const uint32_t *__restrict__ bits,
                                const int2 *__restrict__ ext, int nx, int ny, int wpr, int iy0, int iz0,
                                const RowCursor &c, bool in)
{
    if (!in) return 0;
    const int iy = iy0 + c.iy, iz = iz0 + c.iz;
    int lo, hi;
    RowAffine a;
    bool holes;
    if (!row_span(G, c1_pos, c1_neg, ext, nx, ny, iy, iz, lo, hi, a, holes)) return 0;
    // every voxel between the row's first and last member is one: no mask words needed
    if (!holes) return hi - lo + 1;
    return popcount_range(bits + (size_t)(iz * ny + iy) * wpr, lo, hi);
}

/*
 * Tiles of beamlet j and its row of D's length; one wave.  The beamlet's row
 * block is walked 64 grid rows at a time (lane = row), two such groups per step
 * so that the loads of both are in flight together; each group's members are a
 * block tile's count.  Rows with VOI members are also appended to the
 * beamlet's row list (ascending), whose runs of 64 entries are list tiles with
 * their own counts.  Where fewer than half of the block's rows hold members
 * (a beam crossing air around a body), the fill takes the list tiles, so that
 * no tile set-up is spent on empty rows; otherwise the block tiles, whose rows
 * need no list read.  Everything the loop reads from the plan and the beamlet
 * record is taken into registers first.
 */
struct RowListBuilder {
    int32_t *list;       // the beamlet's row list
    int32_t *tiles;      // its list tiles' member counts
    int n = 0;           // rows in the list so far
    int acc = 0;         // members of the list tile being filled (tile n / 64)

    /* rows of one group of 64: row r (this lane's) with x >= 0 members; returns the group's
     * members.  The group's rows fill tile n / 64 and perhaps start the next (64 rows at most). */
    __device__ int append(int x, int r)
    {
        const uint64_t ne = __ballot(x > 0);
        const int pos = n + mbcnt64(ne);
        if (x > 0) list[pos] = r;
        const int incl = wave_incl_scan(x);                 // members of this lane's row and those below
        const int sum = __builtin_amdgcn_readlane(incl, kWave - 1);
        const int cnt = __popcll(ne), t0 = n >> 6, room = 64 * (t0 + 1) - n;
        if (cnt >= room) {
            // tile t0 is complete: its last row is the one at list position n + room - 1
            const uint64_t last = __ballot(x > 0 && pos == n + room - 1);
            const int sa = __builtin_amdgcn_readlane(incl, (int)__builtin_ctzll(last));
            if (lane_id() == 0) tiles[t0] = acc + sa;
            acc = sum - sa;
        } else {
            acc += sum;
        }
        n += cnt;
        return sum;
    }
    /* the last, partial tile */
    __device__ void finish()
    {
        if ((n & (kRowsPerTile - 1)) != 0 && lane_id() == 0) tiles[n >> 6] = acc;
    }
};
static_assert(kRowsPerTile == kWave, "one list tile per wave of rows");

__device__ void count_beamlet(const PlanDev &P, int j)
{
    const int lane = lane_id();
    const BeamletRec &R = P.rec[j];
    const RowGeom G = row_geom(R);
    const int c1_pos = __builtin_amdgcn_readfirstlane(R.c1_pos), c1_neg = __builtin_amdgcn_readfirstlane(R.c1_neg);
    const int n_iy = R.n_iy, iy0 = R.iy0, iz0 = R.iz0, tile0 = R.tile0, n_tiles = R.n_tiles;
    const int n_rows = n_iy * R.n_iz;
    const int nx = P.nx, ny = P.ny, wpr = P.wpr;
    const uint32_t *__restrict__ bits = P.bits;
    const int2 *__restrict__ ext = P.ext;
    int32_t *__restrict__ tile_count = P.tile_count;
    RowListBuilder L{P.row_list + (int64_t)tile0 * kRowsPerTile, P.list_count + tile0};
    // rows r and r + 64 of this lane, stepped by 128 rows per iteration
    RowCursor ca{lane % n_iy, lane / n_iy};
    RowCursor cb{(lane + kRowsPerTile) % n_iy, (lane + kRowsPerTile) / n_iy};
    const int dy = (2 * kRowsPerTile) % n_iy, dz = (2 * kRowsPerTile) / n_iy;
    int64_t total = 0;
    for (int t = 0; t < n_tiles; t += 2) {
        const int r = t * kRowsPerTile + lane;
        const int x0 = count_row(G, c1_pos, c1_neg, bits, ext, nx, ny, wpr, iy0, iz0, ca, r < n_rows);
        const int x1 = count_row(G, c1_pos, c1_neg, bits, ext, nx, ny, wpr, iy0, iz0, cb, r + kRowsPerTile < n_rows);
        const int c0 = L.append(x0, r), c1 = L.append(x1, r + kRowsPerTile);
        if (lane == 0) {
            tile_count[tile0 + t] = c0;
            if (t + 1 < n_tiles) tile_count[tile0 + t + 1] = c1;
        }
        total += c0 + c1;
        ca.step(dy, dz, n_iy);
        cb.step(dy, dz, n_iy);
    }
    L.finish();
    if (lane == 0) {
        P.row_nnz[j] = total;
        const bool list = P.tiles_mode == 0 ? 2 * L.n < n_rows : P.tiles_mode == 2;
        P.row_ne[j] = list ? L.n : -1;
    }
}

__global__ __launch_bounds__(kBlock) void k_count(const PlanDev *__restrict__ plans)
{
    const PlanDev &P = plans[0];
    const int j = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (j < P.n_beamlets) count_beamlet(P, j);
}

/* ---------------------------------------------------------------- scan */

constexpr int kScanBlock = 1024;

/* Exclusive scan of row_nnz into indptr[0..n]; indptr[n] = nnz.  One workgroup of kScanBlock. */
__device__ void scan_plan(const PlanDev &P, int64_t *indptr)
{
    // each thread takes kScanPer consecutive rows per pass, so one pass covers 8192 rows and
    // all of its loads are issued together
    constexpr int kScanPer = 8;
    __shared__ int64_t wsum[kScanBlock / kWave];
    __shared__ int64_t carry_s;
    const int tid = threadIdx.x, wave = tid >> 6, lane = lane_id();
    const int n = P.n_beamlets;
    const int64_t *__restrict__ row_nnz = P.row_nnz;
    if (tid == 0) carry_s = 0;
    __syncthreads();
    for (int base = 0; base < n; base += kScanBlock * kScanPer) {
        const int i0 = base + tid * kScanPer;
        int64_t v[kScanPer], s = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            v[k] = i0 + k < n ? row_nnz[i0 + k] : 0;
            s += v[k];
        }
        const int64_t inc = wave_incl_scan(s);
        if (lane == kWave - 1) wsum[wave] = inc;
        __syncthreads();
        int64_t woff = 0;
        for (int w = 0; w < wave; ++w) woff += wsum[w];
        const int64_t carry = carry_s;
        int64_t e = carry + woff + inc - s;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            if (i0 + k < n) indptr[i0 + k] = e;
            e += v[k];
        }
        __syncthreads();
        if (tid == kScanBlock - 1) carry_s = carry + woff + inc;
        __syncthreads();
    }
    if (tid == 0) {
        indptr[n] = carry_s;
        P.nnz[0] = carry_s;
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan(const PlanDev *__restrict__ plans,
                                                      const OutDev *__restrict__ outs)
{
    scan_plan(plans[0], outs[0].indptr);
}

/* ---------------------------------------------------------------- fill */

/* Word 3 of a raw (unformatted, stride 0) gfx9 buffer descriptor. */
constexpr int kRawBufferWord3 = 0x00020000;

/* A wave-uniform 64-bit value moved to scalar registers (keeps address arithmetic scalar). */
__device__ inline int64_t uniform64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

/* Global-address-space views of pointers read from plan records (global_* instead of flat_*). */
template <typename T>
using gptr = __attribute__((address_space(1))) T *;

template <typename T>
__device__ inline gptr<T> as_global(T *p)
{
    return (gptr<T>)(p);
}

/*
 * erf(z) at the table coordinate x = z kErfScale from the LDS copy of the
 * fill's table: linear interpolation between nodes 1/256 apart, each interval
 * k stored as the line through its two end nodes in the table coordinate,
 * (intercept c_k, slope s_k), so that erf ~ x s_k + c_k is one FMA of the
 * (clamped) argument and no fractional part is taken.
 *
 * Two forms: compact (7.5 KB, the intervals of [0, kErfMax]; odd symmetry gives
 * negative arguments) and mirrored (15 KB, the intervals of [-kErfMax,
 * kErfMax], arguments offset by kErfIntervals, read with their sign).  The
 * mirrored form's first interval is constant erf(-kErfMax) (slope 0), so an
 * argument below the table reads that entry through a saturating conversion
 * and needs no clamp; beyond the last node the argument is clamped.
 */
constexpr float kErfScale = (float)kErfIntervals / kErfMax;
constexpr float kErfTop = (float)kErfIntervals - 1.0f / 1024.0f;            // below kErfIntervals
constexpr float kErfTopSigned = 2.0f * kErfIntervals - 1.0f / 1024.0f;      // below 2 kErfIntervals

/* compact form, any sign */
__device__ inline float erf_lds(const float2 *__restrict__ tab, float x)
{
    const float xc = fminf(fabsf(x), kErfTop);
    const float2 q = tab[(int)xc];
    return copysignf(fmaf(xc, q.y, q.x), x);
}

/* compact form, x >= 0 */
__device__ inline float erf_lds_pos(const float2 *__restrict__ tab, float x)
{
    const float xc = fminf(x, kErfTop);
    const float2 q = tab[(int)xc];
    return fmaf(xc, q.y, q.x);
}

/* mirrored form, clamped on both sides */
__device__ inline float erf_m(const float2 *__restrict__ tab, float x)
{
    const float xc = __builtin_amdgcn_fmed3f(x, 0.0f, kErfTopSigned);
    const float2 q = tab[(int)xc];
    return fmaf(xc, q.y, q.x);
}

/* mirrored form, x >= 0: clamped above */
__device__ inline float erf_m_hi(const float2 *__restrict__ tab, float x)
{
    const float xc = fminf(x, kErfTopSigned);
    const float2 q = tab[(int)xc];
    return fmaf(xc, q.y, q.x);
}

/* mirrored form, x known to lie below the last node: v_cvt_u32_f32 saturates a
 * negative argument to entry 0, the constant erf(-kErfMax) (x times a zero slope) */
__device__ inline float erf_m_lo(const float2 *__restrict__ tab, float x)
{
    uint32_t k;
    __asm__("v_cvt_u32_f32 %0, %1" : "=v"(k) : "v"(x));
    const float2 q = tab[k];
    return fmaf(x, q.y, q.x);
}

/*
 * How the fill reads erf (a plan-level choice, made on the host):
 *   0  compact table (odd symmetry for negative arguments);
 *   1  mirrored table, both arguments of a bracket clamped;
 *   2  mirrored table, the first argument known to stay below the table's top
 *      (the plan's widest beamlet over its narrowest sigma): no clamp on it;
 *   3  as 2, with square beamlets (a = b), so the u and v brackets of a term
 *      share their offsets, and the second argument read through erf(z) =
 *      -erf(-z) so that it too can only leave the table below (no clamp at
 *      all, and a saturated bracket is exactly 0); in the analytic form the
 *      first term's weight is folded into the staged depth dose.  Only for
 *      kernels with D >= 0 (non-negative weights and depth dose).
 */
constexpr bool erf_mirrored_mode(int em) { return em >= 1; }

/*
 * One bracket of Eq. 3, erf((h - x) is) + erf((h + x) is), with
 * is = 1/(sqrt2 sigma): isk = is kErfScale and hk = h isk put both arguments
 * in table coordinates.  The bracket is even in x, so it is evaluated at |x|,
 * where the second argument is never negative (h > 0).  Mirrored modes: hk
 * already offset by kErfIntervals.
 */
template <int EM>
__device__ inline float edge_pair(const float2 *__restrict__ tab, float x, float hk, float isk)
{
    const float ax = fabsf(x);
    const float x1 = fmaf(-ax, isk, hk), x2 = fmaf(ax, isk, hk);
    if (EM >= 2) return erf_m_lo(tab, x1) + erf_m_hi(tab, x2);
    if (EM == 1) return erf_m(tab, x1) + erf_m_hi(tab, x2);
    return erf_lds(tab, x1) + erf_lds_pos(tab, x2);
}

/* Mode 3: the bracket from hk = h isk + n and hk2 = n - h isk (n = kErfIntervals):
 * erf(x1) - erf(mirror of (h + |x|) is), both read below the table's top. */
__device__ inline float edge_pair_sq(const float2 *__restrict__ tab, float x, float hk, float hk2, float isk)
{
    const float ax = fabsf(x);
    return erf_m_lo(tab, fmaf(-ax, isk, hk)) - erf_m_lo(tab, fmaf(-ax, isk, hk2));
}

/* hk of the bracket: h isk, plus the mirrored table's offset */
template <int EM>
__device__ inline float edge_offset(float h, float isk)
{
    return EM >= 1 ? fmaf(h, isk, (float)kErfIntervals) : h * isk;
}

/* Per-beamlet constants of the fill, held in registers. */
template <int K>
struct FillConst {
    float tA, inv_step, tau_max, pdd_inv, pdd_max;
    bool floor0;                 // D >= 0 holds exactly: negative rounding residue is cut to 0
    int n_terms;
    float w4[K], ha[K], hb[K];
    float sig0[K], sig1[K];      // sigma law divided by kIsScale: 1/sigma' = isk
    // general form (tables): A and c grids, beamlet half sides
    float a_inv, a_max, c_inv, c_max, half_a, half_b;
    int nc;
};

// is kErfScale = kIsScale / sigma
constexpr float kIsScale = 0.70710678118654752f * kErfScale;

/*
 * D of one VOI voxel at s = t' - tA, with U' = (P - S).eu' SAD and
 * V' = (P - S).ev' SAD (the lateral offsets scaled by SAD in advance), so that
 * with r = 1/t' the iso-plane offsets are u = U' r, v = V' r and the inverse
 * square (SAD/t')^2 = SAD^2 r^2 has its SAD^2 folded into the LDS depth dose.
 */
template <int K, bool GUARD, int EM>
__device__ inline float dose_value(const FillConst<K> &c, const float2 *__restrict__ tab,
                                   const float2 *__restrict__ pdd, const float2 *__restrict__ etab,
                                   float s, float U, float V)
{
    const float r = __builtin_amdgcn_rcpf(s + c.tA);   // 1 / t'
    const float u = U * r, v = V * r;
    // radiological depth at O': linear interpolation in the table, one FMA in the intercept form
    // (last entry has slope 0)
    const float tau = __builtin_amdgcn_fmed3f(s * c.inv_step, 0.0f, c.tau_max);
    const float2 q = tab[(int)tau];
    const float d = fmaf(tau, q.y, q.x);
    // depth dose times SAD^2, held at the last node
    const float x = __builtin_amdgcn_fmed3f(d * c.pdd_inv, 0.0f, c.pdd_max);
    const float2 qp = pdd[(int)x];
    const float A = fmaf(x, qp.y, qp.x) * r * r;
    // lateral profile, Eq. 3
    float L = 0.0f;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        if (GUARD && i >= c.n_terms) break;
        const float isk = __builtin_amdgcn_rcpf(fmaf(c.sig1[i], d, c.sig0[i]));
        if (EM == 3) {
            // square beamlets; the first term's weight is in the depth dose, c.w4 relative to it
            const float hk = fmaf(c.ha[i], isk, (float)kErfIntervals), hk2 = fmaf(-c.ha[i], isk, (float)kErfIntervals);
            const float eu = edge_pair_sq(etab, u, hk, hk2, isk), ev = edge_pair_sq(etab, v, hk, hk2, isk);
            L = i == 0 ? eu * ev : fmaf(c.w4[i] * eu, ev, L);
        } else {
            const float eu = edge_pair<EM>(etab, u, edge_offset<EM>(c.ha[i], isk), isk);
            const float ev = edge_pair<EM>(etab, v, edge_offset<EM>(c.hb[i], isk), isk);
            L = i == 0 ? c.w4[0] * eu * ev : fmaf(c.w4[i] * eu, ev, L);   // no add of 0 for the first term
        }
    }
    // with non-negative weights and depth dose D is >= 0 (every bracket is); the table's
    // rounding could otherwise leave a -1e-8-sized value where both brackets saturate
    const float D = A * L;
    if (EM == 3) return fmaxf(D, 0.0f);   // mode 3 implies such a kernel
    return c.floor0 ? fmaxf(D, 0.0f) : D;
}

/*
 * Eq. 2-3 in their general form: A(theta_j, d) SAD^2 from the beamlet's LDS
 * row (already interpolated in theta), c1, c2, c3 of each term from LDS depth
 * tables (value, slope) laid out [c][term][node].
 */
template <int K, int EM>
__device__ inline float dose_value_gen(const FillConst<K> &c, const float2 *__restrict__ tab,
                                       const float2 *__restrict__ sA, const float2 *__restrict__ sc,
                                       const float2 *__restrict__ etab, float s, float U, float V)
{
    const float r = __builtin_amdgcn_rcpf(s + c.tA);
    const float u = U * r, v = V * r;
    const float tau = __builtin_amdgcn_fmed3f(s * c.inv_step, 0.0f, c.tau_max);
    const float2 q = tab[(int)tau];
    const float d = fmaf(tau, q.y, q.x);
    const float xa = __builtin_amdgcn_fmed3f(d * c.a_inv, 0.0f, c.a_max);
    const float2 qa = sA[(int)xa];
    const float A = fmaf(xa, qa.y, qa.x) * r * r;
    const float xc = __builtin_amdgcn_fmed3f(d * c.c_inv, 0.0f, c.c_max);
    const int kc = (int)xc;
    const float fc = __builtin_amdgcn_fractf(xc);
    float L = 0.0f;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const float2 q1 = sc[i * c.nc + kc], q2 = sc[(K + i) * c.nc + kc], q3 = sc[(2 * K + i) * c.nc + kc];
        const float c1 = fmaf(fc, q1.y, q1.x), c2 = fmaf(fc, q2.y, q2.x), c3 = fmaf(fc, q3.y, q3.x);
        const float isk = kIsScale * __builtin_amdgcn_rcpf(c3);
        float eu, ev;
        if (EM == 3) {
            const float h = c2 * c.half_a;
            const float hk = fmaf(h, isk, (float)kErfIntervals), hk2 = fmaf(-h, isk, (float)kErfIntervals);
            eu = edge_pair_sq(etab, u, hk, hk2, isk);
            ev = edge_pair_sq(etab, v, hk, hk2, isk);
        } else {
            eu = edge_pair<EM>(etab, u, edge_offset<EM>(c2 * c.half_a, isk), isk);
            ev = edge_pair<EM>(etab, v, edge_offset<EM>(c2 * c.half_b, isk), isk);
        }
        L = i == 0 ? 0.25f * c1 * eu * ev : fmaf(0.25f * c1 * eu, ev, L);
    }
    const float D = A * L;
    if (EM == 3) return fmaxf(D, 0.0f);   // mode 3 implies such a kernel
    return c.floor0 ? fmaxf(D, 0.0f) : D;
}

/* Entries of the depth-dose region of the fill's LDS: the PDD, or the general
 * form's A row and c tables. */
__host__ __device__ inline int lds_pdd_pairs(const PlanDev &P)
{
    return P.gen ? P.n_adepth + 3 * P.n_terms * P.n_cdepth : P.n_pdd;
}

__device__ inline int readlane(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

/*
 * D_ij of beamlet j (one CSR row) by a workgroup of W waves: LDS-staged
 * tables, then each wave takes tiles of 64 grid rows (64 consecutive rows of
 * the beamlet's row block, or 64 entries of the list of its rows with members,
 * as the count pass chose); a tile's VOI candidates are flattened across its
 * rows, 64 per chunk, members compacted by ballot.
 * K = unrolled term count; GUARD: stop at P.n_terms (plans of mixed K);
 * EM: how erf is read (erf_mirrored_mode).
 */
/* tile_group: consecutive 64-row tiles a wave takes per step (the batched fill's tuned shape). */
template <int K, int W, bool GUARD, bool SURR, bool GEN = false, int EM = 0>
__device__ __attribute__((always_inline)) inline void fill_beamlet(const PlanDev &P, const OutDev &O, int j, unsigned char *smem,
                                                             int tile_group = 1)
{
    const BeamletRec &R = P.rec[j];
    if (R.n_tiles == 0) return;   // the axis misses the grid
    constexpr int kB = W * kWave;
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = lane_id();
    constexpr bool SE = erf_mirrored_mode(EM);
    // mode 3, analytic form: term weights relative to the first, whose weight the depth dose carries
    constexpr bool FOLD_W = EM == 3 && !GEN;

    // ---- constants into registers
    const int n_table = R.n_table, n_pdd = lds_pdd_pairs(P), tile0 = R.tile0;
    const int iy0 = R.iy0, n_iy = R.n_iy, iz0 = R.iz0;
    const gptr<const int32_t> row_list = as_global<const int32_t>(P.row_list + (int64_t)R.tile0 * kRowsPerTile);
    const int nx = P.nx, ny = P.ny, wpr = P.wpr;
    FillConst<K> c;
    c.tA = R.tA_f;
    c.inv_step = R.inv_step_f;
    c.tau_max = R.tau_max_f;
    c.pdd_inv = P.pdd_inv_step;
    c.pdd_max = P.pdd_max;
    c.floor0 = P.d_floor == 0.0f;
    c.n_terms = P.n_terms;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        c.w4[i] = FOLD_W ? P.w4[i] / P.w4[0] : P.w4[i];
        c.sig0[i] = P.sig0[i] * (1.0f / kIsScale);
        c.sig1[i] = P.sig1[i] * (1.0f / kIsScale);
        c.ha[i] = R.ha[i];
        c.hb[i] = R.hb[i];
    }
    if (GEN) {
        c.a_inv = P.a_inv_step;
        c.a_max = P.a_max;
        c.c_inv = P.c_inv_step;
        c.c_max = P.c_max;
        c.half_a = R.half_a;
        c.half_b = R.half_b;
        c.nc = P.n_cdepth;
    }
    const float sad_f = R.sad_f;
    const double tA = R.tA, sad = R.sad;
    // per voxel step along x: t' in float, U and V scaled by SAD (rounded once from FP64)
    const float t1f = R.t1_f, U1f = (float)(R.dx[1] * sad), V1f = (float)(R.dx[2] * sad);
    const gptr<const uint32_t> bits = as_global<const uint32_t>(P.bits);
    const gptr<int32_t> out_idx = as_global<int32_t>(O.indices);
    const gptr<float> out_val = as_global<float>(O.values);
    const int64_t capacity = O.capacity;
    const int64_t row_base = uniform64(O.indptr[j] - O.indptr[O.row0]);

    // ---- LDS: erf table, depth table, depth dose (times SAD^2), tile prefix; the depth table
    // and the depth dose (or the general form's A row) as (intercept, slope) in their own
    // table coordinate, value = x slope + intercept for x in [k, k + 1]
    float2 *s_erf = reinterpret_cast<float2 *>(smem);
    constexpr int kErfPairs = SE ? 2 * kErfIntervals : kErfIntervals;
    float2 *s_tab = s_erf + kErfPairs;
    float2 *s_pdd = s_tab + P.max_table;
    int *s_tpre = reinterpret_cast<int *>(s_pdd + n_pdd);
    __shared__ int wsum[W];
    // the beamlet's VOI row coefficients, read by every tile (LDS keeps them out of registers)
    __shared__ RowGeom s_geom;
    const int c1_pos = __builtin_amdgcn_readfirstlane(R.c1_pos), c1_neg = __builtin_amdgcn_readfirstlane(R.c1_neg);
    // surrogate: per-wave h1 tile after the tile prefix, and W2 fragments in registers
    uint16_t *s_h1 = reinterpret_cast<uint16_t *>(
        smem + ((sizeof(float2) * ((size_t)kErfPairs + P.max_table + n_pdd) +
                 sizeof(int) * ((size_t)P.max_tiles + 1) + 15) & ~(size_t)15)) + wave * (64 * mlp::kH1Stride);
    // and the layer-1 bias with this beamlet's width term folded in, after the W tiles
    float *s_b1x = reinterpret_cast<float *>(s_h1 + (W - wave) * (64 * mlp::kH1Stride));
    mlp::W2Frags wf;
    if (SURR) mlp::load_w2_frags(P.mlp_w2, wf);
    const float a_f = R.a_f;
    const bool mlp_ok = SURR && R.mlp_ok;
    if (SURR && tid < kMlpH)
        s_b1x[tid] = fmaf(P.mlp_p[kOffW1 + tid * kMlpIn + 3], mlp::feature_a(a_f), P.mlp_p[kOffB1 + tid]);

    {
        // the erf table in the form this fill reads (compact, or mirrored after it)
        const float4 *__restrict__ et = reinterpret_cast<const float4 *>(P.erf_tab + (SE ? kErfIntervals : 0));
        float4 *se4 = reinterpret_cast<float4 *>(s_erf);
        for (int i = tid; i < kErfPairs / 2; i += kB) se4[i] = et[i];
        if (tid < kGeomWords) reinterpret_cast<double *>(&s_geom)[tid] = (&R.cu_sad)[tid];
        const gptr<const float> tab = as_global<const float>(P.tables + R.table_off);
        for (int i = tid; i < n_table; i += kB) {
            const float d0 = tab[i];
            const float sl = (i + 1 < n_table ? tab[i + 1] : d0) - d0;
            s_tab[i] = make_float2(fmaf(-(float)i, sl, d0), sl);
        }
        const float sad2 = sad_f * sad_f;
        if (GEN) {
            // this beamlet's A row (interpolated in theta, times SAD^2), then the c tables
            const int na = P.n_adepth, k0 = R.theta_k, k1 = min(R.theta_k + 1, P.n_theta - 1);
            const float ft = R.theta_f;
            const gptr<const float> a0 = as_global<const float>(P.atab + (size_t)k0 * na);
            const gptr<const float> a1 = as_global<const float>(P.atab + (size_t)k1 * na);
            for (int i = tid; i < na; i += kB) {
                const float v0 = fmaf(ft, a1[i] - a0[i], a0[i]);
                const float v1 = i + 1 < na ? fmaf(ft, a1[i + 1] - a0[i + 1], a0[i + 1]) : v0;
                const float sl = (v1 - v0) * sad2;
                s_pdd[i] = make_float2(fmaf(-(float)i, sl, v0 * sad2), sl);
            }
            const int nc = P.n_cdepth, ntab = 3 * P.n_terms * nc;
            const gptr<const float> ct = as_global<const float>(P.ctab);
            for (int i = tid; i < ntab; i += kB) {
                const int node = i % nc;
                const float v0 = ct[i];
                s_pdd[na + i] = make_float2(v0, (node + 1 < nc ? ct[i + 1] : v0) - v0);
            }
        } else {
            const gptr<const float> pd = as_global<const float>(P.pdd);
            const float scale = FOLD_W ? sad2 * P.w4[0] : sad2;
            for (int i = tid; i < n_pdd; i += kB) {
                const float p0 = pd[i];
                const float sl = ((i + 1 < n_pdd ? pd[i + 1] : p0) - p0) * scale;
                s_pdd[i] = make_float2(fmaf(-(float)i, sl, p0 * scale), sl);
            }
        }
    }
    // the tiles the count pass chose (read here, after the table loads have been issued): the
    // row list's (64 rows with members each, the last one partial; its length clamped to the
    // row block's capacity, so that no index can leave it) or the row block's
    const int ne = __builtin_amdgcn_readfirstlane(P.row_ne[j]);
    const bool use_list = ne >= 0;
    const int n_list = use_list ? min(ne, R.n_tiles * kRowsPerTile) : R.n_iy * R.n_iz;
    const int n_tiles = use_list ? (n_list + kRowsPerTile - 1) / kRowsPerTile : R.n_tiles;
    const gptr<const int32_t> tile_count = as_global<const int32_t>(use_list ? P.list_count : P.tile_count);
    // exclusive scan of this beamlet's tile counts
    int carry = 0;
    for (int base = 0; base < n_tiles; base += kB) {
        const int i = base + tid;
        const int v = i < n_tiles ? tile_count[tile0 + i] : 0;
        const int inc = wave_incl_scan(v);
        if (lane == kWave - 1) wsum[wave] = inc;
        __syncthreads();
        int woff = 0;
        for (int w = 0; w < wave; ++w) woff += wsum[w];
        if (i < n_tiles) s_tpre[i] = carry + woff + inc - v;
        int tot = 0;
        for (int w = 0; w < W; ++w) tot += wsum[w];
        carry += tot;
        __syncthreads();
    }

    // the wave's tiles: runs of tile_group consecutive tiles, every W-th run.  Lane = a grid
    // row r of the beamlet's row block (of a block tile, or an entry of the row list); with the
    // list, the next tile's entries are loaded while this tile is walked
    auto next_tile = [&](int t) { return (t + 1) % tile_group != 0 ? t + 1 : t + 1 + (W - 1) * tile_group; };
    auto list_entry = [&](int t) {
        const int li = t * kRowsPerTile + lane;
        return t < n_tiles && li < n_list ? row_list[li] : -1;
    };
    // one tile: row r (this lane's; -1 for none) of tile tl; after_span runs once the rows'
    // extents have been read
    auto tile = [&](const int tl, const int r, auto &&after_span) {
        // row r's VOI interval and FP32 start values; the column of candidate k of the row is
        // cb + k, its mask word wb + ((lo + k) >> 5)
        const int members = __builtin_amdgcn_readfirstlane(tile_count[tile0 + tl]);
        if (members == 0) {           // an empty block tile (list tiles always have members)
            after_span();
            return;
        }
        const int64_t out0 = row_base + __builtin_amdgcn_readfirstlane(s_tpre[tl]);
        int lo = 0, hi = -1, cb = 0, wb = 0;
        float s_lo = 0.0f, U_lo = 0.0f, V_lo = 0.0f;
        if (r >= 0) {
            const int iy = iy0 + (int)((uint32_t)r % (uint32_t)n_iy), iz = iz0 + (int)((uint32_t)r / (uint32_t)n_iy);
            RowAffine a;
            // the block is read from LDS here, tile by tile (an offset the compiler cannot see
            // through keeps it from being held in registers across the tile loop)
            uint32_t goff = 0;
            asm volatile("" : "+s"(goff));
            const RowGeom G = row_geom(reinterpret_cast<const double *>(reinterpret_cast<const char *>(&s_geom) + goff));
            bool holes;
            if (row_span(G, c1_pos, c1_neg, P.ext, P.nx, P.ny, iy, iz, lo, hi, a, holes)) {
                const int grow = iz * ny + iy;
                cb = grow * nx + lo;
                wb = grow * wpr;
                const double x = (double)lo;
                s_lo = (float)(a.t0 + x * G.dx[0] - tA);
                U_lo = (float)(fma(x, G.dx[1], a.U0) * sad);
                V_lo = (float)(fma(x, G.dx[2], a.V0) * sad);
            } else {
                lo = 0;
                hi = -1;
            }
        }
        // the next tile's list entries, loaded once this tile's row extents have arrived: the
        // vector memory counter retires in order, so an earlier issue would make the wait for
        // those extents wait for this load as well
        after_span();
        int cnt = hi - lo + 1;
        {
            // rows with candidates move to the low lanes, in order, empty rows after them
            // (a permutation of the wave), so that row starts are distinct candidates
            const uint64_t ne = __ballot(cnt > 0);
            const int dst = cnt > 0 ? mbcnt64(ne) : __popcll(ne) + mbcnt64(~ne);
            const int a = dst << 2;
            lo = __builtin_amdgcn_ds_permute(a, lo);
            cnt = __builtin_amdgcn_ds_permute(a, cnt);
            cb = __builtin_amdgcn_ds_permute(a, cb);
            wb = __builtin_amdgcn_ds_permute(a, wb);
            s_lo = __int_as_float(__builtin_amdgcn_ds_permute(a, __float_as_int(s_lo)));
            U_lo = __int_as_float(__builtin_amdgcn_ds_permute(a, __float_as_int(U_lo)));
            V_lo = __int_as_float(__builtin_amdgcn_ds_permute(a, __float_as_int(V_lo)));
        }
        const int n_ne = __popcll(__ballot(cnt > 0));
        const int incl = wave_incl_scan(cnt);
        const int excl = incl - cnt;
        const int total = readlane(incl, kWave - 1);   // wave-uniform: the chunk loop stays scalar
        // candidate p of the tile lies on the last row whose exclusive prefix is <= p;
        // rows are walked once, wave-uniformly, as the chunks advance (rcur: row of
        // the first candidate of the next chunk)
        int rcur = 0;
        int64_t written = out0;
        // a tile whose counted members equal its candidates (no masked voxel inside its rows)
        // takes every candidate: no mask read, and member lanes are the low ones of the chunk
        const bool dense = members == total;
        // the tile's entries fit the caller's arrays: no per-chunk capacity test, and they are
        // written through buffer descriptors over exactly the tile's entries (32-bit offsets:
        // the lane's slot in a VGPR, the chunk's start in an SGPR)
        const bool fits = out0 + members <= capacity;
        const __amdgpu_buffer_rsrc_t rs_idx =
            __builtin_amdgcn_make_buffer_rsrc(O.indices + out0, 0, members * 4, kRawBufferWord3);
        const __amdgpu_buffer_rsrc_t rs_val =
            __builtin_amdgcn_make_buffer_rsrc(O.values + out0, 0, members * 4, kRawBufferWord3);
        // one chunk: candidate p of the tile, on row rr of the tile; every lane of the wave calls it
        auto chunk = [&](const int p, const int rr, auto dense_tag, auto fits_tag) {
            constexpr bool DENSE = decltype(dense_tag)::value;
            constexpr bool FITS = decltype(fits_tag)::value;
            // row rr's values, fetched by lane (rr < 64: the byte address needs no wrap)
            const int ra = rr << 2;
            auto from_row = [&](int v) { return __builtin_amdgcn_ds_bpermute(ra, v); };
            auto from_row_f = [&](float v) { return __int_as_float(__builtin_amdgcn_ds_bpermute(ra, __float_as_int(v))); };
            const int k = p - from_row(excl);
            const int col = from_row(cb) + k;
            bool member = false;
            if (DENSE) {
                member = p < total;
            } else {
                const int wr = from_row(wb), ix = from_row(lo) + k;
                if (p < total) {
                    const uint32_t wo = ((uint32_t)wr + ((uint32_t)ix >> 5)) << 2;   // byte offset
                    member = (*(const gptr<const uint32_t>)((gptr<const char>)bits + wo) >> (ix & 31)) & 1u;
                }
            }
            const uint64_t mask = __ballot(member);
            const uint32_t slot = DENSE ? (uint32_t)lane : (uint32_t)mbcnt64(mask);
            const float sl = from_row_f(s_lo);
            const float ul = from_row_f(U_lo);
            const float vl = from_row_f(V_lo);
            // this chunk's entries go to [written, written + popcount); the bases are wave-uniform
            const gptr<char> ip = (gptr<char>)(out_idx + written);
            const gptr<char> vp = (gptr<char>)(out_val + written);
            float D = 0.0f;
            if (SURR) {
                // the network runs on all 64 lanes (matrix cores need the whole wave)
                const float kf = (float)k;
                const float sv = fmaf(kf, t1f, sl), Uv = fmaf(kf, U1f, ul), Vv = fmaf(kf, V1f, vl);
                const float rr_ = __builtin_amdgcn_rcpf(sv + c.tA);
                const float g = sad_f * rr_;
                const float au = fabsf(Uv * rr_), av = fabsf(Vv * rr_);
                const float tau = __builtin_amdgcn_fmed3f(sv * c.inv_step, 0.0f, c.tau_max);
                const float2 q = s_tab[(int)tau];
                const float d = fmaf(tau, q.y, q.x);
                const bool in_box = member && mlp_ok && d <= kMlpDMax && au <= kMlpUVMax &&
                                    av <= kMlpUVMax;
                float x[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                if (in_box) mlp::features(d, au, av, a_f, x);
                // the network only for chunks with a sample inside the training box
                float y = 0.0f;
                if (__ballot(in_box)) y = mlp::forward_wave<true>(P.mlp_p, s_b1x, wf, x, s_h1);
                if (in_box) D = y * g * g;
                else if (member) D = dose_value<K, GUARD, EM>(c, s_tab, s_pdd, s_erf, sv, Uv, Vv);
            }
            if (member) {
                const float kf = (float)k;
                if (GEN)
                    D = dose_value_gen<K, EM>(c, s_tab, s_pdd, s_pdd + P.n_adepth, s_erf, fmaf(kf, t1f, sl),
                                                  fmaf(kf, U1f, ul), fmaf(kf, V1f, vl));
                else if (!SURR)
                    D = dose_value<K, GUARD, EM>(c, s_tab, s_pdd, s_erf, fmaf(kf, t1f, sl), fmaf(kf, U1f, ul),
                                                     fmaf(kf, V1f, vl));
                if (FITS) {
                    const int so = (int)(written - out0) << 2;
                    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)col, rs_idx, (int)(slot << 2), so, 0);
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(D), rs_val, (int)(slot << 2), so, 0);
                } else {
                    // slots below `avail` fit in the caller's arrays
                    const int64_t left = capacity - written;
                    const uint32_t avail = left >= kWave ? (uint32_t)kWave : (left > 0 ? (uint32_t)left : 0u);
                    if (slot < avail) {
                        *(gptr<int32_t>)(ip + (slot << 2)) = col;
                        *(gptr<float>)(vp + (slot << 2)) = D;
                    } else {
                        *O.overflow = 1;
                    }
                }
            }
            written += __popcll(mask);
        };
        auto walk2 = [&](auto dense_tag, auto fits_tag) {
            // two chunks per row walk: lane takes candidates c0 + lane and c0 + 64 + lane.
            // Bit b of (mhi:mlo) marks a row starting at candidate c0 + b (0 < b < 128);
            // a lane's row is rcur plus the row starts at or below its candidate, a
            // masked bit count of the mask shifted down by one
            for (int c0 = 0; c0 < total; c0 += 2 * kWave) {
                uint64_t mlo = 0, mhi = 0;
                int rnext = rcur;
                for (int q = rcur + 1; q < n_ne; ++q) {
                    const int b = readlane(excl, q) - c0;
                    if (b > 2 * kWave) break;
                    rnext = q;
                    if (b == 2 * kWave) break;
                    if (b < kWave) mlo |= 1ull << b;
                    else mhi |= 1ull << (b - kWave);
                }
                const uint64_t nlo = (mlo >> 1) | (mhi << 63), nhi = mhi >> 1;
                const int r1 = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(nlo >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)nlo, (uint32_t)rcur));
                const int r2 = (int)__builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(nhi >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)nhi, (uint32_t)(rcur + __popcll(nlo))));
                chunk(c0 + lane, r1, dense_tag, fits_tag);
                chunk(c0 + kWave + lane, r2, dense_tag, fits_tag);
                rcur = rnext;
            }
        };
        // dense tiles whose entries fit: a lane takes two consecutive candidates of one row
        // (pair slot q of a row holds its candidates 2q and 2q + 1), so that the row lookup,
        // the row walk and the column arithmetic serve two entries; each entry's value is
        // computed exactly as in a chunk of single candidates
        auto pair_chunk = [&](const int q, const int rr, const int pexcl, const int ptotal) {
            const int ra = rr << 2;
            auto from_row = [&](int v) { return __builtin_amdgcn_ds_bpermute(ra, v); };
            auto from_row_f = [&](float v) { return __int_as_float(__builtin_amdgcn_ds_bpermute(ra, __float_as_int(v))); };
            const int k0 = (q - from_row(pexcl)) << 1;
            const int e0 = from_row(excl) + k0;            // tile-local entry of candidate k0
            const int cn = from_row(cnt);
            const int col = from_row(cb) + k0;
            const float sl = from_row_f(s_lo), ul = from_row_f(U_lo), vl = from_row_f(V_lo);
            if (q < ptotal) {
                const bool two = k0 + 1 < cn;
                auto value = [&](float kf) {
                    if (GEN)
                        return dose_value_gen<K, EM>(c, s_tab, s_pdd, s_pdd + P.n_adepth, s_erf, fmaf(kf, t1f, sl),
                                                     fmaf(kf, U1f, ul), fmaf(kf, V1f, vl));
                    return dose_value<K, GUARD, EM>(c, s_tab, s_pdd, s_erf, fmaf(kf, t1f, sl), fmaf(kf, U1f, ul),
                                                    fmaf(kf, V1f, vl));
                };
                // the second candidate of a row's last, odd slot is evaluated at the first (and not stored)
                const float D0 = value((float)k0), D1 = value((float)(two ? k0 + 1 : k0));
                __builtin_amdgcn_raw_buffer_store_b32((uint32_t)col, rs_idx, e0 << 2, 0, 0);
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(D0), rs_val, e0 << 2, 0, 0);
                if (two) {
                    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)(col + 1), rs_idx, (e0 + 1) << 2, 0, 0);
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(D1), rs_val, (e0 + 1) << 2, 0, 0);
                }
            }
        };
        auto walk_pairs = [&]() {
            // the row walk of walk2 over pair slots: bit b of (mhi:mlo) marks a row whose
            // first pair slot is c0 + b
            const int np = (cnt + 1) >> 1;
            const int pincl = wave_incl_scan(np);
            const int pexcl = pincl - np;
            const int ptotal = readlane(pincl, kWave - 1);
            int rc = 0;
            for (int c0 = 0; c0 < ptotal; c0 += 2 * kWave) {
                uint64_t mlo = 0, mhi = 0;
                int rnext = rc;
                for (int q = rc + 1; q < n_ne; ++q) {
                    const int b = readlane(pexcl, q) - c0;
                    if (b > 2 * kWave) break;
                    rnext = q;
                    if (b == 2 * kWave) break;
                    if (b < kWave) mlo |= 1ull << b;
                    else mhi |= 1ull << (b - kWave);
                }
                const uint64_t nlo = (mlo >> 1) | (mhi << 63), nhi = mhi >> 1;
                const int r1 = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(nlo >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)nlo, (uint32_t)rc));
                const int r2 = (int)__builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(nhi >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)nhi, (uint32_t)(rc + __popcll(nlo))));
                pair_chunk(c0 + lane, r1, pexcl, ptotal);
                pair_chunk(c0 + kWave + lane, r2, pexcl, ptotal);
                rc = rnext;
            }
        };
        if (!SURR) {
            if (fits) {
                if (dense) walk_pairs();
                else walk2(std::false_type{}, std::true_type{});
            } else {
                walk2(std::false_type{}, std::false_type{});
            }
        } else {
            for (int c0 = 0; c0 < total; c0 += kWave) {
                while (rcur + 1 < kWave && readlane(excl, rcur + 1) <= c0) ++rcur;
                const int p = c0 + lane;
                int rr = rcur;
                for (int q = rcur + 1; q < kWave; ++q) {
                    const int eq = readlane(excl, q);
                    if (eq > c0 + kWave - 1) break;
                    if (p >= eq) rr = q;
                }
                chunk(p, rr, std::false_type{}, std::false_type{});
            }
        }
    };
    if (!use_list) {
        for (int tg = wave * tile_group; tg < n_tiles; tg += W * tile_group)
            for (int tl = tg; tl < tg + tile_group && tl < n_tiles; ++tl) {
                const int r = tl * kRowsPerTile + lane;
                tile(tl, r < n_list ? r : -1, [] {});
            }
    } else {
        int r_next = list_entry(wave * tile_group);
        for (int tl = wave * tile_group; tl < n_tiles; tl = next_tile(tl)) {
            const int r = r_next;
            tile(tl, r, [&] { r_next = list_entry(next_tile(tl)); });
        }
    }
}

// the analytic form's register budget at one or two terms: six waves per SIMD (80 VGPRs)
template <int K, bool SURR, bool GEN, int EM>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(SURR || GEN || K > 2 ? 1 : 6))) void k_fill(const PlanDev *__restrict__ plans,
                                                  const OutDev *__restrict__ outs)
{
    extern __shared__ __align__(16) unsigned char smem[];
    // launched before the host has read the plan's total: write nothing if it does not fit
    if (outs[0].check_nnz && *plans[0].nnz > outs[0].capacity) return;
    fill_beamlet<K, kWavesPerBlock, false, SURR, GEN, EM>(plans[0], outs[0], outs[0].row0 + (int)blockIdx.x, smem);
}

/* ------------------------------------------------------------ batches */

/*
 * Persistent kernels over many plans.  Wave-level stages walk a global item
 * index grid-stride; item i belongs to the plan p with start[p] <= i <
 * start[p+1] (few plans: a short uniform search).  The fill pulls
 * (plan, beamlet) items from an atomic queue, longest rows first.
 */
__device__ inline int plan_of(const int64_t *__restrict__ start, int n_plans, int64_t i)
{
    int lo = 0, hi = n_plans - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int STAGE>
__global__ __launch_bounds__(kBlock) void kp_wave(const PlanDev *const *__restrict__ plans,
                                                  const int64_t *__restrict__ start, int n_plans)
{
    const int64_t total = start[n_plans];
    const int64_t nw = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); w < total; w += nw) {
        const int p = plan_of(start, n_plans, w);
        const PlanDev &P = *plans[p];
        const int i = (int)(w - start[p]);
        if (STAGE == 0) prep_row(P, i);
        else if (STAGE == 1) raytrace_beamlet(P, i);
        else count_beamlet(P, i);
    }
}

__global__ __launch_bounds__(kScanBlock) void kp_scan(const PlanDev *const *__restrict__ plans,
                                                       const OutDev *__restrict__ outs)
{
    scan_plan(*plans[blockIdx.x], outs[blockIdx.x].indptr);
}

// amdgpu_waves_per_eu(4): a register budget that leaves room for at least four waves per SIMD
// (it is a lower bound on occupancy, not a cap)
// Work items (plan, beamlet) come from a queue, per_item consecutive ones per fetch; a wave
// takes tile_group consecutive tiles of a beamlet per step.
template <int K, int W>
__global__ __launch_bounds__(W * kWave) __attribute__((amdgpu_waves_per_eu(4))) void kp_fill(const PlanDev *const *__restrict__ plans,
                                                     const OutDev *__restrict__ outs,
                                                     const int2 *__restrict__ items, int n_items,
                                                     int *__restrict__ counter, int per_item, int tile_group)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int w0 = s_item * per_item;
        __syncthreads();
        if (w0 >= n_items) break;
        const int w1 = min(n_items, w0 + per_item);
        for (int w = w0; w < w1; ++w) {
            const int2 it = items[w];
            const PlanDev &P = *plans[it.x];
            // each plan in the erf table form of its own fill (identical results to it)
            switch (P.erf_mode) {
            case 3: fill_beamlet<K, W, true, false, false, 3>(P, outs[it.x], it.y, smem, tile_group); break;
            case 2: fill_beamlet<K, W, true, false, false, 2>(P, outs[it.x], it.y, smem, tile_group); break;
            case 1: fill_beamlet<K, W, true, false, false, 1>(P, outs[it.x], it.y, smem, tile_group); break;
            default: fill_beamlet<K, W, true, false, false, 0>(P, outs[it.x], it.y, smem, tile_group); break;
            }
            __syncthreads();
        }
    }
}

__global__ void k_reset(int *__restrict__ counters, int n)
{
    if ((int)threadIdx.x < n) counters[threadIdx.x] = 0;
}

}  // namespace

/* ------------------------------------------------------------ launchers */

static inline unsigned blocks_for(int64_t items, int per_block)
{
    return (unsigned)((items + per_block - 1) / per_block);
}

hipError_t launch_prep(const PlanDev *dplan, const PlanDev &h, hipStream_t s)
{
    const int64_t rows = (int64_t)h.ny * h.nz;
    hipLaunchKernelGGL(k_prep, dim3(blocks_for(rows, kWavesPerBlock)), dim3(kBlock), 0, s, dplan);
    return hipGetLastError();
}

hipError_t launch_raytrace(const PlanDev *dplan, const PlanDev &h, hipStream_t s)
{
    hipLaunchKernelGGL(k_raytrace, dim3(blocks_for(h.n_beamlets, kWavesPerBlock)), dim3(kBlock), 0, s,
                       dplan);
    return hipGetLastError();
}

hipError_t launch_count(const PlanDev *dplan, const PlanDev &h, hipStream_t s)
{
    if (h.n_beamlets == 0) return hipSuccess;
    hipLaunchKernelGGL(k_count, dim3(blocks_for(h.n_beamlets, kWavesPerBlock)), dim3(kBlock), 0, s, dplan);
    return hipGetLastError();
}

hipError_t launch_scan(const PlanDev *dplan, const OutDev *dout, const PlanDev &h, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanBlock), 0, s, dplan, dout);
    return hipGetLastError();
}

size_t fill_shared_bytes(const PlanDev &h, bool mirrored_erf)
{
    size_t b = sizeof(float2) * ((mirrored_erf ? 2 * kErfIntervals : kErfIntervals) + (size_t)h.max_table +
                                 (size_t)lds_pdd_pairs(h)) +
               sizeof(int) * ((size_t)h.max_tiles + 1);
    if (h.use_mlp)
        b = ((b + 15) & ~(size_t)15) + sizeof(uint16_t) * 64 * mlp::kH1Stride * kWavesPerBlock +
            sizeof(float) * kMlpH;
    return b;
}

size_t fill_shared_bytes(const PlanDev &h)
{
    return fill_shared_bytes(h, fill_mirrored_erf(h));
}

bool fill_mirrored_erf(const PlanDev &h) { return h.erf_mirrored && !h.use_mlp; }

int mirrored_erf_mode(const PlanDev &h)
{
    if (!h.erf_nc) return 1;
    return h.erf_square && h.d_floor == 0.0f && (h.gen || h.w4[0] != 0.0f) ? 3 : 2;
}

template <int K, bool GEN>
static const void *fill_kernel_ptr_k(int em)
{
    switch (em) {
    case 3: return (const void *)k_fill<K, false, GEN, 3>;
    case 2: return (const void *)k_fill<K, false, GEN, 2>;
    case 1: return (const void *)k_fill<K, false, GEN, 1>;
    default: return (const void *)k_fill<K, false, GEN, 0>;
    }
}

template <bool GEN>
static const void *fill_kernel_ptr(int K, int em)
{
    switch (K) {
    case 1: return fill_kernel_ptr_k<1, GEN>(em);
    case 2: return fill_kernel_ptr_k<2, GEN>(em);
    case 3: return fill_kernel_ptr_k<3, GEN>(em);
    default: return fill_kernel_ptr_k<4, GEN>(em);
    }
}

/*
 * Workgroups of a fill kernel per CU: the runtime's limit from registers and
 * waves, and an LDS limit computed here with the allocation (static + dynamic)
 * rounded up to 512 bytes and counted in two halves of the CU's LDS.  The
 * halves are what the measured fill times follow: the mirrored table takes
 * the slab (24 KB per workgroup) 2 % faster at five workgroups per CU, and the
 * pelvis (27 KB, three per half would need 83 KB) 7 % slower, though the
 * runtime's query (160 KB, whole) gives five for both.
 */
static int fill_groups_per_cu(const void *f, size_t lds, int lds_per_cu)
{
    int n = 0;
    hipFuncAttributes attr{};
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kBlock, 0) != hipSuccess ||
        hipFuncGetAttributes(&attr, f) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    const size_t need = (lds + attr.sharedSizeBytes + 511) & ~(size_t)511;
    return std::min(n, 2 * (int)((size_t)(lds_per_cu / 2) / need));
}

int choose_erf_form(const PlanDev &h)
{
    const size_t lds_m = fill_shared_bytes(h, true), lds_s = fill_shared_bytes(h, false);
    if (lds_m > 64 * 1024) return 0;
    int dev = 0, lds_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        lds_cu <= 0) {
        (void)hipGetLastError();
        return 0;
    }
    const int em = mirrored_erf_mode(h);
    const void *fm = h.gen ? fill_kernel_ptr<true>(h.n_terms, em) : fill_kernel_ptr<false>(h.n_terms, em);
    const void *fs = h.gen ? fill_kernel_ptr<true>(h.n_terms, 0) : fill_kernel_ptr<false>(h.n_terms, 0);
    const int nm = fill_groups_per_cu(fm, lds_m, lds_cu), ns = fill_groups_per_cu(fs, lds_s, lds_cu);
    return nm > 0 && nm >= ns ? 1 : 0;
}

hipError_t launch_batch_wave(int stage, const PlanDev *const *plans, const int64_t *start, int n_plans,
                             int grid, hipStream_t s)
{
    const dim3 g(grid), b(kBlock);
    switch (stage) {
    case 0: hipLaunchKernelGGL(kp_wave<0>, g, b, 0, s, plans, start, n_plans); break;
    case 1: hipLaunchKernelGGL(kp_wave<1>, g, b, 0, s, plans, start, n_plans); break;
    default: hipLaunchKernelGGL(kp_wave<2>, g, b, 0, s, plans, start, n_plans); break;
    }
    return hipGetLastError();
}

hipError_t launch_batch_scan(const PlanDev *const *plans, const OutDev *outs, int n_plans, hipStream_t s)
{
    hipLaunchKernelGGL(kp_scan, dim3(n_plans), dim3(kScanBlock), 0, s, plans, outs);
    return hipGetLastError();
}

hipError_t launch_batch_reset(int *counters, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, counters, n);
    return hipGetLastError();
}

template <int K>
static hipError_t launch_kp_fill_k(int W, const PlanDev *const *plans, const OutDev *outs, const int2 *items,
                                   int n_items, int *counter, int per_item, int tile_group, int grid, size_t lds,
                                   hipStream_t s)
{
    const dim3 g(grid);
    switch (W) {
    case 2:
        hipLaunchKernelGGL((kp_fill<K, 2>), g, dim3(2 * kWave), lds, s, plans, outs, items, n_items, counter, per_item,
                           tile_group);
        break;
    case 8:
        hipLaunchKernelGGL((kp_fill<K, 8>), g, dim3(8 * kWave), lds, s, plans, outs, items, n_items, counter, per_item,
                           tile_group);
        break;
    default:
        hipLaunchKernelGGL((kp_fill<K, 4>), g, dim3(4 * kWave), lds, s, plans, outs, items, n_items, counter, per_item,
                           tile_group);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_batch_fill(int K, int W, const PlanDev *const *plans, const OutDev *outs, const int2 *items,
                             int n_items, int *counter, int per_item, int tile_group, int grid, size_t lds,
                             hipStream_t s)
{
    switch (K) {
    case 1: return launch_kp_fill_k<1>(W, plans, outs, items, n_items, counter, per_item, tile_group, grid, lds, s);
    case 2: return launch_kp_fill_k<2>(W, plans, outs, items, n_items, counter, per_item, tile_group, grid, lds, s);
    case 3: return launch_kp_fill_k<3>(W, plans, outs, items, n_items, counter, per_item, tile_group, grid, lds, s);
    default: return launch_kp_fill_k<4>(W, plans, outs, items, n_items, counter, per_item, tile_group, grid, lds, s);
    }
}

hipError_t launch_fill(const PlanDev *dplan, const OutDev *dout, const PlanDev &h, int row0, int n_rows,
                       hipStream_t s)
{
    (void)row0;   // read by the kernel from the output record
    if (n_rows <= 0) return hipSuccess;
    const dim3 grid(n_rows), block(kBlock);
    const size_t lds = fill_shared_bytes(h);
    if (h.use_mlp) {
        switch (h.n_terms) {
        case 1: hipLaunchKernelGGL((k_fill<1, true, false, 0>), grid, block, lds, s, dplan, dout); break;
        case 2: hipLaunchKernelGGL((k_fill<2, true, false, 0>), grid, block, lds, s, dplan, dout); break;
        case 3: hipLaunchKernelGGL((k_fill<3, true, false, 0>), grid, block, lds, s, dplan, dout); break;
        default: hipLaunchKernelGGL((k_fill<4, true, false, 0>), grid, block, lds, s, dplan, dout); break;
        }
        return hipGetLastError();
    }
    const int em = h.erf_mode;
    const void *f = h.gen ? fill_kernel_ptr<true>(h.n_terms, em) : fill_kernel_ptr<false>(h.n_terms, em);
    void *args[] = {const_cast<PlanDev **>(&dplan), const_cast<OutDev **>(&dout)};
    return hipLaunchKernel(f, grid, block, args, lds, s);
}

}  // namespace fspb
