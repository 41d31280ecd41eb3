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
 * The FP64 beamlet and grid quantities the VOI row interval needs, read once
 * per beamlet (or tile) into registers, and the four inequalities
 * c0 + c1 x <= 0 in the column x of a grid row: c1 (and 1/c1) are the same for
 * every row of the beamlet.
 */
struct RowGeom {
    double wx, oy, oz, sy, sz, Sy, Sz;    // org0 - S0; org1, org2; spacing y, z; S1, S2
    double e[3], eu[3], ev[3], cu, cv;
    double c1[4], r1[4];
};

__device__ inline RowGeom row_geom(const PlanDev &P, const BeamletRec &R)
{
    RowGeom G;
    G.wx = P.org[0] - R.S[0];
    G.oy = P.org[1];
    G.oz = P.org[2];
    G.sy = P.sp[1];
    G.sz = P.sp[2];
    G.Sy = R.S[1];
    G.Sz = R.S[2];
    for (int k = 0; k < 3; ++k) {
        G.e[k] = R.e[k];
        G.eu[k] = R.eu[k];
        G.ev[k] = R.ev[k];
    }
    G.cu = R.cu_sad;
    G.cv = R.cv_sad;
    const double t1 = P.sp[0] * R.e[0];
    const double U1 = P.sp[0] * R.eu[0];
    const double V1 = P.sp[0] * R.ev[0];
    G.c1[0] = U1 - G.cu * t1;
    G.c1[1] = -U1 - G.cu * t1;
    G.c1[2] = V1 - G.cv * t1;
    G.c1[3] = -V1 - G.cv * t1;
#pragma unroll
    for (int c = 0; c < 4; ++c) G.r1[c] = G.c1[c] != 0.0 ? 1.0 / G.c1[c] : 0.0;
    return G;
}

__device__ inline RowAffine row_affine(const RowGeom &G, int iy, int iz)
{
    const double wx = G.wx;
    const double wy = fma((double)iy, G.sy, G.oy) - G.Sy;
    const double wz = fma((double)iz, G.sz, G.oz) - G.Sz;
    RowAffine a;
    a.t0 = wx * G.e[0] + wy * G.e[1] + wz * G.e[2];
    a.U0 = wx * G.eu[0] + wy * G.eu[1] + wz * G.eu[2];
    a.V0 = wx * G.ev[0] + wy * G.ev[1] + wz * G.ev[2];
    return a;
}

/*
 * Columns [lo, hi] of grid row (iy, iz) whose centres satisfy
 * |U| <= (cu/SAD) t' and |V| <= (cv/SAD) t' (the VOI, which is convex, so an
 * interval), intersected with the row's extent of voxels above rho_min.
 * Solved in FP64 from the four linear inequalities.  Returns false if empty.
 */
__device__ inline bool row_span(const RowGeom &G, const int2 *__restrict__ ext_rows, int nx, int ny, int iy,
                                int iz, int &lo, int &hi, RowAffine &a, bool &holes)
{
    a = row_affine(G, iy, iz);
    const double c0[4] = {a.U0 - G.cu * a.t0, -a.U0 - G.cu * a.t0,
                          a.V0 - G.cv * a.t0, -a.V0 - G.cv * a.t0};
    double xlo = -1.0, xhi = (double)nx;            // already clipped to the grid
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 4; ++c) {                   // c0 + c1 x <= 0
        if (G.c1[c] > 0.0) xhi = fmin(xhi, -c0[c] * G.r1[c]);
        else if (G.c1[c] < 0.0) xlo = fmax(xlo, -c0[c] * G.r1[c]);
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
__device__ inline int count_row(const RowGeom &G, const uint32_t *__restrict__ bits,
                                const int2 *__restrict__ ext, int nx, int ny, int wpr, int iy0, int iz0,
                                const RowCursor &c, bool in)
{
    if (!in) return 0;
    const int iy = iy0 + c.iy, iz = iz0 + c.iz;
    int lo, hi;
    RowAffine a;
    bool holes;
    if (!row_span(G, ext, nx, ny, iy, iz, lo, hi, a, holes)) return 0;
    // every voxel between the row's first and last member is one: no mask words needed
    if (!holes) return hi - lo + 1;
    return popcount_range(bits + (size_t)(iz * ny + iy) * wpr, lo, hi);
}

/*
 * VOI members of every tile of beamlet j (64 grid rows each, lane = row) and
 * of its whole row of D; one wave, two tiles per step so that the loads of
 * both are in flight together.  Everything the loop reads from the plan and
 * the beamlet record is taken into registers first.
 */
__device__ void count_beamlet(const PlanDev &P, int j)
{
    const int lane = lane_id();
    const BeamletRec &R = P.rec[j];
    const RowGeom G = row_geom(P, R);
    const int n_iy = R.n_iy, iy0 = R.iy0, iz0 = R.iz0, tile0 = R.tile0, n_tiles = R.n_tiles;
    const int n_rows = n_iy * R.n_iz;
    const int nx = P.nx, ny = P.ny, wpr = P.wpr;
    const uint32_t *__restrict__ bits = P.bits;
    const int2 *__restrict__ ext = P.ext;
    int32_t *__restrict__ tile_count = P.tile_count;
    // rows r and r + 64 of this lane, stepped by 128 rows per iteration
    RowCursor ca{lane % n_iy, lane / n_iy};
    RowCursor cb{(lane + kRowsPerTile) % n_iy, (lane + kRowsPerTile) / n_iy};
    const int dy = (2 * kRowsPerTile) % n_iy, dz = (2 * kRowsPerTile) / n_iy;
    int64_t total = 0;
    for (int t = 0; t < n_tiles; t += 2) {
        const int r = t * kRowsPerTile + lane;
        const int x0 = count_row(G, bits, ext, nx, ny, wpr, iy0, iz0, ca, r < n_rows);
        const int x1 = count_row(G, bits, ext, nx, ny, wpr, iy0, iz0, cb, r + kRowsPerTile < n_rows);
        const int c0 = wave_sum(x0), c1 = wave_sum(x1);
        if (lane == 0) {
            tile_count[tile0 + t] = c0;
            if (t + 1 < n_tiles) tile_count[tile0 + t + 1] = c1;
        }
        total += c0 + c1;
        ca.step(dy, dz, n_iy);
        cb.step(dy, dz, n_iy);
    }
    if (lane == 0) P.row_nnz[j] = total;
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
 * erf(z) at the table coordinate x = z kErfScale: linear interpolation in the
 * LDS copy of the table on [0, kErfMax] (one 8-byte (value, difference) read),
 * sign restored by odd symmetry, held at +-erf(kErfMax) beyond the table.
 *
 * The fill stages the table in one of two forms: this one (8 KB), or mirrored
 * onto [-kErfMax, kErfMax] (16 KB, arguments offset by kErfIntervals), where a
 * signed argument needs no absolute value or sign restore.  The mirrored form
 * saves four instructions per coefficient of a two-term kernel and is used
 * wherever its larger LDS footprint does not cost the fill a workgroup per CU.
 */
constexpr float kErfScale = (float)kErfIntervals / kErfMax;
constexpr int kErfLdsFloats = 2 * kErfIntervals;
constexpr float kErfTopSigned = 2.0f * kErfIntervals - 1.0f / 1024.0f;   // below 2 kErfIntervals, fract < 1

__device__ inline float erf_lds(const float *__restrict__ tab, float x)
{
    const float xc = fminf(fabsf(x), (float)kErfIntervals - 1.0f / 1024.0f);
    const int k = (int)xc;
    const float f = __builtin_amdgcn_fractf(xc);
    const float2 q = reinterpret_cast<const float2 *>(tab)[k];
    return copysignf(fmaf(q.y, f, q.x), x);
}

/* erf_lds for an argument known to be >= 0 (no sign to restore); SE: in the
 * mirrored table, offset included. */
template <bool SE = false>
__device__ inline float erf_lds_pos(const float *__restrict__ tab, float x)
{
    const float xc = fminf(x, SE ? kErfTopSigned : (float)kErfIntervals - 1.0f / 1024.0f);
    const int k = (int)xc;
    const float f = __builtin_amdgcn_fractf(xc);
    const float2 q = reinterpret_cast<const float2 *>(tab)[k];
    return fmaf(q.y, f, q.x);
}

/* erf in the mirrored table at x + kErfIntervals (the offset is part of the argument). */
__device__ inline float erf_lds_signed(const float *__restrict__ tab, float xo)
{
    const float xc = __builtin_amdgcn_fmed3f(xo, 0.0f, kErfTopSigned);
    const int k = (int)xc;
    const float f = __builtin_amdgcn_fractf(xc);
    const float2 q = reinterpret_cast<const float2 *>(tab)[k];
    return fmaf(q.y, f, q.x);
}

/*
 * One bracket of Eq. 3, erf((h - x) is) + erf((h + x) is), with
 * is = 1/(sqrt2 sigma): isk = is kErfScale and hk = h isk put both arguments
 * in table coordinates.  The bracket is even in x, so it is evaluated at |x|,
 * where the second argument is never negative (h > 0).  SE: mirrored table,
 * hk already offset by kErfIntervals.
 */
template <bool SE>
__device__ inline float edge_pair(const float *__restrict__ tab, float x, float hk, float isk)
{
    const float ax = fabsf(x);
    if (SE) return erf_lds_signed(tab, fmaf(-ax, isk, hk)) + erf_lds_pos<true>(tab, fmaf(ax, isk, hk));
    return erf_lds(tab, fmaf(-ax, isk, hk)) + erf_lds_pos(tab, fmaf(ax, isk, hk));
}

/* hk of the bracket: h isk, plus the mirrored table's offset */
template <bool SE>
__device__ inline float edge_offset(float h, float isk)
{
    return SE ? fmaf(h, isk, (float)kErfIntervals) : h * isk;
}

/* Per-beamlet constants of the fill, held in registers. */
template <int K>
struct FillConst {
    float sad, tA, inv_step, tau_max, pdd_inv, pdd_max;
    int n_terms;
    float w4[K], ha[K], hb[K];
    float sig0[K], sig1[K];      // sigma law divided by kIsScale: 1/sigma' = isk
    // general form (tables): A and c grids, beamlet half sides
    float a_inv, a_max, c_inv, c_max, half_a, half_b;
    int nc;
};

// is kErfScale = kIsScale / sigma
constexpr float kIsScale = 0.70710678118654752f * kErfScale;

template <int K, bool GUARD, bool SE>
__device__ inline float dose_value(const FillConst<K> &c, const float2 *__restrict__ tab,
                                   const float2 *__restrict__ pdd, const float *__restrict__ etab,
                                   float s, float U, float V)
{
    const float tp = s + c.tA;                      // t' = |SO'|
    const float g = c.sad * __builtin_amdgcn_rcpf(tp);   // SAD / t'
    const float u = U * g, v = V * g;
    // radiological depth at O': linear interpolation in the table (last entry has slope 0)
    const float tau = __builtin_amdgcn_fmed3f(s * c.inv_step, 0.0f, c.tau_max);
    const float2 q = tab[(int)tau];
    const float d = fmaf(__builtin_amdgcn_fractf(tau), q.y, q.x);
    // depth dose, held at the last node
    const float x = __builtin_amdgcn_fmed3f(d * c.pdd_inv, 0.0f, c.pdd_max);
    const float2 qp = pdd[(int)x];
    const float A = fmaf(__builtin_amdgcn_fractf(x), qp.y, qp.x) * g * g;
    // lateral profile, Eq. 3
    float L = 0.0f;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        if (GUARD && i >= c.n_terms) break;
        const float isk = __builtin_amdgcn_rcpf(fmaf(c.sig1[i], d, c.sig0[i]));
        const float eu = edge_pair<SE>(etab, u, edge_offset<SE>(c.ha[i], isk), isk);
        const float ev = edge_pair<SE>(etab, v, edge_offset<SE>(c.hb[i], isk), isk);
        L = i == 0 ? c.w4[0] * eu * ev : fmaf(c.w4[i] * eu, ev, L);   // no add of 0 for the first term
    }
    return A * L;
}

/*
 * Eq. 2-3 in their general form: A(theta_j, d) from the beamlet's LDS row
 * (already interpolated in theta), c1, c2, c3 of each term from LDS depth
 * tables (value, slope) laid out [c][term][node].
 */
template <int K, bool SE>
__device__ inline float dose_value_gen(const FillConst<K> &c, const float2 *__restrict__ tab,
                                       const float2 *__restrict__ sA, const float2 *__restrict__ sc,
                                       const float *__restrict__ etab, float s, float U, float V)
{
    const float tp = s + c.tA;
    const float g = c.sad * __builtin_amdgcn_rcpf(tp);
    const float u = U * g, v = V * g;
    const float tau = __builtin_amdgcn_fmed3f(s * c.inv_step, 0.0f, c.tau_max);
    const float2 q = tab[(int)tau];
    const float d = fmaf(__builtin_amdgcn_fractf(tau), q.y, q.x);
    const float xa = __builtin_amdgcn_fmed3f(d * c.a_inv, 0.0f, c.a_max);
    const float2 qa = sA[(int)xa];
    const float A = fmaf(__builtin_amdgcn_fractf(xa), qa.y, qa.x) * g * g;
    const float xc = __builtin_amdgcn_fmed3f(d * c.c_inv, 0.0f, c.c_max);
    const int kc = (int)xc;
    const float fc = __builtin_amdgcn_fractf(xc);
    float L = 0.0f;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const float2 q1 = sc[i * c.nc + kc], q2 = sc[(K + i) * c.nc + kc], q3 = sc[(2 * K + i) * c.nc + kc];
        const float c1 = fmaf(fc, q1.y, q1.x), c2 = fmaf(fc, q2.y, q2.x), c3 = fmaf(fc, q3.y, q3.x);
        const float isk = kIsScale * __builtin_amdgcn_rcpf(c3);
        const float eu = edge_pair<SE>(etab, u, edge_offset<SE>(c2 * c.half_a, isk), isk);
        const float ev = edge_pair<SE>(etab, v, edge_offset<SE>(c2 * c.half_b, isk), isk);
        L = i == 0 ? 0.25f * c1 * eu * ev : fmaf(0.25f * c1 * eu, ev, L);
    }
    return A * L;
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
 * tables, then each wave takes tiles of 64 grid rows; a tile's VOI candidates
 * are flattened across its rows, 64 per chunk, members compacted by ballot.
 * K = unrolled term count; GUARD: stop at P.n_terms (plans of mixed K);
 * SE: mirrored erf table.
 */
template <int K, int W, bool GUARD, bool SURR, bool GEN = false, bool SE = false>
__device__ void fill_beamlet(const PlanDev &P, const OutDev &O, int j, unsigned char *smem)
{
    const BeamletRec &R = P.rec[j];
    const int n_tiles = R.n_tiles;
    if (n_tiles == 0) return;
    constexpr int kB = W * kWave;
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = lane_id();

    // ---- constants into registers
    const int n_table = R.n_table, n_pdd = lds_pdd_pairs(P), tile0 = R.tile0;
    const int iy0 = R.iy0, n_iy = R.n_iy, iz0 = R.iz0, n_rows = R.n_iy * R.n_iz;
    const int nx = P.nx, ny = P.ny, wpr = P.wpr;
    FillConst<K> c;
    c.sad = R.sad_f;
    c.tA = R.tA_f;
    c.inv_step = R.inv_step_f;
    c.tau_max = R.tau_max_f;
    c.pdd_inv = P.pdd_inv_step;
    c.pdd_max = P.pdd_max;
    c.n_terms = P.n_terms;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        c.w4[i] = P.w4[i];
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
    const double tA = R.tA;
    const double t1 = P.sp[0] * R.e[0], u1 = P.sp[0] * R.eu[0], v1 = P.sp[0] * R.ev[0];
    const float t1f = R.t1_f, U1f = R.U1_f, V1f = R.V1_f;
    const gptr<const uint32_t> bits = as_global<const uint32_t>(P.bits);
    const gptr<const int32_t> tile_count = as_global<const int32_t>(P.tile_count);
    const gptr<int32_t> out_idx = as_global<int32_t>(O.indices);
    const gptr<float> out_val = as_global<float>(O.values);
    const int64_t capacity = O.capacity;
    const int64_t row_base = uniform64(O.indptr[j] - O.indptr[O.row0]);

    // ---- LDS: erf table, depth table, depth dose, tile prefix
    float *s_erf = reinterpret_cast<float *>(smem);
    constexpr int kErfFloats = SE ? 2 * kErfLdsFloats : kErfLdsFloats;
    float2 *s_tab = reinterpret_cast<float2 *>(s_erf + kErfFloats);
    float2 *s_pdd = s_tab + P.max_table;
    int *s_tpre = reinterpret_cast<int *>(s_pdd + n_pdd);
    __shared__ int wsum[W];
    // surrogate: per-wave h1 tile after the tile prefix, and W2 fragments in registers
    uint16_t *s_h1 = reinterpret_cast<uint16_t *>(
        smem + ((sizeof(float) * kErfFloats + sizeof(float2) * ((size_t)P.max_table + n_pdd) +
                 sizeof(int) * ((size_t)P.max_tiles + 1) + 15) & ~(size_t)15)) + wave * (64 * mlp::kH1Stride);
    mlp::W2Frags wf;
    if (SURR) mlp::load_w2_frags(P.mlp_w2, wf);
    const float a_f = R.a_f;
    const bool mlp_ok = SURR && R.mlp_ok;

    {
        const float2 *et = P.erf_tab;
        if (SE) {
            // [0, n): erf on [-kErfMax, 0) from the odd symmetry; [n, 2n): the table
            for (int i = tid; i < 2 * kErfIntervals; i += kB) {
                float2 q;
                if (i >= kErfIntervals) {
                    q = et[i - kErfIntervals];
                } else {
                    const float2 m = et[kErfIntervals - 1 - i];
                    q = make_float2(-(m.x + m.y), m.y);
                }
                reinterpret_cast<float2 *>(s_erf)[i] = q;
            }
        } else {
            for (int i = tid; i < kErfIntervals; i += kB) reinterpret_cast<float2 *>(s_erf)[i] = et[i];
        }
        const gptr<const float> tab = as_global<const float>(P.tables + R.table_off);
        for (int i = tid; i < n_table; i += kB) {
            const float d0 = tab[i];
            s_tab[i] = make_float2(d0, (i + 1 < n_table ? tab[i + 1] : d0) - d0);
        }
        if (GEN) {
            // this beamlet's A row (interpolated in theta), then the c tables
            const int na = P.n_adepth, k0 = R.theta_k, k1 = min(R.theta_k + 1, P.n_theta - 1);
            const float ft = R.theta_f;
            const gptr<const float> a0 = as_global<const float>(P.atab + (size_t)k0 * na);
            const gptr<const float> a1 = as_global<const float>(P.atab + (size_t)k1 * na);
            for (int i = tid; i < na; i += kB) {
                const float v0 = fmaf(ft, a1[i] - a0[i], a0[i]);
                const float v1 = i + 1 < na ? fmaf(ft, a1[i + 1] - a0[i + 1], a0[i + 1]) : v0;
                s_pdd[i] = make_float2(v0, v1 - v0);
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
            for (int i = tid; i < n_pdd; i += kB) {
                const float p0 = pd[i];
                s_pdd[i] = make_float2(p0, (i + 1 < n_pdd ? pd[i + 1] : p0) - p0);
            }
        }
    }
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

    for (int tl = wave; tl < n_tiles; tl += W) {
        if (tile_count[tile0 + tl] == 0) continue;
        const int64_t out0 = row_base + __builtin_amdgcn_readfirstlane(s_tpre[tl]);
        // lane = grid row of this tile: its VOI interval and FP32 start values
        const int r = tl * kRowsPerTile + lane;
        int lo = 0, hi = -1, grow = 0;
        float s_lo = 0.0f, U_lo = 0.0f, V_lo = 0.0f;
        if (r < n_rows) {
            const int iy = iy0 + r % n_iy, iz = iz0 + r / n_iy;
            RowAffine a;
            const RowGeom G = row_geom(P, R);
            bool holes;
            if (row_span(G, P.ext, P.nx, P.ny, iy, iz, lo, hi, a, holes)) {
                grow = iz * ny + iy;
                const double x = (double)lo;
                s_lo = (float)(a.t0 + x * t1 - tA);
                U_lo = (float)(a.U0 + x * u1);
                V_lo = (float)(a.V0 + x * v1);
            } else {
                lo = 0;
                hi = -1;
            }
        }
        int cnt = hi - lo + 1;
        {
            // rows with candidates move to the low lanes, in order, empty rows after them
            // (a permutation of the wave), so that row starts are distinct candidates
            const uint64_t ne = __ballot(cnt > 0);
            const int dst = cnt > 0 ? mbcnt64(ne) : __popcll(ne) + mbcnt64(~ne);
            const int a = dst << 2;
            lo = __builtin_amdgcn_ds_permute(a, lo);
            cnt = __builtin_amdgcn_ds_permute(a, cnt);
            grow = __builtin_amdgcn_ds_permute(a, grow);
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
        // one chunk: candidate p of the tile, on row rr of the tile; every lane of the wave calls it
        // a tile whose counted members equal its candidates (no masked voxel inside its rows)
        // takes every candidate: no mask read, and member lanes are the low ones of the chunk
        const bool dense = tile_count[tile0 + tl] == total;
        auto chunk = [&](const int p, const int rr, auto dense_tag) {
            constexpr bool DENSE = decltype(dense_tag)::value;
            const int k = p - __shfl(excl, rr, kWave);
            const int ix = __shfl(lo, rr, kWave) + k;
            const int gr = __shfl(grow, rr, kWave);
            bool member = false;
            if (DENSE) {
                member = p < total;
            } else if (p < total) {
                const uint32_t wo = ((uint32_t)(gr * wpr) + ((uint32_t)ix >> 5)) << 2;   // byte offset
                member = (*(const gptr<const uint32_t>)((gptr<const char>)bits + wo) >> (ix & 31)) & 1u;
            }
            const uint64_t mask = __ballot(member);
            const uint32_t slot = DENSE ? (uint32_t)lane : (uint32_t)mbcnt64(mask);
            const float sl = __shfl(s_lo, rr, kWave);
            const float ul = __shfl(U_lo, rr, kWave);
            const float vl = __shfl(V_lo, rr, kWave);
            // this chunk's entries go to [written, written + popcount); the bases are wave-uniform
            const gptr<char> ip = (gptr<char>)(out_idx + written);
            const gptr<char> vp = (gptr<char>)(out_val + written);
            // slots below `avail` fit in the caller's arrays (scalar: no 64-bit compare per lane)
            const int64_t left = capacity - written;
            const uint32_t avail = left >= kWave ? (uint32_t)kWave : (left > 0 ? (uint32_t)left : 0u);
            float D = 0.0f;
            if (SURR) {
                // the network runs on all 64 lanes (matrix cores need the whole wave)
                const float kf = (float)k;
                const float sv = fmaf(kf, t1f, sl), Uv = fmaf(kf, U1f, ul), Vv = fmaf(kf, V1f, vl);
                const float g = c.sad * __builtin_amdgcn_rcpf(sv + c.tA);
                const float au = fabsf(Uv * g), av = fabsf(Vv * g);
                const float tau = __builtin_amdgcn_fmed3f(sv * c.inv_step, 0.0f, c.tau_max);
                const float2 q = s_tab[(int)tau];
                const float d = fmaf(__builtin_amdgcn_fractf(tau), q.y, q.x);
                const bool in_box = member && mlp_ok && d <= kMlpDMax && au <= kMlpUVMax &&
                                    av <= kMlpUVMax;
                float x[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                if (in_box) mlp::features(d, au, av, a_f, x);
                const float y = mlp::forward_wave(P.mlp_p, wf, x, s_h1);
                if (in_box) D = y * g * g;
                else if (member) D = dose_value<K, GUARD, SE>(c, s_tab, s_pdd, s_erf, sv, Uv, Vv);
            }
            if (member) {
                const float kf = (float)k;
                if (GEN)
                    D = dose_value_gen<K, SE>(c, s_tab, s_pdd, s_pdd + P.n_adepth, s_erf, fmaf(kf, t1f, sl),
                                          fmaf(kf, U1f, ul), fmaf(kf, V1f, vl));
                else if (!SURR)
                    D = dose_value<K, GUARD, SE>(c, s_tab, s_pdd, s_erf, fmaf(kf, t1f, sl), fmaf(kf, U1f, ul),
                                             fmaf(kf, V1f, vl));
                if (slot < avail) {
                    *(gptr<int32_t>)(ip + (slot << 2)) = gr * nx + ix;
                    *(gptr<float>)(vp + (slot << 2)) = D;
                } else {
                    *O.overflow = 1;
                }
            }
            written += __popcll(mask);
        };
        auto walk2 = [&](auto dense_tag) {
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
                chunk(c0 + lane, r1, dense_tag);
                chunk(c0 + kWave + lane, r2, dense_tag);
                rcur = rnext;
            }
        };
        if (!SURR) {
            if (dense) walk2(std::true_type{});
            else walk2(std::false_type{});
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
                chunk(p, rr, std::false_type{});
            }
        }
    }
}

template <int K, bool SURR, bool GEN, bool SE>
__global__ __launch_bounds__(kBlock) void k_fill(const PlanDev *__restrict__ plans,
                                                  const OutDev *__restrict__ outs)
{
    extern __shared__ __align__(16) unsigned char smem[];
    // launched before the host has read the plan's total: write nothing if it does not fit
    if (outs[0].check_nnz && *plans[0].nnz > outs[0].capacity) return;
    fill_beamlet<K, kWavesPerBlock, false, SURR, GEN, SE>(plans[0], outs[0], outs[0].row0 + (int)blockIdx.x, smem);
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

template <int K, int W>
__global__ __launch_bounds__(W * kWave) __attribute__((amdgpu_waves_per_eu(4))) void kp_fill(const PlanDev *const *__restrict__ plans,
                                                     const OutDev *__restrict__ outs,
                                                     const int2 *__restrict__ items, int n_items,
                                                     int *__restrict__ counter)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int w = s_item;
        __syncthreads();
        if (w >= n_items) break;
        const int2 it = items[w];
        const PlanDev &P = *plans[it.x];
        // each plan in the erf table form of its own fill (identical results to it)
        if (P.erf_mirrored && !P.use_mlp) fill_beamlet<K, W, true, false, false, true>(P, outs[it.x], it.y, smem);
        else fill_beamlet<K, W, true, false>(P, outs[it.x], it.y, smem);
        __syncthreads();
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
    size_t b = sizeof(float) * (mirrored_erf ? 2 * kErfLdsFloats : kErfLdsFloats) + sizeof(float2) * ((size_t)h.max_table + (size_t)lds_pdd_pairs(h)) +
               sizeof(int) * ((size_t)h.max_tiles + 1);
    if (h.use_mlp) b = ((b + 15) & ~(size_t)15) + sizeof(uint16_t) * 64 * mlp::kH1Stride * kWavesPerBlock;
    return b;
}

size_t fill_shared_bytes(const PlanDev &h)
{
    return fill_shared_bytes(h, fill_mirrored_erf(h));
}

bool fill_mirrored_erf(const PlanDev &h) { return h.erf_mirrored && !h.use_mlp; }

template <bool GEN>
static const void *fill_kernel_ptr(int K, bool se)
{
    switch (K) {
    case 1: return se ? (const void *)k_fill<1, false, GEN, true> : (const void *)k_fill<1, false, GEN, false>;
    case 2: return se ? (const void *)k_fill<2, false, GEN, true> : (const void *)k_fill<2, false, GEN, false>;
    case 3: return se ? (const void *)k_fill<3, false, GEN, true> : (const void *)k_fill<3, false, GEN, false>;
    default: return se ? (const void *)k_fill<4, false, GEN, true> : (const void *)k_fill<4, false, GEN, false>;
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
    const void *fm = h.gen ? fill_kernel_ptr<true>(h.n_terms, true) : fill_kernel_ptr<false>(h.n_terms, true);
    const void *fs = h.gen ? fill_kernel_ptr<true>(h.n_terms, false) : fill_kernel_ptr<false>(h.n_terms, false);
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
                                   int n_items, int *counter, int grid, size_t lds, hipStream_t s)
{
    const dim3 g(grid);
    switch (W) {
    case 2: hipLaunchKernelGGL((kp_fill<K, 2>), g, dim3(2 * kWave), lds, s, plans, outs, items, n_items, counter); break;
    case 8: hipLaunchKernelGGL((kp_fill<K, 8>), g, dim3(8 * kWave), lds, s, plans, outs, items, n_items, counter); break;
    default: hipLaunchKernelGGL((kp_fill<K, 4>), g, dim3(4 * kWave), lds, s, plans, outs, items, n_items, counter); break;
    }
    return hipGetLastError();
}

hipError_t launch_batch_fill(int K, int W, const PlanDev *const *plans, const OutDev *outs, const int2 *items,
                             int n_items, int *counter, int grid, size_t lds, hipStream_t s)
{
    switch (K) {
    case 1: return launch_kp_fill_k<1>(W, plans, outs, items, n_items, counter, grid, lds, s);
    case 2: return launch_kp_fill_k<2>(W, plans, outs, items, n_items, counter, grid, lds, s);
    case 3: return launch_kp_fill_k<3>(W, plans, outs, items, n_items, counter, grid, lds, s);
    default: return launch_kp_fill_k<4>(W, plans, outs, items, n_items, counter, grid, lds, s);
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
        case 1: hipLaunchKernelGGL((k_fill<1, true, false, false>), grid, block, lds, s, dplan, dout); break;
        case 2: hipLaunchKernelGGL((k_fill<2, true, false, false>), grid, block, lds, s, dplan, dout); break;
        case 3: hipLaunchKernelGGL((k_fill<3, true, false, false>), grid, block, lds, s, dplan, dout); break;
        default: hipLaunchKernelGGL((k_fill<4, true, false, false>), grid, block, lds, s, dplan, dout); break;
        }
        return hipGetLastError();
    }
    const void *f = h.gen ? fill_kernel_ptr<true>(h.n_terms, fill_mirrored_erf(h))
                          : fill_kernel_ptr<false>(h.n_terms, fill_mirrored_erf(h));
    void *args[] = {const_cast<PlanDev **>(&dplan), const_cast<OutDev **>(&dout)};
    return hipLaunchKernel(f, grid, block, args, lds, s);
}

}  // namespace fspb
