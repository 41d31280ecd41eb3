/*
 * gfx950 kernels for Eq. 1 on the dose-coefficient matrix D_ij.
 *
 *   beamlet-row CSR (what the fill writes: row j = beamlet, columns = voxels)
 *     k_fluence_dose      dose_i += w_j D_ij with FP32 atomics   -- one wave per row
 *     k_fluence_gradient  g_j = sum_i D_ij r_i, fixed order      -- one workgroup per row
 *   voxel-row CSR (row i = voxel, columns = beamlets): the transpose, a stable
 *   sort of the row-major entries by column
 *     k_run_count, scan, k_run_sizes   runs of each row (stretches within one
 *                                      32-column bucket), their pointers, the
 *                                      path flags
 *     run path (the default for D, whose rows are long stretches of columns):
 *       k_run_emit                     run records: bucket, row, first entry and a
 *                                      32-bit column mask (ascending rows) or length
 *       k_rs_hist, scan, k_rs_scatter  stable LSD radix sort of the runs by bucket
 *       k_bucket_bounds                bucket pointers
 *       rows ascending:   scan of the lengths, k_place_sorted -- one wave per
 *                         bucket: column counts from the masks (the voxel-row
 *                         pointers), batches reordered in LDS and written out
 *       rows in any order: k_key_count + scan (pointers), k_place_any
 *     entry path (short stretches): k_key_count + scan, k_expand_rows, then
 *       k_rs_hist, scan, k_rs_scatter per 8 bits of the column
 *     k_voxel_dose        dose_i = sum_j D_ij w_j, fixed order  -- 16 lanes per voxel row
 *
 * Both sorts are stable and the input rows are in ascending beamlet order, so
 * every voxel row lists its beamlets in ascending order: the transpose is
 * canonical and bit-reproducible.  It runs without host synchronisation.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "fspb_device.h"

namespace fspb {

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;          // digits per pass; one thread per digit
constexpr int kSortItems = 16;                   // items per thread per tile
constexpr int kSortTile = kBlock * kSortItems;   // 4096 entries per sort tile
constexpr int kScanItems = 16;
constexpr int kScanChunk = kBlock * kScanItems;  // 4096 values per scan block
constexpr int kScanTop = 1024;

static_assert(kRadix == kBlock, "one thread per digit");

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ inline int mbcnt64(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <typename T>
__device__ inline T wave_sum(T x)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

/*
 * Inclusive scan of a wave's 32-bit integers by DPP: row shifts by 1, 2, 4 and
 * 8 lanes scan each row of 16 lanes (lanes shifted in from outside the row read
 * 0); rows 1 and 3 then add the last lane of the row below (row_bcast:15) and
 * rows 2 and 3 add lane 31 (row_bcast:31).  Every lane of the wave must be
 * active.
 */
__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return (uint32_t)x;
}

/* Wave total of 32-bit integers (every lane active), the same on every lane. */
__device__ inline uint32_t wave_sum(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(x), kWave - 1);
}

/* Exclusive scan of one value per thread over the block; *total gets the sum. */
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *s_w, uint32_t *total)
{
    const int l = lane_id(), w = threadIdx.x >> 6;
    uint32_t x = wave_incl_scan(v);
    if (l == kWave - 1) s_w[w] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kWavesPerBlock; ++k) {
        const uint32_t t = s_w[k];
        off += k < w ? t : 0u;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

/* ------------------------------------------------------------ Eq. 1 */

__global__ __launch_bounds__(kBlock) void k_zero(float *__restrict__ x, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = 0.0f;
}

__global__ __launch_bounds__(kBlock) void k_zero_u32(uint32_t *__restrict__ x, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = 0u;
}

/* dose[i] += w_j D_ij over row j; one wave per row.  Columns outside
 * [0, n_voxels) are skipped. */
__global__ __launch_bounds__(kBlock) void k_fluence_dose(const int64_t *__restrict__ indptr,
                                                         const int32_t *__restrict__ indices,
                                                         const float *__restrict__ values, int n_rows,
                                                         int n_voxels, const float *__restrict__ w,
                                                         float *__restrict__ dose)
{
    const int j = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (j >= n_rows) return;
    const float wj = w[j];
    if (wj == 0.0f) return;
    const int64_t e1 = indptr[j + 1];
    int64_t e = indptr[j] + lane_id();
    // four entries per lane in flight, then the tail
    for (; e + 3 * kWave < e1; e += 4 * kWave) {
        uint32_t i[4];
        float v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            i[k] = (uint32_t)indices[e + k * kWave];
            v[k] = values[e + k * kWave];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i[k] < (uint32_t)n_voxels) atomicAdd(dose + i[k], wj * v[k]);
    }
    for (; e < e1; e += kWave) {
        const uint32_t i = (uint32_t)indices[e];
        if (i < (uint32_t)n_voxels) atomicAdd(dose + i, wj * values[e]);
    }
}

/*
 * Entries [e0, e1) of a CSR row split for 16-byte loads: [e0, a) head, [a, b) whole
 * steps of `step` entries (4 consecutive per lane), [b, e1) tail; the head is
 * shorter than 4 entries.  Only when indices and values have the same offset
 * modulo 16 bytes; otherwise head and steps are empty and the whole row is tail.
 */
struct RowSplit { int64_t a, b; };

__device__ inline RowSplit row_split(const int32_t *indices, const float *values, int64_t e0, int64_t e1,
                                     int step)
{
    const uintptr_t oi = (uintptr_t)indices, ov = (uintptr_t)values;
    if ((oi & 3) || (ov & 3) || ((oi ^ ov) & 15)) return {e0, e0};
    const int64_t mis = (int64_t)((oi >> 2) & 3);          // element offset of the array modulo 4
    const int64_t a = min(e1, ((e0 + mis + 3) & ~(int64_t)3) - mis);
    return {a, a + (e1 - a) / step * step};
}

typedef int vi4 __attribute__((ext_vector_type(4)));
typedef float vf4 __attribute__((ext_vector_type(4)));

/*
 * g_j = sum_i D_ij r_i; one workgroup per row.  The row's middle goes in steps
 * of 4 kBlock entries: lane l of wave w takes entries 256 w + l + 64 k
 * (k < 4) of a step, so that each gather of r reads 64 consecutive columns;
 * the next step's indices and values are loaded (non-temporal: streamed once,
 * kept from displacing r in the caches) after this step's gathers are issued,
 * so they are in flight while the gathered values are awaited.  The tail is
 * lane-strided; lane partial sums, a fixed butterfly per wave and the wave
 * totals added in wave order.  Columns outside [0, n_voxels) are skipped.
 */
__global__ __launch_bounds__(kBlock) void k_fluence_gradient(const int64_t *__restrict__ indptr,
                                                             const int32_t *__restrict__ indices,
                                                             const float *__restrict__ values, int n_rows,
                                                             int n_voxels, const float *__restrict__ r,
                                                             float *__restrict__ g)
{
    constexpr int kStep = 4 * kBlock;
    __shared__ float s_w[kWavesPerBlock];
    const int j = blockIdx.x;
    const int t = threadIdx.x;
    const uint32_t n = (uint32_t)n_voxels;
    const int64_t e0 = indptr[j], e1 = indptr[j + 1];
    // whole steps from the row's start (4-byte loads need no alignment), then the tail
    const int64_t b = e0 + (e1 - e0) / kStep * kStep;
    float acc0 = 0.0f, acc1 = 0.0f;
    if (e0 < b) {   // the same for the whole workgroup, as is every step test below
        int64_t e = e0 + 4 * kWave * (t >> 6) + (t & (kWave - 1));
        uint32_t i0[4];
        float v0[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            i0[k] = (uint32_t)__builtin_nontemporal_load(indices + e + kWave * k);
            v0[k] = __builtin_nontemporal_load(values + e + kWave * k);
        }
        for (;;) {
            const int64_t en = e + kStep;
            float x[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) x[k] = i0[k] < n ? r[i0[k]] : 0.0f;
            uint32_t i1[4];
            float v1[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                i1[k] = i0[k];
                v1[k] = v0[k];
            }
            if (en < b) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    i1[k] = (uint32_t)__builtin_nontemporal_load(indices + en + kWave * k);
                    v1[k] = __builtin_nontemporal_load(values + en + kWave * k);
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (i0[k] < n) acc0 = fmaf(v0[k], x[k], acc0);
            if (en >= b) break;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                i0[k] = i1[k];
                v0[k] = v1[k];
            }
            e = en;
        }
    }
    for (int64_t q = b + t; q < e1; q += kBlock) {
        const uint32_t i = (uint32_t)indices[q];
        if (i < n) acc1 = fmaf(values[q], r[i], acc1);
    }
    const float s = wave_sum(acc0 + acc1);
    if (lane_id() == 0) s_w[t >> 6] = s;
    __syncthreads();
    if (t == 0) {
        float tot = s_w[0];
        for (int k = 1; k < kWavesPerBlock; ++k) tot += s_w[k];
        g[j] = tot;
    }
}

/* dose_i = sum_j D_ij w_j over voxel row i: 16 lanes per row, 16-byte loads of
 * four consecutive entries per lane, the next step's loads in flight while
 * this step's gathers of w are awaited; lane-strided partial sums and a fixed
 * 16-lane butterfly.  Beamlets outside [0, n_w) are skipped. */
__global__ __launch_bounds__(kBlock) void k_voxel_dose(const int64_t *__restrict__ t_indptr,
                                                       const int32_t *__restrict__ t_indices,
                                                       const float *__restrict__ t_values, int n_voxels, int n_w,
                                                       const float *__restrict__ w, float *__restrict__ dose)
{
    const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 4;
    const int l = threadIdx.x & 15;
    const uint32_t n = (uint32_t)n_w;
    float acc0 = 0.0f, acc1 = 0.0f;
    if (i < n_voxels) {
        // 16-byte loads of four consecutive entries per lane (64 per step), head and tail lane-strided
        const int64_t e0 = t_indptr[i], e1 = t_indptr[i + 1];
        const RowSplit sp = row_split(t_indices, t_values, e0, e1, 64);
        if (e0 + l < sp.a) {
            const uint32_t j = (uint32_t)t_indices[e0 + l];
            if (j < n) acc0 = fmaf(t_values[e0 + l], w[j], acc0);
        }
        // the next step's indices and values are loaded after this step's gathers of w are
        // issued (non-temporal: streamed once), so they are in flight while those are awaited
        int64_t e = sp.a + 4 * l;
        if (e < sp.b) {
            vi4 a = __builtin_nontemporal_load(reinterpret_cast<const vi4 *>(t_indices + e));
            vf4 c = __builtin_nontemporal_load(reinterpret_cast<const vf4 *>(t_values + e));
            for (;;) {
                const int64_t en = e + 64;
                float x0 = 0.0f, x1 = 0.0f, x2 = 0.0f, x3 = 0.0f;
                if ((uint32_t)a.x < n) x0 = w[(uint32_t)a.x];
                if ((uint32_t)a.y < n) x1 = w[(uint32_t)a.y];
                if ((uint32_t)a.z < n) x2 = w[(uint32_t)a.z];
                if ((uint32_t)a.w < n) x3 = w[(uint32_t)a.w];
                vi4 a1 = a;
                vf4 c1 = c;
                if (en < sp.b) {
                    a1 = __builtin_nontemporal_load(reinterpret_cast<const vi4 *>(t_indices + en));
                    c1 = __builtin_nontemporal_load(reinterpret_cast<const vf4 *>(t_values + en));
                }
                if ((uint32_t)a.x < n) acc1 = fmaf(c.x, x0, acc1);
                if ((uint32_t)a.y < n) acc1 = fmaf(c.y, x1, acc1);
                if ((uint32_t)a.z < n) acc1 = fmaf(c.z, x2, acc1);
                if ((uint32_t)a.w < n) acc1 = fmaf(c.w, x3, acc1);
                if (en >= sp.b) break;
                a = a1;
                c = c1;
                e = en;
            }
        }
        for (int64_t e = sp.b + l; e < e1; e += 16) {
            const uint32_t j = (uint32_t)t_indices[e];
            if (j < n) acc0 = fmaf(t_values[e], w[j], acc0);
        }
    }
    float s = acc0 + acc1;
#pragma unroll
    for (int d = 8; d > 0; d >>= 1) s += __shfl_xor(s, d, kWave);
    if (l == 0 && i < n_voxels) dose[i] = s;
}

/* ------------------------------------------------------------ transpose */

/*
 * The transpose never synchronises the host: both of its sort paths are
 * enqueued, and a flag the device computes from the data (how long the
 * stretches of each row within a bucket of columns are) lets one of them run;
 * the other's kernels return at once.  Sizes only the device knows (the number
 * of stretches) are read by the kernels themselves, which walk their work
 * grid-stride from a grid sized by a host bound.
 */
struct Gate {
    const int32_t *flag;   // nullptr: always run
    int32_t want;
};
__device__ inline bool gate_closed(Gate g) { return g.flag && *g.flag != g.want; }

/* An element count known on the host (dev == nullptr) or read from device memory. */
struct Count {
    int64_t n;
    const int64_t *dev;
};
__device__ inline int64_t count_of(Count c) { return c.dev ? *c.dev : c.n; }

/* rows[e] = j for every entry e of row j (clamped to [0, nnz)); one wave per row. */
__global__ __launch_bounds__(kBlock) void k_expand_rows(const int64_t *__restrict__ indptr, int n_rows, int64_t nnz,
                                                        int32_t *__restrict__ rows, Gate g)
{
    if (gate_closed(g)) return;
    const int j = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (j >= n_rows) return;
    const int64_t e0 = indptr[j] > 0 ? indptr[j] : 0, e1 = indptr[j + 1] < nnz ? indptr[j + 1] : nnz;
    for (int64_t e = e0 + lane_id(); e < e1; e += kWave) rows[e] = j;
}

/* Scan, phase 1: sum of each kScanChunk-value chunk (grid-stride over chunks); with
 * POPC the values scanned are the popcounts of the inputs (here and in phase 3). */
template <bool POPC>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t *__restrict__ in, Count n_in,
                                                        uint32_t *__restrict__ partial, Gate g)
{
    if (gate_closed(g)) return;
    __shared__ uint32_t s_w[kWavesPerBlock];
    const int64_t n = count_of(n_in), nch = (n + kScanChunk - 1) / kScanChunk;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const int64_t base = c * kScanChunk + (int64_t)threadIdx.x * kScanItems;
        uint32_t v = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const uint32_t x = base + k < n ? in[base + k] : 0u;
            v += POPC ? (uint32_t)__popc(x) : x;
        }
        v = wave_sum(v);
        if (lane_id() == 0) s_w[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
            for (int k = 0; k < kWavesPerBlock; ++k) t += s_w[k];
            partial[c] = t;
        }
        __syncthreads();
    }
}

/* Scan, phase 2: exclusive scan of the chunk sums in place (one workgroup);
 * partial[nb] = total, also stored to *total64 when given. */
__global__ __launch_bounds__(kScanTop) void k_scan_top(uint32_t *__restrict__ partial, Count n_in,
                                                       int64_t *__restrict__ total64, Gate g)
{
    if (gate_closed(g)) return;
    __shared__ uint32_t s_w[kScanTop / kWave];
    const int64_t nb = (count_of(n_in) + kScanChunk - 1) / kScanChunk;
    const int l = lane_id(), w = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanTop) {
        const int64_t i = b0 + threadIdx.x;
        const uint32_t v = i < nb ? partial[i] : 0u;
        uint32_t x = wave_incl_scan(v);
        if (l == kWave - 1) s_w[w] = x;
        __syncthreads();
        uint32_t off = 0, tot = 0;
        for (int k = 0; k < kScanTop / kWave; ++k) {
            off += k < w ? s_w[k] : 0u;
            tot += s_w[k];
        }
        if (i < nb) partial[i] = carry + off + x - v;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[nb] = carry;
        if (total64) *total64 = (int64_t)carry;
    }
}

/* Scan, phase 3: exclusive (INCL: inclusive) scan within each chunk plus its chunk
 * offset (grid-stride); out may be in (each chunk is read before it is written). */
template <typename OUT, bool INCL, bool POPC>
__global__ __launch_bounds__(kBlock) void k_scan_down(const uint32_t *in, Count n_in, const uint32_t *__restrict__ partial,
                                                      OUT *out, Gate g)
{
    if (gate_closed(g)) return;
    __shared__ uint32_t s_w[kWavesPerBlock];
    const int64_t n = count_of(n_in), nch = (n + kScanChunk - 1) / kScanChunk;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const int64_t base = c * kScanChunk + (int64_t)threadIdx.x * kScanItems;
        uint32_t v[kScanItems];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = base + k < n ? in[base + k] : 0u;
            if (POPC) v[k] = (uint32_t)__popc(v[k]);
            sum += v[k];
        }
        uint32_t total;
        uint32_t run = partial[c] + block_excl_scan(sum, s_w, &total);
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            run += INCL ? v[k] : 0u;
            if (base + k < n) out[base + k] = (OUT)run;
            run += INCL ? 0u : v[k];
        }
    }
}

/* Radix pass, phase 1: digit histogram of each kSortTile-entry tile, stored
 * digit-major (hist[d * n_tiles + tile]) so that one exclusive scan gives every
 * (digit, tile) its first output slot.  Keys above `clamp` count as `clamp`
 * (the sentinel that sorts entries with an invalid column last). */
__global__ __launch_bounds__(kBlock) void k_rs_hist(const uint32_t *__restrict__ keys, Count n_in, uint32_t clamp,
                                                    int shift, uint32_t *__restrict__ hist, Gate g)
{
    if (gate_closed(g)) return;
    __shared__ uint32_t h[kRadix];
    const int64_t n = count_of(n_in), n_tiles = (n + kSortTile - 1) / kSortTile;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        h[threadIdx.x] = 0u;
        __syncthreads();
        const int64_t base = tile * kSortTile + threadIdx.x;
#pragma unroll 4
        for (int r = 0; r < kSortItems; ++r) {
            const int64_t i = base + (int64_t)r * kBlock;
            if (i < n) atomicAdd(&h[(min(keys[i], clamp) >> shift) & (kRadix - 1)], 1u);
        }
        __syncthreads();
        hist[(int64_t)threadIdx.x * n_tiles + tile] = h[threadIdx.x];
        __syncthreads();
    }
}

/*
 * Radix pass, phase 2: stable scatter (of a fourth uint32 payload too with XTRA).  Wave w of a block owns the w-th
 * quarter of the tile (kSortItems rounds of 64 consecutive entries) and
 * ranks it on its own: in a round, ballots on the 8 digit bits group the
 * lanes holding the same digit, a lane's rank is the number of lower peers,
 * and the wave's per-digit counter in LDS (read by the group, advanced by its
 * lowest lane) orders the rounds.  The entries stay in registers; one block
 * scan turns the waves' counts into tile-local slots (digit-major, lower
 * waves first), the tile is sorted by digit in LDS and written out in that
 * order, so each digit's run goes to consecutive addresses.  keys_out may be
 * NULL (last pass).  Grid-stride over the tiles.
 */
template <bool XTRA>
__global__ __launch_bounds__(kBlock) void k_rs_scatter(const uint32_t *__restrict__ keys_in,
                                                       const int32_t *__restrict__ rows_in,
                                                       const float *__restrict__ vals_in,
                                                       const uint32_t *__restrict__ xs_in, Count n_in, uint32_t clamp,
                                                       int shift, const uint32_t *__restrict__ offs,
                                                       uint32_t *__restrict__ keys_out,
                                                       int32_t *__restrict__ rows_out,
                                                       float *__restrict__ vals_out, uint32_t *__restrict__ xs_out,
                                                       Gate g)
{
    if (gate_closed(g)) return;
    __shared__ uint32_t s_key[kSortTile];
    __shared__ int32_t s_row[kSortTile];
    __shared__ float s_val[kSortTile];
    __shared__ uint32_t s_x[XTRA ? kSortTile : 1];
    __shared__ uint32_t cnt[kWavesPerBlock][kRadix];   // per wave: digit counts, then first tile-local slot
    __shared__ uint32_t goff[kRadix];                  // global slot of tile-local slot 0 of each digit's run
    __shared__ uint32_t s_w[kWavesPerBlock];
    constexpr int kSub = kSortTile / kWavesPerBlock;    // entries per wave
    const int t = threadIdx.x, wave = t >> 6, lane = t & (kWave - 1);
    const int64_t n = count_of(n_in), n_tiles = (n + kSortTile - 1) / kSortTile;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t tile0 = tile * kSortTile;
        const int64_t sub0 = tile0 + (int64_t)wave * kSub;
#pragma unroll
        for (int w = 0; w < kWavesPerBlock; ++w) cnt[w][t] = 0u;
        __syncthreads();

        uint32_t key[kSortItems], pos[kSortItems], xv[kSortItems];
        int32_t row[kSortItems];
        float val[kSortItems];
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const int64_t i = sub0 + (int64_t)r * kWave + lane;
            const bool valid = i < n;
            key[r] = valid ? min(keys_in[i], clamp) : 0u;
            row[r] = valid ? rows_in[i] : 0;
            val[r] = valid ? vals_in[i] : 0.0f;
            xv[r] = (XTRA && valid) ? xs_in[i] : 0u;
            const uint32_t d = (key[r] >> shift) & (kRadix - 1);
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < kRadixBits; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            const uint32_t rank = (uint32_t)mbcnt64(peers);
            uint32_t before = 0u;
            if (valid) before = cnt[wave][d];                 // every lane of the group reads the old count
            if (valid && rank == 0) cnt[wave][d] = before + (uint32_t)__popcll(peers);
            pos[r] = before + rank;
        }
        __syncthreads();
        {
            // thread t = digit t: tile-local start of the digit, then of each wave's part of it
            uint32_t c[kWavesPerBlock], tot = 0;
#pragma unroll
            for (int w = 0; w < kWavesPerBlock; ++w) {
                c[w] = cnt[w][t];
                tot += c[w];
            }
            uint32_t total;
            const uint32_t start = block_excl_scan(tot, s_w, &total);
            uint32_t b = start;
#pragma unroll
            for (int w = 0; w < kWavesPerBlock; ++w) {
                cnt[w][t] = b;
                b += c[w];
            }
            goff[t] = offs[(int64_t)t * n_tiles + tile] - start;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const int64_t i = sub0 + (int64_t)r * kWave + lane;
            if (i < n) {
                const uint32_t lp = cnt[wave][(key[r] >> shift) & (kRadix - 1)] + pos[r];
                s_key[lp] = key[r];
                s_row[lp] = row[r];
                s_val[lp] = val[r];
                if (XTRA) s_x[lp] = xv[r];
            }
        }
        __syncthreads();
        const int64_t rem = n - tile0;
        const int m = rem < kSortTile ? (int)rem : kSortTile;
        for (int lp = t; lp < m; lp += kBlock) {
            const uint32_t key_ = s_key[lp];
            const uint32_t p = goff[(key_ >> shift) & (kRadix - 1)] + (uint32_t)lp;
            if (keys_out) keys_out[p] = key_;
            rows_out[p] = s_row[lp];
            vals_out[p] = s_val[lp];
            if (XTRA) xs_out[p] = s_x[lp];
        }
        __syncthreads();
    }
}

}  // namespace

static inline unsigned blocks_of(int64_t items, int per_block)
{
    return (unsigned)((items + per_block - 1) / per_block);
}

hipError_t launch_fluence_dose(const int64_t *indptr, const int32_t *indices, const float *values, int n_rows,
                               int n_voxels, const float *w, float *dose, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero, dim3(blocks_of(n_voxels, kBlock)), dim3(kBlock), 0, s, dose, (int64_t)n_voxels);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_rows == 0) return e;
    hipLaunchKernelGGL(k_fluence_dose, dim3(blocks_of(n_rows, kWavesPerBlock)), dim3(kBlock), 0, s, indptr, indices,
                       values, n_rows, n_voxels, w, dose);
    return hipGetLastError();
}

hipError_t launch_fluence_gradient(const int64_t *indptr, const int32_t *indices, const float *values, int n_rows,
                                   int n_voxels, const float *r, float *g, hipStream_t s)
{
    if (n_rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fluence_gradient, dim3(n_rows), dim3(kBlock), 0, s, indptr,
                       indices, values, n_rows, n_voxels, r, g);
    return hipGetLastError();
}

hipError_t launch_voxel_dose(const int64_t *t_indptr, const int32_t *t_indices, const float *t_values, int n_voxels,
                             int n_w, const float *w, float *dose, hipStream_t s)
{
    hipLaunchKernelGGL(k_voxel_dose, dim3(blocks_of((int64_t)n_voxels * 16, kBlock)), dim3(kBlock), 0, s, t_indptr,
                       t_indices, t_values, n_voxels, n_w, w, dose);
    return hipGetLastError();
}

namespace {

/*
 * Run transpose.  A run is a maximal stretch of consecutive entries of one row
 * whose columns share a bucket of kBucketCols columns (col >> kBucketShift);
 * entries whose column lies outside [0, n_voxels) form runs of their own,
 * flagged (row id with its top bit set) and never placed.  The runs are
 * sorted by bucket (stably, so a bucket's runs keep row order) and the
 * entries of each bucket are then placed by one wave, in that order, with a
 * stable counting sort on the column's low bits: the output is the stable sort
 * of the row-major entries by column, as the radix path gives.
 *
 * When every row's columns ascend strictly (a plan's D) a run holds at most
 * one entry per column of its bucket, so a 32-bit mask of its columns
 * describes it: its length is the mask's popcount, its k-th entry lies in the
 * column of the mask's k-th set bit, and the entries of a bucket that fall in
 * column c are counted by popcounts of masks.  The placement then reads only
 * the values, and the voxel-row pointers come from the bucket counts.
 */
constexpr int kBucketShift = 5;
constexpr int kBucketCols = 1 << kBucketShift;
constexpr uint32_t kRunFlag = 0x80000000u;   // run of invalid columns (in the run's row id)
constexpr int kRowChunks = 4;                // chunks of 64 entries whose loads are in flight together
constexpr int kXcds = 8;                     // workgroups are handed to the 8 XCDs in turn

/* Value of the lane below (above), through a whole-wave DPP shift; lane 0 (63) takes `edge`. */
__device__ inline int from_lane_below(int v, int edge) { return __builtin_amdgcn_update_dpp(edge, v, 0x138, 0xf, 0xf, false); }
__device__ inline int from_lane_above(int v, int edge) { return __builtin_amdgcn_update_dpp(edge, v, 0x130, 0xf, 0xf, false); }

/* Run key of a column: its bucket, or -2 (outside [0, n_voxels)). */
__device__ inline int run_key(int col, int n_voxels)
{
    return (uint32_t)col < (uint32_t)n_voxels ? (col >> kBucketShift) : -2;
}

/* Flags the transpose computes on the device (one 64-byte slot of the workspace). */
struct Flags {
    int32_t unsorted;      // some row's columns do not ascend strictly
    int32_t use_runs;      // runs are at most half the entries: a run path
    int64_t hist_len;      // digit-histogram length of the run sort
    int32_t need_counts;   // entries per column counted by atomics (entry path, unsorted rows)
    int32_t sorted;        // run path with masks (rows ascending)
    int32_t any;           // run path for rows in any column order
    int32_t pad;
    int64_t total;         // placed entries (sorted run path)
};

/* counts[k] += 1 for every key k in [0, n_valid) among the first n keys; other keys are skipped. */
__global__ __launch_bounds__(kBlock) void k_key_count(const int32_t *__restrict__ keys, int64_t n, int n_valid,
                                                      uint32_t *__restrict__ counts, Gate g)
{
    if (gate_closed(g)) return;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += stride) {
        const uint32_t i = (uint32_t)keys[e];
        if (i < (uint32_t)n_valid) atomicAdd(counts + i, 1u);
    }
}

/* Per row (one wave, kRowChunks chunks of 64 entries loaded together): the
 * number of runs (run_cnt[j]), and the unsorted flag when the row's columns do
 * not ascend strictly. */
__global__ __launch_bounds__(kBlock) void k_run_count(const int64_t *__restrict__ indptr,
                                                      const int32_t *__restrict__ indices, int n_rows, int n_voxels,
                                                      uint32_t *__restrict__ run_cnt, Flags *__restrict__ fl)
{
    const int j = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (j >= n_rows) return;
    const int lane = lane_id();
    const int64_t e0 = indptr[j], e1 = indptr[j + 1];
    uint32_t runs = 0;
    int prev_col = 0, prev_k = -1;                     // entry before the chunk (key -1: none)
    bool down = false;
    for (int64_t c = e0; c < e1; c += kRowChunks * kWave) {
        int cols[kRowChunks];
#pragma unroll
        for (int u = 0; u < kRowChunks; ++u) {
            const int64_t e = c + u * kWave + lane;
            cols[u] = e < e1 ? indices[e] : 0;
        }
#pragma unroll
        for (int u = 0; u < kRowChunks; ++u) {
            const int64_t e = c + u * kWave + lane;
            const bool in = e < e1;
            const int col = cols[u];
            const int k = in ? run_key(col, n_voxels) : -3;
            const int cp = from_lane_below(col, prev_col), kp = from_lane_below(k, prev_k);
            runs += (uint32_t)__popcll(__ballot(in && k != kp));
            down = down || (in && kp != -1 && col <= cp);
            prev_col = __builtin_amdgcn_readlane(col, kWave - 1);
            prev_k = __builtin_amdgcn_readlane(k, kWave - 1);
        }
    }
    if (lane == 0) run_cnt[j] = runs;
    if (__ballot(down) && lane == 0) fl->unsorted = 1;
}

/* The path flags (one thread): a run path when the runs are at most half the
 * entries, with masks when the rows ascend; else the radix sort of the entries. */
__global__ void k_run_sizes(const int64_t *__restrict__ n_runs, int64_t nnz, Flags *__restrict__ fl)
{
    const int64_t R = *n_runs;
    const int32_t use = 2 * R <= nnz ? 1 : 0, uns = fl->unsorted ? 1 : 0;
    fl->use_runs = use;
    fl->hist_len = (int64_t)kRadix * ((R + kSortTile - 1) / kSortTile);
    fl->need_counts = (!use || uns) ? 1 : 0;
    fl->sorted = (use && !uns) ? 1 : 0;
    fl->any = (use && uns) ? 1 : 0;
}

/*
 * Records of every run (row-major run ids from run_ptr): its bucket key (an
 * invalid run takes the bucket of its column clamped into the grid), row
 * (flagged when invalid), first entry, and an auxiliary word: with ascending
 * rows the mask of its columns (OR of 1 << (col mod 32) over its entries, 0 for
 * an invalid run), else its length (0 for an invalid run).  A lane's run
 * starts at the highest start lane at or below it, or in an earlier chunk
 * (carried); when the columns from that start to the lane are consecutive, as
 * they are on a VOI row without holes, the lane's partial mask is a range of
 * bits, else a segmented OR over the lanes gives it.
 */
__global__ __launch_bounds__(kBlock) void k_run_emit(const int64_t *__restrict__ indptr,
                                                     const int32_t *__restrict__ indices, int n_rows, int n_voxels,
                                                     const int64_t *__restrict__ run_ptr, const Flags *__restrict__ fl,
                                                     uint32_t *__restrict__ run_key_out, int32_t *__restrict__ run_row,
                                                     float *__restrict__ run_src, uint32_t *__restrict__ run_aux,
                                                     Gate g)
{
    if (gate_closed(g)) return;
    const int j = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (j >= n_rows) return;
    const bool masks = fl->unsorted == 0;
    const int lane = lane_id();
    const uint64_t upto_lane = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull);   // lanes <= this one
    const int64_t e0 = indptr[j], e1 = indptr[j + 1];
    uint32_t r = (uint32_t)run_ptr[j];
    int prev_k = -1;                                   // run key of the entry before the chunk
    int open_first = 0;                                // run open at the chunk start: its first column,
    uint32_t open_len = 0, open_mask = 0;              // its entries and mask so far
    for (int64_t c = e0; c < e1; c += kRowChunks * kWave) {
        int cols[kRowChunks];
#pragma unroll
        for (int u = 0; u < kRowChunks; ++u) {
            const int64_t e = c + u * kWave + lane;
            cols[u] = e < e1 ? indices[e] : 0;
        }
        const int64_t en = c + kRowChunks * kWave;     // first entry after this group (uniform address)
        const int after = en < e1 ? indices[en] : 0;
#pragma unroll
        for (int u = 0; u < kRowChunks; ++u) {
            const int64_t e = c + u * kWave + lane;
            const bool in = e < e1;
            const int col = cols[u];
            const int k = in ? run_key(col, n_voxels) : -3;
            const int kp = from_lane_below(k, prev_k);
            // key of the entry after lane 63 (the next chunk's first, or none at the row's end)
            const int64_t e_next = c + (u + 1) * kWave;
            const int nx = u + 1 < kRowChunks ? __builtin_amdgcn_readlane(cols[u + 1 < kRowChunks ? u + 1 : u], 0) : after;
            const int kn = from_lane_above(k, e_next < e1 ? run_key(nx, n_voxels) : -3);
            const bool start = in && k != kp;
            const bool end = in && kn != k;
            const uint64_t m = __ballot(start);
            const uint64_t upto = m & upto_lane;
            const int sl = upto ? kWave - 1 - (int)__builtin_clzll(upto) : -1;   // start lane of this lane's run
            const int fc_here = __shfl(col, sl < 0 ? 0 : sl, kWave);
            const int fc = sl >= 0 ? fc_here : open_first;
            const uint32_t len = sl >= 0 ? (uint32_t)(lane - sl + 1) : open_len + (uint32_t)lane + 1u;
            uint32_t x = 0u;
            if (masks) {
                const bool valid = in && k >= 0;
                const bool ok = !valid || col - fc + 1 == (int)len;
                if (__ballot(!ok) == 0) {
                    // columns fc .. col of the bucket
                    const uint32_t hi = (2u << (col & (kBucketCols - 1))) - 1u;
                    const uint32_t lo = (1u << (fc & (kBucketCols - 1))) - 1u;
                    x = valid ? (hi & ~lo) : 0u;
                } else {
                    // segmented inclusive OR over the lanes, segments opened by run starts
                    x = valid ? 1u << (col & (kBucketCols - 1)) : 0u;
                    int f = start ? 1 : 0;
#pragma unroll
                    for (int d = 1; d < kWave; d <<= 1) {
                        const uint32_t y = __shfl_up(x, d, kWave);
                        const int fy = __shfl_up(f, d, kWave);
                        if (lane >= d && !f) {
                            x |= y;
                            f = fy;
                        }
                    }
                    if (!f) x |= open_mask;            // no start at or below this lane: the open run
                }
            }
            const uint32_t id = r + (uint32_t)mbcnt64(m) + (start ? 1u : 0u) - 1u;
            if (start) {
                const int clamped = col < 0 ? 0 : (col >= n_voxels ? n_voxels - 1 : col);
                run_key_out[id] = (uint32_t)(clamped >> kBucketShift);
                run_row[id] = k >= 0 ? j : (int32_t)((uint32_t)j | kRunFlag);
                run_src[id] = __uint_as_float((uint32_t)e);
            }
            if (end) run_aux[id] = masks ? x : (k >= 0 ? len : 0u);
            open_first = __builtin_amdgcn_readlane(fc, kWave - 1);
            open_len = (uint32_t)__builtin_amdgcn_readlane((int)len, kWave - 1);
            open_mask = (uint32_t)__builtin_amdgcn_readlane((int)x, kWave - 1);
            r += (uint32_t)__popcll(m);
            prev_k = __builtin_amdgcn_readlane(k, kWave - 1);
        }
    }
}

/* Bucket pointers from the sorted bucket keys: b_ptr[b] = first run of bucket b
 * (b_ptr[n_buckets] = R).  Keys ascend, so each b is written once. */
__global__ __launch_bounds__(kBlock) void k_bucket_bounds(const uint32_t *__restrict__ keys, Count n_runs,
                                                          int n_buckets, int64_t *__restrict__ b_ptr, Gate g)
{
    if (gate_closed(g)) return;
    const int64_t R = count_of(n_runs);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q <= R; q += stride) {
        const int64_t kq = q < R ? (int64_t)keys[q] : n_buckets;
        const int64_t kp = q > 0 ? (int64_t)keys[q - 1] : -1;
        for (int64_t b = kp + 1; b <= kq; ++b) b_ptr[b] = q;
    }
}

/* Bucket handled by workgroup blockIdx.x: groups of kXcdGroup consecutive
 * buckets go to one XCD (workgroups are dealt to the XCDs in turn), so that
 * the runs of neighbouring buckets, which share cache lines of a row, meet in
 * one L2; the groups themselves are dealt to the XCDs in turn, which keeps the
 * XCDs evenly loaded when the entries crowd into part of the grid. */
constexpr int kXcdGroup = 16;
__device__ inline int xcd_bucket()
{
    const int x = (int)(blockIdx.x % kXcds), k = (int)(blockIdx.x / kXcds);
    return ((k / kXcdGroup) * kXcds + x) * kXcdGroup + k % kXcdGroup;
}
static unsigned xcd_grid(int n_buckets)
{
    const int per = kXcds * kXcdGroup;
    return (unsigned)(((n_buckets + per - 1) / per) * per);
}

constexpr int kPlaceCap = 1024;     // entries of one batch staged in LDS
constexpr int kStageUnroll = 8;     // staging chunks whose loads are in flight together

/*
 * Placement for rows with ascending columns, one wave per bucket.
 *
 * First the bucket's entries per column: popcounts of ballots over the run
 * masks; their prefix from the bucket's first entry (the exclusive sum of the
 * lengths of all earlier runs) gives the voxel-row pointers of its columns.
 * Then batches of runs (in row order, at most kPlaceCap entries): for column c,
 * the ballot of the runs holding c ranks them, so the entry of run r in column
 * c goes to position (entries of the batch in columns below c) + (runs below r
 * holding c) of the batch's LDS image, which lists the batch's entries column
 * by column.  The image is then written out: each column's part is contiguous
 * after the entries of that column from earlier batches.
 */
__global__ __launch_bounds__(kWave) void k_place_sorted(
    const float *__restrict__ values, int n_voxels, int n_buckets, const int64_t *__restrict__ b_ptr,
    const int32_t *__restrict__ b_rows, const float *__restrict__ b_src, const uint32_t *__restrict__ b_mask,
    const uint32_t *__restrict__ b_off, const Flags *__restrict__ fl, int64_t *__restrict__ t_indptr, uint32_t nnz,
    int32_t *__restrict__ t_indices, float *__restrict__ t_values, Gate g)
{
    if (gate_closed(g)) return;
    const int b = xcd_bucket();
    if (b >= n_buckets) return;
    __shared__ uint16_t s_ent[kPlaceCap];        // batch entry p: (run lane << 5) | column
    __shared__ int32_t s_orow[kPlaceCap];        // LDS image, column by column
    __shared__ float s_oval[kPlaceCap];
    __shared__ uint8_t s_ocol[kPlaceCap];
    __shared__ uint64_t s_cm[kBucketCols];       // runs of the batch holding column c
    __shared__ uint32_t s_cst[kBucketCols];      // first image position of column c
    __shared__ uint32_t s_pos[kBucketCols];      // next output position of column c
    const int lane = lane_id();
    const int64_t q0 = b_ptr[b], q1 = b_ptr[b + 1], R = b_ptr[n_buckets];
    const uint32_t total = (uint32_t)fl->total;
    const uint32_t base = q0 < R ? b_off[q0] : total;

    // entries per column of the bucket (lane c), the voxel-row pointers
    uint32_t acc = 0;
    for (int64_t qb = q0; qb < q1; qb += kWave) {
        const uint32_t mask = qb + lane < q1 ? b_mask[qb + lane] : 0u;
#pragma unroll
        for (int c = 0; c < kBucketCols; ++c) {
            const uint32_t n = (uint32_t)__popcll(__ballot((mask >> c) & 1u));
            acc += lane == c ? n : 0u;
        }
    }
    uint32_t incl = wave_incl_scan(acc);
    if (lane < kBucketCols) {
        const uint32_t pos = base + incl - acc;
        s_pos[lane] = pos;
        const int col = (b << kBucketShift) + lane;
        if (col < n_voxels) t_indptr[col] = pos;
    }
    if (b == n_buckets - 1 && lane == 0) t_indptr[n_voxels] = total;
    __builtin_amdgcn_wave_barrier();

    for (int64_t qb = q0; qb < q1;) {
        const int64_t q = qb + lane;
        const bool have = q < q1;
        const int row = have ? (int)((uint32_t)b_rows[q] & ~kRunFlag) : 0;
        const uint32_t src = have ? __float_as_uint(b_src[q]) : 0u;
        uint32_t mask = have ? b_mask[q] : 0u;   // 0 for an invalid run
        uint32_t len = (uint32_t)__popc(mask);
        uint32_t end = wave_incl_scan(len);
        // the batch: the leading runs whose entries fit (at least one: a run holds <= 32)
        const bool fit = have && end <= (uint32_t)kPlaceCap;
        const int take = __popcll(__ballot(fit));
        const uint32_t T = (uint32_t)__shfl(end, take - 1, kWave);
        if (!fit) {
            mask = 0u;
            len = 0u;
        }
        const uint32_t excl = end - len;
        // runs of the batch per column, and the columns' first image positions
        uint64_t cm = 0;
#pragma unroll
        for (int c = 0; c < kBucketCols; ++c) {
            const uint64_t m = __ballot((mask >> c) & 1u);
            cm = lane == c ? m : cm;
        }
        const uint32_t cnt = (uint32_t)__popcll(cm);
        uint32_t cinc = wave_incl_scan(cnt);
        const uint32_t cst = cinc - cnt;
        if (lane < kBucketCols) {
            s_cm[lane] = cm;
            s_cst[lane] = cst;
        }
        // batch entries in run order: entry excl + i of run `lane` is its mask's i-th column
        {
            uint32_t x = mask, p = excl;
            while (__ballot(x != 0u)) {
                if (x != 0u) {
                    const uint32_t c = (uint32_t)__builtin_ctz(x);
                    x &= x - 1u;
                    s_ent[p] = (uint16_t)(((uint32_t)lane << kBucketShift) | c);
                    ++p;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        // stage the values into the image, kStageUnroll chunks of loads at a time
        for (uint32_t g0 = 0; g0 < T; g0 += kStageUnroll * kWave) {
            uint32_t ent[kStageUnroll];
            float v[kStageUnroll];
#pragma unroll
            for (int u = 0; u < kStageUnroll; ++u) {
                const uint32_t p = g0 + u * kWave + lane;
                const bool in = p < T;
                ent[u] = in ? (uint32_t)s_ent[p] : 0u;
                const int rr = (int)(ent[u] >> kBucketShift);
                // shuffles on every lane; loads only for entries of the batch
                const uint32_t e = __shfl(src, rr, kWave) + (p - __shfl(excl, rr, kWave));
                v[u] = in ? values[e] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kStageUnroll; ++u) {
                const uint32_t p = g0 + u * kWave + lane;
                const int rr = (int)(ent[u] >> kBucketShift);
                const int c = (int)(ent[u] & (kBucketCols - 1));
                const int rowr = __shfl(row, rr, kWave);
                if (p < T) {
                    const uint64_t below = (1ull << rr) - 1ull;
                    const uint32_t d = s_cst[c] + (uint32_t)__popcll(s_cm[c] & below);
                    s_orow[d] = rowr;
                    s_oval[d] = v[u];
                    s_ocol[d] = (uint8_t)c;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        // write the image out
        for (uint32_t i = lane; i < T; i += kWave) {
            const int c = s_ocol[i];
            const uint32_t gp = s_pos[c] + (i - s_cst[c]);
            if (gp < nnz) {   // always true for consistent runs; keeps every store in bounds
                t_indices[gp] = s_orow[i];
                t_values[gp] = s_oval[i];
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < kBucketCols) s_pos[lane] += cnt;
        __builtin_amdgcn_wave_barrier();
        qb += take;
    }
}

/* The runs of bucket b, taken 64 at a time: lane i holds run q0 + i (its row,
 * first entry and length), with the batch's exclusive prefix of lengths. */
struct RunBatch {
    int row;
    uint32_t src, len, excl, total;
};

__device__ inline RunBatch load_runs(int64_t qb, int64_t q1, const int32_t *__restrict__ b_rows,
                                     const float *__restrict__ b_src, const uint32_t *__restrict__ b_len)
{
    const int lane = lane_id();
    const int64_t q = qb + lane;
    RunBatch B{0, 0u, 0u, 0u, 0u};
    if (q < q1) {
        B.row = (int)((uint32_t)b_rows[q] & ~kRunFlag);
        B.src = __float_as_uint(b_src[q]);
        B.len = b_len[q];   // 0 for an invalid run
    }
    uint32_t incl = wave_incl_scan(B.len);
    B.excl = incl - B.len;
    B.total = __shfl(incl, kWave - 1, kWave);
    return B;
}

/* Lane of the run holding batch entry p = c0 + lane: the last lane whose
 * exclusive prefix is <= p, walked wave-uniformly from *rcur. */
__device__ inline int run_of(const RunBatch &B, uint32_t c0, int &rcur)
{
    while (rcur + 1 < kWave && (uint32_t)__builtin_amdgcn_readlane((int)B.excl, rcur + 1) <= c0) ++rcur;
    const uint32_t p = c0 + lane_id();
    int rr = rcur;
    for (int k = rcur + 1; k < kWave; ++k) {
        const uint32_t ek = (uint32_t)__builtin_amdgcn_readlane((int)B.excl, k);
        if (ek > c0 + kWave - 1) break;
        if (p >= ek) rr = k;
    }
    return rr;
}

/*
 * Placement for rows in any column order, one wave per bucket: the bucket's
 * runs are taken 64 at a time, their entries flattened over the lanes in run
 * order; an entry of column col goes to t_indptr[col] + (entries of col placed
 * before it), counted per column in LDS.  Equal columns within a 64-entry
 * chunk are ranked by lane with five ballots over the column's low bits.
 */
__global__ __launch_bounds__(kWave) void k_place_any(
    const int32_t *__restrict__ indices, const float *__restrict__ values, int n_voxels, int n_buckets,
    const int64_t *__restrict__ b_ptr, const int32_t *__restrict__ b_rows, const float *__restrict__ b_src,
    const uint32_t *__restrict__ b_len, const int64_t *__restrict__ t_indptr, uint32_t nnz,
    int32_t *__restrict__ t_indices, float *__restrict__ t_values, Gate g)
{
    if (gate_closed(g)) return;
    const int b = xcd_bucket();
    if (b >= n_buckets) return;
    __shared__ uint32_t base[kBucketCols];
    __shared__ uint32_t cnt[kBucketCols];
    const int lane = lane_id();
    for (int c = lane; c < kBucketCols; c += kWave) {
        const int col = (b << kBucketShift) + c;
        base[c] = col < n_voxels ? (uint32_t)t_indptr[col] : 0u;
        cnt[c] = 0u;
    }
    __builtin_amdgcn_wave_barrier();
    const int64_t q0 = b_ptr[b], q1 = b_ptr[b + 1];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));   // lanes under this one
    for (int64_t qb = q0; qb < q1; qb += kWave) {
        const RunBatch B = load_runs(qb, q1, b_rows, b_src, b_len);
        int rcur = 0;
        for (uint32_t c0 = 0; c0 < B.total; c0 += kWave) {
            const uint32_t p = c0 + lane;
            const int rr = run_of(B, c0, rcur);
            const bool in = p < B.total;
            const uint32_t e = __shfl(B.src, rr, kWave) + (p - __shfl(B.excl, rr, kWave));
            const int rowj = __shfl(B.row, rr, kWave);
            const int col = in ? indices[e] : 0;
            const float v = in ? values[e] : 0.0f;
            const int bin = col & (kBucketCols - 1);
            uint64_t eq = __ballot(in);
#pragma unroll
            for (int k = 0; k < kBucketShift; ++k) {
                const bool bit = (bin >> k) & 1;
                const uint64_t m = __ballot(bit);
                eq &= bit ? m : ~m;
            }
            const uint32_t rank = (uint32_t)__popcll(eq & below);
            const uint32_t n_eq = (uint32_t)__popcll(eq);
            const uint32_t pos = base[bin] + cnt[bin] + rank;
            if (in && pos < nnz) {   // always true for consistent runs; keeps every store in bounds
                t_indices[pos] = rowj;
                t_values[pos] = v;
            }
            __builtin_amdgcn_wave_barrier();
            if (in && rank + 1 == n_eq) cnt[bin] += n_eq;   // the last lane of each column group
            __builtin_amdgcn_wave_barrier();
        }
    }
}

}  // namespace

/* Workspace layout of the transpose (offsets from a 256-byte aligned base). */
struct TransposeLayout {
    size_t key[2], row[2], val[2], hist, offs, partial, counts, bptr, flags, run_cnt, run_ptr, total;
};

static TransposeLayout transpose_layout(int64_t nnz, int n_voxels, int n_rows)
{
    TransposeLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const int64_t n_tiles = (nnz + kSortTile - 1) / kSortTile;
    const int64_t n_hist = (int64_t)kRadix * (n_tiles > 0 ? n_tiles : 1);
    const int64_t nb = (n_voxels + kBucketCols - 1) >> kBucketShift;
    int64_t n_scan = std::max<int64_t>(std::max<int64_t>(n_hist, n_voxels), std::max<int64_t>(n_rows, (nnz + 1) / 2));
    const size_t e = (size_t)(nnz > 0 ? nnz : 1);
    for (int b = 0; b < 2; ++b) {
        L.key[b] = take(sizeof(uint32_t) * e);
        L.row[b] = take(sizeof(int32_t) * e);
        L.val[b] = take(sizeof(float) * e);
    }
    L.hist = take(sizeof(uint32_t) * (size_t)n_hist);
    L.offs = take(sizeof(uint32_t) * (size_t)n_hist);
    L.partial = take(sizeof(uint32_t) * (size_t)((n_scan + kScanChunk - 1) / kScanChunk + 1));
    L.counts = take(sizeof(uint32_t) * ((size_t)n_voxels + 1));
    L.bptr = take(sizeof(int64_t) * (size_t)(nb + 1));
    L.flags = take(sizeof(Flags));
    L.run_cnt = take(sizeof(uint32_t) * (size_t)(n_rows > 0 ? n_rows : 1));
    L.run_ptr = take(sizeof(int64_t) * ((size_t)n_rows + 1));
    L.total = off;
    return L;
}

size_t transpose_workspace(int64_t nnz, int n_voxels, int n_rows)
{
    return transpose_layout(nnz, n_voxels, n_rows).total;
}

int transpose_passes(int n_keys)
{
    int bits = 0;
    while (bits < 31 && ((int64_t)1 << bits) < (int64_t)n_keys) ++bits;
    const int p = (bits + kRadixBits - 1) / kRadixBits;
    return p > 0 ? p : 1;
}

/* Persistent grid of a grid-stride launch over `items` units of work. */
static unsigned stride_grid(int64_t items)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(items, 4096));
}

/* Exclusive (inclusive with INCL) scan of n uint32 values in -> out (OUT =
 * uint32_t or int64_t; out may be in); n is a host count or, with n.dev, a
 * device count at most n_max.  partial[nblocks] receives the total, and
 * *total64 too when given. */
template <typename OUT, bool INCL = false, bool POPC = false>
static hipError_t scan_excl(const uint32_t *in, Count n, int64_t n_max, uint32_t *partial, OUT *out,
                            int64_t *total64, Gate g, hipStream_t s)
{
    const unsigned nb = stride_grid((n_max + kScanChunk - 1) / kScanChunk);
    hipLaunchKernelGGL(k_scan_reduce<POPC>, dim3(nb), dim3(kBlock), 0, s, in, n, partial, g);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanTop), 0, s, partial, n, total64, g);
    hipLaunchKernelGGL((k_scan_down<OUT, INCL, POPC>), dim3(nb), dim3(kBlock), 0, s, in, n, partial, out, g);
    return hipGetLastError();
}

/* Optional fourth payload of a radix sort: input, ping-pong buffers, output. */
struct Extra {
    const uint32_t *in;
    uint32_t *b0, *b1, *out;
};

/*
 * One stable LSD radix sort of (key, row, value) triples by key: `passes`
 * passes of 8 bits, keys above clamp sorted as clamp, ping-pong through
 * (k1, r1, v1) and (k0, r0, v0) (the input may be separate), the last pass
 * writing rows and values to (rows_out, vals_out), and with keys_out its keys
 * to the pass's own key buffer (*keys_out = that buffer); with x.in a fourth
 * payload rides along (through x.b1, x.b0, to x.out).  n is a host or device
 * count, at most n_max.
 */
static hipError_t radix_sort(const uint32_t *keys, const int32_t *rows, const float *vals, Count n, int64_t n_max,
                             uint32_t clamp, int passes, uint32_t *k0, int32_t *r0, float *v0, uint32_t *k1,
                             int32_t *r1, float *v1, int32_t *rows_out, float *vals_out, uint32_t **keys_out,
                             Extra x, uint32_t *hist, uint32_t *offs, uint32_t *partial, int64_t *hist_len_dev, Gate g,
                             hipStream_t s)
{
    const int64_t tiles_max = (n_max + kSortTile - 1) / kSortTile;
    const unsigned grid = stride_grid(tiles_max);
    const Count hn = hist_len_dev ? Count{0, hist_len_dev} : Count{(int64_t)kRadix * tiles_max, nullptr};
    const uint32_t *kin = keys;
    const int32_t *rin = rows;
    const float *vin = vals;
    const uint32_t *xin = x.in;
    hipError_t e;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kRadixBits;
        const bool last = p == passes - 1;
        uint32_t *kbuf = (p & 1) ? k0 : k1;
        uint32_t *kout = last ? (keys_out ? kbuf : nullptr) : kbuf;
        int32_t *rout = last ? rows_out : ((p & 1) ? r0 : r1);
        float *vout = last ? vals_out : ((p & 1) ? v0 : v1);
        uint32_t *xout = last ? x.out : ((p & 1) ? x.b0 : x.b1);
        hipLaunchKernelGGL(k_rs_hist, dim3(grid), dim3(kBlock), 0, s, kin, n, clamp, shift, hist, g);
        if ((e = scan_excl<uint32_t>(hist, hn, (int64_t)kRadix * tiles_max, partial, offs, nullptr, g, s)) !=
            hipSuccess)
            return e;
        if (x.in)
            hipLaunchKernelGGL(k_rs_scatter<true>, dim3(grid), dim3(kBlock), 0, s, kin, rin, vin, xin, n, clamp, shift,
                               offs, kout, rout, vout, xout, g);
        else
            hipLaunchKernelGGL(k_rs_scatter<false>, dim3(grid), dim3(kBlock), 0, s, kin, rin, vin, nullptr, n, clamp,
                               shift, offs, kout, rout, vout, nullptr, g);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (last && keys_out) *keys_out = kout;
        kin = kout;
        rin = rout;
        vin = vout;
        xin = xout;
    }
    return hipSuccess;
}

hipError_t launch_transpose(const int64_t *indptr, const int32_t *indices, const float *values, int n_rows,
                            int n_voxels, int64_t nnz, int64_t *t_indptr, int32_t *t_indices, float *t_values,
                            void *workspace, hipStream_t s)
{
    const TransposeLayout L = transpose_layout(nnz, n_voxels, n_rows);
    char *ws = static_cast<char *>(workspace);
    uint32_t *key[2] = {reinterpret_cast<uint32_t *>(ws + L.key[0]), reinterpret_cast<uint32_t *>(ws + L.key[1])};
    int32_t *row[2] = {reinterpret_cast<int32_t *>(ws + L.row[0]), reinterpret_cast<int32_t *>(ws + L.row[1])};
    float *val[2] = {reinterpret_cast<float *>(ws + L.val[0]), reinterpret_cast<float *>(ws + L.val[1])};
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    uint32_t *offs = reinterpret_cast<uint32_t *>(ws + L.offs);
    uint32_t *partial = reinterpret_cast<uint32_t *>(ws + L.partial);
    uint32_t *counts = reinterpret_cast<uint32_t *>(ws + L.counts);
    Flags *fl = reinterpret_cast<Flags *>(ws + L.flags);
    uint32_t *run_cnt = reinterpret_cast<uint32_t *>(ws + L.run_cnt);
    int64_t *run_ptr = reinterpret_cast<int64_t *>(ws + L.run_ptr);
    const Gate always{nullptr, 0};
    hipError_t e;

    if (nnz == 0 || n_rows == 0) {   // empty voxel rows
        hipLaunchKernelGGL(k_zero_u32, dim3(blocks_of((int64_t)n_voxels + 1, kBlock)), dim3(kBlock), 0, s, counts,
                           (int64_t)n_voxels + 1);
        return scan_excl<int64_t>(counts, Count{n_voxels, nullptr}, n_voxels, partial, t_indptr, t_indptr + n_voxels,
                                  always, s);
    }

    // runs of every row and the unsorted flag; run pointers; the path flags
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kBlock), 0, s, reinterpret_cast<uint32_t *>(fl),
                       (int64_t)(sizeof(Flags) / 4));
    hipLaunchKernelGGL(k_run_count, dim3(blocks_of(n_rows, kWavesPerBlock)), dim3(kBlock), 0, s, indptr, indices,
                       n_rows, n_voxels, run_cnt, fl);
    if ((e = scan_excl<int64_t>(run_cnt, Count{n_rows, nullptr}, n_rows, partial, run_ptr, run_ptr + n_rows, always,
                                s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_run_sizes, dim3(1), dim3(1), 0, s, run_ptr + n_rows, nnz, fl);
    const Gate runs{&fl->use_runs, 1}, entries{&fl->use_runs, 0}, counted{&fl->need_counts, 1},
        masked{&fl->sorted, 1}, any{&fl->any, 1};

    // entry path and unsorted rows: entries per column by atomics, the voxel-row pointers
    hipLaunchKernelGGL(k_zero_u32, dim3(blocks_of((int64_t)n_voxels + 1, kBlock)), dim3(kBlock), 0, s, counts,
                       (int64_t)n_voxels + 1);
    hipLaunchKernelGGL(k_key_count, dim3(stride_grid(blocks_of(nnz, kBlock))), dim3(kBlock), 0, s, indices, nnz,
                       n_voxels, counts, counted);
    if ((e = scan_excl<int64_t>(counts, Count{n_voxels, nullptr}, n_voxels, partial, t_indptr, t_indptr + n_voxels,
                                counted, s)) != hipSuccess)
        return e;

    // run paths: at most nnz / 2 runs.  Run records (bucket, row, first entry, mask or
    // length) in the first halves of key[0], row[0], val[0] and in key[0] + half; the
    // sort's other buffers are the first halves of key/row/val[1] and key[1] + half; the
    // sorted rows, first entries and masks or lengths go to row[0] + half, val[0] + half
    // and row[1] + half, the entry offsets of the sorted runs to val[1] + half
    const int nb = (n_voxels + kBucketCols - 1) >> kBucketShift;
    {
        const int64_t half = (nnz + 1) / 2;
        int32_t *brow = row[0] + half;
        float *bsrc = val[0] + half;
        uint32_t *baux = reinterpret_cast<uint32_t *>(row[1]) + half;
        uint32_t *boff = reinterpret_cast<uint32_t *>(val[1]) + half;
        int64_t *bptr = reinterpret_cast<int64_t *>(ws + L.bptr);
        const Count n_runs{0, run_ptr + n_rows};
        hipLaunchKernelGGL(k_run_emit, dim3(blocks_of(n_rows, kWavesPerBlock)), dim3(kBlock), 0, s, indptr, indices,
                           n_rows, n_voxels, run_ptr, fl, key[0], row[0], val[0], key[0] + half, runs);
        // stable sort of the runs by bucket
        uint32_t *skeys = nullptr;
        const Extra aux{key[0] + half, key[0] + half, key[1] + half, baux};
        if ((e = radix_sort(key[0], row[0], val[0], n_runs, half, 0xffffffffu, transpose_passes(nb), key[0], row[0],
                            val[0], key[1], row[1], val[1], brow, bsrc, &skeys, aux, hist, offs, partial,
                            &fl->hist_len, runs, s)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_bucket_bounds, dim3(stride_grid(blocks_of(half + 1, kBlock))), dim3(kBlock), 0, s, skeys,
                           n_runs, nb, bptr, runs);
        // rows ascending: entry offset of every sorted run, then the placement (and the pointers)
        if ((e = scan_excl<uint32_t, false, true>(baux, n_runs, half, partial, boff, &fl->total, masked, s)) !=
            hipSuccess)
            return e;
        hipLaunchKernelGGL(k_place_sorted, dim3(xcd_grid(nb)), dim3(kWave), 0, s, values, n_voxels, nb, bptr, brow,
                           bsrc, baux, boff, fl, t_indptr, (uint32_t)nnz, t_indices, t_values, masked);
        // rows in any order
        hipLaunchKernelGGL(k_place_any, dim3(xcd_grid(nb)), dim3(kWave), 0, s, indices, values, n_voxels, nb, bptr,
                           brow, bsrc, baux, t_indptr, (uint32_t)nnz, t_indices, t_values, any);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }

    // entry path: row id of every entry (into row[0]), then a radix sort of the entries by
    // column (invalid columns as n_voxels, sorted last)
    hipLaunchKernelGGL(k_expand_rows, dim3(blocks_of(n_rows, kWavesPerBlock)), dim3(kBlock), 0, s, indptr, n_rows, nnz,
                       row[0], entries);
    return radix_sort(reinterpret_cast<const uint32_t *>(indices), row[0], values, Count{nnz, nullptr}, nnz,
                      (uint32_t)n_voxels, transpose_passes(n_voxels + 1), key[0], row[0], val[0], key[1], row[1],
                      val[1], t_indices, t_values, nullptr, Extra{nullptr, nullptr, nullptr, nullptr}, hist, offs,
                      partial, nullptr, entries, s);
}

/*
 * Scratch of the allocation-free transpose: a file-scope device array, one
 * copy per GPU, held until the process ends.  Host code never passes the
 * array's name to a kernel (on the host it is only a stand-in for the
 * symbol): its device address is taken once per device with
 * hipGetSymbolAddress and kept in noalloc_scratch_ptr.
 */
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_ptr(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace fspb
