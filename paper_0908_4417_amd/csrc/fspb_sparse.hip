/*
 * gfx950 kernels for Eq. 1 on the dose-coefficient matrix D_ij.
 *
 *   beamlet-row CSR (what the fill writes: row j = beamlet, columns = voxels)
 *     k_fluence_dose      dose_i += w_j D_ij with FP32 atomics   -- one wave per row
 *     k_fluence_gradient  g_j = sum_i D_ij r_i, fixed order      -- one wave per row
 *   voxel-row CSR (row i = voxel, columns = beamlets): the transpose, a stable
 *   sort of the row-major entries by column
 *     k_run_count         per row: runs (stretches within one 32-column bucket),
 *                         the unsorted flag, entries per column as a difference
 *                         array (two atomics per stretch of consecutive columns)
 *     scans               entries per column, voxel-row pointers, run pointers
 *     k_run_sizes         the path flag
 *     run path (the default for D, whose rows are long stretches of columns):
 *       k_run_emit                             run records
 *       k_rs_hist, scan, k_rs_scatter          stable LSD radix sort of the runs by bucket
 *       k_bucket_bounds, k_run_gather          bucket pointers; each sorted run's
 *                                              first entry and length
 *       k_bucket_place                         one wave per bucket places its runs'
 *                                              entries by a counting sort on the column
 *     entry path (short stretches):
 *       k_expand_rows, then k_rs_hist, scan, k_rs_scatter per 8 bits of the column
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

/* Exclusive scan of one value per thread over the block; *total gets the sum. */
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *s_w, uint32_t *total)
{
    const int l = lane_id(), w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, kWave);
        if (l >= d) x += y;
    }
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

__device__ inline float dot4(int4 i, float4 v, const float *__restrict__ x, uint32_t n, float acc)
{
    if ((uint32_t)i.x < n) acc = fmaf(v.x, x[(uint32_t)i.x], acc);
    if ((uint32_t)i.y < n) acc = fmaf(v.y, x[(uint32_t)i.y], acc);
    if ((uint32_t)i.z < n) acc = fmaf(v.z, x[(uint32_t)i.z], acc);
    if ((uint32_t)i.w < n) acc = fmaf(v.w, x[(uint32_t)i.w], acc);
    return acc;
}

/* g_j = sum_i D_ij r_i; one wave per row: 16-byte loads of four consecutive
 * entries per lane, two steps in flight, lane partial sums then a fixed
 * butterfly.  Columns outside [0, n_voxels) are skipped. */
__global__ __launch_bounds__(kBlock) void k_fluence_gradient(const int64_t *__restrict__ indptr,
                                                             const int32_t *__restrict__ indices,
                                                             const float *__restrict__ values, int n_rows,
                                                             int n_voxels, const float *__restrict__ r,
                                                             float *__restrict__ g)
{
    const int j = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (j >= n_rows) return;
    const int lane = lane_id();
    const uint32_t n = (uint32_t)n_voxels;
    const int64_t e0 = indptr[j], e1 = indptr[j + 1];
    const RowSplit sp = row_split(indices, values, e0, e1, 4 * kWave);
    float acc0 = 0.0f, acc1 = 0.0f;
    if (e0 + lane < sp.a) {
        const uint32_t i = (uint32_t)indices[e0 + lane];
        if (i < n) acc0 = fmaf(values[e0 + lane], r[i], acc0);
    }
    int64_t e = sp.a + 4 * lane;
    for (; e + 4 * kWave < sp.b; e += 8 * kWave) {
        const int4 i0 = *reinterpret_cast<const int4 *>(indices + e);
        const float4 v0 = *reinterpret_cast<const float4 *>(values + e);
        const int4 i1 = *reinterpret_cast<const int4 *>(indices + e + 4 * kWave);
        const float4 v1 = *reinterpret_cast<const float4 *>(values + e + 4 * kWave);
        acc0 = dot4(i0, v0, r, n, acc0);
        acc1 = dot4(i1, v1, r, n, acc1);
    }
    if (e < sp.b) {
        const int4 i0 = *reinterpret_cast<const int4 *>(indices + e);
        const float4 v0 = *reinterpret_cast<const float4 *>(values + e);
        acc0 = dot4(i0, v0, r, n, acc0);
    }
    for (int64_t t = sp.b + lane; t < e1; t += kWave) {
        const uint32_t i = (uint32_t)indices[t];
        if (i < n) acc1 = fmaf(values[t], r[i], acc1);
    }
    float s = wave_sum(acc0 + acc1);
    if (lane == 0) g[j] = s;
}

/* dose_i = sum_j D_ij w_j over voxel row i: 16 lanes per row, lane-strided
 * partial sums and a fixed 16-lane butterfly.  Beamlets outside [0, n_w) are
 * skipped. */
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
        for (int64_t e = sp.a + 4 * l; e < sp.b; e += 64) {
            const int4 j4 = *reinterpret_cast<const int4 *>(t_indices + e);
            const float4 v4 = *reinterpret_cast<const float4 *>(t_values + e);
            acc1 = dot4(j4, v4, w, n, acc1);
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

/* Scan, phase 1: sum of each kScanChunk-value chunk (grid-stride over chunks). */
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
        for (int k = 0; k < kScanItems; ++k) v += base + k < n ? in[base + k] : 0u;
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
        uint32_t x = v;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, kWave);
            if (l >= d) x += y;
        }
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
template <typename OUT, bool INCL>
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
 * Radix pass, phase 2: stable scatter.  Wave w of a block owns the w-th
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
__global__ __launch_bounds__(kBlock) void k_rs_scatter(const uint32_t *__restrict__ keys_in,
                                                       const int32_t *__restrict__ rows_in,
                                                       const float *__restrict__ vals_in, Count n_in, uint32_t clamp,
                                                       int shift, const uint32_t *__restrict__ offs,
                                                       uint32_t *__restrict__ keys_out,
                                                       int32_t *__restrict__ rows_out,
                                                       float *__restrict__ vals_out, Gate g)
{
    if (gate_closed(g)) return;
    __shared__ uint32_t s_key[kSortTile];
    __shared__ int32_t s_row[kSortTile];
    __shared__ float s_val[kSortTile];
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

        uint32_t key[kSortItems], pos[kSortItems];
        int32_t row[kSortItems];
        float val[kSortItems];
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const int64_t i = sub0 + (int64_t)r * kWave + lane;
            const bool valid = i < n;
            key[r] = valid ? min(keys_in[i], clamp) : 0u;
            row[r] = valid ? rows_in[i] : 0;
            val[r] = valid ? vals_in[i] : 0.0f;
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
    hipLaunchKernelGGL(k_fluence_gradient, dim3(blocks_of(n_rows, kWavesPerBlock)), dim3(kBlock), 0, s, indptr,
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

/* Workspace layout of the transpose (offsets from a 256-byte aligned base). */
namespace {

/*
 * Run transpose.  A run is a maximal stretch of consecutive entries of one row
 * whose columns share a bucket of kBucketCols columns (col >> kBucketShift);
 * entries whose column lies outside [0, n_voxels) form runs of their own,
 * flagged (row id with its top bit set) and never placed.  The transpose sorts
 * the runs by bucket (stably, so a bucket's runs keep row order), then one wave
 * per bucket walks its runs' entries in that order and places each with a
 * stable counting sort on the column's low bits: the output is the stable sort
 * of the row-major entries by column, as the radix path gives, for about two
 * reads and one write of the matrix.
 */
constexpr int kBucketShift = 5;
constexpr int kBucketCols = 1 << kBucketShift;
constexpr uint32_t kRunFlag = 0x80000000u;   // run of invalid columns (in the run's row id)
constexpr int kRowChunks = 4;                // chunks of 64 entries whose loads are in flight together

/* Run key of a column: its bucket, or -2 (outside [0, n_voxels)); -1 marks "no entry before". */
__device__ inline int run_key(int col, int n_voxels)
{
    return (uint32_t)col < (uint32_t)n_voxels ? (col >> kBucketShift) : -2;
}

/*
 * Per row (one wave, kRowChunks chunks of 64 entries loaded together): the
 * number of runs (run_cnt[j]); *unsorted when the row's columns are not
 * strictly ascending; and the row's entries per column as a difference array:
 * every maximal stretch of entries with consecutive valid columns c .. c+m-1
 * adds 1 at c and -1 at c+m (two atomics per stretch, where one per entry
 * would be needed otherwise; a plan's D has stretches of tens of entries).
 */
__global__ __launch_bounds__(kBlock) void k_run_count(const int64_t *__restrict__ indptr,
                                                      const int32_t *__restrict__ indices, int n_rows, int n_voxels,
                                                      uint32_t *__restrict__ run_cnt, int32_t *__restrict__ unsorted,
                                                      uint32_t *__restrict__ diff)
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
        // first entry after this group (uniform address)
        const int64_t en = c + kRowChunks * kWave;
        const int after = en < e1 ? indices[en] : 0;
#pragma unroll
        for (int u = 0; u < kRowChunks; ++u) {
            const int64_t e = c + u * kWave + lane;
            const bool in = e < e1;
            const int col = cols[u];
            const int k = in ? run_key(col, n_voxels) : -3;
            int cp = __shfl_up(col, 1, kWave), kp = __shfl_up(k, 1, kWave);
            if (lane == 0) {
                cp = prev_col;
                kp = prev_k;
            }
            int cn = __shfl_down(col, 1, kWave), kn = __shfl_down(k, 1, kWave);
            if (lane == kWave - 1) {
                const int nx = u + 1 < kRowChunks ? __builtin_amdgcn_readlane(cols[u + 1 < kRowChunks ? u + 1 : u], 0)
                                                  : after;
                cn = nx;
                kn = e + 1 < e1 ? run_key(nx, n_voxels) : -3;
            }
            runs += (uint32_t)__popcll(__ballot(in && k != kp));
            down = down || (in && kp != -1 && col <= cp);
            const bool valid = in && k >= 0;
            if (valid && !(kp >= 0 && col == cp + 1)) atomicAdd(diff + col, 1u);
            if (valid && !(kn >= 0 && cn == col + 1)) atomicAdd(diff + col + 1, 0xffffffffu);
            prev_col = __shfl(col, kWave - 1, kWave);
            prev_k = __shfl(k, kWave - 1, kWave);
        }
    }
    if (lane == 0) run_cnt[j] = runs;
    if (__ballot(down) && lane == 0) *unsorted = 1;
}

/*
 * The path flag: the run transpose when the runs are at most half the entries,
 * else the radix sort of the entries; and the length of the run sort's digit
 * histograms.  One thread.
 */
__global__ void k_run_sizes(const int64_t *__restrict__ n_runs, int64_t nnz, int32_t *__restrict__ use_runs,
                            int64_t *__restrict__ hist_len)
{
    const int64_t R = *n_runs;
    *use_runs = 2 * R <= nnz ? 1 : 0;
    *hist_len = (int64_t)kRadix * ((R + kSortTile - 1) / kSortTile);
}

/* Records of every run (row-major run ids from run_ptr): its bucket (an invalid
 * run takes the bucket of its column clamped into the grid), row (flagged when
 * invalid), id (as the value payload of the run sort) and first entry. */
__global__ __launch_bounds__(kBlock) void k_run_emit(const int64_t *__restrict__ indptr,
                                                     const int32_t *__restrict__ indices, int n_rows, int n_voxels,
                                                     const int64_t *__restrict__ run_ptr,
                                                     uint32_t *__restrict__ run_bucket, int32_t *__restrict__ run_row,
                                                     float *__restrict__ run_id, uint32_t *__restrict__ run_src,
                                                     Gate g)
{
    if (gate_closed(g)) return;
    const int j = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (j >= n_rows) return;
    const int lane = lane_id();
    const int64_t e0 = indptr[j], e1 = indptr[j + 1];
    uint32_t r = (uint32_t)run_ptr[j];
    int prev_k = -1;                                   // run key of the entry before the chunk
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
            int kp = __shfl_up(k, 1, kWave);
            if (lane == 0) kp = prev_k;
            const bool start = in && k != kp;
            const uint64_t m = __ballot(start);
            if (start) {
                const uint32_t id = r + (uint32_t)mbcnt64(m);
                const int clamped = col < 0 ? 0 : (col >= n_voxels ? n_voxels - 1 : col);
                run_bucket[id] = (uint32_t)(clamped >> kBucketShift);
                run_row[id] = k >= 0 ? j : (int32_t)((uint32_t)j | kRunFlag);
                run_id[id] = __uint_as_float(id);
                run_src[id] = (uint32_t)e;
            }
            r += (uint32_t)__popcll(m);
            prev_k = __shfl(k, kWave - 1, kWave);
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

/* Sorted run q: its first entry and length (0 for an invalid run), and its row
 * without the flag; the length runs to the next run of the row or the row's end. */
__global__ __launch_bounds__(kBlock) void k_run_gather(const float *__restrict__ b_ids, int32_t *__restrict__ b_rows,
                                                       const uint32_t *__restrict__ run_src,
                                                       const int64_t *__restrict__ run_ptr,
                                                       const int64_t *__restrict__ indptr, Count n_runs,
                                                       uint32_t *__restrict__ b_src, uint32_t *__restrict__ b_len,
                                                       Gate g)
{
    if (gate_closed(g)) return;
    const int64_t R = count_of(n_runs);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < R; q += stride) {
        const uint32_t id = __float_as_uint(b_ids[q]);
        const uint32_t rw = (uint32_t)b_rows[q];
        const int row = (int)(rw & ~kRunFlag);
        const uint32_t src = run_src[id];
        const uint32_t end = (int64_t)id + 1 < run_ptr[row + 1] ? run_src[id + 1] : (uint32_t)indptr[row + 1];
        b_src[q] = src;
        b_len[q] = (rw & kRunFlag) ? 0u : end - src;
        b_rows[q] = row;
    }
}

constexpr int kColWaves = 2;                               // waves per workgroup of k_bucket_place
constexpr int kStageUnroll = 8;                            // staging chunks whose loads are in flight together

/* The runs of bucket b, taken 64 at a time: lane i holds run q0 + i (its row,
 * first entry and length), with the batch's exclusive prefix of lengths. */
struct RunBatch {
    int row;
    uint32_t src, len, excl, total;
};

__device__ inline RunBatch load_runs(int64_t qb, int64_t q1, const int32_t *__restrict__ b_rows,
                                     const uint32_t *__restrict__ b_src, const uint32_t *__restrict__ b_len,
                                     uint32_t max_len)
{
    const int lane = lane_id();
    const int64_t q = qb + lane;
    RunBatch B{0, 0u, 0u, 0u, 0u};
    if (q < q1) {
        B.row = b_rows[q];
        B.src = b_src[q];
        B.len = min(b_len[q], max_len);
    }
    uint32_t incl = B.len;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += y;
    }
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
 * Placement for rows with strictly ascending columns, column by column.  A
 * batch of 64 runs of the bucket (rows ascending; each at most 32 entries,
 * one per column) is first copied into LDS, the runs' entries flattened over
 * the lanes, kStageUnroll chunks of 64 at a time with all their loads issued
 * together; then each lane holds one run and, at column c, the lanes whose
 * next entry has column c write it, ranked by lane, so each column's entries
 * from the batch go out as one contiguous stretch.
 */
__device__ void place_columns(int b, int wave, const int32_t *__restrict__ indices, const float *__restrict__ values,
                              int n_voxels, const int64_t *__restrict__ b_ptr, const int32_t *__restrict__ b_rows,
                              const uint32_t *__restrict__ b_src, const uint32_t *__restrict__ b_len,
                              const int64_t *__restrict__ t_indptr, uint32_t nnz, int32_t *__restrict__ t_indices,
                              float *__restrict__ t_values)
{
    constexpr int kStage = kWave * kBucketCols;            // 64 runs of at most 32 entries
    __shared__ uint32_t s_pos[kColWaves][kBucketCols];
    __shared__ float s_val[kColWaves][kStage];
    __shared__ uint8_t s_col[kColWaves][kStage];
    const int lane = lane_id();
    uint32_t *pos = s_pos[wave];                           // next free position of each column's list
    float *sv = s_val[wave];
    uint8_t *sc = s_col[wave];
    for (int c = lane; c < kBucketCols; c += kWave) {
        const int col = (b << kBucketShift) + c;
        pos[c] = col < n_voxels ? (uint32_t)t_indptr[col] : 0u;
    }
    const int col0 = b << kBucketShift;
    const int64_t q0 = b_ptr[b], q1 = b_ptr[b + 1];
    for (int64_t qb = q0; qb < q1; qb += kWave) {
        const RunBatch B = load_runs(qb, q1, b_rows, b_src, b_len, kBucketCols);
        // stage: entry p of the batch -> LDS
        int rcur = 0;
        for (uint32_t g0 = 0; g0 < B.total; g0 += kStageUnroll * kWave) {
            uint32_t e[kStageUnroll];
#pragma unroll
            for (int u = 0; u < kStageUnroll; ++u) {
                const uint32_t c0 = g0 + u * kWave;
                e[u] = 0u;
                if (c0 < B.total) {
                    const int rr = run_of(B, c0, rcur);
                    // shuffles on every lane: the source lane rr may be past the end of the batch's entries
                    e[u] = __shfl(B.src, rr, kWave) + (c0 + lane - __shfl(B.excl, rr, kWave));
                }
            }
            int cols[kStageUnroll];
            float vals[kStageUnroll];
#pragma unroll
            for (int u = 0; u < kStageUnroll; ++u) {
                const bool in = g0 + u * kWave + lane < B.total;
                cols[u] = in ? indices[e[u]] : col0;
                vals[u] = in ? values[e[u]] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kStageUnroll; ++u) {
                const uint32_t p = g0 + u * kWave + lane;
                if (p < B.total) {
                    sc[p] = (uint8_t)(cols[u] - col0);
                    sv[p] = vals[u];
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        // place: lane = run, its entries sc/sv[excl, excl + len)
        uint32_t k = B.excl;
        const uint32_t end = B.excl + B.len;
        int ca = k < end ? (int)sc[k] : kBucketCols;
        for (int c = 0; c < kBucketCols; ++c) {
            const bool has = ca == c;
            const uint64_t m = __ballot(has);
            if (m == 0) continue;
            const uint32_t p0 = pos[c];
            if (has) {
                const uint32_t p = p0 + (uint32_t)mbcnt64(m);
                if (p < nnz) {   // always true for consistent runs; keeps every store in bounds
                    t_indices[p] = B.row;
                    t_values[p] = sv[k];
                }
                ++k;
                ca = k < end ? (int)sc[k] : kBucketCols;
            }
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) pos[c] = p0 + (uint32_t)__popcll(m);
            __builtin_amdgcn_wave_barrier();
        }
        __builtin_amdgcn_wave_barrier();
    }
}

/*
 * Placement for rows in any column order: the bucket's runs are taken 64 at a
 * time, their entries flattened over the lanes in run order; an entry of
 * column col goes to t_indptr[col] + (entries of col placed before it),
 * counted per column in LDS.  Equal columns within a 64-entry chunk are
 * ranked by lane with five ballots over the column's low bits.
 */
__device__ void place_any(int b, int wave, const int32_t *__restrict__ indices, const float *__restrict__ values,
                          int n_voxels, const int64_t *__restrict__ b_ptr, const int32_t *__restrict__ b_rows,
                          const uint32_t *__restrict__ b_src, const uint32_t *__restrict__ b_len,
                          const int64_t *__restrict__ t_indptr, uint32_t nnz, int32_t *__restrict__ t_indices,
                          float *__restrict__ t_values)
{
    __shared__ uint32_t s_base[kColWaves][kBucketCols];
    __shared__ uint32_t s_cnt[kColWaves][kBucketCols];
    const int lane = lane_id();
    uint32_t *base = s_base[wave];
    uint32_t *cnt = s_cnt[wave];
    for (int c = lane; c < kBucketCols; c += kWave) {
        const int col = (b << kBucketShift) + c;
        base[c] = col < n_voxels ? (uint32_t)t_indptr[col] : 0u;
        cnt[c] = 0u;
    }
    const int64_t q0 = b_ptr[b], q1 = b_ptr[b + 1];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));   // lanes under this one
    for (int64_t qb = q0; qb < q1; qb += kWave) {
        const RunBatch B = load_runs(qb, q1, b_rows, b_src, b_len, 0xffffffffu);
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

/* One wave per bucket of columns. */
__global__ __launch_bounds__(kColWaves * kWave) void k_bucket_place(
    const int32_t *__restrict__ indices, const float *__restrict__ values, int n_voxels, int n_buckets,
    const int64_t *__restrict__ b_ptr, const int32_t *__restrict__ b_rows, const uint32_t *__restrict__ b_src,
    const uint32_t *__restrict__ b_len, const int64_t *__restrict__ t_indptr, uint32_t nnz,
    int32_t *__restrict__ t_indices, float *__restrict__ t_values, const int32_t *__restrict__ unsorted, Gate g)
{
    if (gate_closed(g)) return;
    const int wave = threadIdx.x >> 6;
    const int b = blockIdx.x * kColWaves + wave;
    if (b >= n_buckets) return;
    if (*unsorted)
        place_any(b, wave, indices, values, n_voxels, b_ptr, b_rows, b_src, b_len, t_indptr, nnz, t_indices,
                  t_values);
    else
        place_columns(b, wave, indices, values, n_voxels, b_ptr, b_rows, b_src, b_len, t_indptr, nnz, t_indices,
                      t_values);
}

}  // namespace

struct TransposeLayout {
    size_t key[2], row[2], val[2], hist, offs, partial, counts, bptr, scal, run_cnt, run_ptr, total;
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
    int64_t n_scan = n_hist > n_voxels ? n_hist : n_voxels;
    if (n_rows > n_scan) n_scan = n_rows;
    const size_t e = (size_t)(nnz > 0 ? nnz : 1);
    for (int b = 0; b < 2; ++b) {
        L.key[b] = take(sizeof(uint32_t) * e);
        L.row[b] = take(sizeof(int32_t) * e);
        L.val[b] = take(sizeof(float) * e);
    }
    L.hist = take(sizeof(uint32_t) * (size_t)n_hist);
    L.offs = take(sizeof(uint32_t) * (size_t)n_hist);
    L.partial = take(sizeof(uint32_t) * (size_t)((n_scan + kScanChunk - 1) / kScanChunk + 1));
    L.counts = take(sizeof(uint32_t) * ((size_t)n_voxels + 1));   // difference array, then counts
    L.bptr = take(sizeof(int64_t) * (size_t)(nb + 1));
    L.scal = take(64);   // unsorted-rows flag, path flag, run histogram length
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
template <typename OUT, bool INCL = false>
static hipError_t scan_excl(const uint32_t *in, Count n, int64_t n_max, uint32_t *partial, OUT *out,
                            int64_t *total64, Gate g, hipStream_t s)
{
    const unsigned nb = stride_grid((n_max + kScanChunk - 1) / kScanChunk);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s, in, n, partial, g);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanTop), 0, s, partial, n, total64, g);
    hipLaunchKernelGGL((k_scan_down<OUT, INCL>), dim3(nb), dim3(kBlock), 0, s, in, n, partial, out, g);
    return hipGetLastError();
}

/*
 * One stable LSD radix sort of (key, row, value) triples by key: `passes`
 * passes of 8 bits, keys above clamp sorted as clamp, ping-pong through
 * (k1, r1, v1) and (k0, r0, v0) (the input may be separate), the last pass
 * writing rows and values to (rows_out, vals_out), and with keys_out its keys
 * to the pass's own key buffer (*keys_out = that buffer).  n is a host or
 * device count, at most n_max.
 */
static hipError_t radix_sort(const uint32_t *keys, const int32_t *rows, const float *vals, Count n, int64_t n_max,
                             uint32_t clamp, int passes, uint32_t *k0, int32_t *r0, float *v0, uint32_t *k1,
                             int32_t *r1, float *v1, int32_t *rows_out, float *vals_out, uint32_t **keys_out,
                             uint32_t *hist, uint32_t *offs, uint32_t *partial, int64_t *hist_len_dev, Gate g,
                             hipStream_t s)
{
    const int64_t tiles_max = (n_max + kSortTile - 1) / kSortTile;
    const unsigned grid = stride_grid(tiles_max);
    const Count hn = hist_len_dev ? Count{0, hist_len_dev} : Count{(int64_t)kRadix * tiles_max, nullptr};
    const uint32_t *kin = keys;
    const int32_t *rin = rows;
    const float *vin = vals;
    hipError_t e;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kRadixBits;
        const bool last = p == passes - 1;
        uint32_t *kbuf = (p & 1) ? k0 : k1;
        uint32_t *kout = last ? (keys_out ? kbuf : nullptr) : kbuf;
        int32_t *rout = last ? rows_out : ((p & 1) ? r0 : r1);
        float *vout = last ? vals_out : ((p & 1) ? v0 : v1);
        hipLaunchKernelGGL(k_rs_hist, dim3(grid), dim3(kBlock), 0, s, kin, n, clamp, shift, hist, g);
        if ((e = scan_excl<uint32_t>(hist, hn, (int64_t)kRadix * tiles_max, partial, offs, nullptr, g, s)) !=
            hipSuccess)
            return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3(grid), dim3(kBlock), 0, s, kin, rin, vin, n, clamp, shift, offs, kout,
                           rout, vout, g);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (last && keys_out) *keys_out = kout;
        kin = kout;
        rin = rout;
        vin = vout;
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
    int32_t *unsorted = reinterpret_cast<int32_t *>(ws + L.scal);
    int32_t *use_runs = unsorted + 1;
    int64_t *hist_len = reinterpret_cast<int64_t *>(ws + L.scal + 8);
    uint32_t *run_cnt = reinterpret_cast<uint32_t *>(ws + L.run_cnt);
    int64_t *run_ptr = reinterpret_cast<int64_t *>(ws + L.run_ptr);
    const Gate always{nullptr, 0};
    hipError_t e;

    // runs of every row, the unsorted flag and the entries per column as a difference
    // array; then entries per column (inclusive scan) and the voxel-row pointers
    hipLaunchKernelGGL(k_zero_u32, dim3(blocks_of((int64_t)n_voxels + 1, kBlock)), dim3(kBlock), 0, s, counts,
                       (int64_t)n_voxels + 1);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kBlock), 0, s, reinterpret_cast<uint32_t *>(unsorted), (int64_t)1);
    if (nnz > 0 && n_rows > 0)
        hipLaunchKernelGGL(k_run_count, dim3(blocks_of(n_rows, kWavesPerBlock)), dim3(kBlock), 0, s, indptr, indices,
                           n_rows, n_voxels, run_cnt, unsorted, counts);
    if ((e = scan_excl<uint32_t, true>(counts, Count{n_voxels, nullptr}, n_voxels, partial, counts, nullptr, always,
                                       s)) != hipSuccess)
        return e;
    if ((e = scan_excl<int64_t>(counts, Count{n_voxels, nullptr}, n_voxels, partial, t_indptr, t_indptr + n_voxels,
                                always, s)) != hipSuccess)
        return e;
    if (nnz == 0 || n_rows == 0) return hipSuccess;

    const int nb = (n_voxels + kBucketCols - 1) >> kBucketShift;
    if ((e = scan_excl<int64_t>(run_cnt, Count{n_rows, nullptr}, n_rows, partial, run_ptr, run_ptr + n_rows, always,
                                s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_run_sizes, dim3(1), dim3(1), 0, s, run_ptr + n_rows, nnz, use_runs, hist_len);
    const Gate runs{use_runs, 1}, entries{use_runs, 0};

    // run path: at most nnz / 2 runs.  Run records in the first half of key[0], row[0],
    // val[0]; first entries and the sorted rows and ids from `half` on; the sort's other
    // buffers are key/row/val[1]; after the sort, each run's first entry and length go to
    // row[1] and val[1] (free then: the sorted keys are in key[0] or key[1])
    {
        const int64_t half = (nnz + 1) / 2;
        uint32_t *rkey = key[0];
        int32_t *rrow = row[0];
        float *rid = val[0];
        uint32_t *rsrc = key[0] + half;
        int32_t *brow = row[0] + half;
        float *bid = val[0] + half;
        uint32_t *bsrc = reinterpret_cast<uint32_t *>(row[1]);
        uint32_t *blen = reinterpret_cast<uint32_t *>(val[1]);
        int64_t *bptr = reinterpret_cast<int64_t *>(ws + L.bptr);
        const Count n_runs{0, run_ptr + n_rows};
        hipLaunchKernelGGL(k_run_emit, dim3(blocks_of(n_rows, kWavesPerBlock)), dim3(kBlock), 0, s, indptr, indices,
                           n_rows, n_voxels, run_ptr, rkey, rrow, rid, rsrc, runs);
        // stable sort of the runs by bucket
        uint32_t *skeys = nullptr;
        if ((e = radix_sort(rkey, rrow, rid, n_runs, half, 0xffffffffu, transpose_passes(nb), key[0], row[0], val[0],
                            key[1], row[1], val[1], brow, bid, &skeys, hist, offs, partial, hist_len, runs, s)) !=
            hipSuccess)
            return e;
        hipLaunchKernelGGL(k_bucket_bounds, dim3(stride_grid(blocks_of(half + 1, kBlock))), dim3(kBlock), 0, s, skeys,
                           n_runs, nb, bptr, runs);
        hipLaunchKernelGGL(k_run_gather, dim3(stride_grid(blocks_of(half, kBlock))), dim3(kBlock), 0, s, bid, brow,
                           rsrc, run_ptr, indptr, n_runs, bsrc, blen, runs);
        hipLaunchKernelGGL(k_bucket_place, dim3(blocks_of(nb, kColWaves)), dim3(kColWaves * kWave), 0, s, indices,
                           values, n_voxels, nb, bptr, brow, bsrc, blen, t_indptr, (uint32_t)nnz, t_indices, t_values,
                           unsorted, runs);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }

    // entry path: row id of every entry (into row[0]), then a radix sort of the entries by
    // column (invalid columns as n_voxels, sorted last)
    hipLaunchKernelGGL(k_expand_rows, dim3(blocks_of(n_rows, kWavesPerBlock)), dim3(kBlock), 0, s, indptr, n_rows, nnz,
                       row[0], entries);
    return radix_sort(reinterpret_cast<const uint32_t *>(indices), row[0], values, Count{nnz, nullptr}, nnz,
                      (uint32_t)n_voxels, transpose_passes(n_voxels + 1), key[0], row[0], val[0], key[1], row[1],
                      val[1], t_indices, t_values, nullptr, hist, offs, partial, nullptr, entries, s);
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
