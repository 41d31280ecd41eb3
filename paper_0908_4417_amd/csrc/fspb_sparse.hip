/*
 * gfx950 kernels for Eq. 1 on the dose-coefficient matrix D_ij.
 *
 *   beamlet-row CSR (what the fill writes: row j = beamlet, columns = voxels)
 *     k_fluence_dose      dose_i += w_j D_ij with FP32 atomics   -- one wave per row
 *     k_fluence_gradient  g_j = sum_i D_ij r_i, fixed order      -- one wave per row
 *   voxel-row CSR (row i = voxel, columns = beamlets), built by
 *     k_expand_rows, k_col_count + scan         row ids of the entries, voxel-row pointers
 *     k_rs_hist, scan, k_rs_scatter             one pass of a stable LSD radix sort on the
 *                                               voxel index, 8 bits per pass
 *     k_voxel_dose        dose_i = sum_j D_ij w_j, fixed order  -- 16 lanes per voxel row
 *
 * The radix sort is stable and the input rows are in ascending beamlet order,
 * so every voxel row lists its beamlets in ascending order: the transpose is
 * canonical and bit-reproducible.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

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

/* rows[e] = j for every entry e of row j (clamped to [0, nnz)); one wave per row. */
__global__ __launch_bounds__(kBlock) void k_expand_rows(const int64_t *__restrict__ indptr, int n_rows, int64_t nnz,
                                                        int32_t *__restrict__ rows)
{
    const int j = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (j >= n_rows) return;
    const int64_t e0 = indptr[j] > 0 ? indptr[j] : 0, e1 = indptr[j + 1] < nnz ? indptr[j + 1] : nnz;
    for (int64_t e = e0 + lane_id(); e < e1; e += kWave) rows[e] = j;
}

/* Entries per voxel; an index outside [0, n_voxels) raises *bad. */
__global__ __launch_bounds__(kBlock) void k_col_count(const int32_t *__restrict__ indices, int64_t nnz,
                                                      int n_voxels, uint32_t *__restrict__ counts,
                                                      int32_t *__restrict__ bad)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz; e += stride) {
        const uint32_t i = (uint32_t)indices[e];
        if (i < (uint32_t)n_voxels) atomicAdd(counts + i, 1u);
        else *bad = 1;
    }
}

/* Scan, phase 1: sum of each kScanChunk-value chunk. */
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t *__restrict__ in, int64_t n,
                                                        uint32_t *__restrict__ partial)
{
    __shared__ uint32_t s_w[kWavesPerBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) v += base + k < n ? in[base + k] : 0u;
    v = wave_sum(v);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kWavesPerBlock; ++k) t += s_w[k];
        partial[blockIdx.x] = t;
    }
}

/* Scan, phase 2: exclusive scan of the chunk sums in place (one workgroup);
 * partial[nb] = total, also stored to *total64 when given. */
__global__ __launch_bounds__(kScanTop) void k_scan_top(uint32_t *__restrict__ partial, int nb,
                                                       int64_t *__restrict__ total64)
{
    __shared__ uint32_t s_w[kScanTop / kWave];
    const int l = lane_id(), w = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += kScanTop) {
        const int i = b0 + threadIdx.x;
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

/* Scan, phase 3: exclusive scan within each chunk plus its chunk offset. */
template <typename OUT>
__global__ __launch_bounds__(kBlock) void k_scan_down(const uint32_t *__restrict__ in, int64_t n,
                                                      const uint32_t *__restrict__ partial, OUT *__restrict__ out)
{
    __shared__ uint32_t s_w[kWavesPerBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        sum += v[k];
    }
    uint32_t total;
    uint32_t run = partial[blockIdx.x] + block_excl_scan(sum, s_w, &total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = (OUT)run;
        run += v[k];
    }
}

/* Radix pass, phase 1: digit histogram of each kSortTile-entry tile, stored
 * digit-major (hist[d * n_tiles + tile]) so that one exclusive scan gives every
 * (digit, tile) its first output slot. */
__global__ __launch_bounds__(kBlock) void k_rs_hist(const uint32_t *__restrict__ keys, int64_t n, int shift,
                                                    uint32_t *__restrict__ hist, int n_tiles)
{
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile + threadIdx.x;
#pragma unroll 4
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = base + (int64_t)r * kBlock;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
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
 * NULL (last pass).
 */
__global__ __launch_bounds__(kBlock) void k_rs_scatter(const uint32_t *__restrict__ keys_in,
                                                       const int32_t *__restrict__ rows_in,
                                                       const float *__restrict__ vals_in, int64_t n, int shift,
                                                       const uint32_t *__restrict__ offs, int n_tiles,
                                                       uint32_t *__restrict__ keys_out,
                                                       int32_t *__restrict__ rows_out,
                                                       float *__restrict__ vals_out)
{
    __shared__ uint32_t s_key[kSortTile];
    __shared__ int32_t s_row[kSortTile];
    __shared__ float s_val[kSortTile];
    __shared__ uint32_t cnt[kWavesPerBlock][kRadix];   // per wave: digit counts, then first tile-local slot
    __shared__ uint32_t goff[kRadix];                  // global slot of tile-local slot 0 of each digit's run
    __shared__ uint32_t s_w[kWavesPerBlock];
    constexpr int kSub = kSortTile / kWavesPerBlock;    // entries per wave
    const int t = threadIdx.x, wave = t >> 6, lane = t & (kWave - 1);
    const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
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
        key[r] = valid ? keys_in[i] : 0u;
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
        goff[t] = offs[(int64_t)t * n_tiles + blockIdx.x] - start;
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
 * whose columns share a bucket of kBucketCols columns (col >> kBucketShift).
 * The transpose sorts the runs by bucket (stably, so a bucket's runs keep row
 * order), then one wave per bucket walks its runs' entries in that order and
 * places each with a stable counting sort on the column's low bits: the
 * output is the stable sort of the row-major entries by column, as the radix
 * path gives, for about two reads and one write of the matrix.  Buckets of 32
 * columns: with 128 the slab's transpose took 29 ms, with 32 20 ms, with 16 19 ms
 * (the pelvis 22, 14 and 17 ms; the radix path 30 and 18 ms); staging each batch
 * of runs in LDS brought the 32-column case to 12.6 ms (pelvis 11.9 ms).
 */
constexpr int kBucketShift = 5;
constexpr int kBucketCols = 1 << kBucketShift;

/* run_cnt[j] = runs of row j; one wave per row.  *unsorted is set when a row's
 * columns are not strictly ascending. */
__global__ __launch_bounds__(kBlock) void k_run_count(const int64_t *__restrict__ indptr,
                                                      const int32_t *__restrict__ indices, int n_rows,
                                                      uint32_t *__restrict__ run_cnt, int32_t *__restrict__ unsorted)
{
    const int j = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (j >= n_rows) return;
    const int lane = lane_id();
    const int64_t e0 = indptr[j], e1 = indptr[j + 1];
    uint32_t runs = 0;
    int prev = -1;                                     // column of the entry before the chunk
    bool down = false;
    for (int64_t c = e0; c < e1; c += kWave) {
        const int64_t e = c + lane;
        const bool in = e < e1;
        const int col = in ? indices[e] : 0;
        int cp = __shfl_up(col, 1, kWave);
        if (lane == 0) cp = prev;
        const int b = col >> kBucketShift;
        runs += (uint32_t)__popcll(__ballot(in && (cp < 0 || b != (cp >> kBucketShift))));
        down = down || (in && cp >= 0 && col <= cp);
        prev = __shfl(col, kWave - 1, kWave);
    }
    if (lane == 0) run_cnt[j] = runs;
    if (__ballot(down) && lane == 0) *unsorted = 1;
}

/* Records of every run (row-major run ids from run_ptr): its bucket, row, id
 * (as the value payload of the run sort) and first entry. */
__global__ __launch_bounds__(kBlock) void k_run_emit(const int64_t *__restrict__ indptr,
                                                     const int32_t *__restrict__ indices, int n_rows,
                                                     const int64_t *__restrict__ run_ptr,
                                                     uint32_t *__restrict__ run_key, int32_t *__restrict__ run_row,
                                                     float *__restrict__ run_id, uint32_t *__restrict__ run_src)
{
    const int j = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (j >= n_rows) return;
    const int lane = lane_id();
    const int64_t e0 = indptr[j], e1 = indptr[j + 1];
    uint32_t r = (uint32_t)run_ptr[j];
    int prev = -1;                                     // column of the entry before the chunk
    for (int64_t c = e0; c < e1; c += kWave) {
        const int64_t e = c + lane;
        const bool in = e < e1;
        const int col = in ? indices[e] : 0;
        int cp = __shfl_up(col, 1, kWave);
        if (lane == 0) cp = prev;
        const int b = col >> kBucketShift;
        const bool start = in && (cp < 0 || b != (cp >> kBucketShift));
        const uint64_t m = __ballot(start);
        if (start) {
            const uint32_t id = r + (uint32_t)mbcnt64(m);
            run_key[id] = (uint32_t)b;
            run_row[id] = j;
            run_id[id] = __uint_as_float(id);
            run_src[id] = (uint32_t)e;
        }
        r += (uint32_t)__popcll(m);
        prev = __shfl(col, kWave - 1, kWave);
    }
}

/*
 * The same placement for rows with strictly ascending columns, column by
 * column.  A batch of 64 runs of the bucket (rows ascending; each at most 32
 * entries, one per column) is first copied into LDS, the runs' entries
 * flattened over the lanes so that all loads are independent; then each lane
 * holds one run and, at column c, the lanes whose next entry has column c write
 * it, ranked by lane, so each column's entries from the batch go out as one
 * contiguous stretch.
 */
constexpr int kColWaves = 2;                               // waves per workgroup of k_bucket_columns

__global__ __launch_bounds__(kColWaves * kWave) void k_bucket_columns(
    const int64_t *__restrict__ indptr, const int32_t *__restrict__ indices, const float *__restrict__ values,
    int n_voxels, int n_buckets, const int64_t *__restrict__ run_ptr, const uint32_t *__restrict__ run_src,
    const int64_t *__restrict__ b_ptr, const int32_t *__restrict__ b_rows, const float *__restrict__ b_ids,
    const int64_t *__restrict__ t_indptr, uint32_t nnz, int32_t *__restrict__ t_indices,
    float *__restrict__ t_values)
{
    constexpr int kStage = kWave * kBucketCols;            // 64 runs of at most 32 entries
    __shared__ uint32_t s_pos[kColWaves][kBucketCols];
    __shared__ float s_val[kColWaves][kStage];
    __shared__ uint8_t s_col[kColWaves][kStage];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int b = blockIdx.x * kColWaves + wave;
    if (b >= n_buckets) return;
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
        // lane i: run qb + i (row, first entry, length)
        const int64_t q = qb + lane;
        int row = 0;
        uint32_t src = 0u, len = 0u;
        if (q < q1) {
            row = b_rows[q];
            const uint32_t id = __float_as_uint(b_ids[q]);
            src = run_src[id];
            const uint32_t end = (int64_t)id + 1 < run_ptr[row + 1] ? run_src[id + 1] : (uint32_t)indptr[row + 1];
            len = min(end - src, (uint32_t)kBucketCols);   // at most 32 for strictly ascending rows
        }
        uint32_t incl = len;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d, kWave);
            if (lane >= d) incl += y;
        }
        const uint32_t excl = incl - len;
        const uint32_t total = __shfl(incl, kWave - 1, kWave);   // <= kStage
        // stage: entry p of the batch (run walked wave-uniformly) -> LDS
        int rcur = 0;
        for (uint32_t c0 = 0; c0 < total; c0 += kWave) {
            while (rcur + 1 < kWave && (uint32_t)__builtin_amdgcn_readlane((int)excl, rcur + 1) <= c0) ++rcur;
            const uint32_t p = c0 + lane;
            int rr = rcur;
            for (int k = rcur + 1; k < kWave; ++k) {
                const uint32_t ek = (uint32_t)__builtin_amdgcn_readlane((int)excl, k);
                if (ek > c0 + kWave - 1) break;
                if (p >= ek) rr = k;
            }
            // shuffles on every lane: the source lane rr may be past the end of the batch's entries
            const uint32_t e = __shfl(src, rr, kWave) + (p - __shfl(excl, rr, kWave));
            if (p < total) {
                sc[p] = (uint8_t)(indices[e] - col0);
                sv[p] = values[e];
            }
        }
        __builtin_amdgcn_wave_barrier();
        // place: lane = run, its entries sc/sv[excl, excl + len)
        uint32_t k = excl;
        const uint32_t end = excl + len;
        int ca = k < end ? (int)sc[k] : kBucketCols;
        for (int c = 0; c < kBucketCols; ++c) {
            const bool has = ca == c;
            const uint64_t m = __ballot(has);
            if (m == 0) continue;
            const uint32_t p0 = pos[c];
            if (has) {
                const uint32_t p = p0 + (uint32_t)mbcnt64(m);
                if (p < nnz) {   // always true for consistent runs; keeps every store in bounds
                    t_indices[p] = row;
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
 * Bucket b's entries into the voxel-row arrays; one wave per bucket.  Its runs
 * (positions b_ptr[b] .. b_ptr[b + 1] of the run sort's output, rows ascending)
 * are taken 64 at a time, their entries flattened over the lanes in run
 * order; an entry of column col goes to t_indptr[col] + (entries of col placed
 * before it), counted per column in LDS.  Equal columns within a 64-entry
 * chunk are ranked by lane with seven ballots over the column's low bits.
 */
__global__ __launch_bounds__(kBlock) void k_bucket_scatter(const int64_t *__restrict__ indptr,
                                                           const int32_t *__restrict__ indices,
                                                           const float *__restrict__ values, int n_voxels,
                                                           int n_buckets, const int64_t *__restrict__ run_ptr,
                                                           const uint32_t *__restrict__ run_src,
                                                           const int64_t *__restrict__ b_ptr,
                                                           const int32_t *__restrict__ b_rows,
                                                           const float *__restrict__ b_ids,
                                                           const int64_t *__restrict__ t_indptr, uint32_t nnz,
                                                           int32_t *__restrict__ t_indices, float *__restrict__ t_values)
{
    __shared__ uint32_t s_base[kWavesPerBlock][kBucketCols];
    __shared__ uint32_t s_cnt[kWavesPerBlock][kBucketCols];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int b = blockIdx.x * kWavesPerBlock + wave;
    if (b >= n_buckets) return;
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
        // lane i: run qb + i (row, first entry, length)
        const int64_t q = qb + lane;
        int row = 0;
        uint32_t src = 0u, len = 0u;
        if (q < q1) {
            row = b_rows[q];
            const uint32_t id = __float_as_uint(b_ids[q]);
            src = run_src[id];
            const uint32_t end = (int64_t)id + 1 < run_ptr[row + 1] ? run_src[id + 1] : (uint32_t)indptr[row + 1];
            len = end - src;
        }
        uint32_t incl = len;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d, kWave);
            if (lane >= d) incl += y;
        }
        const uint32_t excl = incl - len;
        const uint32_t total = __shfl(incl, kWave - 1, kWave);
        int rcur = 0;
        for (uint32_t c0 = 0; c0 < total; c0 += kWave) {
            // run of entry p: the last lane whose exclusive prefix is <= p (walked wave-uniformly)
            while (rcur + 1 < kWave && (uint32_t)__builtin_amdgcn_readlane((int)excl, rcur + 1) <= c0) ++rcur;
            const uint32_t p = c0 + lane;
            int rr = rcur;
            for (int k = rcur + 1; k < kWave; ++k) {
                const uint32_t ek = (uint32_t)__builtin_amdgcn_readlane((int)excl, k);
                if (ek > c0 + kWave - 1) break;
                if (p >= ek) rr = k;
            }
            const bool in = p < total;
            const uint32_t e = __shfl(src, rr, kWave) + (p - __shfl(excl, rr, kWave));
            const int rowj = __shfl(row, rr, kWave);
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

struct TransposeLayout {
    size_t key[2], row[2], val[2], hist, offs, partial, counts, bad, run_cnt, run_ptr, total;
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
    L.counts = take(sizeof(uint32_t) * (size_t)n_voxels);
    L.bad = take(2 * sizeof(int32_t));   // bad column flag, unsorted-rows flag
    L.run_cnt = take(sizeof(uint32_t) * (size_t)(n_rows > 0 ? n_rows : 1));
    L.run_ptr = take(sizeof(int64_t) * ((size_t)n_rows + 1));
    L.total = off;
    return L;
}

size_t transpose_workspace(int64_t nnz, int n_voxels, int n_rows)
{
    return transpose_layout(nnz, n_voxels, n_rows).total;
}

int transpose_passes(int n_voxels)
{
    int bits = 0;
    while (bits < 31 && ((int64_t)1 << bits) < (int64_t)n_voxels) ++bits;
    const int p = (bits + kRadixBits - 1) / kRadixBits;
    return p > 0 ? p : 1;
}

/* Exclusive scan of n uint32 values in -> out (OUT = uint32_t or int64_t);
 * partial[nblocks] receives the total, and *total64 too when given. */
template <typename OUT>
static hipError_t scan_excl(const uint32_t *in, int64_t n, uint32_t *partial, OUT *out, int64_t *total64,
                            hipStream_t s)
{
    const unsigned nb = blocks_of(n, kScanChunk);
    if (nb > 0) hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s, in, n, partial);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanTop), 0, s, partial, (int)nb, total64);
    if (nb > 0) hipLaunchKernelGGL((k_scan_down<OUT>), dim3(nb), dim3(kBlock), 0, s, in, n, partial, out);
    return hipGetLastError();
}

hipError_t launch_transpose(const int64_t *indptr, const int32_t *indices, const float *values, int n_rows,
                            int n_voxels, int64_t nnz, int64_t *t_indptr, int32_t *t_indices, float *t_values,
                            void *workspace, int32_t *bad_host, hipStream_t s)
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
    int32_t *bad = reinterpret_cast<int32_t *>(ws + L.bad);
    hipError_t e;

    // voxel-row pointers: entries per voxel, exclusive scan, total at t_indptr[n_voxels]
    hipLaunchKernelGGL(k_zero_u32, dim3(blocks_of(n_voxels, kBlock)), dim3(kBlock), 0, s, counts, (int64_t)n_voxels);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kBlock), 0, s, reinterpret_cast<uint32_t *>(bad), (int64_t)1);
    if (nnz > 0) {
        const int64_t want = (nnz + kBlock - 1) / kBlock;
        const unsigned g = (unsigned)(want < 65536 ? want : 65536);
        hipLaunchKernelGGL(k_col_count, dim3(g), dim3(kBlock), 0, s, indices, nnz, n_voxels, counts, bad);
    }
    if ((e = scan_excl<int64_t>(counts, n_voxels, partial, t_indptr, t_indptr + n_voxels, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(bad_host, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    if (*bad || nnz == 0) return hipSuccess;

    // runs (stretches of a row within one bucket of columns): the run transpose when they are
    // at most half the entries (a plan's D has tens of entries per run), else the radix sort
    uint32_t *run_cnt = reinterpret_cast<uint32_t *>(ws + L.run_cnt);
    int64_t *run_ptr = reinterpret_cast<int64_t *>(ws + L.run_ptr);
    int32_t *unsorted = bad + 1;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kBlock), 0, s, reinterpret_cast<uint32_t *>(unsorted), (int64_t)1);
    hipLaunchKernelGGL(k_run_count, dim3(blocks_of(n_rows, kWavesPerBlock)), dim3(kBlock), 0, s, indptr, indices,
                       n_rows, run_cnt, unsorted);
    if ((e = scan_excl<int64_t>(run_cnt, n_rows, partial, run_ptr, run_ptr + n_rows, s)) != hipSuccess) return e;
    int64_t n_runs = 0;
    int32_t rows_unsorted = 0;
    if ((e = hipMemcpyAsync(&n_runs, run_ptr + n_rows, sizeof(int64_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(&rows_unsorted, unsorted, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    if (2 * n_runs <= nnz) {
        const int64_t R = n_runs;
        const int nb = (n_voxels + kBucketCols - 1) >> kBucketShift;
        // run records in the first half of key[0], row[0], val[0]; first entries and the
        // sorted runs in their second half; bucket counts and pointers in `counts`
        uint32_t *rkey = key[0];
        int32_t *rrow = row[0];
        float *rid = val[0];
        uint32_t *rsrc = key[0] + R;
        int32_t *brow = row[0] + R;
        float *bid = val[0] + R;
        uint32_t *bcnt = counts;
        int64_t *bptr = reinterpret_cast<int64_t *>(ws + L.counts + ((sizeof(uint32_t) * (size_t)nb + 7) & ~(size_t)7));
        hipLaunchKernelGGL(k_run_emit, dim3(blocks_of(n_rows, kWavesPerBlock)), dim3(kBlock), 0, s, indptr, indices,
                           n_rows, run_ptr, rkey, rrow, rid, rsrc);
        hipLaunchKernelGGL(k_zero_u32, dim3(blocks_of(nb, kBlock)), dim3(kBlock), 0, s, bcnt, (int64_t)nb);
        {
            const int64_t want = (R + kBlock - 1) / kBlock;
            const unsigned g = (unsigned)(want < 65536 ? want : 65536);
            hipLaunchKernelGGL(k_col_count, dim3(g), dim3(kBlock), 0, s, reinterpret_cast<const int32_t *>(rkey), R,
                               nb, bcnt, bad);
        }
        if ((e = scan_excl<int64_t>(bcnt, nb, partial, bptr, bptr + nb, s)) != hipSuccess) return e;
        // stable sort of the runs by bucket: passes alternate between key/row/val[1] and the
        // first half of key/row/val[0]; the last one writes rows and ids to brow, bid
        const int rt = (int)blocks_of(R, kSortTile);
        const int rpasses = transpose_passes(nb);
        const uint32_t *kin = rkey;
        const int32_t *rin = rrow;
        const float *vin = rid;
        for (int p = 0; p < rpasses; ++p) {
            const int shift = p * kRadixBits;
            const bool last = p == rpasses - 1;
            const int o = (p & 1) ? 0 : 1;
            uint32_t *kout = last ? nullptr : key[o];
            int32_t *rout = last ? brow : row[o];
            float *vout = last ? bid : val[o];
            hipLaunchKernelGGL(k_rs_hist, dim3(rt), dim3(kBlock), 0, s, kin, R, shift, hist, rt);
            if ((e = scan_excl<uint32_t>(hist, (int64_t)kRadix * rt, partial, offs, nullptr, s)) != hipSuccess)
                return e;
            hipLaunchKernelGGL(k_rs_scatter, dim3(rt), dim3(kBlock), 0, s, kin, rin, vin, R, shift, offs, rt, kout,
                               rout, vout);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            kin = kout;
            rin = rout;
            vin = vout;
        }
        if (rows_unsorted)
            hipLaunchKernelGGL(k_bucket_scatter, dim3(blocks_of(nb, kWavesPerBlock)), dim3(kBlock), 0, s, indptr,
                               indices, values, n_voxels, nb, run_ptr, rsrc, bptr, brow, bid, t_indptr, (uint32_t)nnz,
                               t_indices, t_values);
        else
            hipLaunchKernelGGL(k_bucket_columns, dim3(blocks_of(nb, kColWaves)), dim3(kColWaves * kWave), 0, s, indptr,
                               indices, values, n_voxels, nb, run_ptr, rsrc, bptr, brow, bid, t_indptr, (uint32_t)nnz,
                               t_indices, t_values);
        return hipGetLastError();
    }

    // row id of every entry (into row[1], free until the second pass writes it)
    hipLaunchKernelGGL(k_expand_rows, dim3(blocks_of(n_rows, kWavesPerBlock)), dim3(kBlock), 0, s, indptr, n_rows, nnz,
                       row[1]);
    const int n_tiles = (int)blocks_of(nnz, kSortTile);
    const int passes = transpose_passes(n_voxels);
    const uint32_t *kin = reinterpret_cast<const uint32_t *>(indices);
    const int32_t *rin = row[1];
    const float *vin = values;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kRadixBits;
        const bool last = p == passes - 1;
        uint32_t *kout = last ? nullptr : key[p & 1];
        int32_t *rout = last ? t_indices : row[p & 1];
        float *vout = last ? t_values : val[p & 1];
        hipLaunchKernelGGL(k_rs_hist, dim3(n_tiles), dim3(kBlock), 0, s, kin, nnz, shift, hist, n_tiles);
        if ((e = scan_excl<uint32_t>(hist, (int64_t)kRadix * n_tiles, partial, offs, nullptr, s)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3(n_tiles), dim3(kBlock), 0, s, kin, rin, vin, nnz, shift, offs, n_tiles,
                           kout, rout, vout);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        kin = kout;
        rin = rout;
        vin = vout;
    }
    return hipSuccess;
}

}  // namespace fspb
