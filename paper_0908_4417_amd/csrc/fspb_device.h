/*
 * Internal records shared by the host plan code and the gfx950 kernels.
 * Not part of the public ABI.
 */
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fspb {

constexpr int kWave = 64;            // CDNA wavefront
constexpr int kRowsPerTile = 64;     // grid rows (iy, iz) per count/fill tile: one per lane
constexpr int kMaxTerms = 4;
// flag in PlanDev::ext[].x: the grid row has non-member voxels between its first and last member
constexpr int kExtHoles = 1 << 30;
// erfc on [0, kErfcMax] by piecewise quadratics on kErfcIntervals equal intervals
// (training targets of the kernel surrogate)
constexpr int kErfcIntervals = 512;
constexpr float kErfcMax = 4.0f;
// erf on [0, kErfMax] by linear interpolation between kErfIntervals + 1 equally
// spaced nodes, 256 per unit of argument (the fill; held at +-erf(kErfMax)
// beyond the last node: erfc(3.75) = 1.1e-7, below 1e-5 of any bracket of Eq. 3
// that enters a coefficient above 1 % of the maximum).  The table holds each interval as (intercept, slope) in
// the table coordinate: kErfIntervals entries on [0, kErfMax] (compact form, odd
// symmetry for negative arguments), then 2 kErfIntervals on [-kErfMax, kErfMax]
// (mirrored form, coordinate offset by kErfIntervals, first entry constant)
constexpr int kErfIntervals = 960;
constexpr float kErfMax = 3.75f;

/* Per-beamlet record, built in FP64 on the host (Fig. 1 geometry). */
struct alignas(16) BeamletRec {
    double S[3];          // source
    double e[3];          // unit central axis
    double eu[3], ev[3];  // unit lateral axes (x', z')
    double tA, tB;        // entry / exit distances from S
    double step;          // spacing of the table points on AB
    double sad;
    // VOI row interval (one block, copied as a whole by the fill): the cutoffs over SAD
    // (|U| <= cu_sad t', |V| <= cv_sad t'); t', U and V of the centre of voxel (0, iy, iz),
    // relative to S, as row_t[0] + iy row_t[1] + iz row_t[2] (likewise row_u, row_v); the
    // row's four conditions c0 + c1[c] x <= 0 as r1[c] = 1 / c1[c] (0 if c1[c] = 0) and the
    // signs of c1 (c1_pos, c1_neg below); dx: the change of t', U, V per column
    double cu_sad, cv_sad;
    double row_t[3], row_u[3], row_v[3];
    double r1[4];
    double dx[3];
    float half_a, half_b;   // a/2, b/2 at the iso plane
    float tA_f, inv_step_f;
    float sad_f, tau_max_f;   // SAD; n_table - 1
    float t1_f, U1_f, V1_f;   // change of t', U, V per voxel step along x
    float pad_f;
    float ha[kMaxTerms], hb[kMaxTerms];   // c2_k a/2, c2_k b/2
    float a_f;                // beamlet side a (the surrogate's fourth input)
    int32_t mlp_ok;           // square beamlet with a inside the surrogate's training box
    int32_t theta_k;          // general kernel: A row below this beamlet's angle
    float theta_f;            //   and the fraction towards the next row
    int32_t n_table;      // table points (0: axis misses the grid)
    int32_t table_off;    // first entry in the plan's table array
    int32_t iy0, n_iy;    // bounding rows of the VOI
    int32_t iz0, n_iz;
    int32_t tile0;        // first tile (plan-local)
    int32_t n_tiles;
    int32_t c1_pos, c1_neg;   // bit c set where c1[c] > 0, where c1[c] < 0
};

/* Everything a kernel needs about one plan; lives in device memory. */
struct alignas(16) PlanDev {
    // grid
    int32_t nx, ny, nz, wpr;     // wpr = 32-bit mask words per grid row
    double org[3], sp[3];
    double lo[3];                // lower corner of the bounding box
    const float *density;
    uint32_t *bits;              // [nz*ny][wpr] density > rho_min
    int2 *ext;                   // [nz*ny] first / last member column of each grid row; bit 30
                                 // of .x set: non-member voxels lie between them
    float rho_min;
    // kernel
    int32_t n_terms, n_pdd;
    float w4[kMaxTerms];         // c1 / 4
    float sig0[kMaxTerms], sig1[kMaxTerms];
    float c2[kMaxTerms];
    float pdd_inv_step, pdd_max;   // 1/step; n_pdd - 1
    const float *pdd;
    const float2 *erf_tab;       // [3 kErfIntervals]: compact form, then mirrored form
    // general kernel form (0: the analytic form above): c tables [3][n_terms][n_cdepth]
    // (c1, c2, c3), A [n_theta][n_adepth]
    int32_t gen, n_cdepth, n_theta, n_adepth;
    float c_inv_step, c_max, a_inv_step, a_max;
    const float *ctab;
    const float *atab;
    // beamlets and tables
    int32_t n_beamlets, max_table;
    int32_t ray_iters;           // bound on the per-interval Siddon loop
    int32_t n_tiles;
    int32_t max_tiles;           // most tiles of any beamlet
    int32_t depth_mode;          // 0: exact path integral; 1: trilinear samples + trapezoids
    int32_t tiles_mode;          // fill tiles: 0 chosen per beamlet, 1 row block, 2 row list
    const BeamletRec *rec;
    float *tables;
    // Fill tiles, from the count pass: either the beamlet's row block in runs of kRowsPerTile
    // grid rows, or, where most of the block's rows hold no VOI member, its list of the rows
    // that do (row index in the block, ascending) in runs of kRowsPerTile list entries
    int32_t *tile_count;         // [n_tiles] members of each block tile
    int32_t *row_list;           // [n_tiles kRowsPerTile]: beamlet j's list at tile0 kRowsPerTile
    int32_t *list_count;         // [n_tiles] members of each list tile (first ceil(row_ne / 64) of a beamlet's)
    int32_t *row_ne;             // [n_beamlets] length of beamlet j's list, -1: block tiles
    int64_t *row_nnz;            // [n_beamlets]
    int64_t *nnz;                // [1]
    // attached kernel surrogate (use_mlp = 0: analytic fill)
    const float *mlp_p;          // FP32 parameters
    const uint16_t *mlp_w2;      // BF16 W2 [out][in]
    int32_t use_mlp;
    int32_t erf_mirrored;        // fill stages erf on [-kErfMax, kErfMax] (analytic and tabulated forms)
    int32_t erf_nc;              // every term's c2 a/2 over sigma stays below kErfMax: the first
                                 // argument of a bracket never passes the mirrored table's top
    float d_floor;               // lower bound applied to D: 0 when every weight (c1) and every
                                 // depth-dose (A) entry is >= 0, so that D >= 0 exactly; else -inf
    int32_t erf_square;          // every beam's beamlets are square (a = b)
    int32_t erf_mode;            // how the fill reads erf (0..3, see erf_mirrored_mode in the kernels)
};

/* Caller-owned CSR output of one plan (device pointers). */
struct alignas(16) OutDev {
    int64_t *indptr;             // n_beamlets + 1
    int32_t *indices;            // capacity
    float *values;               // capacity
    int64_t capacity;
    int32_t *overflow;           // set to 1 if a fill would exceed capacity
    int32_t row0;                // first row written: entry positions are relative to indptr[row0]
    int32_t check_nnz;           // whole-plan fill: write nothing when PlanDev::nnz > capacity
};

/* Launchers (fspb_kernels.hip).  Each returns the launch's hipError_t. */
hipError_t launch_prep(const PlanDev *dplan, const PlanDev &h, hipStream_t s);
hipError_t launch_raytrace(const PlanDev *dplan, const PlanDev &h, hipStream_t s);
hipError_t launch_count(const PlanDev *dplan, const PlanDev &h, hipStream_t s);
hipError_t launch_scan(const PlanDev *dplan, const OutDev *dout, const PlanDev &h, hipStream_t s);
/* Fill rows row0 .. row0 + n_rows - 1 (dout->row0 must equal row0). */
hipError_t launch_fill(const PlanDev *dplan, const OutDev *dout, const PlanDev &h, int row0, int n_rows,
                       hipStream_t s);
/* Dynamic LDS of one fill workgroup: in the form launch_fill uses, or in a given erf table form. */
size_t fill_shared_bytes(const PlanDev &h);
size_t fill_shared_bytes(const PlanDev &h, bool mirrored_erf);
bool fill_mirrored_erf(const PlanDev &h);
/* The erf mode of the plan's fill when it stages the mirrored table (1, 2 or 3). */
int mirrored_erf_mode(const PlanDev &h);
/* 1 when the mirrored erf table keeps the plan's fill at the same workgroups per CU as the
 * compact table (occupancy query for the current device); 0 otherwise. */
int choose_erf_form(const PlanDev &h);

/* Eq. 1 and its adjoint on a CSR. */
/* Eq. 1 on a beamlet-row CSR and on its voxel-row transpose (fspb_sparse.hip). */
hipError_t launch_fluence_dose(const int64_t *indptr, const int32_t *indices, const float *values, int n_rows,
                               int n_voxels, const float *w, float *dose, hipStream_t s);
hipError_t launch_fluence_gradient(const int64_t *indptr, const int32_t *indices, const float *values, int n_rows,
                                   int n_voxels, const float *r, float *g, hipStream_t s);
hipError_t launch_voxel_dose(const int64_t *t_indptr, const int32_t *t_indices, const float *t_values, int n_voxels,
                             int n_w, const float *w, float *dose, hipStream_t s);
size_t transpose_workspace(int64_t nnz, int n_voxels, int n_rows);
int transpose_passes(int n_keys);
/* Stream-ordered (no host synchronisation); entries whose column lies outside
 * [0, n_voxels) are left out of the voxel rows. */
hipError_t launch_transpose(const int64_t *indptr, const int32_t *indices, const float *values, int n_rows,
                            int n_voxels, int64_t nnz, int64_t *t_indptr, int32_t *t_indices, float *t_values,
                            void *workspace, hipStream_t s);
/* Size of the static device scratch of the allocation-free transpose, and its
 * device address on the current device (looked up once per device). */
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
hipError_t noalloc_scratch_ptr(void **out);

/* Batched launches over n_plans plans (persistent grids). */
hipError_t launch_batch_wave(int stage, const PlanDev *const *plans, const int64_t *start, int n_plans,
                             int grid, hipStream_t s);   // stage 0 prep, 1 raytrace, 2 count
hipError_t launch_batch_scan(const PlanDev *const *plans, const OutDev *outs, int n_plans, hipStream_t s);
hipError_t launch_batch_reset(int *counters, int n, hipStream_t s);
/* per_item work items per queue fetch; tile_group consecutive tiles per wave step. */
hipError_t launch_batch_fill(int K, int W, const PlanDev *const *plans, const OutDev *outs, const int2 *items,
                             int n_items, int *counter, int per_item, int tile_group, int grid, size_t lds,
                             hipStream_t s);

}  // namespace fspb
