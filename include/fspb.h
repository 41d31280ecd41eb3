/*
 * fspb.h -- dose-deposition coefficients D_ij of a finite-size pencil-beam
 * (FSPB) model on an AMD Instinct MI355X (gfx950).
 *
 * The library computes, for every beamlet j of a set of coplanar IMRT beams
 * and every voxel i inside that beamlet's volume of interest, the coefficient
 *
 *     D_ij = A(d) F(u, v, d)                      (Eq. 2 of Gu et al. 2009,
 *                                                   arXiv:0908.4417)
 *     A(d) = PDD(d) (SAD / t')^2                   depth dose x inverse square
 *     F    = sum_k c1_k / 4 [erf((c2_k a/2 - u)/(sqrt2 c3_k(d)))
 *                            + erf((c2_k a/2 + u)/(sqrt2 c3_k(d)))]
 *                          [same in v with b]       (Eq. 3, K <= 4 terms)
 *
 * and returns them as an FP32 CSR matrix, one row per beamlet, columns =
 * voxel linear index (iz * ny + iy) * nx + ix in strictly ascending order.
 *
 * Geometry (Fig. 1 of the paper; Sec. 2.1 and 2.2):
 *   - gantry angle g rotates about the patient z axis; the source is at
 *     S = iso + SAD (sin g, -cos g, 0); the beam's lateral axes are
 *     eu = (cos g, sin g, 0) and ev = (0, 0, 1);
 *   - beamlet (iu, iv) of a beam is centred at iso + (u0 + iu a) eu +
 *     (v0 + iv b) ev on the iso plane; its central axis runs from S through
 *     that point; row j = (sum of nu*nv over earlier beams) + iv * nu + iu;
 *   - for a voxel centre P: t' = (P - S).e (distance from S to O', the
 *     projection of P on the axis), u = (P - S).eu' SAD / t',
 *     v = (P - S).ev' SAD / t' (iso-plane lateral offsets), where eu' is eu
 *     made perpendicular to the axis e and ev' = eu' x e;
 *   - the VOI (Sec. 2.1, last paragraph) is |u| <= cutoff_u, |v| <= cutoff_v
 *     (default 3a, 3b: a co-axial beamlet six times wider) and density >
 *     rho_min;
 *   - the radiological depth d at O' is read by linear interpolation from a
 *     per-beamlet table of n equally spaced points on AB (A, B = entry and
 *     exit of the axis through the grid's bounding box; Sec. 2.2), each
 *     point's depth being the Siddon (1985) path integral of density from A
 *     (or, with FSPB_DEPTH_TRILINEAR, the trapezoid sum of trilinear density
 *     samples at the table points, as the paper builds the table);
 *     d = 0 before A and d = depth(B) beyond B.
 *
 * Units: cm, g/cc relative to water, degrees.
 *
 * Conventions for every entry point:
 *   - all functions return an fspb_status; nothing aborts or throws;
 *   - arguments are validated before any device work; on error nothing is
 *     written to caller memory and fspb_last_error() describes the problem;
 *   - device work is ordered on the caller's stream (a hipStream_t passed as
 *     void*, NULL = the null stream); the only host synchronisation in the
 *     plain path is the 8-byte nonzero count read by fspb_dose_coeffs;
 *   - a plan is not thread-safe; distinct plans are independent.
 */
#ifndef FSPB_H
#define FSPB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fspb_status;
#define FSPB_OK             0
#define FSPB_ERR_INVALID   (-1)   /* an argument failed validation */
#define FSPB_ERR_STATE     (-2)   /* call out of order (e.g. dose before raytrace) */
#define FSPB_ERR_CAPACITY  (-3)   /* caller buffer too small; the size needed was reported */
#define FSPB_ERR_HIP       (-4)   /* a HIP runtime call failed */
#define FSPB_ERR_NOMEM     (-5)   /* host allocation failed */
#define FSPB_ERR_OVERFLOW  (-6)   /* a replayed batch produced more nonzeros than its buffers */

typedef struct fspb_plan fspb_plan;

/* CT-derived density grid (Sec. 2.2: the CT images and their bounding prism). */
typedef struct {
    int32_t nx, ny, nz;          /* voxels per axis, each >= 1, nx < 2^30, nx*ny*nz < 2^31 */
    int32_t reserved;            /* must be 0 */
    double spacing[3];           /* voxel size (cm), each > 0 */
    double origin[3];            /* centre of voxel (0,0,0) (cm) */
    const float *density;        /* DEVICE pointer, [nz][ny][nx] x fastest, finite and >= 0.
                                    BORROWED: must stay valid while the plan lives; its
                                    contents are read by every fspb_raytrace call. */
} fspb_grid;

/* One broad beam split into identical beamlets (Sec. 2.1, assumption 1). */
typedef struct {
    double gantry_deg;           /* gantry angle (degrees) */
    double isocenter[3];         /* (cm) */
    double sad;                  /* source-axis distance (cm), > 0; the source must lie
                                    outside the grid's bounding box */
    double beamlet_a, beamlet_b; /* beamlet side lengths at the iso plane along eu, ev (cm) */
    double u0, v0;               /* iso-plane centre of beamlet (0,0) (cm) */
    int32_t nu, nv;              /* beamlets along eu and ev, each >= 1 */
} fspb_beam;

/*
 * Eq. 2-3 in their general form (the paper's C(d) and A(theta, d)): every
 * term's c1, c2, c3 tabulated against depth, and A(theta, d) against theta,
 * the angle between a beamlet's axis and its broad beam's central axis (S
 * towards the isocentre), and depth.  Linear interpolation in each variable,
 * held at the first and last nodes.  With these tables
 *   D = A(theta, d) (SAD/t')^2 sum_k c1_k(d)/4 [E_u][E_v],
 * E_u = erf((c2_k(d) a/2 - u)/(sqrt2 c3_k(d))) + erf((c2_k(d) a/2 + u)/(sqrt2 c3_k(d))),
 * so the analytic form is the special case of constant c1, c2, c3 linear in
 * d and A = PDD.  All arrays are HOST memory, COPIED at plan creation.
 */
typedef struct {
    int32_t n_depth;             /* c nodes, >= 2, at depths k * depth_step */
    int32_t n_theta;             /* A rows, >= 1, at angles k * theta_step */
    int32_t n_adepth;            /* A columns, >= 2, at depths k * adepth_step */
    int32_t reserved;            /* must be 0 */
    double depth_step;           /* > 0 (cm) */
    double theta_step;           /* > 0 (radians) */
    double adepth_step;          /* > 0 (cm) */
    const float *c1;             /* [n_terms][n_depth], finite */
    const float *c2;             /* [n_terms][n_depth], > 0 */
    const float *c3;             /* [n_terms][n_depth], > 0 */
    const float *A;              /* [n_theta][n_adepth], finite */
} fspb_kernel_tables;

/* FSPB kernel parameters (Eq. 2-3) and VOI / table settings. */
typedef struct {
    int32_t n_terms;             /* K, 1..4 (Eq. 3 uses 3) */
    int32_t n_pdd;               /* entries of pdd, >= 2 */
    double weight[4];            /* c1_k (finite) */
    double sigma0[4];            /* c3_k(d) = sigma0_k + sigma_slope_k d; sigma0 > 0 */
    double sigma_slope[4];       /* >= 0 */
    double width_scale[4];       /* c2_k > 0 */
    const float *pdd;            /* HOST pointer: depth dose at depths k * pdd_step; linear
                                    interpolation, held at the last entry. COPIED at create. */
    double pdd_step;             /* > 0 (cm) */
    double cutoff_u, cutoff_v;   /* VOI half-widths at the iso plane; <= 0 selects 3a, 3b */
    double table_step;           /* nominal depth-table element; <= 0 selects half the
                                    smallest voxel spacing (Sec. 3.2) */
    float rho_min;               /* voxels with density <= rho_min are in no VOI */
    uint32_t flags;              /* 0, or FSPB_DEPTH_TRILINEAR, at most one of
                                    FSPB_ERF_COMPACT, FSPB_ERF_MIRRORED, and at most
                                    one of FSPB_TILES_BLOCK, FSPB_TILES_LIST */
    const fspb_kernel_tables *tables;   /* NULL: the analytic form above (weight, sigma0,
                                           sigma_slope, width_scale, pdd); else these tables
                                           replace them (pdd is still validated, unused) */
} fspb_kernel;

/*
 * kernel.flags: build the radiological-depth table as Sec. 2.2 describes it,
 * from densities sampled by trilinear interpolation of the voxel centres at
 * the n table points (each coordinate held at the outermost centre plane)
 * and summed by the trapezoid rule, instead of the exact path integral
 * through the voxels (the default).
 */
#define FSPB_DEPTH_TRILINEAR 1u

/*
 * kernel.flags: the form in which the fill stages its erf table (linear
 * interpolation between 961 nodes on [0, 3.75], the same interpolant in both
 * forms, so the coefficients agree to rounding).  By default plan creation
 * takes the mirrored form (15 KB, the table extended onto [-3.75, 3.75] so that a
 * signed argument is read directly) unless its larger LDS footprint would
 * cost the fill workgroups per CU on the current device, and the compact form
 * (7.5 KB on [0, 3.75], the sign restored by odd symmetry) otherwise.  These flags
 * force one form; FSPB_ERF_MIRRORED fails with FSPB_ERR_INVALID when the
 * fill's LDS would then exceed 64 KB.
 */
#define FSPB_ERF_COMPACT  2u
#define FSPB_ERF_MIRRORED 4u

/*
 * kernel.flags: how the fill walks a beamlet's VOI rows (the coefficients are
 * the same either way, bit for bit).  By default the count pass chooses per
 * beamlet: tiles of 64 consecutive grid rows of the beamlet's bounding row
 * block, or, where fewer than half of those rows hold a VOI member, tiles of
 * 64 entries of the list of rows that do.  These flags force one kind for
 * every beamlet of the plan (for testing both; the default is the faster).
 */
#define FSPB_TILES_BLOCK  8u
#define FSPB_TILES_LIST  16u

/* Static description of a created plan. */
typedef struct {
    int32_t n_beamlets;          /* rows of D */
    int32_t n_voxels;            /* columns of D (nx*ny*nz) */
    int64_t table_entries;       /* sum of depth-table lengths */
    int64_t n_tiles;             /* units of work of the count and fill kernels */
    int32_t max_table;           /* longest depth table */
    int32_t fill_lds_bytes;      /* LDS of one fill workgroup: the erf table (7.5 KB on [0, 3.75],
                                    or 15 KB mirrored onto [-3.75, 3.75] where that does not lower the
                                    fill's workgroups per CU on this device), the longest depth
                                    table and the depth dose as (value, slope) pairs, and the
                                    tile offsets of the beamlet with most tiles */
    int32_t fill_erf_mode;       /* how the fill reads erf: 0 the compact table (sign by odd
                                    symmetry); 1 the mirrored table with clamped arguments;
                                    2 mirrored, the first argument of each bracket unclamped
                                    (the plan's widest beamlet over its narrowest sigma keeps
                                    it inside the table); 3 as 2 with square beamlets and a
                                    non-negative kernel, no argument clamped */
} fspb_plan_desc;

/*
 * Create a plan: validate, compute the FP64 beamlet geometry (Fig. 1) on the
 * host, carve the caller's device workspace and upload the beamlet records
 * and the depth-dose table.  Nothing is sent to the device here: the
 * host-written part of the workspace is assembled in a pinned staging buffer
 * of the library (pooled per device, kept until the process ends), which the
 * plan holds until its first fspb_raytrace or fspb_batch_create copies it
 * (one asynchronous copy, on that call's stream, so ordered like the rest of
 * the plan's work).
 *
 * workspace        DEVICE pointer of workspace_bytes bytes (256-byte aligned), owned by
 *                  the caller, kept for the plan's life.  NULL: only *workspace_needed is
 *                  set and FSPB_ERR_CAPACITY is returned (no plan is created).
 * workspace_needed HOST out, may be NULL when workspace is given.
 * out              HOST out: the plan (owns host metadata only).
 * Errors: INVALID (bad argument), CAPACITY (workspace missing or too small, size
 * reported), HIP (upload failed), NOMEM.
 */
fspb_status fspb_plan_create(const fspb_grid *grid, const fspb_beam *beams, int32_t n_beams,
                             const fspb_kernel *kernel, void *workspace, size_t workspace_bytes,
                             size_t *workspace_needed, fspb_plan **out);

/*
 * Radiological-depth tables (Sec. 2.2): for every beamlet, trace its central
 * axis from A to B through the density grid (Siddon; crossing parameters in
 * FP64, path sums in FP32 with compensation) and tabulate the depth at the
 * table points; with FSPB_DEPTH_TRILINEAR the density is instead sampled by
 * trilinear interpolation at the table points (FP64) and summed by
 * trapezoids.  Also derives the density mask (density > rho_min) used by the
 * VOI test and counts every beamlet's VOI members (Sec. 2.1), which
 * fspb_dose_coeffs turns into row pointers.  Reads the borrowed density;
 * enqueues work on `stream` (on the plan's first call, after the copy of the
 * plan's records into the workspace).  Invalidates the row pointers of an
 * earlier fspb_dose_coeffs.
 */
fspb_status fspb_raytrace(fspb_plan *plan, void *stream);

/*
 * D_ij as FP32 CSR (Eq. 2-3 over every beamlet's VOI).  Requires a prior
 * fspb_raytrace on the plan.
 *
 * indptr   DEVICE, n_beamlets + 1 int64 (always written on OK or CAPACITY).
 * indices  DEVICE, capacity int32 voxel indices; NULL = size query.
 * values   DEVICE, capacity floats.
 * nnz_out  HOST out: number of nonzeros.
 * Returns CAPACITY (after writing indptr and *nnz_out, no values) when indices
 * or values is NULL or capacity < nnz.  The fill is enqueued right behind the
 * count (it checks the total against capacity on the device and writes
 * nothing if it does not fit); the call then waits for the count only, not
 * for the fill.
 */
fspb_status fspb_dose_coeffs(fspb_plan *plan, int64_t *indptr, int32_t *indices, float *values,
                             int64_t capacity, int64_t *nnz_out, void *stream);

/*
 * Rows j0 .. j1-1 of D only, for callers whose memory holds a part of the
 * matrix at a time (the paper computes the beams of a plan in turns on a
 * small card, Sec. 4).  fspb_dose_coeffs must have counted the rows of the
 * current trace first (NULL indices only count): indptr is the row-pointer
 * array it wrote (DEVICE, n_beamlets + 1, unchanged since).  Entry e of row j
 * is written at indptr[j] - indptr[j0] + e of indices / values (DEVICE,
 * capacity entries each); *nnz_out = indptr[j1] - indptr[j0] (HOST).
 * Synchronises `stream` once (to read the two row pointers).
 * Errors: INVALID (bad range or arguments), STATE (rows not counted since the
 * last fspb_raytrace), CAPACITY (arrays too small; *nnz_out reports the size).
 * The same plan's calls share one output record: run them in stream order.
 */
fspb_status fspb_dose_coeffs_rows(fspb_plan *plan, int32_t j0, int32_t j1, const int64_t *indptr,
                                  int32_t *indices, float *values, int64_t capacity, int64_t *nnz_out,
                                  void *stream);

/*
 * The partition of a plan's rows for the small-memory mode (Sec. 4: a plan
 * computed a few beams at a time, each part copied out before the next):
 * consecutive beamlet ranges [bounds[k], bounds[k + 1]), k < *n_ranges, each
 * of whose entries take at most max_bytes (8 bytes per entry: FP32 value and
 * int32 column), to be filled one after another with fspb_dose_coeffs_rows.
 * Each range is as long as the budget allows (greedy from row 0).  With
 * beam_rows (n_beams > 0; beam_rows[b] = nu * nv of beam b, summing to
 * n_rows) a range ends at the furthest beam boundary that fits, and only a
 * range that cannot hold the rest of its beam ends inside it; with n_beams =
 * 0 every row boundary is a candidate.  Host-only: no device work.
 *
 * indptr     HOST, n_rows + 1 non-decreasing int64 row pointers (the counts of
 *            fspb_dose_coeffs with NULL indices, copied to the host).
 * bounds     HOST out, max_ranges + 1 int32 (bounds[0] = 0, bounds[*n_ranges] = n_rows);
 *            NULL = size query.
 * n_ranges   HOST out: number of ranges.
 * Errors: INVALID (bad arguments, or a single row larger than the budget:
 * nothing written), CAPACITY (bounds NULL or more than max_ranges ranges;
 * *n_ranges reports the count, bounds is not written).
 */
fspb_status fspb_row_ranges(const int64_t *indptr, int32_t n_rows, const int32_t *beam_rows, int32_t n_beams,
                            int64_t max_bytes, int32_t *bounds, int32_t max_ranges, int32_t *n_ranges);

/* Release the plan's host metadata (the workspace stays the caller's). NULL is a no-op. */
void fspb_plan_destroy(fspb_plan *plan);

/* Static sizes of a plan. */
fspb_status fspb_plan_info(const fspb_plan *plan, fspb_plan_desc *desc);

/*
 * Copy the depth tables to HOST memory for inspection: tables gets
 * desc.table_entries floats, offsets n_beamlets + 1 int64 (row j's table is
 * tables[offsets[j] .. offsets[j+1])); synchronises `stream`.  Requires a prior
 * fspb_raytrace.  Either pointer may be NULL.
 */
fspb_status fspb_plan_get_tables(fspb_plan *plan, float *tables, int64_t *offsets, void *stream);

/* Device time of the kernels of the most recent fspb_raytrace / fspb_dose_coeffs calls. */
typedef struct {
    float prep_ms;               /* density mask and row extents */
    float raytrace_ms;           /* depth tables */
    float count_ms;              /* VOI members per tile */
    float scan_ms;               /* row sums and row pointers */
    float fill_ms;               /* dose values and CSR columns */
    int32_t valid;               /* 1 if every interval above was recorded */
} fspb_timing;

/*
 * Enable (1) or disable (0) HIP-event timing of the plan's kernels.  When on,
 * every launch is bracketed by events recorded on the caller's stream.
 */
fspb_status fspb_plan_set_timing(fspb_plan *plan, int32_t enable);

/* Wait for the last recorded events and report the intervals (HOST out). */
fspb_status fspb_plan_get_timing(fspb_plan *plan, fspb_timing *out);

/* ------------------------------------------------------------------------
 * Batches: many plans (uneven grids, beams, beamlet sizes) computed by one
 * captured HIP graph of persistent kernels.  Each stage (mask, depth tables,
 * counts, row sums, row pointers, fill) is one launch over all plans; the
 * fill pulls (plan, beamlet) work items from a device queue, longest rows
 * first.  Output sizes are fixed by a counting pass at creation, so a run
 * needs no host synchronisation and can be replayed.  Plans stay owned by
 * the caller and must outlive the batch; while a plan belongs to a batch it
 * must not be run on its own concurrently with the batch (they share its
 * workspace).  A batch computes Eq. 2-3 analytically: plans with kernel
 * tables or with a surrogate attached are rejected at creation, and a
 * surrogate cannot be attached to a plan while a batch holds it.
 * ------------------------------------------------------------------------ */
typedef struct fspb_batch fspb_batch;

/* Launch shape of the batched fill. */
typedef struct {
    int32_t waves_per_group;     /* fill workgroup size in 64-wide waves: 2, 4 or 8 */
    int32_t groups_per_cu;       /* persistent fill grid = groups_per_cu x compute units, 1..16 */
    int32_t order;               /* 0: longest beamlet rows first, 1: plan order */
    int32_t tuned;               /* out: 1 if the shape came from fspb_batch_tune or its cache */
    float fill_ms;               /* out: fill time measured for this shape by the tuner (0 if none) */
    int32_t tile_rows;           /* grid rows a wave takes per step through a beamlet's tiles of 64
                                    rows: 64, 128 or 256 (0 = 64) */
    int32_t beamlets_per_item;   /* beamlets a workgroup takes per fetch from the queue: 1, 2 or 4
                                    (0 = 1) */
    int32_t reserved;
} fspb_batch_config;

/*
 * Create a batch over plans[0..n_plans) (each created by fspb_plan_create;
 * density grids in place).  Runs the mask, ray-trace and counting stages once
 * on `stream` and synchronises to size every plan's output.
 * workspace: DEVICE, 256-byte aligned, caller-owned; NULL = size query
 * (returns CAPACITY with *workspace_needed set).
 */
fspb_status fspb_batch_create(fspb_plan *const *plans, int32_t n_plans, void *workspace,
                              size_t workspace_bytes, size_t *workspace_needed, void *stream,
                              fspb_batch **out);

/* Nonzeros of plan `plan` (index into the creation array) found by the sizing pass. */
fspb_status fspb_batch_nnz(const fspb_batch *batch, int32_t plan, int64_t *nnz);

/*
 * Bind the CSR outputs of plan `plan`: DEVICE indptr (n_beamlets + 1 int64),
 * indices (int32) and values (float) of `capacity` entries, capacity >=
 * fspb_batch_nnz.  Every plan must be bound before fspb_batch_run.
 */
fspb_status fspb_batch_bind(fspb_batch *batch, int32_t plan, int64_t *indptr, int32_t *indices,
                            float *values, int64_t capacity);

/*
 * Time fill launch shapes on this batch (outputs must be bound), keep the
 * fastest and remember it for batches of the same shape class in this process
 * (number of plans, beamlets and nonzeros rounded to two digits, term count).
 * First every workgroup size, grid and queue order (tile_rows 64, one beamlet
 * per item), then every tile_rows and beamlets_per_item for the best of those.
 * Every shape gives the same bits.  Synchronises `stream`.
 */
fspb_status fspb_batch_tune(fspb_batch *batch, void *stream);

fspb_status fspb_batch_get_config(const fspb_batch *batch, fspb_batch_config *cfg);
/* Set the launch shape explicitly (the graph is captured again on the next run). */
fspb_status fspb_batch_set_config(fspb_batch *batch, const fspb_batch_config *cfg);

/*
 * Enqueue the whole batch on `stream` as one graph launch (captured on first
 * use).  No host synchronisation.
 */
fspb_status fspb_batch_run(fspb_batch *batch, void *stream);

/*
 * Synchronise `stream` and report whether any plan produced more nonzeros than
 * its bound capacity since the last check (possible only if densities changed
 * after creation): OVERFLOW, with the plan's excess entries dropped.  Clears
 * the flags.
 */
fspb_status fspb_batch_check(fspb_batch *batch, void *stream);

/* Release the batch's host state (graph included). NULL is a no-op. */
void fspb_batch_destroy(fspb_batch *batch);

/* ------------------------------------------------------------------------
 * Learned kernel surrogate.  A 4 -> 64 -> 64 -> 1 perceptron with SiLU
 * activations approximates K(d, u, v, a) = PDD(d) F(u, v; a, a, d) (Eq. 2-3
 * without the inverse square) for square beamlets over the training box
 * d in [0, 30] cm, |u|, |v| <= 3 cm, a in [0.25, 1] cm.  It is trained on
 * the GPU by the library's own forward and backward kernels (BF16 matrix
 * cores with FP32 accumulation for the 64 x 64 layer, FP32 elsewhere, Adam on
 * FP32 master weights) from kernel values the analytic path generates.  A
 * plan with a surrogate attached evaluates it inside the fill for every VOI
 * voxel within the box and falls back to Eq. 2-3 outside it.
 *
 * Parameter vector (4545 FP32 values): W1[64][4], b1[64], W2[64][64], b2[64],
 * W3[64], b3; W[o][i] maps input i to output o.  Inputs are the features
 * 2 sqrt(d/30) - 1, 2 sqrt(|u|/3) - 1, 2 sqrt(|v|/3) - 1, (a - 0.625)/0.375.
 * ------------------------------------------------------------------------ */
typedef struct fspb_surrogate fspb_surrogate;

#define FSPB_SURROGATE_PARAMS 4545

typedef struct {
    int32_t epochs;              /* passes over the sample set, >= 1 */
    int32_t batch;               /* samples per step, multiple of 64, <= the max_batch of create */
    float lr_max, lr_min;        /* cosine learning-rate schedule over all steps */
    float beta1, beta2, eps;     /* Adam */
    int32_t reserved;
    uint64_t seed;               /* seeds the per-epoch sample order (SplitMix64 of seed, epoch) */
} fspb_train_config;

/*
 * Create a surrogate for the kernel parameters `kernel` (its depth-dose table
 * is copied; cutoffs and table_step are ignored) with initial parameters
 * init_params (HOST, FSPB_SURROGATE_PARAMS floats).  max_batch bounds the
 * training batch (multiple of 64).  workspace: DEVICE, 256-byte aligned,
 * caller-owned; NULL = size query (returns CAPACITY).
 */
fspb_status fspb_surrogate_create(const fspb_kernel *kernel, const float *init_params, int32_t max_batch,
                                  void *workspace, size_t workspace_bytes, size_t *workspace_needed,
                                  fspb_surrogate **out);

/*
 * Training data from the analytic kernel: for n samples (DEVICE, [n][4] =
 * d, u, v, a) write their features (DEVICE, [n][4]) and targets K (DEVICE, [n]).
 */
fspb_status fspb_surrogate_targets(fspb_surrogate *sur, const float *samples, int64_t n, float *features,
                                   float *targets, void *stream);

/* Outputs of the network for n feature rows (DEVICE in, DEVICE out). */
fspb_status fspb_surrogate_forward(fspb_surrogate *sur, const float *features, int64_t n, float *out,
                                   void *stream);

/*
 * Gradient of the mean squared error over n samples (n <= max_batch) with
 * respect to every parameter: grad (DEVICE, FSPB_SURROGATE_PARAMS floats),
 * *loss (HOST).  Synchronises `stream`.
 */
fspb_status fspb_surrogate_gradient(fspb_surrogate *sur, const float *features, const float *targets, int64_t n,
                                    float *grad, float *loss, void *stream);

/*
 * Train on n samples (features/targets on the DEVICE).  loss_per_epoch (HOST,
 * cfg->epochs floats, may be NULL) receives the mean squared error of each
 * epoch's last batch.  Synchronises `stream` once per epoch.
 */
fspb_status fspb_surrogate_train(fspb_surrogate *sur, const float *features, const float *targets, int64_t n,
                                 const fspb_train_config *cfg, float *loss_per_epoch, void *stream);

/* Copy the parameters to / from HOST memory (FSPB_SURROGATE_PARAMS floats). */
fspb_status fspb_surrogate_get_params(fspb_surrogate *sur, float *params, void *stream);
fspb_status fspb_surrogate_set_params(fspb_surrogate *sur, const float *params);

/*
 * Attach a surrogate to a plan (NULL detaches it: analytic fill).  The plan's
 * kernel parameters must equal the surrogate's (same terms, widths, sigma
 * law and depth-dose table); the surrogate must outlive the attachment.
 * INVALID when the plan uses kernel tables or belongs to a live batch.
 * After the plan's first fspb_raytrace this waits for all device work, then
 * replaces the device copy of the plan record.
 */
fspb_status fspb_plan_set_surrogate(fspb_plan *plan, const fspb_surrogate *sur);

/* Release the surrogate's host state. NULL is a no-op. */
void fspb_surrogate_destroy(fspb_surrogate *sur);

/* ------------------------------------------------------------------------
 * Dose superposition (Eq. 1: D(x) = sum_j w_j D_j(x)) and its adjoint, on
 * the beamlet-row CSR produced above (rows = beamlets, columns = voxels) and
 * on its voxel-row transpose (rows = voxels, columns = beamlets).
 * ------------------------------------------------------------------------ */

/*
 * dose[i] = sum_j w[j] D_ij.  indptr (n_rows + 1), indices, values, w (n_rows)
 * and dose (n_voxels) are DEVICE pointers; dose is overwritten.  Entries are
 * added with FP32 atomics, so the rounding of each voxel's sum depends on
 * the order in which rows land (the value itself is the same to FP32
 * precision; fspb_voxel_dose is the bit-reproducible form).  Entries whose
 * column lies outside [0, n_voxels) are skipped.  indices and values are
 * read only where indptr says there are entries (they may be NULL for a
 * matrix without any).
 */
fspb_status fspb_fluence_dose(const int64_t *indptr, const int32_t *indices, const float *values, int32_t n_rows,
                              int32_t n_voxels, const float *w, float *dose, void *stream);

/*
 * g[j] = sum_i D_ij r[i] (the gradient of sum_i r_i D_i with respect to the
 * beamlet weights).  DEVICE pointers; r has n_voxels entries, g has n_rows
 * and is overwritten.  Each row is summed by one wave in a fixed order:
 * deterministic.  Entries whose column lies outside [0, n_voxels) are skipped;
 * indices and values may be NULL for a matrix without entries.
 */
fspb_status fspb_fluence_gradient(const int64_t *indptr, const int32_t *indices, const float *values,
                                  int32_t n_rows, int32_t n_voxels, const float *r, float *g, void *stream);

/*
 * Voxel-row form of D: the transpose of a beamlet-row CSR (n_rows beamlets,
 * nnz entries, columns in [0, n_voxels)): a stable sort of the entries by
 * voxel index.  When a row's entries form long stretches within 32-column
 * buckets (as in D), the stretches are sorted by bucket and each bucket's
 * entries placed by a counting sort; otherwise a radix sort of the entries.
 * Each voxel row lists its beamlets in ascending order, so the result is
 * canonical and bit-reproducible.
 *   indptr (n_rows + 1, int64), indices (nnz), values (nnz): DEVICE, input;
 *   t_indptr (n_voxels + 1, int64), t_indices (nnz, beamlet ids),
 *   t_values (nnz): DEVICE, written.
 * workspace: DEVICE, 256-byte aligned, caller-owned, about 24 bytes per
 * entry; NULL = size query (returns FSPB_ERR_CAPACITY and sets
 * *workspace_needed).  nnz must be below 2^32.  Stream-ordered: no host
 * synchronisation, so the call can be captured in a HIP graph.  An entry
 * whose column lies outside [0, n_voxels) is left out: t_indptr counts the
 * valid entries only (t_indptr[n_voxels] < nnz tells the caller), and
 * t_indices / t_values past t_indptr[n_voxels] are unspecified.
 */
fspb_status fspb_csr_transpose(const int64_t *indptr, const int32_t *indices, const float *values, int32_t n_rows,
                               int32_t n_voxels, int64_t nnz, int64_t *t_indptr, int32_t *t_indices,
                               float *t_values, void *workspace, size_t workspace_bytes, size_t *workspace_needed,
                               void *stream);

/*
 * fspb_csr_transpose for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): no workspace argument, and no allocation of any kind.  Its
 * scratch is a static device array of FSPB_NOALLOC_SCRATCH_BYTES (64 MiB)
 * in the library, one per GPU, kept until the process ends.  Same arguments
 * (minus the workspace), kernels and results as fspb_csr_transpose.
 * Returns FSPB_ERR_CAPACITY (before any device work) when the transpose of
 * these sizes needs more scratch than that: about 24 bytes per entry plus 4
 * per voxel and 12 per row, i.e. up to roughly 2.5 million entries.  Every
 * call on a GPU shares that GPU's array and leaves its contents behind: calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller.
 */
#define FSPB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
fspb_status fspb_csr_transpose_noalloc(const int64_t *indptr, const int32_t *indices, const float *values,
                                       int32_t n_rows, int32_t n_voxels, int64_t nnz, int64_t *t_indptr,
                                       int32_t *t_indices, float *t_values, void *stream);

/*
 * dose[i] = sum_j D_ij w[j] over the voxel-row CSR of fspb_csr_transpose:
 * each voxel row is summed by 16 lanes in a fixed order (bit-reproducible, no
 * atomics).  DEVICE pointers; w has n_beamlets entries, dose n_voxels and is
 * overwritten.  Entries whose beamlet lies outside [0, n_beamlets) are
 * skipped; t_indices and t_values may be NULL for a matrix without entries.
 */
fspb_status fspb_voxel_dose(const int64_t *t_indptr, const int32_t *t_indices, const float *t_values,
                            int32_t n_voxels, int32_t n_beamlets, const float *w, float *dose, void *stream);

/* Human-readable name of a status code (static storage). */
const char *fspb_status_string(fspb_status s);

/* Message of the last failing call on this thread ("" if none). */
const char *fspb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FSPB_H */
