/*
 * Host side of the fspb C ABI: argument validation, FP64 beamlet geometry
 * (Fig. 1 of Gu et al. 2009), VOI row bounds, workspace layout and kernel
 * launches.  See include/fspb.h for the contract of each entry point.
 */
#include "../../include/fspb.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fspb_device.h"
#include "fspb_mlp.h"

using fspb::BeamletRec;
using fspb::OutDev;
using fspb::PlanDev;

namespace {

thread_local std::string g_last_error;

fspb_status fail(fspb_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

fspb_status hip_fail(hipError_t e, const char *what)
{
    return fail(FSPB_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define FSPB_HIP(call, what)                              \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, what);  \
    } while (0)

/* ------------------------------------------------------------ vec3 */
struct V3 {
    double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline V3 unit(V3 a) { return (1.0 / std::sqrt(dot(a, a))) * a; }
inline double comp(V3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }
inline void store(V3 a, double *p) { p[0] = a.x; p[1] = a.y; p[2] = a.z; }

bool finite(double v) { return std::isfinite(v); }

constexpr double kPi = 3.14159265358979323846;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

/* Workspace carve: offsets of every device array.  The arrays the host
 * writes come first, so that one copy of [0, upload) uploads all of them. */
struct Layout {
    size_t plan, scal, rec, pdd, erf, ctab, atab, upload;
    size_t out, tile_count, row_list, list_count, row_ne, row_nnz, tables, bits, ext, total;
};

/*
 * Pinned host buffers for plan uploads.  fspb_plan_create writes a plan's
 * upload image into one of them and keeps it claimed; the plan's first
 * fspb_raytrace (or fspb_batch_create) sends it with a single asynchronous
 * copy on that call's stream and releases the claim.  A released buffer is
 * reused once the event recorded after its copy has completed.  When
 * kStagingPerDevice buffers exist on a device, creation waits for a released
 * one rather than allocating (unless every buffer is claimed by a plan whose
 * upload is still pending); buffers are kept until the process ends.
 */
struct Staging {
    void *host = nullptr;
    size_t cap = 0;
    int device = -1;
    bool claimed = false;
    hipEvent_t done = nullptr;
};
constexpr int kStagingPerDevice = 8;
std::mutex g_stage_mu;
std::vector<std::unique_ptr<Staging>> g_stage;

bool stage_idle(Staging &b)
{
    const hipError_t e = hipEventQuery(b.done);
    if (e == hipErrorNotReady) (void)hipGetLastError();   // not an error: clear it
    return e != hipErrorNotReady;
}

void stage_release(Staging *b)
{
    std::lock_guard<std::mutex> lk(g_stage_mu);
    b->claimed = false;
}

/* erf table of the fill (built once). */
const std::vector<float2> &fill_erf_table();

/*
 * Pinned 64-byte host slots, one per plan, that a plan's nonzero count is
 * copied back into: an asynchronous copy into pinned memory lets
 * fspb_dose_coeffs queue the fill before it waits for the count.  Slots are
 * carved from pinned pages and recycled; the pages are kept until the process
 * ends.
 */
std::mutex g_slot_mu;
std::vector<void *> g_slot_pages;
std::vector<int64_t *> g_slot_free;
constexpr size_t kSlotBytes = 64, kSlotPage = 64 * 1024;

fspb_status slot_acquire(int64_t **out)
{
    std::lock_guard<std::mutex> lk(g_slot_mu);
    if (g_slot_free.empty()) {
        void *page = nullptr;
        FSPB_HIP(hipHostMalloc(&page, kSlotPage, hipHostMallocDefault), "allocate pinned slots");
        g_slot_pages.push_back(page);
        for (size_t o = kSlotPage; o >= kSlotBytes; o -= kSlotBytes)
            g_slot_free.push_back(reinterpret_cast<int64_t *>(static_cast<char *>(page) + o - kSlotBytes));
    }
    *out = g_slot_free.back();
    g_slot_free.pop_back();
    return FSPB_OK;
}

void slot_release(int64_t *slot)
{
    std::lock_guard<std::mutex> lk(g_slot_mu);
    g_slot_free.push_back(slot);
}

}  // namespace

struct fspb_plan {
    PlanDev h{};                  // host image of the device record (device pointers inside)
    OutDev out{};                 // host image of the output record
    PlanDev *d_plan = nullptr;
    OutDev *d_out = nullptr;
    int64_t *d_nnz = nullptr;
    int32_t *d_overflow = nullptr;
    std::vector<BeamletRec> recs;
    int64_t table_entries = 0;
    int32_t n_voxels = 0;
    bool traced = false;
    bool counted = false;         // row counts and pointers of the current trace are known
    // kernel parameters (to check a surrogate against)
    int32_t n_terms = 0;
    double weight[4] = {}, sigma0[4] = {}, sigma_slope[4] = {}, width_scale[4] = {}, pdd_step = 0.0;
    std::vector<float> pdd;
    // optional kernel timing: events bracket prep, raytrace, count, scan, fill
    bool timing = false;
    hipEvent_t ev[8] = {};
    bool have_trace_ev = false, have_dose_ev = false;
    Staging *upload = nullptr;          // claimed staging buffer of a pending upload
    size_t upload_bytes = 0;            // its length: workspace bytes [0, upload_bytes)
    int32_t batches = 0;                // live batches holding this plan
    int64_t *nnz_host = nullptr;        // pinned slot the nonzero count is read into
    hipEvent_t nnz_ready = nullptr;     // recorded after that read
    ~fspb_plan()
    {
        for (hipEvent_t &e : ev)
            if (e) (void)hipEventDestroy(e);
        if (nnz_ready) (void)hipEventDestroy(nnz_ready);
        if (nnz_host) slot_release(nnz_host);
        if (upload) stage_release(upload);
    }
};

namespace {

/* Enqueue a plan's pending upload (its pinned image) on `s`, then release the image. */
fspb_status plan_upload(fspb_plan *p, hipStream_t s)
{
    if (!p->upload) return FSPB_OK;
    FSPB_HIP(hipMemcpyAsync(static_cast<void *>(p->d_plan), p->upload->host, p->upload_bytes,
                            hipMemcpyHostToDevice, s),
             "upload plan");
    FSPB_HIP(hipEventRecord(p->upload->done, s), "record upload");
    stage_release(p->upload);
    p->upload = nullptr;
    return FSPB_OK;
}

fspb_status validate(const fspb_grid *g, const fspb_beam *beams, int32_t n_beams, const fspb_kernel *K)
{
    if (!g) return fail(FSPB_ERR_INVALID, "grid is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1)
        return fail(FSPB_ERR_INVALID, "grid dimensions must be >= 1 (got %d x %d x %d)", g->nx, g->ny, g->nz);
    if ((int64_t)g->nx * g->ny * g->nz >= (int64_t)1 << 31)
        return fail(FSPB_ERR_INVALID, "grid has 2^31 or more voxels");
    if (g->nx >= 1 << 30) return fail(FSPB_ERR_INVALID, "grid.nx must be < 2^30 (got %d)", g->nx);
    if (g->reserved != 0) return fail(FSPB_ERR_INVALID, "grid.reserved must be 0");
    for (int k = 0; k < 3; ++k) {
        if (!(finite(g->spacing[k]) && g->spacing[k] > 0.0))
            return fail(FSPB_ERR_INVALID, "grid.spacing[%d] must be finite and > 0", k);
        if (!finite(g->origin[k])) return fail(FSPB_ERR_INVALID, "grid.origin[%d] is not finite", k);
    }
    if (!g->density) return fail(FSPB_ERR_INVALID, "grid.density is NULL");
    if (!beams) return fail(FSPB_ERR_INVALID, "beams is NULL");
    if (n_beams < 1) return fail(FSPB_ERR_INVALID, "n_beams must be >= 1");
    int64_t nbl = 0;
    const double lo[3] = {g->origin[0] - 0.5 * g->spacing[0], g->origin[1] - 0.5 * g->spacing[1],
                          g->origin[2] - 0.5 * g->spacing[2]};
    const int nn[3] = {g->nx, g->ny, g->nz};
    for (int32_t b = 0; b < n_beams; ++b) {
        const fspb_beam &B = beams[b];
        if (!finite(B.gantry_deg) || !finite(B.isocenter[0]) || !finite(B.isocenter[1]) ||
            !finite(B.isocenter[2]) || !finite(B.u0) || !finite(B.v0))
            return fail(FSPB_ERR_INVALID, "beam %d: non-finite angle, isocentre or offset", b);
        if (!(finite(B.sad) && B.sad > 0.0)) return fail(FSPB_ERR_INVALID, "beam %d: sad must be > 0", b);
        if (!(finite(B.beamlet_a) && B.beamlet_a > 0.0 && finite(B.beamlet_b) && B.beamlet_b > 0.0))
            return fail(FSPB_ERR_INVALID, "beam %d: beamlet sizes must be > 0", b);
        if (B.nu < 1 || B.nv < 1) return fail(FSPB_ERR_INVALID, "beam %d: nu and nv must be >= 1", b);
        nbl += (int64_t)B.nu * B.nv;
        const double g_rad = B.gantry_deg * kPi / 180.0;
        const double S[3] = {B.isocenter[0] + B.sad * std::sin(g_rad), B.isocenter[1] - B.sad * std::cos(g_rad),
                             B.isocenter[2]};
        bool inside = true;
        for (int k = 0; k < 3; ++k) inside = inside && S[k] >= lo[k] && S[k] < lo[k] + nn[k] * g->spacing[k];
        if (inside) return fail(FSPB_ERR_INVALID, "beam %d: the source lies inside the grid", b);
    }
    if (nbl >= (int64_t)1 << 28) return fail(FSPB_ERR_INVALID, "too many beamlets (%lld)", (long long)nbl);
    if (!K) return fail(FSPB_ERR_INVALID, "kernel is NULL");
    if (K->n_terms < 1 || K->n_terms > fspb::kMaxTerms)
        return fail(FSPB_ERR_INVALID, "kernel.n_terms must be 1..4 (got %d)", K->n_terms);
    for (int i = 0; i < K->n_terms && !K->tables; ++i) {
        if (!finite(K->weight[i])) return fail(FSPB_ERR_INVALID, "kernel.weight[%d] is not finite", i);
        if (!(finite(K->sigma0[i]) && K->sigma0[i] > 0.0))
            return fail(FSPB_ERR_INVALID, "kernel.sigma0[%d] must be > 0", i);
        if (!(finite(K->sigma_slope[i]) && K->sigma_slope[i] >= 0.0))
            return fail(FSPB_ERR_INVALID, "kernel.sigma_slope[%d] must be >= 0", i);
        if (!(finite(K->width_scale[i]) && K->width_scale[i] > 0.0))
            return fail(FSPB_ERR_INVALID, "kernel.width_scale[%d] must be > 0", i);
    }
    if (!K->pdd) return fail(FSPB_ERR_INVALID, "kernel.pdd is NULL");
    if (K->n_pdd < 2 || K->n_pdd > 4096) return fail(FSPB_ERR_INVALID, "kernel.n_pdd must be 2..4096");
    for (int i = 0; i < K->n_pdd; ++i)
        if (!std::isfinite(K->pdd[i])) return fail(FSPB_ERR_INVALID, "kernel.pdd[%d] is not finite", i);
    if (!(finite(K->pdd_step) && K->pdd_step > 0.0)) return fail(FSPB_ERR_INVALID, "kernel.pdd_step must be > 0");
    if (!finite(K->cutoff_u) || !finite(K->cutoff_v) || !finite(K->table_step))
        return fail(FSPB_ERR_INVALID, "kernel cutoffs and table_step must be finite");
    if (!std::isfinite(K->rho_min)) return fail(FSPB_ERR_INVALID, "kernel.rho_min must be finite");
    if (K->flags & ~(FSPB_DEPTH_TRILINEAR | FSPB_ERF_COMPACT | FSPB_ERF_MIRRORED | FSPB_TILES_BLOCK | FSPB_TILES_LIST))
        return fail(FSPB_ERR_INVALID, "kernel.flags has unknown bits");
    if ((K->flags & FSPB_ERF_COMPACT) && (K->flags & FSPB_ERF_MIRRORED))
        return fail(FSPB_ERR_INVALID, "kernel.flags: FSPB_ERF_COMPACT and FSPB_ERF_MIRRORED exclude each other");
    if ((K->flags & FSPB_TILES_BLOCK) && (K->flags & FSPB_TILES_LIST))
        return fail(FSPB_ERR_INVALID, "kernel.flags: FSPB_TILES_BLOCK and FSPB_TILES_LIST exclude each other");
    if (const fspb_kernel_tables *T = K->tables) {
        if (T->n_depth < 2 || T->n_adepth < 2 || T->n_theta < 1 || T->reserved != 0)
            return fail(FSPB_ERR_INVALID, "kernel.tables: n_depth, n_adepth must be >= 2, n_theta >= 1, reserved 0");
        if ((int64_t)T->n_depth * K->n_terms > 16384 || (int64_t)T->n_theta * T->n_adepth > (1 << 22))
            return fail(FSPB_ERR_INVALID, "kernel.tables are too large");
        if (!(finite(T->depth_step) && T->depth_step > 0.0 && finite(T->adepth_step) && T->adepth_step > 0.0 &&
              finite(T->theta_step) && T->theta_step > 0.0))
            return fail(FSPB_ERR_INVALID, "kernel.tables steps must be finite and > 0");
        if (!T->c1 || !T->c2 || !T->c3 || !T->A) return fail(FSPB_ERR_INVALID, "kernel.tables arrays are NULL");
        for (int64_t i = 0; i < (int64_t)K->n_terms * T->n_depth; ++i) {
            if (!std::isfinite(T->c1[i])) return fail(FSPB_ERR_INVALID, "kernel.tables.c1[%lld] is not finite", (long long)i);
            if (!(std::isfinite(T->c2[i]) && T->c2[i] > 0.0f))
                return fail(FSPB_ERR_INVALID, "kernel.tables.c2[%lld] must be > 0", (long long)i);
            if (!(std::isfinite(T->c3[i]) && T->c3[i] > 0.0f))
                return fail(FSPB_ERR_INVALID, "kernel.tables.c3[%lld] must be > 0", (long long)i);
        }
        for (int64_t i = 0; i < (int64_t)T->n_theta * T->n_adepth; ++i)
            if (!std::isfinite(T->A[i])) return fail(FSPB_ERR_INVALID, "kernel.tables.A[%lld] is not finite", (long long)i);
    }
    return FSPB_OK;
}

/* Entry and exit of S + t e through the box [lo, hi) (slab method). */
bool clip_box(V3 S, V3 e, const double lo[3], const double hi[3], double &tA, double &tB)
{
    double t0 = 0.0, t1 = HUGE_VAL;
    for (int k = 0; k < 3; ++k) {
        const double s = comp(S, k), d = comp(e, k);
        if (d == 0.0) {
            if (s < lo[k] || s >= hi[k]) return false;
            continue;
        }
        double a = (lo[k] - s) / d, b = (hi[k] - s) / d;
        if (a > b) std::swap(a, b);
        t0 = std::max(t0, a);
        t1 = std::min(t1, b);
    }
    if (!(t1 > t0)) return false;
    tA = t0;
    tB = t1;
    return true;
}

/*
 * Conservative index bounds of the VOI along y and z.  The VOI inside the grid
 * lies in the pyramid |U| <= cu t'/SAD, |V| <= cv t'/SAD between the smallest
 * and largest t' of the grid's corners; its 8 corner points bound it.
 */
void voi_rows(const fspb_grid *g, V3 S, V3 e, V3 eu, V3 ev, double cu_sad, double cv_sad, int &iy0, int &n_iy,
              int &iz0, int &n_iz)
{
    const double lo[3] = {g->origin[0] - 0.5 * g->spacing[0], g->origin[1] - 0.5 * g->spacing[1],
                          g->origin[2] - 0.5 * g->spacing[2]};
    const int nn[3] = {g->nx, g->ny, g->nz};
    double tmin = HUGE_VAL, tmax = -HUGE_VAL;
    for (int c = 0; c < 8; ++c) {
        V3 P = {lo[0] + ((c & 1) ? nn[0] * g->spacing[0] : 0.0), lo[1] + ((c & 2) ? nn[1] * g->spacing[1] : 0.0),
                lo[2] + ((c & 4) ? nn[2] * g->spacing[2] : 0.0)};
        const double t = dot(P - S, e);
        tmin = std::min(tmin, t);
        tmax = std::max(tmax, t);
    }
    n_iy = n_iz = 0;
    iy0 = iz0 = 0;
    if (!(tmax > 0.0)) return;
    tmin = std::max(tmin, 0.0);
    double bmin[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, bmax[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
    for (int c = 0; c < 8; ++c) {
        const double t = (c & 1) ? tmax : tmin;
        const double su = (c & 2) ? cu_sad : -cu_sad, sv = (c & 4) ? cv_sad : -cv_sad;
        V3 P = S + t * (e + su * eu + sv * ev);
        for (int k = 0; k < 3; ++k) {
            bmin[k] = std::min(bmin[k], comp(P, k));
            bmax[k] = std::max(bmax[k], comp(P, k));
        }
    }
    int first[3], last[3];
    for (int k = 1; k < 3; ++k) {
        const double a = (bmin[k] - g->origin[k]) / g->spacing[k];
        const double b = (bmax[k] - g->origin[k]) / g->spacing[k];
        first[k] = (int)std::max(0.0, std::floor(a) - 1.0);
        last[k] = (int)std::min((double)nn[k] - 1.0, std::ceil(b) + 1.0);
    }
    if (first[1] > last[1] || first[2] > last[2]) return;
    iy0 = first[1];
    n_iy = last[1] - first[1] + 1;
    iz0 = first[2];
    n_iz = last[2] - first[2] + 1;
}

/*
 * Piecewise-quadratic erfc used for the surrogate's training targets: on interval k of
 * [0, kErfcMax] (width w) the quadratic through erfc at the interval's two
 * ends and midpoint, in the local coordinate f in [0, 1]:
 *   erfc(z_k + f w) ~ c0 + f (c1 + f c2).
 * The interpolation error is below w^3 max|d3 erfc/dz3| / (72 sqrt3), about
 * 2e-8 for w = 1/128; the FP32 coefficients add about one ulp of erfc.
 */
void erfc_table(std::vector<float4> &t)
{
    const int n = fspb::kErfcIntervals;
    const double w = (double)fspb::kErfcMax / n;
    t.resize(n);
    for (int k = 0; k < n; ++k) {
        const double y0 = std::erfc(k * w), ym = std::erfc((k + 0.5) * w), y1 = std::erfc((k + 1) * w);
        t[k] = make_float4((float)y0, (float)(4.0 * ym - 3.0 * y0 - y1), (float)(2.0 * (y1 + y0 - 2.0 * ym)), 0.0f);
    }
}

/*
 * Piecewise-linear erf used by the fill kernel, nodes w = 1/256 apart, each
 * interval stored as the line through its end nodes in the table coordinate
 * x = z / w: (intercept, slope) = (erf(z_k) - k s_k, s_k) with s_k =
 * erf(z_{k+1}) - erf(z_k), so the kernel evaluates x s_k + intercept with one
 * FMA (computed in FP64, rounded once).  First the compact form (intervals of
 * [0, kErfMax], k = 0 .. n-1), then the mirrored form (intervals of [-kErfMax,
 * kErfMax] in the coordinate x = z / w + n, k = 0 .. 2n-1), whose first
 * interval is replaced by the constant erf(-kErfMax) (it differs from the line
 * there by 6e-10) so that arguments below the table can read it unclamped.
 */
void erf_table(std::vector<float2> &t)
{
    const int n = fspb::kErfIntervals;
    const double w = (double)fspb::kErfMax / n;
    t.resize((size_t)3 * n);
    for (int k = 0; k < n; ++k) {
        const double e0 = std::erf(k * w), e1 = std::erf((k + 1) * w), sl = e1 - e0;
        t[k] = make_float2((float)(e0 - k * sl), (float)sl);
    }
    for (int k = 0; k < 2 * n; ++k) {
        const double e0 = std::erf((k - n) * w), e1 = std::erf((k + 1 - n) * w), sl = e1 - e0;
        t[(size_t)n + k] = k == 0 ? make_float2((float)e0, 0.0f) : make_float2((float)(e0 - k * sl), (float)sl);
    }
}

const std::vector<float2> &fill_erf_table()
{
    static const std::vector<float2> t = [] {
        std::vector<float2> v;
        erf_table(v);
        return v;
    }();
    return t;
}

/*
 * True when the first argument of every bracket of Eq. 3, (c2 a/2 - |x|) /
 * (sqrt2 c3), stays below the mirrored erf table's top (kErfMax) with a margin
 * of 24 table intervals for FP32 rounding: the fill then reads it without a
 * clamp.  c3 (sigma) is smallest at its first node (analytic form: sigma0,
 * the slope being >= 0); for tables, c2 / c3 is a ratio of two linear
 * functions on each depth interval, so its largest value sits on a node.
 */
/* True when every weight (c1) and every depth-dose (A) value of the kernel is
 * >= 0: then each coefficient of Eq. 2-3 is >= 0 (each bracket of Eq. 3 is). */
bool nonnegative_kernel(const fspb_kernel *K)
{
    if (const fspb_kernel_tables *T = K->tables) {
        for (int64_t i = 0; i < (int64_t)K->n_terms * T->n_depth; ++i)
            if (T->c1[i] < 0.0f) return false;
        for (int64_t i = 0; i < (int64_t)T->n_theta * T->n_adepth; ++i)
            if (T->A[i] < 0.0f) return false;
        return true;
    }
    for (int i = 0; i < K->n_terms; ++i)
        if (K->weight[i] < 0.0) return false;
    for (int i = 0; i < K->n_pdd; ++i)
        if (K->pdd[i] < 0.0f) return false;
    return true;
}

bool erf_args_bounded(const fspb_kernel *K, const fspb_beam *beams, int32_t n_beams)
{
    double half = 0.0;
    for (int32_t b = 0; b < n_beams; ++b) half = std::max(half, 0.5 * std::max(beams[b].beamlet_a, beams[b].beamlet_b));
    const double per_unit = fspb::kErfIntervals / (double)fspb::kErfMax;    // table intervals per unit of argument
    const double limit = (fspb::kErfIntervals - 24) / per_unit;
    double worst = 0.0;
    if (const fspb_kernel_tables *T = K->tables) {
        for (int i = 0; i < K->n_terms; ++i)
            for (int m = 0; m < T->n_depth; ++m) {
                const size_t q = (size_t)i * T->n_depth + m;
                worst = std::max(worst, (double)T->c2[q] * half / (std::sqrt(2.0) * (double)T->c3[q]));
            }
    } else {
        for (int i = 0; i < K->n_terms; ++i)
            worst = std::max(worst, K->width_scale[i] * half / (std::sqrt(2.0) * K->sigma0[i]));
    }
    return worst < limit;
}

/*
 * The fill's erf table form for a plan (fspb::choose_erf_form), remembered per
 * device, kernel shape and LDS size: plans of one geometry share the answer.
 */
std::mutex g_form_mu;
std::map<std::array<int64_t, 5>, int> g_form;

int erf_form(const fspb::PlanDev &h, int device)
{
    const std::array<int64_t, 5> key{device, h.n_terms, h.gen, fspb::mirrored_erf_mode(h),
                                     (int64_t)fspb::fill_shared_bytes(h, false)};
    std::lock_guard<std::mutex> lk(g_form_mu);
    auto it = g_form.find(key);
    if (it != g_form.end()) return it->second;
    const int f = fspb::choose_erf_form(h);
    g_form.emplace(key, f);
    return f;
}

/* A staging buffer of at least `bytes` on `device`, claimed for the caller. */
fspb_status stage_acquire(size_t bytes, int device, Staging **out)
{
    std::lock_guard<std::mutex> lk(g_stage_mu);
    int on_device = 0;
    Staging *reuse = nullptr;
    for (auto &b : g_stage) {
        if (b->device != device) continue;
        ++on_device;
        if (b->claimed) continue;
        if (b->cap >= bytes && stage_idle(*b)) {
            b->claimed = true;
            *out = b.get();
            return FSPB_OK;
        }
        if (!reuse) reuse = b.get();
    }
    if (on_device >= kStagingPerDevice && reuse) {
        // every buffer is busy or small: wait for one, grow it if needed
        FSPB_HIP(hipEventSynchronize(reuse->done), "wait for an earlier upload");
        if (reuse->cap < bytes) {
            FSPB_HIP(hipHostFree(reuse->host), "free staging buffer");
            reuse->host = nullptr;
            reuse->cap = 0;
            const size_t cap = align_up(bytes, (size_t)1 << 20);
            FSPB_HIP(hipHostMalloc(&reuse->host, cap, hipHostMallocDefault), "allocate staging buffer");
            reuse->cap = cap;
        }
        reuse->claimed = true;
        *out = reuse;
        return FSPB_OK;
    }
    std::unique_ptr<Staging> b(new (std::nothrow) Staging);
    if (!b) return fail(FSPB_ERR_NOMEM, "cannot allocate a staging record");
    b->device = device;
    FSPB_HIP(hipEventCreateWithFlags(&b->done, hipEventDisableTiming), "create staging event");
    const size_t cap = align_up(bytes, (size_t)1 << 20);
    hipError_t e = hipHostMalloc(&b->host, cap, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipEventDestroy(b->done);
        return hip_fail(e, "allocate staging buffer");
    }
    b->cap = cap;
    b->claimed = true;
    *out = b.get();
    g_stage.push_back(std::move(b));
    return FSPB_OK;
}


}  // namespace

extern "C" {

const char *fspb_status_string(fspb_status s)
{
    switch (s) {
    case FSPB_OK: return "FSPB_OK";
    case FSPB_ERR_INVALID: return "FSPB_ERR_INVALID";
    case FSPB_ERR_STATE: return "FSPB_ERR_STATE";
    case FSPB_ERR_CAPACITY: return "FSPB_ERR_CAPACITY";
    case FSPB_ERR_HIP: return "FSPB_ERR_HIP";
    case FSPB_ERR_NOMEM: return "FSPB_ERR_NOMEM";
    case FSPB_ERR_OVERFLOW: return "FSPB_ERR_OVERFLOW";
    default: return "FSPB_ERR_UNKNOWN";
    }
}

const char *fspb_last_error(void) { return g_last_error.c_str(); }

fspb_status fspb_plan_create(const fspb_grid *g, const fspb_beam *beams, int32_t n_beams, const fspb_kernel *K,
                             void *workspace, size_t workspace_bytes, size_t *workspace_needed, fspb_plan **out)
{
    g_last_error.clear();
    if (!out) return fail(FSPB_ERR_INVALID, "out is NULL");
    *out = nullptr;
    fspb_status st = validate(g, beams, n_beams, K);
    if (st != FSPB_OK) return st;
    if (!workspace && !workspace_needed)
        return fail(FSPB_ERR_INVALID, "workspace and workspace_needed are both NULL");

    fspb_plan *p = new (std::nothrow) fspb_plan;
    if (!p) return fail(FSPB_ERR_NOMEM, "cannot allocate the plan");
    struct Guard {
        fspb_plan *p;
        ~Guard() { delete p; }
    } guard{p};

    // ---- grid and kernel constants
    PlanDev &h = p->h;
    h.nx = g->nx;
    h.ny = g->ny;
    h.nz = g->nz;
    h.wpr = (g->nx + 31) / 32;
    for (int k = 0; k < 3; ++k) {
        h.org[k] = g->origin[k];
        h.sp[k] = g->spacing[k];
        h.lo[k] = g->origin[k] - 0.5 * g->spacing[k];
    }
    double hi[3] = {h.lo[0] + g->nx * g->spacing[0], h.lo[1] + g->ny * g->spacing[1], h.lo[2] + g->nz * g->spacing[2]};
    h.density = g->density;
    h.rho_min = K->rho_min;
    h.depth_mode = (K->flags & FSPB_DEPTH_TRILINEAR) ? 1 : 0;
    h.tiles_mode = (K->flags & FSPB_TILES_BLOCK) ? 1 : ((K->flags & FSPB_TILES_LIST) ? 2 : 0);
    h.n_terms = K->n_terms;
    h.n_pdd = K->n_pdd;
    for (int i = 0; i < fspb::kMaxTerms; ++i) {
        const bool on = i < K->n_terms;
        h.w4[i] = on ? (float)(0.25 * K->weight[i]) : 0.0f;
        h.sig0[i] = on ? (float)K->sigma0[i] : 1.0f;
        h.sig1[i] = on ? (float)K->sigma_slope[i] : 0.0f;
        h.c2[i] = on ? (float)K->width_scale[i] : 1.0f;
    }
    h.pdd_inv_step = (float)(1.0 / K->pdd_step);
    h.pdd_max = (float)(K->n_pdd - 1);
    if (const fspb_kernel_tables *T = K->tables) {
        h.gen = 1;
        h.n_cdepth = T->n_depth;
        h.n_theta = T->n_theta;
        h.n_adepth = T->n_adepth;
        h.c_inv_step = (float)(1.0 / T->depth_step);
        h.c_max = (float)(T->n_depth - 1);
        h.a_inv_step = (float)(1.0 / T->adepth_step);
        h.a_max = (float)(T->n_adepth - 1);
    }
    p->n_terms = K->n_terms;
    for (int i = 0; i < K->n_terms; ++i) {
        p->weight[i] = K->weight[i];
        p->sigma0[i] = K->sigma0[i];
        p->sigma_slope[i] = K->sigma_slope[i];
        p->width_scale[i] = K->width_scale[i];
    }
    p->pdd_step = K->pdd_step;
    p->pdd.assign(K->pdd, K->pdd + K->n_pdd);
    p->n_voxels = g->nx * g->ny * g->nz;

    // ---- beamlet geometry (FP64)
    const double minsp = std::min(g->spacing[0], std::min(g->spacing[1], g->spacing[2]));
    const double nominal = K->table_step > 0.0 ? K->table_step : 0.5 * minsp;
    int64_t nbl = 0;
    for (int32_t b = 0; b < n_beams; ++b) nbl += (int64_t)beams[b].nu * beams[b].nv;
    try {
        p->recs.resize((size_t)nbl);
    } catch (...) {
        return fail(FSPB_ERR_NOMEM, "cannot allocate %lld beamlet records", (long long)nbl);
    }
    int64_t table_off = 0, tile_off = 0;
    int32_t max_table = 2, max_tiles = 0;
    double max_step = nominal;
    size_t j = 0;
    for (int32_t b = 0; b < n_beams; ++b) {
        const fspb_beam &B = beams[b];
        const double gr = B.gantry_deg * kPi / 180.0;
        const V3 iso = {B.isocenter[0], B.isocenter[1], B.isocenter[2]};
        const V3 S = iso + B.sad * V3{std::sin(gr), -std::cos(gr), 0.0};
        const V3 beu = {std::cos(gr), std::sin(gr), 0.0};
        const V3 bev = {0.0, 0.0, 1.0};
        const double cu = K->cutoff_u > 0.0 ? K->cutoff_u : 3.0 * B.beamlet_a;
        const double cv = K->cutoff_v > 0.0 ? K->cutoff_v : 3.0 * B.beamlet_b;
        for (int32_t iv = 0; iv < B.nv; ++iv) {
            for (int32_t iu = 0; iu < B.nu; ++iu, ++j) {
                BeamletRec &R = p->recs[j];
                std::memset(&R, 0, sizeof R);
                const V3 Q = iso + (B.u0 + iu * B.beamlet_a) * beu + (B.v0 + iv * B.beamlet_b) * bev;
                const V3 e = unit(Q - S);
                const V3 eu = unit(beu - dot(beu, e) * e);
                const V3 ev = cross(eu, e);
                store(S, R.S);
                store(e, R.e);
                store(eu, R.eu);
                store(ev, R.ev);
                R.sad = B.sad;
                R.cu_sad = cu / B.sad;
                R.cv_sad = cv / B.sad;
                {
                    // VOI row interval coefficients, once per beamlet (the count and the fill
                    // solve every grid row from them)
                    const V3 w0 = V3{g->origin[0], g->origin[1], g->origin[2]} - S;
                    const V3 axis[3] = {e, eu, ev};
                    double *row[3] = {R.row_t, R.row_u, R.row_v};
                    for (int k = 0; k < 3; ++k) {
                        row[k][0] = dot(w0, axis[k]);
                        row[k][1] = g->spacing[1] * axis[k].y;
                        row[k][2] = g->spacing[2] * axis[k].z;
                        R.dx[k] = g->spacing[0] * axis[k].x;
                    }
                    const double c1[4] = {R.dx[1] - R.cu_sad * R.dx[0], -R.dx[1] - R.cu_sad * R.dx[0],
                                          R.dx[2] - R.cv_sad * R.dx[0], -R.dx[2] - R.cv_sad * R.dx[0]};
                    for (int c = 0; c < 4; ++c) {
                        R.r1[c] = c1[c] != 0.0 ? 1.0 / c1[c] : 0.0;
                        if (c1[c] > 0.0) R.c1_pos |= 1 << c;
                        if (c1[c] < 0.0) R.c1_neg |= 1 << c;
                    }
                }
                R.half_a = (float)(0.5 * B.beamlet_a);
                R.half_b = (float)(0.5 * B.beamlet_b);
                double tA, tB;
                if (!clip_box(S, e, h.lo, hi, tA, tB)) continue;   // axis misses: empty row
                const double L = tB - tA;
                int32_t segs = (int32_t)std::ceil(L / nominal - 1e-9);
                if (segs < 1) segs = 1;
                R.tA = tA;
                R.tB = tB;
                R.step = L / segs;
                R.n_table = segs + 1;
                R.table_off = (int32_t)table_off;
                R.tA_f = (float)tA;
                R.inv_step_f = (float)(1.0 / R.step);
                R.sad_f = (float)B.sad;
                R.tau_max_f = (float)(R.n_table - 1);
                R.t1_f = (float)(g->spacing[0] * e.x);
                R.U1_f = (float)(g->spacing[0] * eu.x);
                R.V1_f = (float)(g->spacing[0] * ev.x);
                R.a_f = (float)B.beamlet_a;
                if (const fspb_kernel_tables *T = K->tables) {
                    // Fig. 1a: theta between SS' (S towards the isocentre) and the beamlet axis
                    const double ct = dot(unit(iso - S), e);
                    const double theta = std::acos(std::max(-1.0, std::min(1.0, ct)));
                    if (T->n_theta == 1) {
                        R.theta_k = 0;
                        R.theta_f = 0.0f;
                    } else {
                        const double y = std::min(theta / T->theta_step, (double)(T->n_theta - 1));
                        const int32_t k = std::min((int32_t)std::floor(y), T->n_theta - 2);
                        R.theta_k = k;
                        R.theta_f = (float)(y - k);
                    }
                }
                R.mlp_ok = (B.beamlet_a == B.beamlet_b && B.beamlet_a >= fspb::kMlpAMin &&
                            B.beamlet_a <= fspb::kMlpAMax) ? 1 : 0;
                for (int i = 0; i < fspb::kMaxTerms; ++i) {
                    const double c2 = i < K->n_terms ? K->width_scale[i] : 1.0;
                    R.ha[i] = (float)(0.5 * c2 * B.beamlet_a);
                    R.hb[i] = (float)(0.5 * c2 * B.beamlet_b);
                }
                table_off += R.n_table;
                max_table = std::max(max_table, R.n_table);
                max_step = std::max(max_step, R.step);
                voi_rows(g, S, e, eu, ev, R.cu_sad, R.cv_sad, R.iy0, R.n_iy, R.iz0, R.n_iz);
                const int64_t rows = (int64_t)R.n_iy * R.n_iz;
                R.n_tiles = (int32_t)((rows + fspb::kRowsPerTile - 1) / fspb::kRowsPerTile);
                R.tile0 = (int32_t)tile_off;
                tile_off += R.n_tiles;
                max_tiles = std::max(max_tiles, R.n_tiles);
            }
        }
    }
    if (table_off >= (int64_t)1 << 31 || tile_off >= (int64_t)1 << 31)
        return fail(FSPB_ERR_INVALID, "plan too large (%lld table entries, %lld tiles)", (long long)table_off,
                    (long long)tile_off);
    h.n_beamlets = (int32_t)nbl;
    h.max_table = max_table;
    h.n_tiles = (int32_t)tile_off;
    h.max_tiles = max_tiles;
    // Siddon steps inside one table interval: crossings per axis plus the final segment
    h.ray_iters = 2;
    for (int k = 0; k < 3; ++k) h.ray_iters += (int32_t)std::ceil(max_step / g->spacing[k]) + 1;
    p->table_entries = table_off;
    if (fspb::fill_shared_bytes(h) > 64 * 1024)
        return fail(FSPB_ERR_INVALID, "depth tables too long for the fill kernel's LDS (%zu bytes)",
                    fspb::fill_shared_bytes(h));

    // ---- workspace layout
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    const int64_t grow = (int64_t)g->ny * g->nz;
    L.plan = take(sizeof(PlanDev));
    L.scal = take(64);
    L.rec = take(sizeof(BeamletRec) * (size_t)nbl);
    L.pdd = take(sizeof(float) * (size_t)K->n_pdd);
    L.erf = take(sizeof(float2) * 3 * fspb::kErfIntervals);
    if (K->tables) {
        L.ctab = take(sizeof(float) * 3 * (size_t)K->n_terms * K->tables->n_depth);
        L.atab = take(sizeof(float) * (size_t)K->tables->n_theta * K->tables->n_adepth);
    }
    L.upload = off;
    L.out = take(sizeof(OutDev));
    L.tile_count = take(sizeof(int32_t) * (size_t)std::max<int64_t>(tile_off, 1));
    L.row_list = take(sizeof(int32_t) * (size_t)std::max<int64_t>(tile_off * fspb::kRowsPerTile, 1));
    L.list_count = take(sizeof(int32_t) * (size_t)std::max<int64_t>(tile_off, 1));
    L.row_ne = take(sizeof(int32_t) * (size_t)std::max<int64_t>(nbl, 1));
    L.row_nnz = take(sizeof(int64_t) * (size_t)nbl);
    L.tables = take(sizeof(float) * (size_t)std::max<int64_t>(table_off, 1));
    L.bits = take(sizeof(uint32_t) * (size_t)grow * h.wpr);
    L.ext = take(sizeof(int2) * (size_t)grow);
    L.total = off;
    if (workspace_needed) *workspace_needed = L.total;
    if (!workspace) return fail(FSPB_ERR_CAPACITY, "workspace query: %zu bytes needed", L.total);
    if (workspace_bytes < L.total)
        return fail(FSPB_ERR_CAPACITY, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes,
                    L.total);
    if ((uintptr_t)workspace % 256 != 0) return fail(FSPB_ERR_INVALID, "workspace must be 256-byte aligned");

    // density and workspace must be device memory
    hipPointerAttribute_t attr;
    for (const void *ptr : {(const void *)g->density, (const void *)workspace}) {
        hipError_t e = hipPointerGetAttributes(&attr, ptr);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(FSPB_ERR_INVALID, "density and workspace must be device pointers (%s)", hipGetErrorString(e));
        }
        if (attr.type != hipMemoryTypeDevice)
            return fail(FSPB_ERR_INVALID, "density and workspace must be device memory");
    }

    char *ws = static_cast<char *>(workspace);
    p->d_plan = reinterpret_cast<PlanDev *>(ws + L.plan);
    p->d_out = reinterpret_cast<OutDev *>(ws + L.out);
    p->d_nnz = reinterpret_cast<int64_t *>(ws + L.scal);
    p->d_overflow = reinterpret_cast<int32_t *>(ws + L.scal + 16);
    h.rec = reinterpret_cast<BeamletRec *>(ws + L.rec);
    h.row_list = reinterpret_cast<int32_t *>(ws + L.row_list);
    h.list_count = reinterpret_cast<int32_t *>(ws + L.list_count);
    h.row_ne = reinterpret_cast<int32_t *>(ws + L.row_ne);
    h.tile_count = reinterpret_cast<int32_t *>(ws + L.tile_count);
    h.row_nnz = reinterpret_cast<int64_t *>(ws + L.row_nnz);
    h.tables = reinterpret_cast<float *>(ws + L.tables);
    h.pdd = reinterpret_cast<float *>(ws + L.pdd);
    h.erf_tab = reinterpret_cast<float2 *>(ws + L.erf);
    if (K->tables) {
        h.ctab = reinterpret_cast<float *>(ws + L.ctab);
        h.atab = reinterpret_cast<float *>(ws + L.atab);
    }
    h.bits = reinterpret_cast<uint32_t *>(ws + L.bits);
    h.ext = reinterpret_cast<int2 *>(ws + L.ext);
    h.nnz = p->d_nnz;

    // ---- every host-written array goes into one pinned image of [0, L.upload); the first
    // fspb_raytrace or fspb_batch_create copies it on its stream
    int dev = 0;
    FSPB_HIP(hipGetDevice(&dev), "get device");
    h.erf_nc = erf_args_bounded(K, beams, n_beams) ? 1 : 0;
    h.d_floor = nonnegative_kernel(K) ? 0.0f : -HUGE_VALF;
    h.erf_square = 1;
    for (int32_t b = 0; b < n_beams; ++b)
        if (beams[b].beamlet_a != beams[b].beamlet_b) h.erf_square = 0;
    if (K->flags & FSPB_ERF_MIRRORED) {
        if (fspb::fill_shared_bytes(h, true) > 64 * 1024)
            return fail(FSPB_ERR_INVALID, "FSPB_ERF_MIRRORED: the fill would need %zu bytes of LDS (64 KB at most)",
                        fspb::fill_shared_bytes(h, true));
        h.erf_mirrored = 1;
    } else if (K->flags & FSPB_ERF_COMPACT) {
        h.erf_mirrored = 0;
    } else {
        h.erf_mirrored = erf_form(h, dev);
    }
    h.erf_mode = h.erf_mirrored ? fspb::mirrored_erf_mode(h) : 0;
    FSPB_HIP(hipEventCreateWithFlags(&p->nnz_ready, hipEventDisableTiming), "create count event");
    st = slot_acquire(&p->nnz_host);
    if (st != FSPB_OK) return st;
    st = stage_acquire(L.upload, dev, &p->upload);
    if (st != FSPB_OK) return st;
    p->upload_bytes = L.upload;
    {
        char *img = static_cast<char *>(p->upload->host);
        std::memcpy(img + L.plan, &h, sizeof(PlanDev));
        std::memset(img + L.scal, 0, 64);   // nonzero count and overflow flag start at zero
        if (nbl > 0) std::memcpy(img + L.rec, p->recs.data(), sizeof(BeamletRec) * (size_t)nbl);
        std::memcpy(img + L.pdd, K->pdd, sizeof(float) * (size_t)K->n_pdd);
        const std::vector<float2> &et = fill_erf_table();
        std::memcpy(img + L.erf, et.data(), sizeof(float2) * et.size());
        if (const fspb_kernel_tables *T = K->tables) {
            const size_t nc = (size_t)K->n_terms * T->n_depth;
            const float *src[3] = {T->c1, T->c2, T->c3};
            for (int m = 0; m < 3; ++m) std::memcpy(img + L.ctab + sizeof(float) * m * nc, src[m], sizeof(float) * nc);
            std::memcpy(img + L.atab, T->A, sizeof(float) * (size_t)T->n_theta * T->n_adepth);
        }
    }
    guard.p = nullptr;
    *out = p;
    return FSPB_OK;
}

fspb_status fspb_raytrace(fspb_plan *p, void *stream)
{
    g_last_error.clear();
    if (!p) return fail(FSPB_ERR_INVALID, "plan is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    fspb_status us = plan_upload(p, s);
    if (us != FSPB_OK) return us;
    // the VOI counts need only the mask, so they run before the depth tables: queued behind
    // another plan's fill, they then get the CUs that fill's last workgroups leave free
    if (p->timing) FSPB_HIP(hipEventRecord(p->ev[0], s), "record event");
    FSPB_HIP(fspb::launch_prep(p->d_plan, p->h, s), "launch prep");
    if (p->timing) FSPB_HIP(hipEventRecord(p->ev[1], s), "record event");
    FSPB_HIP(fspb::launch_count(p->d_plan, p->h, s), "launch count");
    if (p->timing) FSPB_HIP(hipEventRecord(p->ev[3], s), "record event");
    FSPB_HIP(fspb::launch_raytrace(p->d_plan, p->h, s), "launch raytrace");
    if (p->timing) {
        FSPB_HIP(hipEventRecord(p->ev[2], s), "record event");
        p->have_trace_ev = true;
    }
    p->traced = true;
    p->counted = false;
    return FSPB_OK;
}

fspb_status fspb_dose_coeffs(fspb_plan *p, int64_t *indptr, int32_t *indices, float *values, int64_t capacity,
                             int64_t *nnz_out, void *stream)
{
    g_last_error.clear();
    if (!p) return fail(FSPB_ERR_INVALID, "plan is NULL");
    if (!indptr) return fail(FSPB_ERR_INVALID, "indptr is NULL");
    if (!nnz_out) return fail(FSPB_ERR_INVALID, "nnz_out is NULL");
    if (capacity < 0) return fail(FSPB_ERR_INVALID, "capacity must be >= 0");
    if (!p->traced) return fail(FSPB_ERR_STATE, "fspb_raytrace must run before fspb_dose_coeffs");
    hipStream_t s = static_cast<hipStream_t>(stream);
    p->out.indptr = indptr;
    p->out.indices = indices;
    p->out.values = values;
    p->out.capacity = (indices && values) ? capacity : 0;
    p->out.overflow = p->d_overflow;
    p->out.row0 = 0;
    p->out.check_nnz = 1;
    p->counted = false;
    FSPB_HIP(hipMemcpyAsync(p->d_out, &p->out, sizeof(OutDev), hipMemcpyHostToDevice, s), "upload output record");
    p->have_dose_ev = false;
    // tile and row counts were made by fspb_raytrace
    if (p->timing) FSPB_HIP(hipEventRecord(p->ev[4], s), "record event");
    FSPB_HIP(fspb::launch_scan(p->d_plan, p->d_out, p->h, s), "launch scan");
    if (p->timing) FSPB_HIP(hipEventRecord(p->ev[5], s), "record event");
    FSPB_HIP(hipMemcpyAsync(p->nnz_host, p->d_nnz, sizeof(int64_t), hipMemcpyDeviceToHost, s), "read nnz");
    FSPB_HIP(hipEventRecord(p->nnz_ready, s), "record count event");
    // the fill is queued before the count is known; it writes nothing unless the total fits
    const bool fill = indices && values && capacity > 0;
    if (fill) {
        if (p->timing) FSPB_HIP(hipEventRecord(p->ev[6], s), "record event");
        FSPB_HIP(fspb::launch_fill(p->d_plan, p->d_out, p->h, 0, p->h.n_beamlets, s), "launch fill");
        if (p->timing) FSPB_HIP(hipEventRecord(p->ev[7], s), "record event");
    }
    FSPB_HIP(hipEventSynchronize(p->nnz_ready), "wait for nnz");
    const int64_t nnz = *p->nnz_host;
    *nnz_out = nnz;
    p->counted = true;
    if (!fill || capacity < nnz)
        return fail(FSPB_ERR_CAPACITY, "%lld nonzeros do not fit a capacity of %lld", (long long)nnz,
                    (long long)(fill ? capacity : 0));
    p->have_dose_ev = p->timing;
    return FSPB_OK;
}

fspb_status fspb_dose_coeffs_rows(fspb_plan *p, int32_t j0, int32_t j1, const int64_t *indptr, int32_t *indices,
                                  float *values, int64_t capacity, int64_t *nnz_out, void *stream)
{
    g_last_error.clear();
    if (!p) return fail(FSPB_ERR_INVALID, "plan is NULL");
    if (!indptr || !nnz_out) return fail(FSPB_ERR_INVALID, "indptr or nnz_out is NULL");
    if (j0 < 0 || j1 < j0 || j1 > p->h.n_beamlets)
        return fail(FSPB_ERR_INVALID, "row range [%d, %d) outside [0, %d)", j0, j1, p->h.n_beamlets);
    if (capacity < 0) return fail(FSPB_ERR_INVALID, "capacity must be >= 0");
    if (!p->counted) return fail(FSPB_ERR_STATE, "fspb_dose_coeffs must count the rows first");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int64_t ends[2] = {0, 0};
    FSPB_HIP(hipMemcpyAsync(&ends[0], indptr + j0, sizeof(int64_t), hipMemcpyDeviceToHost, s), "read indptr");
    FSPB_HIP(hipMemcpyAsync(&ends[1], indptr + j1, sizeof(int64_t), hipMemcpyDeviceToHost, s), "read indptr");
    FSPB_HIP(hipStreamSynchronize(s), "synchronise for the row range");
    const int64_t nnz = ends[1] - ends[0];
    if (nnz < 0) return fail(FSPB_ERR_INVALID, "indptr is not the counted row-pointer array");
    *nnz_out = nnz;
    if (!indices || !values || capacity < nnz)
        return fail(FSPB_ERR_CAPACITY, "%lld nonzeros do not fit a capacity of %lld", (long long)nnz,
                    (long long)(indices && values ? capacity : 0));
    p->out.indptr = const_cast<int64_t *>(indptr);
    p->out.indices = indices;
    p->out.values = values;
    p->out.capacity = capacity;
    p->out.overflow = p->d_overflow;
    p->out.row0 = j0;
    p->out.check_nnz = 0;   // the range's size was checked above
    FSPB_HIP(hipMemcpyAsync(p->d_out, &p->out, sizeof(OutDev), hipMemcpyHostToDevice, s), "upload output record");
    FSPB_HIP(fspb::launch_fill(p->d_plan, p->d_out, p->h, j0, j1 - j0, s), "launch fill");
    return FSPB_OK;
}

fspb_status fspb_row_ranges(const int64_t *indptr, int32_t n_rows, const int32_t *beam_rows, int32_t n_beams,
                            int64_t max_bytes, int32_t *bounds, int32_t max_ranges, int32_t *n_ranges)
{
    g_last_error.clear();
    if (!indptr || !n_ranges) return fail(FSPB_ERR_INVALID, "indptr or n_ranges is NULL");
    if (n_rows < 0 || n_beams < 0 || max_bytes < 0 || max_ranges < 0)
        return fail(FSPB_ERR_INVALID, "n_rows, n_beams, max_bytes and max_ranges must be >= 0");
    if (n_beams > 0 && !beam_rows) return fail(FSPB_ERR_INVALID, "beam_rows is NULL");
    for (int32_t j = 0; j < n_rows; ++j)
        if (indptr[j + 1] < indptr[j]) return fail(FSPB_ERR_INVALID, "indptr decreases at row %d", j);
    // candidate ends: the beam boundaries (by beam), or every row boundary
    std::vector<int32_t> units;
    if (n_beams > 0) {
        int64_t acc = 0;
        units.push_back(0);
        for (int32_t b = 0; b < n_beams; ++b) {
            if (beam_rows[b] < 0) return fail(FSPB_ERR_INVALID, "beam_rows[%d] < 0", b);
            acc += beam_rows[b];
            units.push_back((int32_t)std::min<int64_t>(acc, INT32_MAX));
        }
        if (acc != n_rows) return fail(FSPB_ERR_INVALID, "beam_rows sum to %lld, not %d rows", (long long)acc, n_rows);
    }
    const int64_t cap = max_bytes / 8;   // FP32 value + int32 column per entry
    int32_t count = 0, j0 = 0;
    size_t u = 0;                        // first beam boundary > j0
    std::vector<int32_t> ends;
    while (j0 < n_rows) {
        const int64_t limit = indptr[j0] + cap;
        while (u < units.size() && units[u] <= j0) ++u;
        int32_t j1 = j0;
        // furthest beam boundary that fits, else furthest row boundary
        for (size_t k = u; k < units.size() && indptr[units[k]] <= limit; ++k) j1 = units[k];
        if (j1 == j0) {
            int32_t r = j0 + 1;
            if (indptr[r] > limit)
                return fail(FSPB_ERR_INVALID, "row %d alone needs %lld bytes, more than the budget of %lld", j0,
                            (long long)(8 * (indptr[r] - indptr[j0])), (long long)max_bytes);
            while (r + 1 <= n_rows && indptr[r + 1] <= limit) ++r;
            j1 = r;
        }
        ends.push_back(j1);
        ++count;
        j0 = j1;
    }
    *n_ranges = count;
    if (!bounds || count > max_ranges)
        return fail(FSPB_ERR_CAPACITY, "%d ranges do not fit max_ranges = %d", count, bounds ? max_ranges : 0);
    bounds[0] = 0;
    for (int32_t k = 0; k < count; ++k) bounds[k + 1] = ends[(size_t)k];
    return FSPB_OK;
}

fspb_status fspb_plan_set_timing(fspb_plan *p, int32_t enable)
{
    g_last_error.clear();
    if (!p) return fail(FSPB_ERR_INVALID, "plan is NULL");
    if (enable && !p->ev[0])
        for (hipEvent_t &e : p->ev) FSPB_HIP(hipEventCreate(&e), "create timing event");
    p->timing = enable != 0;
    p->have_trace_ev = p->have_dose_ev = false;
    return FSPB_OK;
}

fspb_status fspb_plan_get_timing(fspb_plan *p, fspb_timing *t)
{
    g_last_error.clear();
    if (!p || !t) return fail(FSPB_ERR_INVALID, "plan or timing is NULL");
    std::memset(t, 0, sizeof *t);
    if (!p->have_trace_ev || !p->have_dose_ev) return FSPB_OK;
    FSPB_HIP(hipEventSynchronize(p->ev[7]), "wait for timing events");
    FSPB_HIP(hipEventElapsedTime(&t->prep_ms, p->ev[0], p->ev[1]), "elapsed");
    FSPB_HIP(hipEventElapsedTime(&t->count_ms, p->ev[1], p->ev[3]), "elapsed");
    FSPB_HIP(hipEventElapsedTime(&t->raytrace_ms, p->ev[3], p->ev[2]), "elapsed");
    FSPB_HIP(hipEventElapsedTime(&t->scan_ms, p->ev[4], p->ev[5]), "elapsed");
    FSPB_HIP(hipEventElapsedTime(&t->fill_ms, p->ev[6], p->ev[7]), "elapsed");
    t->valid = 1;
    return FSPB_OK;
}

void fspb_plan_destroy(fspb_plan *p) { delete p; }

fspb_status fspb_plan_info(const fspb_plan *p, fspb_plan_desc *d)
{
    g_last_error.clear();
    if (!p || !d) return fail(FSPB_ERR_INVALID, "plan or desc is NULL");
    d->n_beamlets = p->h.n_beamlets;
    d->n_voxels = p->n_voxels;
    d->table_entries = p->table_entries;
    d->n_tiles = p->h.n_tiles;
    d->max_table = p->h.max_table;
    d->fill_lds_bytes = (int32_t)fspb::fill_shared_bytes(p->h);
    d->fill_erf_mode = p->h.use_mlp ? 0 : p->h.erf_mode;
    return FSPB_OK;
}

fspb_status fspb_plan_get_tables(fspb_plan *p, float *tables, int64_t *offsets, void *stream)
{
    g_last_error.clear();
    if (!p) return fail(FSPB_ERR_INVALID, "plan is NULL");
    if (!p->traced) return fail(FSPB_ERR_STATE, "fspb_raytrace must run before fspb_plan_get_tables");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (offsets) {
        int64_t acc = 0;
        for (size_t j = 0; j < p->recs.size(); ++j) {
            offsets[j] = acc;
            acc += p->recs[j].n_table;
        }
        offsets[p->recs.size()] = acc;
    }
    if (tables && p->table_entries > 0) {
        FSPB_HIP(hipMemcpyAsync(tables, p->h.tables, sizeof(float) * (size_t)p->table_entries, hipMemcpyDeviceToHost, s),
                 "read tables");
        FSPB_HIP(hipStreamSynchronize(s), "synchronise tables");
    }
    return FSPB_OK;
}

}  // extern "C"

/* ======================================================================
 * Batches
 * ====================================================================== */

namespace {

struct BatchKey {
    int32_t n_plans, max_terms;
    int64_t beamlets, nnz2;   // nnz rounded to two significant digits
    bool operator<(const BatchKey &o) const
    {
        if (n_plans != o.n_plans) return n_plans < o.n_plans;
        if (max_terms != o.max_terms) return max_terms < o.max_terms;
        if (beamlets != o.beamlets) return beamlets < o.beamlets;
        return nnz2 < o.nnz2;
    }
};

std::mutex g_tune_mu;
std::map<BatchKey, fspb_batch_config> g_tune_cache;

int64_t two_digits(int64_t v)
{
    int64_t scale = 1;
    while (v >= 100) {
        v /= 10;
        scale *= 10;
    }
    return v * scale;
}

}  // namespace

// wave stages of a batch before the scan: mask rows, ray traces, counts
constexpr int kWaveStages = 3;

struct fspb_batch {
    std::vector<fspb_plan *> plans;
    int32_t n = 0;
    // device arrays (caller workspace)
    const PlanDev **d_plans = nullptr;
    OutDev *d_outs = nullptr;
    int64_t *d_start[kWaveStages] = {};   // item prefix per wave stage: rows, beamlets, beamlets
    int2 *d_items[2] = {};        // fill items: longest first, plan order
    int *d_counter = nullptr;
    int32_t n_items = 0;
    int64_t total[kWaveStages] = {};
    std::vector<int64_t> nnz;
    std::vector<OutDev> outs;
    std::vector<bool> bound;
    int32_t max_terms = 1;
    size_t lds = 0;
    int cus = 256;
    fspb_batch_config cfg{4, 4, 0, 0, 0.0f, fspb::kRowsPerTile, 1, 0};
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~fspb_batch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
    void drop_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

namespace {

int wave_grid(const fspb_batch *b, int64_t items)
{
    // persistent grid: enough 4-wave groups to fill the chip several times over
    const int64_t want = (items + fspb::kWave - 1) / 4;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)b->cus * 16));
}

fspb_status launch_fill_only(fspb_batch *b, hipStream_t s, bool reset);

fspb_status enqueue_stages(fspb_batch *b, hipStream_t s, bool with_fill)
{
    FSPB_HIP(fspb::launch_batch_reset(b->d_counter, 1, s), "launch batch reset");
    for (int st = 0; st < kWaveStages; ++st) {
        if (b->total[st] == 0) continue;
        FSPB_HIP(fspb::launch_batch_wave(st, b->d_plans, b->d_start[st], b->n, wave_grid(b, b->total[st]), s),
                 "launch batch stage");
    }
    FSPB_HIP(fspb::launch_batch_scan(b->d_plans, b->d_outs, b->n, s), "launch batch scan");
    if (with_fill && b->n_items > 0) {
        const fspb_status r = launch_fill_only(b, s, false);
        if (r != FSPB_OK) return r;
    }
    return FSPB_OK;
}

/* The batched fill in the current shape (reset: clear the queue counter first). */
fspb_status launch_fill_only(fspb_batch *b, hipStream_t s, bool reset)
{
    if (reset) FSPB_HIP(fspb::launch_batch_reset(b->d_counter, 1, s), "launch batch reset");
    const int per_item = b->cfg.beamlets_per_item > 0 ? b->cfg.beamlets_per_item : 1;
    const int tile_group = b->cfg.tile_rows > 0 ? b->cfg.tile_rows / fspb::kRowsPerTile : 1;
    const int fetches = (b->n_items + per_item - 1) / per_item;
    const int grid = std::max(1, std::min(fetches, b->cfg.groups_per_cu * b->cus));
    FSPB_HIP(fspb::launch_batch_fill(b->max_terms, b->cfg.waves_per_group, b->d_plans, b->d_outs,
                                     b->d_items[b->cfg.order], b->n_items, b->d_counter, per_item, tile_group, grid,
                                     b->lds, s),
             "launch batch fill");
    return FSPB_OK;
}

bool valid_config(const fspb_batch_config &c)
{
    return (c.waves_per_group == 2 || c.waves_per_group == 4 || c.waves_per_group == 8) && c.groups_per_cu >= 1 &&
           c.groups_per_cu <= 16 && (c.order == 0 || c.order == 1) &&
           (c.tile_rows == 0 || c.tile_rows == 64 || c.tile_rows == 128 || c.tile_rows == 256) &&
           (c.beamlets_per_item == 0 || c.beamlets_per_item == 1 || c.beamlets_per_item == 2 ||
            c.beamlets_per_item == 4);
}

BatchKey key_of(const fspb_batch *b)
{
    int64_t beamlets = 0, nnz = 0;
    for (int i = 0; i < b->n; ++i) {
        beamlets += b->plans[i]->h.n_beamlets;
        nnz += b->nnz[i];
    }
    return BatchKey{b->n, b->max_terms, beamlets, two_digits(nnz)};
}

}  // namespace

extern "C" {

fspb_status fspb_batch_create(fspb_plan *const *plans, int32_t n_plans, void *workspace, size_t workspace_bytes,
                              size_t *workspace_needed, void *stream, fspb_batch **out)
{
    g_last_error.clear();
    if (!out) return fail(FSPB_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!plans || n_plans < 1) return fail(FSPB_ERR_INVALID, "plans is NULL or n_plans < 1");
    if (n_plans > 4096) return fail(FSPB_ERR_INVALID, "at most 4096 plans per batch");
    for (int i = 0; i < n_plans; ++i) {
        if (!plans[i]) return fail(FSPB_ERR_INVALID, "plans[%d] is NULL", i);
        if (plans[i]->h.gen) return fail(FSPB_ERR_INVALID, "plans[%d] uses kernel tables (not batched)", i);
        if (plans[i]->h.use_mlp)
            return fail(FSPB_ERR_INVALID, "plans[%d] has a surrogate attached (a batch computes Eq. 2-3 analytically)", i);
        for (int k = 0; k < i; ++k)
            if (plans[k] == plans[i]) return fail(FSPB_ERR_INVALID, "plan %d appears twice", i);
    }
    if (!workspace && !workspace_needed) return fail(FSPB_ERR_INVALID, "workspace and workspace_needed are both NULL");

    int64_t beamlets = 0;
    for (int i = 0; i < n_plans; ++i) beamlets += plans[i]->h.n_beamlets;
    if (beamlets >= (int64_t)1 << 31) return fail(FSPB_ERR_INVALID, "too many beamlets in the batch");
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    const size_t o_plans = take(sizeof(PlanDev *) * n_plans);
    const size_t o_outs = take(sizeof(OutDev) * n_plans);
    size_t o_start[kWaveStages];
    for (int st = 0; st < kWaveStages; ++st) o_start[st] = take(sizeof(int64_t) * (n_plans + 1));
    const size_t o_items0 = take(sizeof(int2) * (size_t)std::max<int64_t>(beamlets, 1));
    const size_t o_items1 = take(sizeof(int2) * (size_t)std::max<int64_t>(beamlets, 1));
    const size_t o_counter = take(64);
    if (workspace_needed) *workspace_needed = off;
    if (!workspace) return fail(FSPB_ERR_CAPACITY, "batch workspace query: %zu bytes needed", off);
    if (workspace_bytes < off)
        return fail(FSPB_ERR_CAPACITY, "batch workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, off);
    if ((uintptr_t)workspace % 256 != 0) return fail(FSPB_ERR_INVALID, "workspace must be 256-byte aligned");

    fspb_batch *b = new (std::nothrow) fspb_batch;
    if (!b) return fail(FSPB_ERR_NOMEM, "cannot allocate the batch");
    std::unique_ptr<fspb_batch> guard(b);
    b->plans.assign(plans, plans + n_plans);
    b->n = n_plans;
    char *ws = static_cast<char *>(workspace);
    b->d_plans = reinterpret_cast<const PlanDev **>(ws + o_plans);
    b->d_outs = reinterpret_cast<OutDev *>(ws + o_outs);
    for (int st = 0; st < kWaveStages; ++st) b->d_start[st] = reinterpret_cast<int64_t *>(ws + o_start[st]);
    b->d_items[0] = reinterpret_cast<int2 *>(ws + o_items0);
    b->d_items[1] = reinterpret_cast<int2 *>(ws + o_items1);
    b->d_counter = reinterpret_cast<int *>(ws + o_counter);
    int dev = 0;
    FSPB_HIP(hipGetDevice(&dev), "get device");
    FSPB_HIP(hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev), "query compute units");

    std::vector<const PlanDev *> pp(n_plans);
    std::vector<int64_t> start[kWaveStages];
    for (int st = 0; st < kWaveStages; ++st) start[st].assign(n_plans + 1, 0);
    b->outs.assign(n_plans, OutDev{});
    b->bound.assign(n_plans, false);
    for (int i = 0; i < n_plans; ++i) {
        const PlanDev &h = plans[i]->h;
        pp[i] = plans[i]->d_plan;
        start[0][i + 1] = start[0][i] + (int64_t)h.ny * h.nz;
        start[1][i + 1] = start[1][i] + h.n_beamlets;
        start[2][i + 1] = start[2][i] + h.n_beamlets;
        b->max_terms = std::max(b->max_terms, h.n_terms);
        b->lds = std::max(b->lds, fspb::fill_shared_bytes(h));   // each plan's erf table form
        b->outs[i].overflow = plans[i]->d_overflow;
    }
    for (int st = 0; st < kWaveStages; ++st) b->total[st] = start[st][n_plans];
    FSPB_HIP(hipMemcpy(b->d_plans, pp.data(), sizeof(PlanDev *) * n_plans, hipMemcpyHostToDevice), "upload plan table");
    for (int st = 0; st < kWaveStages; ++st)
        FSPB_HIP(hipMemcpy(b->d_start[st], start[st].data(), sizeof(int64_t) * (n_plans + 1), hipMemcpyHostToDevice),
                 "upload item ranges");

    // sizing pass: mask, tables, counts, row sums
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int i = 0; i < n_plans; ++i) {
        fspb_status us = plan_upload(plans[i], s);
        if (us != FSPB_OK) return us;
    }
    FSPB_HIP(fspb::launch_batch_reset(b->d_counter, 1, s), "launch batch reset");
    for (int st = 0; st < kWaveStages; ++st)
        if (b->total[st] > 0)
            FSPB_HIP(fspb::launch_batch_wave(st, b->d_plans, b->d_start[st], n_plans, wave_grid(b, b->total[st]), s),
                     "launch batch stage");
    std::vector<std::vector<int64_t>> rn(n_plans);
    for (int i = 0; i < n_plans; ++i) {
        rn[i].resize(plans[i]->h.n_beamlets);
        FSPB_HIP(hipMemcpyAsync(rn[i].data(), plans[i]->h.row_nnz, sizeof(int64_t) * rn[i].size(),
                                hipMemcpyDeviceToHost, s),
                 "read row counts");
    }
    FSPB_HIP(hipStreamSynchronize(s), "synchronise sizing pass");
    b->nnz.assign(n_plans, 0);
    std::vector<std::pair<int64_t, int2>> items;
    items.reserve((size_t)beamlets);
    for (int i = 0; i < n_plans; ++i)
        for (int j = 0; j < (int)rn[i].size(); ++j) {
            b->nnz[i] += rn[i][j];
            if (rn[i][j] > 0) items.push_back({rn[i][j], make_int2(i, j)});
        }
    b->n_items = (int32_t)items.size();
    std::vector<int2> natural(items.size()), longest(items.size());
    for (size_t k = 0; k < items.size(); ++k) natural[k] = items[k].second;
    std::stable_sort(items.begin(), items.end(),
                     [](const std::pair<int64_t, int2> &a, const std::pair<int64_t, int2> &c) { return a.first > c.first; });
    for (size_t k = 0; k < items.size(); ++k) longest[k] = items[k].second;
    if (!items.empty()) {
        FSPB_HIP(hipMemcpy(b->d_items[0], longest.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice),
                 "upload fill queue");
        FSPB_HIP(hipMemcpy(b->d_items[1], natural.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice),
                 "upload fill queue");
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key_of(b));
        if (it != g_tune_cache.end()) b->cfg = it->second;
    }
    FSPB_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "create capture stream");
    for (fspb_plan *q : b->plans) ++q->batches;
    *out = guard.release();
    return FSPB_OK;
}

fspb_status fspb_batch_nnz(const fspb_batch *b, int32_t plan, int64_t *nnz)
{
    g_last_error.clear();
    if (!b || !nnz) return fail(FSPB_ERR_INVALID, "batch or nnz is NULL");
    if (plan < 0 || plan >= b->n) return fail(FSPB_ERR_INVALID, "plan index %d out of range", plan);
    *nnz = b->nnz[plan];
    return FSPB_OK;
}

fspb_status fspb_batch_bind(fspb_batch *b, int32_t plan, int64_t *indptr, int32_t *indices, float *values,
                            int64_t capacity)
{
    g_last_error.clear();
    if (!b) return fail(FSPB_ERR_INVALID, "batch is NULL");
    if (plan < 0 || plan >= b->n) return fail(FSPB_ERR_INVALID, "plan index %d out of range", plan);
    if (!indptr || ((!indices || !values) && b->nnz[plan] > 0))
        return fail(FSPB_ERR_INVALID, "output pointers are NULL");
    if (capacity < b->nnz[plan])
        return fail(FSPB_ERR_CAPACITY, "plan %d needs %lld entries, capacity %lld", plan, (long long)b->nnz[plan],
                    (long long)capacity);
    OutDev &o = b->outs[plan];
    o.indptr = indptr;
    o.indices = indices;
    o.values = values;
    o.capacity = capacity;
    FSPB_HIP(hipMemcpy(b->d_outs + plan, &o, sizeof(OutDev), hipMemcpyHostToDevice), "upload output record");
    b->bound[plan] = true;
    b->drop_graph();
    return FSPB_OK;
}

fspb_status fspb_batch_get_config(const fspb_batch *b, fspb_batch_config *cfg)
{
    g_last_error.clear();
    if (!b || !cfg) return fail(FSPB_ERR_INVALID, "batch or cfg is NULL");
    *cfg = b->cfg;
    return FSPB_OK;
}

fspb_status fspb_batch_set_config(fspb_batch *b, const fspb_batch_config *cfg)
{
    g_last_error.clear();
    if (!b || !cfg) return fail(FSPB_ERR_INVALID, "batch or cfg is NULL");
    if (!valid_config(*cfg)) return fail(FSPB_ERR_INVALID, "invalid launch shape");
    b->cfg = *cfg;
    if (b->cfg.tile_rows == 0) b->cfg.tile_rows = fspb::kRowsPerTile;
    if (b->cfg.beamlets_per_item == 0) b->cfg.beamlets_per_item = 1;
    b->cfg.tuned = 0;
    b->cfg.fill_ms = 0.0f;
    b->drop_graph();
    return FSPB_OK;
}

fspb_status fspb_batch_tune(fspb_batch *b, void *stream)
{
    g_last_error.clear();
    if (!b) return fail(FSPB_ERR_INVALID, "batch is NULL");
    for (int i = 0; i < b->n; ++i)
        if (!b->bound[i]) return fail(FSPB_ERR_STATE, "plan %d has no bound outputs", i);
    hipStream_t s = static_cast<hipStream_t>(stream);
    fspb_status st = enqueue_stages(b, s, false);
    if (st != FSPB_OK) return st;
    hipEvent_t e0, e1;
    FSPB_HIP(hipEventCreate(&e0), "create event");
    FSPB_HIP(hipEventCreate(&e1), "create event");
    fspb_batch_config best = b->cfg;
    float best_ms = 1e30f;
    auto trial = [&](const fspb_batch_config &c) -> fspb_status {
        b->cfg = c;
        float ms = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
            FSPB_HIP(hipEventRecord(e0, s), "record event");
            const fspb_status r = launch_fill_only(b, s, true);
            if (r != FSPB_OK) return r;
            FSPB_HIP(hipEventRecord(e1, s), "record event");
            FSPB_HIP(hipEventSynchronize(e1), "wait event");
            float t = 0.0f;
            FSPB_HIP(hipEventElapsedTime(&t, e0, e1), "elapsed");
            ms = std::min(ms, t);
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
        return FSPB_OK;
    };
    const fspb_batch_config saved = b->cfg;
    // workgroup size, grid and queue order at the base tile shape
    for (int order = 0; order < 2 && st == FSPB_OK; ++order)
        for (int w : {2, 4, 8})
            for (int g : {1, 2, 4, 8})
                if (st == FSPB_OK) st = trial(fspb_batch_config{w, g, order, 0, 0.0f, fspb::kRowsPerTile, 1, 0});
    // then the tile rows per wave step and the beamlets per work item for that launch
    const fspb_batch_config base = best;
    for (int rows : {64, 128, 256})
        for (int per : {1, 2, 4}) {
            if (st != FSPB_OK || (rows == fspb::kRowsPerTile && per == 1)) continue;
            fspb_batch_config c = base;
            c.tile_rows = rows;
            c.beamlets_per_item = per;
            st = trial(c);
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FSPB_OK) {
        b->cfg = saved;
        return st;
    }
    best.tuned = 1;
    best.fill_ms = best_ms;
    b->cfg = best;
    b->drop_graph();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key_of(b)] = best;
    return FSPB_OK;
}

fspb_status fspb_batch_run(fspb_batch *b, void *stream)
{
    g_last_error.clear();
    if (!b) return fail(FSPB_ERR_INVALID, "batch is NULL");
    for (int i = 0; i < b->n; ++i)
        if (!b->bound[i]) return fail(FSPB_ERR_STATE, "plan %d has no bound outputs", i);
    if (!b->exec) {
        FSPB_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
        fspb_status st = enqueue_stages(b, b->cap_stream, true);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
        if (st != FSPB_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        b->graph = g;
        FSPB_HIP(hipGraphInstantiateWithFlags(&b->exec, b->graph, 0), "instantiate graph");
    }
    FSPB_HIP(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)), "launch graph");
    return FSPB_OK;
}

fspb_status fspb_batch_check(fspb_batch *b, void *stream)
{
    g_last_error.clear();
    if (!b) return fail(FSPB_ERR_INVALID, "batch is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int32_t> flags(b->n, 0);
    for (int i = 0; i < b->n; ++i)
        FSPB_HIP(hipMemcpyAsync(&flags[i], b->plans[i]->d_overflow, sizeof(int32_t), hipMemcpyDeviceToHost, s),
                 "read overflow flag");
    FSPB_HIP(hipStreamSynchronize(s), "synchronise check");
    int first = -1;
    for (int i = 0; i < b->n; ++i)
        if (flags[i]) {
            if (first < 0) first = i;
            FSPB_HIP(hipMemset(b->plans[i]->d_overflow, 0, sizeof(int32_t)), "clear overflow flag");
        }
    if (first >= 0) return fail(FSPB_ERR_OVERFLOW, "plan %d produced more nonzeros than its capacity", first);
    return FSPB_OK;
}

void fspb_batch_destroy(fspb_batch *b)
{
    if (!b) return;
    for (fspb_plan *q : b->plans) --q->batches;
    delete b;
}

}  // extern "C"

/* ======================================================================
 * Kernel surrogate
 * ====================================================================== */

struct fspb_surrogate {
    fspb::MlpTargetDev tk{};
    float *params = nullptr, *m1 = nullptr, *m2 = nullptr, *partials = nullptr, *grad = nullptr;
    uint16_t *w2 = nullptr, *w2t = nullptr;
    int32_t max_batch = 0;
    int64_t adam_step = 0;
    int32_t n_terms = 0;
    double weight[4] = {}, sigma0[4] = {}, sigma_slope[4] = {}, width_scale[4] = {}, pdd_step = 0.0;
    std::vector<float> pdd;
};

namespace {

fspb::MlpDev mlp_view(const fspb_surrogate *s) { return fspb::MlpDev{s->params, s->w2, s->w2t}; }

/* SplitMix64 (Steele, Lea and Flood 2014): the per-epoch sample order. */
uint64_t splitmix64(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

uint64_t gcd_u64(uint64_t a, uint64_t b)
{
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

}  // namespace

extern "C" {

fspb_status fspb_surrogate_create(const fspb_kernel *K, const float *init, int32_t max_batch, void *workspace,
                                  size_t workspace_bytes, size_t *workspace_needed, fspb_surrogate **out)
{
    g_last_error.clear();
    if (!out) return fail(FSPB_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!K || !init) return fail(FSPB_ERR_INVALID, "kernel or init_params is NULL");
    if (K->n_terms < 1 || K->n_terms > 4) return fail(FSPB_ERR_INVALID, "kernel.n_terms must be 1..4");
    for (int i = 0; i < K->n_terms; ++i)
        if (!(K->sigma0[i] > 0.0) || !(K->sigma_slope[i] >= 0.0) || !(K->width_scale[i] > 0.0) ||
            !std::isfinite(K->weight[i]))
            return fail(FSPB_ERR_INVALID, "kernel term %d has invalid parameters", i);
    if (!K->pdd || K->n_pdd < 2 || K->n_pdd > 4096 || !(K->pdd_step > 0.0))
        return fail(FSPB_ERR_INVALID, "kernel depth-dose table is invalid");
    if (max_batch < 64 || max_batch % 64 != 0 || max_batch > (1 << 20))
        return fail(FSPB_ERR_INVALID, "max_batch must be a positive multiple of 64 (<= 2^20)");
    for (int i = 0; i < fspb::kMlpParams; ++i)
        if (!std::isfinite(init[i])) return fail(FSPB_ERR_INVALID, "init_params[%d] is not finite", i);
    if (!workspace && !workspace_needed) return fail(FSPB_ERR_INVALID, "workspace and workspace_needed are both NULL");
    const int waves = max_batch / 64;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    const size_t o_p = take(sizeof(float) * fspb::kPartialStride), o_m1 = take(sizeof(float) * fspb::kPartialStride);
    const size_t o_m2 = take(sizeof(float) * fspb::kPartialStride), o_g = take(sizeof(float) * fspb::kPartialStride);
    const size_t o_w2 = take(2 * fspb::kMlpH * fspb::kMlpH), o_w2t = take(2 * fspb::kMlpH * fspb::kMlpH);
    const size_t o_pdd = take(sizeof(float) * K->n_pdd), o_erfc = take(sizeof(float4) * fspb::kErfcIntervals);
    const size_t o_part = take(sizeof(float) * fspb::kPartialStride * (size_t)waves);
    if (workspace_needed) *workspace_needed = off;
    if (!workspace) return fail(FSPB_ERR_CAPACITY, "surrogate workspace query: %zu bytes needed", off);
    if (workspace_bytes < off) return fail(FSPB_ERR_CAPACITY, "surrogate workspace too small (%zu < %zu)", workspace_bytes, off);
    if ((uintptr_t)workspace % 256 != 0) return fail(FSPB_ERR_INVALID, "workspace must be 256-byte aligned");
    fspb_surrogate *s = new (std::nothrow) fspb_surrogate;
    if (!s) return fail(FSPB_ERR_NOMEM, "cannot allocate the surrogate");
    std::unique_ptr<fspb_surrogate> guard(s);
    char *ws = static_cast<char *>(workspace);
    s->params = reinterpret_cast<float *>(ws + o_p);
    s->m1 = reinterpret_cast<float *>(ws + o_m1);
    s->m2 = reinterpret_cast<float *>(ws + o_m2);
    s->grad = reinterpret_cast<float *>(ws + o_g);
    s->w2 = reinterpret_cast<uint16_t *>(ws + o_w2);
    s->w2t = reinterpret_cast<uint16_t *>(ws + o_w2t);
    s->partials = reinterpret_cast<float *>(ws + o_part);
    s->max_batch = max_batch;
    s->n_terms = K->n_terms;
    s->tk.n_terms = K->n_terms;
    s->tk.n_pdd = K->n_pdd;
    for (int i = 0; i < 4; ++i) {
        const bool on = i < K->n_terms;
        s->weight[i] = on ? K->weight[i] : 0.0;
        s->sigma0[i] = on ? K->sigma0[i] : 0.0;
        s->sigma_slope[i] = on ? K->sigma_slope[i] : 0.0;
        s->width_scale[i] = on ? K->width_scale[i] : 0.0;
        s->tk.w4[i] = on ? (float)(0.25 * K->weight[i]) : 0.0f;
        s->tk.sig0[i] = on ? (float)K->sigma0[i] : 1.0f;
        s->tk.sig1[i] = on ? (float)K->sigma_slope[i] : 0.0f;
        s->tk.c2[i] = on ? (float)K->width_scale[i] : 1.0f;
    }
    s->pdd_step = K->pdd_step;
    s->pdd.assign(K->pdd, K->pdd + K->n_pdd);
    s->tk.pdd_inv_step = (float)(1.0 / K->pdd_step);
    s->tk.pdd_max = (float)(K->n_pdd - 1);
    s->tk.pdd = reinterpret_cast<float *>(ws + o_pdd);
    s->tk.erfc_tab = reinterpret_cast<float4 *>(ws + o_erfc);
    FSPB_HIP(hipMemcpy((void *)s->tk.pdd, K->pdd, sizeof(float) * K->n_pdd, hipMemcpyHostToDevice), "upload depth dose");
    std::vector<float4> et;
    erfc_table(et);
    FSPB_HIP(hipMemcpy((void *)s->tk.erfc_tab, et.data(), sizeof(float4) * et.size(), hipMemcpyHostToDevice),
             "upload erfc table");
    FSPB_HIP(hipMemcpy(s->params, init, sizeof(float) * fspb::kMlpParams, hipMemcpyHostToDevice), "upload parameters");
    FSPB_HIP(hipMemset(s->m1, 0, sizeof(float) * fspb::kPartialStride), "clear Adam moments");
    FSPB_HIP(hipMemset(s->m2, 0, sizeof(float) * fspb::kPartialStride), "clear Adam moments");
    FSPB_HIP(fspb::launch_mlp_bf16_copies(s->params, s->w2, s->w2t, nullptr), "launch bf16 copies");
    FSPB_HIP(hipDeviceSynchronize(), "synchronise surrogate creation");
    *out = guard.release();
    return FSPB_OK;
}

fspb_status fspb_surrogate_targets(fspb_surrogate *s, const float *samples, int64_t n, float *features, float *targets,
                                   void *stream)
{
    g_last_error.clear();
    if (!s || !samples || !features || !targets || n < 0) return fail(FSPB_ERR_INVALID, "invalid arguments");
    FSPB_HIP(fspb::launch_mlp_targets(s->tk, samples, n, features, targets, static_cast<hipStream_t>(stream)),
             "launch targets");
    return FSPB_OK;
}

fspb_status fspb_surrogate_forward(fspb_surrogate *s, const float *features, int64_t n, float *out, void *stream)
{
    g_last_error.clear();
    if (!s || !features || !out || n < 0) return fail(FSPB_ERR_INVALID, "invalid arguments");
    FSPB_HIP(fspb::launch_mlp_forward(mlp_view(s), features, n, out, static_cast<hipStream_t>(stream)),
             "launch forward");
    return FSPB_OK;
}

fspb_status fspb_surrogate_gradient(fspb_surrogate *s, const float *features, const float *targets, int64_t n,
                                    float *grad, float *loss, void *stream)
{
    g_last_error.clear();
    if (!s || !features || !targets || !grad || !loss) return fail(FSPB_ERR_INVALID, "invalid arguments");
    if (n < 1 || n > s->max_batch) return fail(FSPB_ERR_INVALID, "n must be 1..max_batch");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int waves = (int)((n + 63) / 64);
    FSPB_HIP(fspb::launch_mlp_grad(mlp_view(s), features, targets, n, 0, n, 1, 0, 1.0f / (float)n, s->partials, st),
             "launch gradient");
    FSPB_HIP(fspb::launch_mlp_reduce(s->params, s->m1, s->m2, s->w2, s->w2t, s->partials, waves, 0, 0.f, 0.f, 0.f, 0.f,
                                     1.f, 1.f, s->grad, st),
             "launch reduce");
    FSPB_HIP(hipMemcpyAsync(grad, s->grad, sizeof(float) * fspb::kMlpParams, hipMemcpyDeviceToDevice, st), "copy gradient");
    float lsum = 0.0f;
    FSPB_HIP(hipMemcpyAsync(&lsum, s->grad + fspb::kMlpParams, sizeof(float), hipMemcpyDeviceToHost, st), "read loss");
    FSPB_HIP(hipStreamSynchronize(st), "synchronise gradient");
    *loss = lsum / (float)n;
    return FSPB_OK;
}

fspb_status fspb_surrogate_train(fspb_surrogate *s, const float *features, const float *targets, int64_t n,
                                 const fspb_train_config *cfg, float *loss_per_epoch, void *stream)
{
    g_last_error.clear();
    if (!s || !features || !targets || !cfg) return fail(FSPB_ERR_INVALID, "invalid arguments");
    if (cfg->epochs < 1 || cfg->batch < 64 || cfg->batch % 64 != 0 || cfg->batch > s->max_batch)
        return fail(FSPB_ERR_INVALID, "epochs >= 1 and batch a multiple of 64 up to max_batch are required");
    if (n < cfg->batch) return fail(FSPB_ERR_INVALID, "fewer samples than one batch");
    if (!(cfg->lr_max > 0.0f) || !(cfg->lr_min >= 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) ||
        !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) || !(cfg->eps > 0.0f))
        return fail(FSPB_ERR_INVALID, "invalid optimiser settings");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t steps = n / cfg->batch;
    const int64_t total = steps * cfg->epochs;
    const int waves = cfg->batch / 64;
    int64_t k = 0;
    for (int e = 0; e < cfg->epochs; ++e) {
        // sample order of this epoch: i -> (offset + i stride) mod n with gcd(stride, n) = 1
        const uint64_t r1 = splitmix64(cfg->seed ^ (0x51ed2701ull * (uint64_t)(e + 1)));
        const uint64_t r2 = splitmix64(r1);
        uint64_t stride = 1 + r1 % (uint64_t)(n - 1 > 0 ? n - 1 : 1);
        while (gcd_u64(stride, (uint64_t)n) != 1) ++stride;
        const uint64_t offset = r2 % (uint64_t)n;
        for (int64_t b = 0; b < steps; ++b, ++k) {
            const double frac = total > 1 ? (double)k / (double)(total - 1) : 1.0;
            const float lr = (float)(cfg->lr_min + 0.5 * (cfg->lr_max - cfg->lr_min) * (1.0 + std::cos(kPi * frac)));
            ++s->adam_step;
            const float bc1 = (float)(1.0 - std::pow((double)cfg->beta1, (double)s->adam_step));
            const float bc2 = (float)(1.0 - std::pow((double)cfg->beta2, (double)s->adam_step));
            FSPB_HIP(fspb::launch_mlp_grad(mlp_view(s), features, targets, n, b * cfg->batch, cfg->batch, stride, offset,
                                           1.0f / (float)cfg->batch, s->partials, st),
                     "launch gradient");
            FSPB_HIP(fspb::launch_mlp_reduce(s->params, s->m1, s->m2, s->w2, s->w2t, s->partials, waves, 1, lr,
                                             cfg->beta1, cfg->beta2, cfg->eps, bc1, bc2,
                                             b == steps - 1 ? s->grad : nullptr, st),
                     "launch Adam");
        }
        float lsum = 0.0f;
        FSPB_HIP(hipMemcpyAsync(&lsum, s->grad + fspb::kMlpParams, sizeof(float), hipMemcpyDeviceToHost, st), "read loss");
        FSPB_HIP(hipStreamSynchronize(st), "synchronise epoch");
        if (loss_per_epoch) loss_per_epoch[e] = lsum / (float)cfg->batch;
    }
    return FSPB_OK;
}

fspb_status fspb_surrogate_get_params(fspb_surrogate *s, float *params, void *stream)
{
    g_last_error.clear();
    if (!s || !params) return fail(FSPB_ERR_INVALID, "invalid arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    FSPB_HIP(hipMemcpyAsync(params, s->params, sizeof(float) * fspb::kMlpParams, hipMemcpyDeviceToHost, st), "read parameters");
    FSPB_HIP(hipStreamSynchronize(st), "synchronise parameters");
    return FSPB_OK;
}

fspb_status fspb_surrogate_set_params(fspb_surrogate *s, const float *params)
{
    g_last_error.clear();
    if (!s || !params) return fail(FSPB_ERR_INVALID, "invalid arguments");
    for (int i = 0; i < fspb::kMlpParams; ++i)
        if (!std::isfinite(params[i])) return fail(FSPB_ERR_INVALID, "params[%d] is not finite", i);
    FSPB_HIP(hipMemcpy(s->params, params, sizeof(float) * fspb::kMlpParams, hipMemcpyHostToDevice), "upload parameters");
    FSPB_HIP(fspb::launch_mlp_bf16_copies(s->params, s->w2, s->w2t, nullptr), "launch bf16 copies");
    FSPB_HIP(hipDeviceSynchronize(), "synchronise parameters");
    return FSPB_OK;
}

fspb_status fspb_plan_set_surrogate(fspb_plan *p, const fspb_surrogate *s)
{
    g_last_error.clear();
    if (!p) return fail(FSPB_ERR_INVALID, "plan is NULL");
    if (s && p->h.gen)
        return fail(FSPB_ERR_INVALID, "the surrogate models the analytic kernel; this plan uses kernel tables");
    if (s && p->batches > 0)
        return fail(FSPB_ERR_INVALID, "the plan belongs to %d batch(es), which compute Eq. 2-3 analytically", p->batches);
    if (s) {
        bool same = s->n_terms == p->n_terms && s->pdd_step == p->pdd_step && s->pdd == p->pdd;
        for (int i = 0; same && i < p->n_terms; ++i)
            same = s->weight[i] == p->weight[i] && s->sigma0[i] == p->sigma0[i] &&
                   s->sigma_slope[i] == p->sigma_slope[i] && s->width_scale[i] == p->width_scale[i];
        if (!same) return fail(FSPB_ERR_INVALID, "the surrogate was built for different kernel parameters");
    }
    p->h.mlp_p = s ? s->params : nullptr;
    p->h.mlp_w2 = s ? s->w2 : nullptr;
    p->h.use_mlp = s ? 1 : 0;
    if (p->upload) {   // not uploaded yet: the record goes with the rest of the image
        std::memcpy(p->upload->host, &p->h, sizeof(PlanDev));
    } else {
        // the upload or a fill may still be in flight on any stream
        FSPB_HIP(hipDeviceSynchronize(), "synchronise before replacing the plan record");
        FSPB_HIP(hipMemcpy(p->d_plan, &p->h, sizeof(PlanDev), hipMemcpyHostToDevice), "upload plan record");
    }
    return FSPB_OK;
}

void fspb_surrogate_destroy(fspb_surrogate *s) { delete s; }

}  // extern "C"

/* ======================================================================
 * Eq. 1: dose of a fluence, and its adjoint
 * ====================================================================== */

extern "C" {

fspb_status fspb_fluence_dose(const int64_t *indptr, const int32_t *indices, const float *values, int32_t n_rows,
                              int32_t n_voxels, const float *w, float *dose, void *stream)
{
    g_last_error.clear();
    if (!indptr || !w || !dose || n_rows < 0 || n_voxels < 1) return fail(FSPB_ERR_INVALID, "invalid arguments");
    FSPB_HIP(fspb::launch_fluence_dose(indptr, indices, values, n_rows, n_voxels, w, dose,
                                       static_cast<hipStream_t>(stream)),
             "launch fluence dose");
    return FSPB_OK;
}

fspb_status fspb_fluence_gradient(const int64_t *indptr, const int32_t *indices, const float *values, int32_t n_rows,
                                  int32_t n_voxels, const float *r, float *g, void *stream)
{
    g_last_error.clear();
    if (!indptr || !r || !g || n_rows < 0 || n_voxels < 1) return fail(FSPB_ERR_INVALID, "invalid arguments");
    FSPB_HIP(fspb::launch_fluence_gradient(indptr, indices, values, n_rows, n_voxels, r, g,
                                           static_cast<hipStream_t>(stream)),
             "launch fluence gradient");
    return FSPB_OK;
}

fspb_status fspb_csr_transpose(const int64_t *indptr, const int32_t *indices, const float *values, int32_t n_rows,
                               int32_t n_voxels, int64_t nnz, int64_t *t_indptr, int32_t *t_indices,
                               float *t_values, void *workspace, size_t workspace_bytes, size_t *workspace_needed,
                               void *stream)
{
    g_last_error.clear();
    if (n_rows < 0 || n_voxels < 1 || nnz < 0) return fail(FSPB_ERR_INVALID, "n_rows, n_voxels or nnz out of range");
    if (nnz >= ((int64_t)1 << 32) - 1) return fail(FSPB_ERR_INVALID, "nnz must be below 2^32");
    const size_t need = fspb::transpose_workspace(nnz, n_voxels, n_rows);
    if (workspace_needed) *workspace_needed = need;
    if (!workspace) return fail(FSPB_ERR_CAPACITY, "workspace query: %zu bytes needed", need);
    if (workspace_bytes < need)
        return fail(FSPB_ERR_CAPACITY, "workspace of %zu bytes; %zu needed", workspace_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(FSPB_ERR_INVALID, "workspace is not 256-byte aligned");
    if (!indptr || !t_indptr) return fail(FSPB_ERR_INVALID, "indptr or t_indptr is NULL");
    if (nnz > 0 && (!indices || !values || !t_indices || !t_values))
        return fail(FSPB_ERR_INVALID, "entry arrays are NULL");
    FSPB_HIP(fspb::launch_transpose(indptr, indices, values, n_rows, n_voxels, nnz, t_indptr, t_indices, t_values,
                                    workspace, static_cast<hipStream_t>(stream)),
             "launch transpose");
    return FSPB_OK;
}

fspb_status fspb_csr_transpose_noalloc(const int64_t *indptr, const int32_t *indices, const float *values,
                                       int32_t n_rows, int32_t n_voxels, int64_t nnz, int64_t *t_indptr,
                                       int32_t *t_indices, float *t_values, void *stream)
{
    g_last_error.clear();
    if (n_rows < 0 || n_voxels < 1 || nnz < 0) return fail(FSPB_ERR_INVALID, "n_rows, n_voxels or nnz out of range");
    if (nnz >= ((int64_t)1 << 32) - 1) return fail(FSPB_ERR_INVALID, "nnz must be below 2^32");
    const size_t need = fspb::transpose_workspace(nnz, n_voxels, n_rows);
    if (need > fspb::kNoAllocScratchBytes)
        return fail(FSPB_ERR_CAPACITY, "transpose needs %zu bytes of scratch; the static scratch holds %zu", need,
                    fspb::kNoAllocScratchBytes);
    if (!indptr || !t_indptr) return fail(FSPB_ERR_INVALID, "indptr or t_indptr is NULL");
    if (nnz > 0 && (!indices || !values || !t_indices || !t_values))
        return fail(FSPB_ERR_INVALID, "entry arrays are NULL");
    void *ws = nullptr;
    FSPB_HIP(fspb::noalloc_scratch_ptr(&ws), "address of the static scratch");
    FSPB_HIP(fspb::launch_transpose(indptr, indices, values, n_rows, n_voxels, nnz, t_indptr, t_indices, t_values, ws,
                                    static_cast<hipStream_t>(stream)),
             "launch transpose");
    return FSPB_OK;
}

fspb_status fspb_voxel_dose(const int64_t *t_indptr, const int32_t *t_indices, const float *t_values,
                            int32_t n_voxels, int32_t n_beamlets, const float *w, float *dose, void *stream)
{
    g_last_error.clear();
    if (!t_indptr || !w || !dose || n_voxels < 1 || n_beamlets < 0) return fail(FSPB_ERR_INVALID, "invalid arguments");
    FSPB_HIP(fspb::launch_voxel_dose(t_indptr, t_indices, t_values, n_voxels, n_beamlets, w, dose,
                                     static_cast<hipStream_t>(stream)),
             "launch voxel dose");
    return FSPB_OK;
}

}  // extern "C"
