/*
 * FSPB dose-deposition coefficients -- plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct reference
 * the HIP library is checked against.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It includes nothing
 * from the library and the library never links or calls it.
 *
 * Method: Gu, Choi, Men, Pan, Majumdar and Jiang, "GPU-based ultra fast dose
 * calculation using a finite pencil beam model" (arXiv:0908.4417).
 *   - Eq. 2: D^p = A(theta, d) F(x', d, z', C), here A = PDD(d) (SAD/t')^2.
 *   - Eq. 3: F = sum_i c1_i/4 [erf + erf]_x' [erf + erf]_z' (Jiang 1998).
 *   - Sec. 2.1 (last paragraph): volume of interest = a co-axial beamlet
 *     six times wider, i.e. half-width 3a at the iso plane by default.
 *   - Sec. 2.2 (radiological depth): Siddon ray trace of the beamlet central
 *     axis from its entry point A to its exit point B of the CT bounding prism,
 *     tabulated at n equally spaced points on AB and read by linear
 *     interpolation at O', the projection of the voxel onto the axis.
 *   - Fig. 1 caption: geometry (S, A, B, O', x', z').
 *   - Sec. 3.2: table element length of half a voxel.
 *   - Fig. 2a / Eq. 4: loop over beamlets, build the table, loop over the
 *     beamlet's VOI voxels.  The oracle follows exactly that structure.
 *
 * Everything is double precision; densities and the depth-dose table are read
 * as float and promoted.  Library routines used: erf, erfc, floor, sqrt, qsort.
 *
 * Parity unpinned: absolute coefficient values against the paper, which prints
 * no D_ij, no fitted kernel parameters and no worked example.  The functions
 * here are pinned instead by closed forms, symmetries, limits and brute force
 * (tests/test_oracle_*.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---------------------------------------------------------------- inputs */

typedef struct {
    int32_t nx, ny, nz, pad_;
    double spacing[3];
    double origin[3];          /* centre of voxel (0,0,0) */
    const float *density;      /* [nz][ny][nx], x fastest */
} ofs_grid;

typedef struct {
    double gantry_deg;
    double iso[3];
    double sad;
    double a, b;               /* beamlet side lengths at the iso plane */
    double u0, v0;             /* centre of beamlet (0,0) on the iso plane */
    int32_t nu, nv;
} ofs_beam;

/*
 * Eq. 2-3 in their general form: c1, c2, c3 of every term tabulated against
 * depth, and A(theta, d) against the beamlet's angle to the broad beam's
 * central axis and depth.  Linear interpolation, held at the last node.
 */
typedef struct {
    int32_t n_depth, n_theta, n_adepth, pad_;
    double depth_step, theta_step, adepth_step;
    const float *c1, *c2, *c3;     /* [n_terms][n_depth] */
    const float *A;                /* [n_theta][n_adepth] */
} ofs_tables;

typedef struct {
    int32_t n_terms, n_pdd;
    double weight[4];          /* c1 of Eq. 3 */
    double sigma0[4];          /* c3(d) = sigma0 + sigma_slope d */
    double sigma_slope[4];
    double width_scale[4];     /* c2 of Eq. 3 */
    const float *pdd;          /* depth dose, node k at depth k*pdd_step */
    double pdd_step;
    double cutoff_u, cutoff_v; /* VOI half-widths at iso; <= 0 means 3a, 3b */
    double table_step;         /* nominal table element; <= 0 means half the smallest spacing */
    double rho_min;            /* voxels with density <= rho_min are not in any VOI */
    int32_t depth_mode;        /* 0: exact path integral (Siddon); 1: trilinear samples + trapezoid */
    int32_t pad_;
    const ofs_tables *tables;  /* NULL: c1, c2 constant, c3 linear in d, A = PDD(d) */
} ofs_kernel;

/* One beamlet: pencil-beam frame of Fig. 1b plus its depth-table layout. */
typedef struct {
    int32_t beam, iu, iv, n;   /* n = number of table points; 0 if the axis misses the grid */
    double S[3];               /* source */
    double e[3];               /* unit central axis, S towards the beamlet centre */
    double eu[3], ev[3];       /* unit lateral axes (x', z' directions) */
    double tA, tB;             /* distances from S to A and to B */
    double step;               /* spacing of the table points on AB */
    double sad, a, b, cu, cv;
    int32_t depth_mode;        /* copied from the kernel: how the depth table is built */
    int32_t pad_;
    double theta;              /* angle between this axis and the broad beam's central axis */
} ofs_beamlet;

/* ------------------------------------------------------------ small vecs */

static double dot3(const double *p, const double *q) { return p[0]*q[0] + p[1]*q[1] + p[2]*q[2]; }

static void normalise3(double *p)
{
    double r = sqrt(dot3(p, p));
    p[0] /= r; p[1] /= r; p[2] /= r;
}

static double grid_lo(const ofs_grid *g, int k) { return g->origin[k] - 0.5 * g->spacing[k]; }
static int grid_n(const ofs_grid *g, int k) { return k == 0 ? g->nx : (k == 1 ? g->ny : g->nz); }
static double grid_hi(const ofs_grid *g, int k) { return grid_lo(g, k) + grid_n(g, k) * g->spacing[k]; }

static double density_at(const ofs_grid *g, int ix, int iy, int iz)
{
    return (double)g->density[((int64_t)iz * g->ny + iy) * g->nx + ix];
}

/* ------------------------------------------------------------- geometry */

int32_t ofs_count_beamlets(const ofs_beam *beams, int32_t n_beams)
{
    int32_t n = 0;
    for (int32_t b = 0; b < n_beams; ++b) n += beams[b].nu * beams[b].nv;
    return n;
}

/*
 * Entry and exit of the ray S + t e through the grid's bounding prism
 * (Fig. 1 caption: A and B).  Slab method; returns 0 if the ray misses.
 */
static int clip_to_grid(const ofs_grid *g, const double *S, const double *e, double *tA, double *tB)
{
    double t0 = 0.0, t1 = INFINITY;
    for (int k = 0; k < 3; ++k) {
        double lo = grid_lo(g, k), hi = grid_hi(g, k);
        if (e[k] == 0.0) {
            if (S[k] < lo || S[k] >= hi) return 0;
            continue;
        }
        double ta = (lo - S[k]) / e[k], tb = (hi - S[k]) / e[k];
        if (ta > tb) { double s = ta; ta = tb; tb = s; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    if (!(t1 > t0)) return 0;
    *tA = t0; *tB = t1;
    return 1;
}

/*
 * Beamlet frames.  Coordinates: gantry rotates about the patient z axis;
 * at gantry g the source sits at iso + SAD (sin g, -cos g, 0), the beam's
 * lateral axes are eu = (cos g, sin g, 0) and ev = (0, 0, 1).  Beamlet
 * (iu, iv) is centred at iso + (u0 + iu a) eu + (v0 + iv b) ev on the iso
 * plane; its axis runs from S through that centre.  The pencil-beam lateral
 * axes (Fig. 1b, x' and z') are eu made perpendicular to the axis, and their
 * cross product.  Rows are numbered beam by beam, iv major, iu minor.
 */
int32_t ofs_geometry(const ofs_grid *g, const ofs_beam *beams, int32_t n_beams,
                     const ofs_kernel *K, ofs_beamlet *out)
{
    double minsp = fmin(g->spacing[0], fmin(g->spacing[1], g->spacing[2]));
    double nominal = K->table_step > 0.0 ? K->table_step : 0.5 * minsp;
    int32_t j = 0;
    for (int32_t bi = 0; bi < n_beams; ++bi) {
        const ofs_beam *bm = &beams[bi];
        double gr = bm->gantry_deg * M_PI / 180.0;
        double S[3] = { bm->iso[0] + bm->sad * sin(gr), bm->iso[1] - bm->sad * cos(gr), bm->iso[2] };
        double beu[3] = { cos(gr), sin(gr), 0.0 };
        double bev[3] = { 0.0, 0.0, 1.0 };
        for (int32_t iv = 0; iv < bm->nv; ++iv) {
            for (int32_t iu = 0; iu < bm->nu; ++iu, ++j) {
                ofs_beamlet *bl = &out[j];
                memset(bl, 0, sizeof *bl);
                bl->beam = bi; bl->iu = iu; bl->iv = iv;
                bl->sad = bm->sad; bl->a = bm->a; bl->b = bm->b;
                bl->cu = K->cutoff_u > 0.0 ? K->cutoff_u : 3.0 * bm->a;
                bl->cv = K->cutoff_v > 0.0 ? K->cutoff_v : 3.0 * bm->b;
                double cu = bm->u0 + iu * bm->a, cv = bm->v0 + iv * bm->b;
                double Q[3];
                for (int k = 0; k < 3; ++k) {
                    Q[k] = bm->iso[k] + cu * beu[k] + cv * bev[k];
                    bl->S[k] = S[k];
                    bl->e[k] = Q[k] - S[k];
                }
                normalise3(bl->e);
                {
                    /* Fig. 1a: theta is the angle between SS' (S towards the isocentre) and the beamlet axis */
                    double c0[3] = { bm->iso[0] - S[0], bm->iso[1] - S[1], bm->iso[2] - S[2] };
                    normalise3(c0);
                    double ct = dot3(c0, bl->e);
                    bl->theta = acos(ct > 1.0 ? 1.0 : (ct < -1.0 ? -1.0 : ct));
                }
                double pr = dot3(beu, bl->e);
                for (int k = 0; k < 3; ++k) bl->eu[k] = beu[k] - pr * bl->e[k];
                normalise3(bl->eu);
                /* ev' = eu' x e (right-handed with ev at the beam centre) */
                bl->ev[0] = bl->eu[1] * bl->e[2] - bl->eu[2] * bl->e[1];
                bl->ev[1] = bl->eu[2] * bl->e[0] - bl->eu[0] * bl->e[2];
                bl->ev[2] = bl->eu[0] * bl->e[1] - bl->eu[1] * bl->e[0];
                double tA, tB;
                bl->depth_mode = K->depth_mode;
                if (!clip_to_grid(g, bl->S, bl->e, &tA, &tB)) { bl->n = 0; continue; }
                bl->tA = tA; bl->tB = tB;
                /* n equally spaced points on AB, both ends included, no further
                 * apart than the nominal element length (a ratio within 1e-9 of
                 * an integer counts as that integer, so |AB| = k * nominal gives
                 * exactly k elements despite rounding in tA and tB) */
                double L = tB - tA;
                int32_t segs = (int32_t)ceil(L / nominal - 1e-9);
                if (segs < 1) segs = 1;
                bl->n = segs + 1;
                bl->step = L / segs;
            }
        }
    }
    return j;
}

/* ---------------------------------------------------------------- Siddon */

static int cmp_double(const void *p, const void *q)
{
    double a = *(const double *)p, b = *(const double *)q;
    return (a > b) - (a < b);
}

/*
 * Siddon (1985), original form: every parametric crossing of the ray with a
 * voxel-boundary plane strictly inside (tA, tB) is collected, merged with tA
 * and tB by sorting, and each gap of positive length is one segment.  A
 * segment belongs to the voxel that contains its midpoint (voxels are
 * half-open).  Writes up to ``cap`` segments; returns the segment count.
 */
int32_t ofs_siddon(const ofs_grid *g, const double *S, const double *e, double tA, double tB,
                   int64_t *vox, double *len, int32_t cap)
{
    int32_t nplanes = g->nx + g->ny + g->nz + 3;
    double *al = (double *)malloc(sizeof(double) * (size_t)(nplanes + 2));
    int32_t na = 0;
    al[na++] = tA;
    al[na++] = tB;
    for (int k = 0; k < 3; ++k) {
        if (e[k] == 0.0) continue;
        for (int p = 0; p <= grid_n(g, k); ++p) {
            double a = (grid_lo(g, k) + p * g->spacing[k] - S[k]) / e[k];
            if (a > tA && a < tB) al[na++] = a;
        }
    }
    qsort(al, (size_t)na, sizeof(double), cmp_double);
    int32_t nseg = 0;
    for (int32_t i = 0; i + 1 < na; ++i) {
        double a0 = al[i], a1 = al[i + 1];
        if (!(a1 > a0)) continue;
        double mid = 0.5 * (a0 + a1);
        int idx[3];
        for (int k = 0; k < 3; ++k) {
            double c = S[k] + mid * e[k];
            int v = (int)floor((c - grid_lo(g, k)) / g->spacing[k]);
            if (v < 0) v = 0;
            if (v > grid_n(g, k) - 1) v = grid_n(g, k) - 1;
            idx[k] = v;
        }
        if (nseg < cap) {
            vox[nseg] = ((int64_t)idx[2] * g->ny + idx[1]) * g->nx + idx[0];
            len[nseg] = a1 - a0;
        }
        ++nseg;
    }
    free(al);
    return nseg;
}

/* Segment list of one beamlet axis with start parameters and densities. */
typedef struct { int32_t n; double *t0; double *len; double *rho; } seglist;

static void trace_axis(const ofs_grid *g, const ofs_beamlet *bl, seglist *sl)
{
    int32_t cap = g->nx + g->ny + g->nz + 4;
    int64_t *vox = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    sl->len = (double *)malloc(sizeof(double) * (size_t)cap);
    sl->t0 = (double *)malloc(sizeof(double) * (size_t)cap);
    sl->rho = (double *)malloc(sizeof(double) * (size_t)cap);
    sl->n = ofs_siddon(g, bl->S, bl->e, bl->tA, bl->tB, vox, sl->len, cap);
    double t = bl->tA;
    for (int32_t s = 0; s < sl->n; ++s) {
        /* segments are contiguous and in order: each starts where the last ended */
        sl->t0[s] = t;
        t += sl->len[s];
        sl->rho[s] = (double)g->density[vox[s]];
    }
    free(vox);
}

static void free_segs(seglist *sl) { free(sl->t0); free(sl->len); free(sl->rho); }

/*
 * Radiological depth table (Sec. 2.2): R at n equally spaced points of AB,
 * R(t) = integral of density from A to S + t e, piecewise linear in t.
 * Returns n.
 */
/*
 * Density at point p from the voxel-centre values by trilinear interpolation
 * (the sampling Sec. 2.2 uses to build the depth table).  Along each axis the
 * position is held at the first / last centre plane, so the half voxel
 * between a centre plane and the box face takes the boundary voxels' values.
 */
double ofs_trilinear_density(const ofs_grid *g, const double p[3])
{
    int i0[3], i1[3];
    double f[3];
    for (int k = 0; k < 3; ++k) {
        int n = grid_n(g, k);
        double c = (p[k] - g->origin[k]) / g->spacing[k];
        if (c < 0.0) c = 0.0;
        if (c > n - 1) c = n - 1;
        int lo = (int)floor(c);
        if (lo > n - 2) lo = n - 2;
        if (lo < 0) lo = 0;
        i0[k] = lo;
        i1[k] = n > 1 ? lo + 1 : lo;
        f[k] = n > 1 ? c - lo : 0.0;
    }
    double r = 0.0;
    for (int corner = 0; corner < 8; ++corner) {
        int ix = (corner & 1) ? i1[0] : i0[0];
        int iy = (corner & 2) ? i1[1] : i0[1];
        int iz = (corner & 4) ? i1[2] : i0[2];
        double w = ((corner & 1) ? f[0] : 1.0 - f[0]) * ((corner & 2) ? f[1] : 1.0 - f[1]) *
                   ((corner & 4) ? f[2] : 1.0 - f[2]);
        r += w * g->density[((int64_t)iz * g->ny + iy) * g->nx + ix];
    }
    return r;
}

/*
 * Depth table of Sec. 2.2 as the paper builds it: the density is sampled by
 * trilinear interpolation at the n table points on AB and the depth from A
 * to point k is the trapezoid sum of the samples over the elements before it.
 */
static void depth_table_trilinear(const ofs_grid *g, const ofs_beamlet *bl, double *table)
{
    double prev_rho = 0.0, prev_t = bl->tA;
    for (int32_t k = 0; k < bl->n; ++k) {
        double t = (k == bl->n - 1) ? bl->tB : bl->tA + k * bl->step;
        double p[3] = { bl->S[0] + t * bl->e[0], bl->S[1] + t * bl->e[1], bl->S[2] + t * bl->e[2] };
        double rho = ofs_trilinear_density(g, p);
        table[k] = k == 0 ? 0.0 : table[k - 1] + 0.5 * (t - prev_t) * (prev_rho + rho);
        prev_rho = rho;
        prev_t = t;
    }
}

int32_t ofs_depth_table(const ofs_grid *g, const ofs_beamlet *bl, double *table)
{
    if (bl->n == 0) return 0;
    if (bl->depth_mode == 1) {
        depth_table_trilinear(g, bl, table);
        return bl->n;
    }
    seglist sl;
    trace_axis(g, bl, &sl);
    int32_t s = 0;
    double acc = 0.0;                    /* R at the start of segment s */
    for (int32_t k = 0; k < bl->n; ++k) {
        double t = (k == bl->n - 1) ? bl->tB : bl->tA + k * bl->step;
        while (s < sl.n && sl.t0[s] + sl.len[s] <= t) { acc += sl.rho[s] * sl.len[s]; ++s; }
        double part = (s < sl.n && t > sl.t0[s]) ? sl.rho[s] * (t - sl.t0[s]) : 0.0;
        table[k] = acc + part;
    }
    free_segs(&sl);
    return bl->n;
}

/* Exact radiological depth R(t) from A (no table); a diagnostic. */
double ofs_exact_depth(const ofs_grid *g, const ofs_beamlet *bl, double t)
{
    if (bl->n == 0) return 0.0;
    if (t > bl->tB) t = bl->tB;
    seglist sl;
    trace_axis(g, bl, &sl);
    double r = 0.0;
    for (int32_t s = 0; s < sl.n; ++s) {
        double l = t - sl.t0[s];
        if (l <= 0.0) break;
        r += sl.rho[s] * (l < sl.len[s] ? l : sl.len[s]);
    }
    free_segs(&sl);
    return r;
}

/* ------------------------------------------------------------ the kernel */

/* Depth at a point whose projection on the axis is at distance t from S. */
double ofs_table_depth(const ofs_beamlet *bl, const double *table, double t)
{
    double tau = (t - bl->tA) / bl->step;
    if (tau <= 0.0) return table[0];
    if (tau >= bl->n - 1) return table[bl->n - 1];
    int32_t k = (int32_t)floor(tau);
    double f = tau - k;
    return (1.0 - f) * table[k] + f * table[k + 1];
}

/* Depth dose, linear interpolation in the table, held at the last node. */
/* Linear interpolation of a table of n nodes at x (in node units), held at both ends. */
static double lerp_table(const float *t, int32_t n, double x)
{
    if (x <= 0.0) return (double)t[0];
    if (x >= n - 1) return (double)t[n - 1];
    int32_t k = (int32_t)floor(x);
    double f = x - k;
    return (1.0 - f) * (double)t[k] + f * (double)t[k + 1];
}

/* c_m(d) of term i (m = 1, 2, 3) from the tables. */
double ofs_table_c(const ofs_tables *T, int32_t m, int32_t i, double d)
{
    const float *base = m == 1 ? T->c1 : (m == 2 ? T->c2 : T->c3);
    return lerp_table(base + (int64_t)i * T->n_depth, T->n_depth, d / T->depth_step);
}

/* A(theta, d): linear in theta between rows, each row linear in d. */
double ofs_table_A(const ofs_tables *T, double theta, double d)
{
    double y = T->n_theta > 1 ? theta / T->theta_step : 0.0;
    if (y <= 0.0 || T->n_theta == 1) return lerp_table(T->A, T->n_adepth, d / T->adepth_step);
    if (y >= T->n_theta - 1)
        return lerp_table(T->A + (int64_t)(T->n_theta - 1) * T->n_adepth, T->n_adepth, d / T->adepth_step);
    int32_t k = (int32_t)floor(y);
    double f = y - k;
    return (1.0 - f) * lerp_table(T->A + (int64_t)k * T->n_adepth, T->n_adepth, d / T->adepth_step) +
           f * lerp_table(T->A + (int64_t)(k + 1) * T->n_adepth, T->n_adepth, d / T->adepth_step);
}

double ofs_pdd(const ofs_kernel *K, double d)
{
    double x = d / K->pdd_step;
    if (x <= 0.0) return (double)K->pdd[0];
    if (x >= K->n_pdd - 1) return (double)K->pdd[K->n_pdd - 1];
    int32_t k = (int32_t)floor(x);
    double f = x - k;
    return (1.0 - f) * (double)K->pdd[k] + f * (double)K->pdd[k + 1];
}

/*
 * One bracket of Eq. 3: erf((w/2 - x)/(sqrt2 s)) + erf((w/2 + x)/(sqrt2 s)).
 * Outside the beamlet edge the same quantity is written as a difference of
 * erfc so that the tail keeps its relative accuracy.
 */
double ofs_edge_pair(double x, double w, double s)
{
    double r = sqrt(2.0) * s, h = 0.5 * w, ax = fabs(x);
    if (ax <= h) return erf((h - ax) / r) + erf((h + ax) / r);
    return erfc((ax - h) / r) - erfc((ax + h) / r);
}

/* Lateral profile F of Eq. 3 at iso-plane offsets (u, v), depth d. */
double ofs_lateral(const ofs_kernel *K, double u, double v, double a, double b, double d)
{
    double sum = 0.0;
    for (int32_t i = 0; i < K->n_terms; ++i) {
        double c1, c2, c3;
        if (K->tables) {
            c1 = ofs_table_c(K->tables, 1, i, d);
            c2 = ofs_table_c(K->tables, 2, i, d);
            c3 = ofs_table_c(K->tables, 3, i, d);
        } else {
            c1 = K->weight[i];
            c2 = K->width_scale[i];
            c3 = K->sigma0[i] + K->sigma_slope[i] * d;
        }
        sum += 0.25 * c1 * ofs_edge_pair(u, c2 * a, c3) * ofs_edge_pair(v, c2 * b, c3);
    }
    return sum;
}

/* Eq. 2 with A = PDD(d) (SAD/t')^2, or A(theta, d) (SAD/t')^2 from the tables. */
double ofs_dose(const ofs_kernel *K, const ofs_beamlet *bl, double d, double tp, double u, double v)
{
    double m = bl->sad / tp;
    double A = K->tables ? ofs_table_A(K->tables, bl->theta, d) : ofs_pdd(K, d);
    return A * m * m * ofs_lateral(K, u, v, bl->a, bl->b, d);
}

/* The learned surrogate's target: PDD(d) F(u, v; a, a, d). */
double ofs_kernel_value(const ofs_kernel *K, double d, double u, double v, double a)
{
    return ofs_pdd(K, d) * ofs_lateral(K, u, v, a, a, d);
}

/* ofs_kernel_value at n points pts[n][4] = (d, u, v, a). */
void ofs_kernel_values(const ofs_kernel *K, const double *pts, int64_t n, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = ofs_kernel_value(K, pts[4 * i], pts[4 * i + 1], pts[4 * i + 2], pts[4 * i + 3]);
}

/*
 * VOI membership of the voxel centre P (Sec. 2.1, last paragraph): with
 * w = P - S, t' = w.e, u = (w.eu) SAD / t', v = (w.ev) SAD / t', the voxel
 * belongs iff t' > 0, |u| <= cu, |v| <= cv and its density exceeds rho_min.
 */
int32_t ofs_voi_member(const ofs_grid *g, const ofs_kernel *K, const ofs_beamlet *bl,
                       int32_t ix, int32_t iy, int32_t iz, double *tp, double *u, double *v)
{
    double P[3] = { g->origin[0] + ix * g->spacing[0], g->origin[1] + iy * g->spacing[1],
                    g->origin[2] + iz * g->spacing[2] };
    double w[3] = { P[0] - bl->S[0], P[1] - bl->S[1], P[2] - bl->S[2] };
    double t = dot3(w, bl->e);
    if (!(t > 0.0)) return 0;
    double uu = dot3(w, bl->eu) * bl->sad / t;
    double vv = dot3(w, bl->ev) * bl->sad / t;
    if (tp) *tp = t;
    if (u) *u = uu;
    if (v) *v = vv;
    if (fabs(uu) > bl->cu || fabs(vv) > bl->cv) return 0;
    if (!(density_at(g, ix, iy, iz) > K->rho_min)) return 0;
    return 1;
}

/*
 * Candidate range of ix on the grid row (iy, iz).  Every member satisfies
 * |w.eu| SAD <= cu t' and |w.ev| SAD <= cv t', which are linear in ix; the
 * real solution interval is widened by two voxels and every candidate is then
 * tested with ofs_voi_member itself.  Returns 0 if the row has no candidate.
 */
static int row_candidates(const ofs_grid *g, const ofs_beamlet *bl, int32_t iy, int32_t iz,
                          int32_t *lo, int32_t *hi)
{
    double w0[3] = { g->origin[0] - bl->S[0], g->origin[1] + iy * g->spacing[1] - bl->S[1],
                     g->origin[2] + iz * g->spacing[2] - bl->S[2] };
    double t0 = dot3(w0, bl->e), t1 = g->spacing[0] * bl->e[0];
    double U0 = dot3(w0, bl->eu), U1 = g->spacing[0] * bl->eu[0];
    double V0 = dot3(w0, bl->ev), V1 = g->spacing[0] * bl->ev[0];
    double c0[4] = { bl->sad * U0 - bl->cu * t0, -bl->sad * U0 - bl->cu * t0,
                     bl->sad * V0 - bl->cv * t0, -bl->sad * V0 - bl->cv * t0 };
    double c1[4] = { bl->sad * U1 - bl->cu * t1, -bl->sad * U1 - bl->cu * t1,
                     bl->sad * V1 - bl->cv * t1, -bl->sad * V1 - bl->cv * t1 };
    double xlo = -INFINITY, xhi = INFINITY;
    for (int c = 0; c < 4; ++c) {           /* c0 + c1 x <= 0 */
        if (c1[c] > 0.0) xhi = fmin(xhi, -c0[c] / c1[c]);
        else if (c1[c] < 0.0) xlo = fmax(xlo, -c0[c] / c1[c]);
        else if (c0[c] > 0.0) return 0;
    }
    if (xlo > xhi) return 0;
    double a = fmax(xlo, -4.0) , b = fmin(xhi, g->nx + 4.0);
    int32_t l = (int32_t)ceil(a) - 2, h = (int32_t)floor(b) + 2;
    if (l < 0) l = 0;
    if (h > g->nx - 1) h = g->nx - 1;
    if (l > h) return 0;
    *lo = l; *hi = h;
    return 1;
}

/*
 * One row of D_ij (Fig. 2a inner loop): every VOI voxel of beamlet ``bl`` in
 * ascending linear index (iz ny + iy) nx + ix, with its coefficient.  If
 * ``idx`` is NULL only the count is returned; otherwise up to ``cap`` entries
 * are written.  ``table`` is the beamlet's depth table.
 */
int64_t ofs_beamlet_row(const ofs_grid *g, const ofs_kernel *K, const ofs_beamlet *bl,
                        const double *table, int32_t *idx, double *val, int64_t cap)
{
    if (bl->n == 0) return 0;
    int64_t count = 0;
    for (int32_t iz = 0; iz < g->nz; ++iz) {
        for (int32_t iy = 0; iy < g->ny; ++iy) {
            int32_t lo, hi;
            if (!row_candidates(g, bl, iy, iz, &lo, &hi)) continue;
            for (int32_t ix = lo; ix <= hi; ++ix) {
                double tp, u, v;
                if (!ofs_voi_member(g, K, bl, ix, iy, iz, &tp, &u, &v)) continue;
                if (idx && count < cap) {
                    double d = ofs_table_depth(bl, table, tp);
                    idx[count] = (int32_t)(((int64_t)iz * g->ny + iy) * g->nx + ix);
                    val[count] = ofs_dose(K, bl, d, tp, u, v);
                }
                ++count;
            }
        }
    }
    return count;
}

/* Brute force over every voxel of the grid; the enumerator's pin. */
int64_t ofs_beamlet_row_bruteforce(const ofs_grid *g, const ofs_kernel *K, const ofs_beamlet *bl,
                                   int32_t *idx, int64_t cap)
{
    if (bl->n == 0) return 0;
    int64_t count = 0;
    for (int32_t iz = 0; iz < g->nz; ++iz)
        for (int32_t iy = 0; iy < g->ny; ++iy)
            for (int32_t ix = 0; ix < g->nx; ++ix) {
                if (!ofs_voi_member(g, K, bl, ix, iy, iz, NULL, NULL, NULL)) continue;
                if (idx && count < cap) idx[count] = (int32_t)(((int64_t)iz * g->ny + iy) * g->nx + ix);
                ++count;
            }
    return count;
}

/* ---------------------------------------------------------- plan drivers */

void ofs_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int32_t ofs_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Depth tables of every beamlet, concatenated; table_off has N_b + 1 entries. */
int32_t ofs_plan_tables(const ofs_grid *g, const ofs_beam *beams, int32_t n_beams, const ofs_kernel *K,
                        double *tables, int64_t *table_off)
{
    int32_t nb = ofs_count_beamlets(beams, n_beams);
    ofs_beamlet *bl = (ofs_beamlet *)malloc(sizeof(ofs_beamlet) * (size_t)nb);
    ofs_geometry(g, beams, n_beams, K, bl);
    table_off[0] = 0;
    for (int32_t j = 0; j < nb; ++j) table_off[j + 1] = table_off[j] + bl[j].n;
    if (tables) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int32_t j = 0; j < nb; ++j) ofs_depth_table(g, &bl[j], tables + table_off[j]);
    }
    free(bl);
    return nb;
}

/* Nonzeros of each beamlet row. */
int32_t ofs_plan_counts(const ofs_grid *g, const ofs_beam *beams, int32_t n_beams, const ofs_kernel *K,
                        int64_t *counts)
{
    int32_t nb = ofs_count_beamlets(beams, n_beams);
    ofs_beamlet *bl = (ofs_beamlet *)malloc(sizeof(ofs_beamlet) * (size_t)nb);
    ofs_geometry(g, beams, n_beams, K, bl);
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t j = 0; j < nb; ++j) counts[j] = ofs_beamlet_row(g, K, &bl[j], NULL, NULL, NULL, 0);
    free(bl);
    return nb;
}

/* Nonzeros of the selected beamlet rows sel[0..nsel). */
int32_t ofs_plan_counts_sel(const ofs_grid *g, const ofs_beam *beams, int32_t n_beams, const ofs_kernel *K,
                            const int32_t *sel, int32_t nsel, int64_t *counts)
{
    int32_t nb = ofs_count_beamlets(beams, n_beams);
    ofs_beamlet *bl = (ofs_beamlet *)malloc(sizeof(ofs_beamlet) * (size_t)nb);
    ofs_geometry(g, beams, n_beams, K, bl);
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t s = 0; s < nsel; ++s) counts[s] = ofs_beamlet_row(g, K, &bl[sel[s]], NULL, NULL, NULL, 0);
    free(bl);
    return nsel;
}

/*
 * Rows of the selected beamlets (sel[0..nsel)), row sel[s] written at
 * idx/val + off[s]; off has nsel + 1 entries and must come from the counts.
 * Returns 0, or -1 if a row's length disagrees with off.
 */
int32_t ofs_plan_rows(const ofs_grid *g, const ofs_beam *beams, int32_t n_beams, const ofs_kernel *K,
                      const int32_t *sel, int32_t nsel, const int64_t *off, int32_t *idx, double *val)
{
    int32_t nb = ofs_count_beamlets(beams, n_beams);
    ofs_beamlet *bl = (ofs_beamlet *)malloc(sizeof(ofs_beamlet) * (size_t)nb);
    ofs_geometry(g, beams, n_beams, K, bl);
    int32_t bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int32_t s = 0; s < nsel; ++s) {
        const ofs_beamlet *b = &bl[sel[s]];
        double *table = (double *)malloc(sizeof(double) * (size_t)(b->n > 0 ? b->n : 1));
        ofs_depth_table(g, b, table);
        int64_t cap = off[s + 1] - off[s];
        int64_t got = ofs_beamlet_row(g, K, b, table, idx + off[s], val + off[s], cap);
        if (got != cap) bad |= 1;
        free(table);
    }
    free(bl);
    return bad ? -1 : 0;
}

/*
 * Dose of a fluence (Eq. 1): dose[i] = sum_j w[j] D_ij over every beamlet row,
 * and the adjoint g[j] = sum_i D_ij r[i] (g or r may be NULL to skip it).
 * dose is overwritten.  Rows are computed independently and added under an
 * atomic update per voxel.
 */
int32_t ofs_plan_fluence(const ofs_grid *g, const ofs_beam *beams, int32_t n_beams, const ofs_kernel *K,
                         const double *w, double *dose, const double *r, double *grad)
{
    int32_t nb = ofs_count_beamlets(beams, n_beams);
    ofs_beamlet *bl = (ofs_beamlet *)malloc(sizeof(ofs_beamlet) * (size_t)nb);
    ofs_geometry(g, beams, n_beams, K, bl);
    int64_t nvox = (int64_t)g->nx * g->ny * g->nz;
    if (dose) memset(dose, 0, sizeof(double) * (size_t)nvox);
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t j = 0; j < nb; ++j) {
        const ofs_beamlet *b = &bl[j];
        double *table = (double *)malloc(sizeof(double) * (size_t)(b->n > 0 ? b->n : 1));
        ofs_depth_table(g, b, table);
        int64_t n = ofs_beamlet_row(g, K, b, table, NULL, NULL, 0);
        int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        double *val = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        ofs_beamlet_row(g, K, b, table, idx, val, n);
        double acc = 0.0;
        for (int64_t e = 0; e < n; ++e) {
            if (dose && w) {
#pragma omp atomic
                dose[idx[e]] += w[j] * val[e];
            }
            if (r) acc += val[e] * r[idx[e]];
        }
        if (grad) grad[j] = acc;
        free(idx);
        free(val);
        free(table);
    }
    free(bl);
    return nb;
}
