"""FP64 CPU oracle for the FSPB dose-coefficient path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never imports it and it
imports nothing from the library; both consume the seeded inputs of
``fspb_inputs`` and nothing else in common.

The C sources (``fspb_oracle.c``, ``mlp_oracle.c``) hold the arithmetic; this
module only marshals numpy arrays through ctypes.  ``build()`` compiles them
with gcc (IEEE semantics: no fast-math, no FMA contraction).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["fspb_oracle.c", "mlp_oracle.c"]

MLP_HIDDEN = 64
MLP_NPARAM = 4545


def build(verbose: bool = False) -> str:
    """Compile the oracle shared library in place (gcc, OpenMP, -O2)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", _LIB_PATH + ".tmp"] + srcs + ["-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + r.stderr)
    if verbose and r.stderr:
        print(r.stderr)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class OGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pad_", C.c_int32),
                ("spacing", C.c_double * 3), ("origin", C.c_double * 3),
                ("density", C.POINTER(C.c_float))]


class OBeam(C.Structure):
    _fields_ = [("gantry_deg", C.c_double), ("iso", C.c_double * 3), ("sad", C.c_double),
                ("a", C.c_double), ("b", C.c_double), ("u0", C.c_double), ("v0", C.c_double),
                ("nu", C.c_int32), ("nv", C.c_int32)]


# how the radiological-depth table is built (Sec. 2.2): the exact path
# integral through the voxels, or trilinear samples summed by trapezoids
DEPTH_MODES = {"siddon": 0, "trilinear": 1}


class OTables(C.Structure):
    _fields_ = [("n_depth", C.c_int32), ("n_theta", C.c_int32), ("n_adepth", C.c_int32), ("pad_", C.c_int32),
                ("depth_step", C.c_double), ("theta_step", C.c_double), ("adepth_step", C.c_double),
                ("c1", C.POINTER(C.c_float)), ("c2", C.POINTER(C.c_float)), ("c3", C.POINTER(C.c_float)),
                ("A", C.POINTER(C.c_float))]


class OKernel(C.Structure):
    _fields_ = [("n_terms", C.c_int32), ("n_pdd", C.c_int32),
                ("weight", C.c_double * 4), ("sigma0", C.c_double * 4),
                ("sigma_slope", C.c_double * 4), ("width_scale", C.c_double * 4),
                ("pdd", C.POINTER(C.c_float)), ("pdd_step", C.c_double),
                ("cutoff_u", C.c_double), ("cutoff_v", C.c_double),
                ("table_step", C.c_double), ("rho_min", C.c_double),
                ("depth_mode", C.c_int32), ("pad_", C.c_int32), ("tables", C.POINTER(OTables))]


class OBeamlet(C.Structure):
    _fields_ = [("beam", C.c_int32), ("iu", C.c_int32), ("iv", C.c_int32), ("n", C.c_int32),
                ("S", C.c_double * 3), ("e", C.c_double * 3), ("eu", C.c_double * 3),
                ("ev", C.c_double * 3), ("tA", C.c_double), ("tB", C.c_double),
                ("step", C.c_double), ("sad", C.c_double), ("a", C.c_double), ("b", C.c_double),
                ("cu", C.c_double), ("cv", C.c_double),
                ("depth_mode", C.c_int32), ("pad_", C.c_int32), ("theta", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER
        d, i32, i64 = C.c_double, C.c_int32, C.c_int64
        sig = {
            "ofs_count_beamlets": (i32, [P(OBeam), i32]),
            "ofs_geometry": (i32, [P(OGrid), P(OBeam), i32, P(OKernel), P(OBeamlet)]),
            "ofs_siddon": (i32, [P(OGrid), P(d), P(d), d, d, P(i64), P(d), i32]),
            "ofs_depth_table": (i32, [P(OGrid), P(OBeamlet), P(d)]),
            "ofs_exact_depth": (d, [P(OGrid), P(OBeamlet), d]),
            "ofs_trilinear_density": (d, [P(OGrid), P(d)]),
            "ofs_table_depth": (d, [P(OBeamlet), P(d), d]),
            "ofs_pdd": (d, [P(OKernel), d]),
            "ofs_edge_pair": (d, [d, d, d]),
            "ofs_lateral": (d, [P(OKernel), d, d, d, d, d]),
            "ofs_dose": (d, [P(OKernel), P(OBeamlet), d, d, d, d]),
            "ofs_kernel_value": (d, [P(OKernel), d, d, d, d]),
            "ofs_kernel_values": (None, [P(OKernel), P(d), i64, P(d)]),
            "ofs_voi_member": (i32, [P(OGrid), P(OKernel), P(OBeamlet), i32, i32, i32,
                                     P(d), P(d), P(d)]),
            "ofs_beamlet_row": (i64, [P(OGrid), P(OKernel), P(OBeamlet), P(d), P(C.c_int32),
                                      P(d), i64]),
            "ofs_beamlet_row_bruteforce": (i64, [P(OGrid), P(OKernel), P(OBeamlet),
                                                 P(C.c_int32), i64]),
            "ofs_set_threads": (None, [i32]),
            "ofs_max_threads": (i32, []),
            "ofs_plan_tables": (i32, [P(OGrid), P(OBeam), i32, P(OKernel), P(d), P(i64)]),
            "ofs_plan_counts": (i32, [P(OGrid), P(OBeam), i32, P(OKernel), P(i64)]),
            "ofs_plan_counts_sel": (i32, [P(OGrid), P(OBeam), i32, P(OKernel), P(i32), i32, P(i64)]),
            "ofs_plan_fluence": (i32, [P(OGrid), P(OBeam), i32, P(OKernel), P(d), P(d), P(d), P(d)]),
            "ofs_plan_rows": (i32, [P(OGrid), P(OBeam), i32, P(OKernel), P(i32), i32, P(i64),
                                    P(i32), P(d)]),
            "ofs_mlp_nparams": (i32, []),
            "ofs_bf16_round": (d, [d]),
            "ofs_surrogate_features": (None, [P(d), i64, P(d)]),
            "ofs_mlp_forward": (None, [P(d), P(d), i64, P(d), i32]),
            "ofs_mlp_loss_grad": (d, [P(d), P(d), P(d), i64, P(d), i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class OraclePlan:
    """Marshalled inputs of one problem (a ``fspb_inputs.Problem``)."""

    def __init__(self, problem):
        g = problem.grid
        self.density = np.ascontiguousarray(g.density, dtype=np.float32)
        nz, ny, nx = self.density.shape
        self.grid = OGrid(nx, ny, nz, 0, (C.c_double * 3)(*g.spacing), (C.c_double * 3)(*g.origin),
                          _ptr(self.density, C.c_float))
        self.beams = (OBeam * len(problem.beams))()
        for k, b in enumerate(problem.beams):
            self.beams[k] = OBeam(b.gantry_deg, (C.c_double * 3)(*b.isocenter), b.sad, b.beamlet_a,
                                  b.beamlet_b, b.u0, b.v0, b.nu, b.nv)
        kp = problem.kernel
        self.pdd = np.ascontiguousarray(kp.pdd, dtype=np.float32)
        pad = lambda v: (C.c_double * 4)(*(list(v) + [0.0] * (4 - len(v))))
        self.kernel = OKernel(kp.n_terms, len(self.pdd), pad(kp.weight), pad(kp.sigma0),
                              pad(kp.sigma_slope), pad(kp.width_scale), _ptr(self.pdd, C.c_float),
                              kp.pdd_step, kp.cutoff_u, kp.cutoff_v, kp.table_step, kp.rho_min,
                              DEPTH_MODES[kp.depth], 0, None)
        kt = getattr(kp, "tables", None)
        if kt is not None:
            self._tab_arrays = [np.ascontiguousarray(x, dtype=np.float32) for x in (kt.c1, kt.c2, kt.c3, kt.A)]
            c1, c2, c3, A = self._tab_arrays
            self._tables = OTables(c1.shape[1], A.shape[0], A.shape[1], 0, kt.depth_step, kt.theta_step,
                                   kt.adepth_step, _ptr(c1, C.c_float), _ptr(c2, C.c_float),
                                   _ptr(c3, C.c_float), _ptr(A, C.c_float))
            self.kernel.tables = C.pointer(self._tables)
        self.n_beams = len(problem.beams)
        self.n_beamlets = lib().ofs_count_beamlets(self.beams, self.n_beams)
        self._beamlets = None

    @property
    def beamlets(self):
        if self._beamlets is None:
            arr = (OBeamlet * self.n_beamlets)()
            lib().ofs_geometry(C.byref(self.grid), self.beams, self.n_beams, C.byref(self.kernel), arr)
            self._beamlets = arr
        return self._beamlets

    # -- depth tables --------------------------------------------------
    def tables(self):
        off = np.zeros(self.n_beamlets + 1, dtype=np.int64)
        lib().ofs_plan_tables(C.byref(self.grid), self.beams, self.n_beams, C.byref(self.kernel),
                              None, _ptr(off, C.c_int64))
        tab = np.zeros(int(off[-1]), dtype=np.float64)
        lib().ofs_plan_tables(C.byref(self.grid), self.beams, self.n_beams, C.byref(self.kernel),
                              _ptr(tab, C.c_double), _ptr(off, C.c_int64))
        return tab, off

    def table(self, j):
        bl = self.beamlets[j]
        t = np.zeros(max(bl.n, 1), dtype=np.float64)
        lib().ofs_depth_table(C.byref(self.grid), C.byref(bl), _ptr(t, C.c_double))
        return t[:bl.n]

    # -- rows ----------------------------------------------------------
    def counts(self):
        c = np.zeros(self.n_beamlets, dtype=np.int64)
        lib().ofs_plan_counts(C.byref(self.grid), self.beams, self.n_beams, C.byref(self.kernel),
                              _ptr(c, C.c_int64))
        return c

    def counts_of(self, sel):
        sel = np.ascontiguousarray(sel, dtype=np.int32)
        c = np.zeros(len(sel), dtype=np.int64)
        lib().ofs_plan_counts_sel(C.byref(self.grid), self.beams, self.n_beams, C.byref(self.kernel),
                                  _ptr(sel, C.c_int32), len(sel), _ptr(c, C.c_int64))
        return c

    def rows(self, sel, counts=None):
        """CSR (indptr, indices int32, values float64) of the selected beamlet rows."""
        sel = np.ascontiguousarray(sel, dtype=np.int32)
        if counts is None:
            counts = self.counts_of(sel)
        off = np.zeros(len(sel) + 1, dtype=np.int64)
        off[1:] = np.cumsum(counts)
        idx = np.zeros(max(int(off[-1]), 1), dtype=np.int32)
        val = np.zeros(max(int(off[-1]), 1), dtype=np.float64)
        rc = lib().ofs_plan_rows(C.byref(self.grid), self.beams, self.n_beams, C.byref(self.kernel),
                                 _ptr(sel, C.c_int32), len(sel), _ptr(off, C.c_int64),
                                 _ptr(idx, C.c_int32), _ptr(val, C.c_double))
        if rc != 0:
            raise RuntimeError("oracle row length disagrees with its count")
        return off, idx[:off[-1]], val[:off[-1]]

    def row_count(self, j):
        bl = self.beamlets[j]
        return int(lib().ofs_beamlet_row(C.byref(self.grid), C.byref(self.kernel), C.byref(bl),
                                         None, None, None, 0))

    def row(self, j):
        off, idx, val = self.rows([j])
        return idx, val

    def row_bruteforce(self, j):
        bl = self.beamlets[j]
        n = lib().ofs_beamlet_row_bruteforce(C.byref(self.grid), C.byref(self.kernel), C.byref(bl),
                                             None, 0)
        idx = np.zeros(max(n, 1), dtype=np.int32)
        lib().ofs_beamlet_row_bruteforce(C.byref(self.grid), C.byref(self.kernel), C.byref(bl),
                                         _ptr(idx, C.c_int32), n)
        return idx[:n]

    def full(self):
        """Every row (small problems only)."""
        c = self.counts()
        return self.rows(np.arange(self.n_beamlets), c)

    def fluence_dose(self, w):
        """Eq. 1: dose of beamlet weights w (FP64, every row computed)."""
        w = np.ascontiguousarray(w, dtype=np.float64)
        nv = self.grid.nx * self.grid.ny * self.grid.nz
        dose = np.zeros(nv, dtype=np.float64)
        lib().ofs_plan_fluence(C.byref(self.grid), self.beams, self.n_beams, C.byref(self.kernel),
                               _ptr(w, C.c_double), _ptr(dose, C.c_double), None, None)
        return dose

    def fluence_gradient(self, r):
        """g_j = sum_i D_ij r_i."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        g = np.zeros(self.n_beamlets, dtype=np.float64)
        lib().ofs_plan_fluence(C.byref(self.grid), self.beams, self.n_beams, C.byref(self.kernel),
                               None, None, _ptr(r, C.c_double), _ptr(g, C.c_double))
        return g

    # -- point evaluations ---------------------------------------------
    def voi_member(self, j, ix, iy, iz):
        t, u, v = C.c_double(), C.c_double(), C.c_double()
        m = lib().ofs_voi_member(C.byref(self.grid), C.byref(self.kernel), C.byref(self.beamlets[j]),
                                 ix, iy, iz, C.byref(t), C.byref(u), C.byref(v))
        return bool(m), t.value, u.value, v.value

    def trilinear_density(self, p):
        """Density at point p by trilinear interpolation of the voxel centres."""
        q = (C.c_double * 3)(*p)
        return lib().ofs_trilinear_density(C.byref(self.grid), q)

    def exact_depth(self, j, t):
        return lib().ofs_exact_depth(C.byref(self.grid), C.byref(self.beamlets[j]), t)

    def table_depth(self, j, table, t):
        tab = np.ascontiguousarray(table, dtype=np.float64)
        return lib().ofs_table_depth(C.byref(self.beamlets[j]), _ptr(tab, C.c_double), t)

    def pdd_at(self, d):
        return lib().ofs_pdd(C.byref(self.kernel), d)

    def lateral(self, u, v, a, b, d):
        return lib().ofs_lateral(C.byref(self.kernel), u, v, a, b, d)

    def kernel_value(self, d, u, v, a):
        return lib().ofs_kernel_value(C.byref(self.kernel), d, u, v, a)

    def kernel_values(self, pts):
        """K(d, u, v, a) for an [n, 4] array."""
        pts = np.ascontiguousarray(pts, dtype=np.float64)
        out = np.zeros(pts.shape[0], dtype=np.float64)
        lib().ofs_kernel_values(C.byref(self.kernel), _ptr(pts, C.c_double), pts.shape[0],
                                _ptr(out, C.c_double))
        return out


def siddon(problem_or_plan, S, e, tA, tB):
    """Per-segment (voxel index, length) of one ray, in order."""
    p = problem_or_plan if isinstance(problem_or_plan, OraclePlan) else OraclePlan(problem_or_plan)
    S = np.ascontiguousarray(S, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    cap = int(p.grid.nx + p.grid.ny + p.grid.nz + 4)
    vox = np.zeros(cap, dtype=np.int64)
    ln = np.zeros(cap, dtype=np.float64)
    n = lib().ofs_siddon(C.byref(p.grid), _ptr(S, C.c_double), _ptr(e, C.c_double), tA, tB,
                         _ptr(vox, C.c_int64), _ptr(ln, C.c_double), cap)
    return vox[:n], ln[:n]


def csr_transpose(indptr, indices, values, n_cols):
    """Voxel-row form of a beamlet-row CSR: the definition of the transpose.

    Every entry (j, i, v) becomes (i, j, v); entries are ordered by voxel i,
    then beamlet j (a stable sort by column of the row-major entry list).
    Returns (t_indptr int64 [n_cols + 1], t_indices int32, t_values).
    """
    indptr = np.asarray(indptr, dtype=np.int64)
    indices = np.asarray(indices, dtype=np.int64)
    values = np.asarray(values)
    rows = np.repeat(np.arange(len(indptr) - 1, dtype=np.int64), np.diff(indptr))
    order = np.argsort(indices, kind="stable")
    counts = np.bincount(indices, minlength=n_cols)
    t_indptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return t_indptr, rows[order].astype(np.int32), values[order]


def set_threads(n):
    lib().ofs_set_threads(int(n))


def max_threads():
    return int(lib().ofs_max_threads())


# -- surrogate MLP --------------------------------------------------------

def bf16_round(v):
    return lib().ofs_bf16_round(float(v))


def surrogate_features(raw):
    raw = np.ascontiguousarray(raw, dtype=np.float64)
    out = np.zeros_like(raw)
    lib().ofs_surrogate_features(_ptr(raw, C.c_double), raw.shape[0], _ptr(out, C.c_double))
    return out


def mlp_forward(params, feats, bf16=False):
    params = np.ascontiguousarray(params, dtype=np.float64)
    feats = np.ascontiguousarray(feats, dtype=np.float64)
    y = np.zeros(feats.shape[0], dtype=np.float64)
    lib().ofs_mlp_forward(_ptr(params, C.c_double), _ptr(feats, C.c_double), feats.shape[0],
                          _ptr(y, C.c_double), int(bf16))
    return y


def mlp_loss_grad(params, feats, target, bf16=False):
    params = np.ascontiguousarray(params, dtype=np.float64)
    feats = np.ascontiguousarray(feats, dtype=np.float64)
    target = np.ascontiguousarray(target, dtype=np.float64)
    g = np.zeros(MLP_NPARAM, dtype=np.float64)
    loss = lib().ofs_mlp_loss_grad(_ptr(params, C.c_double), _ptr(feats, C.c_double),
                                   _ptr(target, C.c_double), feats.shape[0], _ptr(g, C.c_double),
                                   int(bf16))
    return loss, g
