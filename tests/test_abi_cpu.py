"""C ABI checks that need no GPU: the library loads, exports every symbol that
include/fspb.h declares, and validates arguments before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import fspb_inputs as fi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def fspb():
    import paper_0908_4417_amd as m
    if not os.path.exists(m.library_path()):
        from paper_0908_4417_amd import build
        build.build()
    m.lib()
    return m


def _declared():
    src = open(os.path.join(ROOT, "include", "fspb.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(fspb_[a-z_]+)\s*\(", src, re.M)))


def test_header_declarations_are_exported(fspb):
    names = _declared()
    assert {"fspb_plan_create", "fspb_raytrace", "fspb_dose_coeffs", "fspb_plan_destroy"} <= set(names)
    L = C.CDLL(fspb.library_path())
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(fspb.EXPORTED)


def test_library_has_gfx950_code(fspb):
    data = open(fspb.library_path(), "rb").read()
    assert b"gfx950" in data


def _structs(fspb, prob, density_ptr=0x1000):
    from paper_0908_4417_amd.plan import _structs
    return _structs(prob, density_ptr)


def _prob():
    g = fi.water_phantom((16, 12, 10), (0.5, 0.5, 0.5))
    return fi.Problem("abi", g, fi.coplanar_beams(2, (0, 0, 0), 100.0, 1.0, 1.0, 3, 2),
                      fi.default_kernel(0))


def _create(fspb, grid, beams, nb, kern, ws=None, nbytes=0):
    need = C.c_size_t(0)
    h = C.c_void_p(None)
    st = fspb.lib().fspb_plan_create(C.byref(grid), beams, nb, C.byref(kern), ws, nbytes,
                                     C.byref(need), C.byref(h))
    return st, need.value, h.value


def test_workspace_query(fspb):
    grid, beams, kern, pdd = _structs(fspb, _prob())
    st, need, h = _create(fspb, grid, beams, 2, kern)
    assert st == fspb.FSPB_ERR_CAPACITY and need > 0 and h is None
    assert "needed" in fspb.fspb_last_error()


@pytest.mark.parametrize("mutate,msg", [
    (lambda g, b, k: setattr(g, "nx", 0), "dimensions"),
    (lambda g, b, k: (setattr(g, "nx", 1 << 30), setattr(g, "ny", 1), setattr(g, "nz", 1)), "nx must be"),
    (lambda g, b, k: setattr(g, "reserved", 3), "reserved"),
    (lambda g, b, k: g.spacing.__setitem__(1, -0.5), "spacing"),
    (lambda g, b, k: g.origin.__setitem__(2, float("nan")), "origin"),
    (lambda g, b, k: setattr(g, "density", None), "density"),
    (lambda g, b, k: setattr(b[0], "sad", 0.0), "sad"),
    (lambda g, b, k: setattr(b[1], "sad", 2.0), "inside the grid"),
    (lambda g, b, k: setattr(b[0], "nu", 0), "nu"),
    (lambda g, b, k: setattr(b[0], "beamlet_a", 0.0), "beamlet sizes"),
    (lambda g, b, k: setattr(k, "n_terms", 5), "n_terms"),
    (lambda g, b, k: k.sigma0.__setitem__(0, 0.0), "sigma0"),
    (lambda g, b, k: k.sigma_slope.__setitem__(1, -1.0), "sigma_slope"),
    (lambda g, b, k: k.width_scale.__setitem__(0, 0.0), "width_scale"),
    (lambda g, b, k: setattr(k, "n_pdd", 1), "n_pdd"),
    (lambda g, b, k: setattr(k, "pdd_step", 0.0), "pdd_step"),
    (lambda g, b, k: setattr(k, "flags", 32), "flags"),
    (lambda g, b, k: setattr(k, "flags", 6), "exclude each other"),
    (lambda g, b, k: setattr(k, "flags", 24), "FSPB_TILES_BLOCK and FSPB_TILES_LIST"),
    (lambda g, b, k: setattr(k, "rho_min", float("inf")), "rho_min"),
])
def test_invalid_arguments_rejected_before_device_work(fspb, mutate, msg):
    grid, beams, kern, pdd = _structs(fspb, _prob())
    mutate(grid, beams, kern)
    st, need, h = _create(fspb, grid, beams, 2, kern)
    assert st == fspb.FSPB_ERR_INVALID and h is None
    assert msg in fspb.fspb_last_error()


def test_null_arguments(fspb):
    L = fspb.lib()
    grid, beams, kern, pdd = _structs(fspb, _prob())
    assert L.fspb_plan_create(None, beams, 2, C.byref(kern), None, 0, None, None) == fspb.FSPB_ERR_INVALID
    st, _, _ = _create(fspb, grid, beams, 0, kern)
    assert st == fspb.FSPB_ERR_INVALID
    assert L.fspb_raytrace(None, None) == fspb.FSPB_ERR_INVALID
    n = C.c_int64(0)
    assert L.fspb_dose_coeffs(None, None, None, None, 0, C.byref(n), None) == fspb.FSPB_ERR_INVALID
    L.fspb_plan_destroy(None)
    assert fspb.fspb_status_string(fspb.FSPB_ERR_STATE) == "FSPB_ERR_STATE"
    assert fspb.fspb_status_string(-99) == "FSPB_ERR_UNKNOWN"


def test_nan_in_depth_dose_rejected(fspb):
    prob = _prob()
    prob.kernel.pdd = prob.kernel.pdd.copy()
    prob.kernel.pdd[7] = np.nan
    grid, beams, kern, pdd = _structs(fspb, prob)
    st, _, _ = _create(fspb, grid, beams, 2, kern)
    assert st == fspb.FSPB_ERR_INVALID and "pdd[7]" in fspb.fspb_last_error()


def test_host_pointer_rejected_as_density(fspb):
    """A host address for the density is refused (pointer attribute check)."""
    prob = _prob()
    host = np.zeros(16 * 12 * 10, dtype=np.float32)
    grid, beams, kern, pdd = _structs(fspb, prob, density_ptr=host.ctypes.data)
    ws = np.zeros(1 << 20, dtype=np.uint8)
    base = (ws.ctypes.data + 255) // 256 * 256
    st, need, h = _create(fspb, grid, beams, 2, kern, ws=base, nbytes=(1 << 20) - 256)
    assert st in (fspb.FSPB_ERR_INVALID, fspb.FSPB_ERR_CAPACITY) and h is None


def test_batch_arguments_rejected(fspb):
    L = fspb.lib()
    h = C.c_void_p(None)
    need = C.c_size_t(0)
    assert L.fspb_batch_create(None, 1, None, 0, C.byref(need), None, C.byref(h)) == fspb.FSPB_ERR_INVALID
    arr = (C.c_void_p * 2)(None, None)
    assert L.fspb_batch_create(arr, 2, None, 0, C.byref(need), None, C.byref(h)) == fspb.FSPB_ERR_INVALID
    assert "plans[0] is NULL" in fspb.fspb_last_error()
    assert L.fspb_batch_create(arr, 0, None, 0, C.byref(need), None, C.byref(h)) == fspb.FSPB_ERR_INVALID
    n = C.c_int64(0)
    assert L.fspb_batch_nnz(None, 0, C.byref(n)) == fspb.FSPB_ERR_INVALID
    assert L.fspb_batch_run(None, None) == fspb.FSPB_ERR_INVALID
    assert L.fspb_batch_check(None, None) == fspb.FSPB_ERR_INVALID
    assert L.fspb_batch_tune(None, None) == fspb.FSPB_ERR_INVALID
    cfg = fspb.FspbBatchConfig(3, 4, 0, 0, 0.0, 0)
    assert L.fspb_batch_set_config(None, C.byref(cfg)) == fspb.FSPB_ERR_INVALID
    L.fspb_batch_destroy(None)


def test_surrogate_arguments_rejected(fspb):
    from paper_0908_4417_amd.plan import _kernel_struct
    L = fspb.lib()
    k, pdd = _kernel_struct(fi.default_kernel(0))
    init = np.zeros(fspb.SURROGATE_PARAMS, dtype=np.float32)
    ip = init.ctypes.data_as(C.POINTER(C.c_float))
    h = C.c_void_p(None)
    need = C.c_size_t(0)
    # size query works without a device
    assert L.fspb_surrogate_create(C.byref(k), ip, 4096, None, 0, C.byref(need), C.byref(h)) == \
        fspb.FSPB_ERR_CAPACITY and need.value > 0
    assert L.fspb_surrogate_create(C.byref(k), ip, 100, None, 0, C.byref(need), C.byref(h)) == \
        fspb.FSPB_ERR_INVALID                                     # not a multiple of 64
    bad = init.copy()
    bad[17] = np.inf
    assert L.fspb_surrogate_create(C.byref(k), bad.ctypes.data_as(C.POINTER(C.c_float)), 4096, None, 0,
                                   C.byref(need), C.byref(h)) == fspb.FSPB_ERR_INVALID
    assert "init_params[17]" in fspb.fspb_last_error()
    k.n_terms = 0
    assert L.fspb_surrogate_create(C.byref(k), ip, 4096, None, 0, C.byref(need), C.byref(h)) == \
        fspb.FSPB_ERR_INVALID
    assert L.fspb_plan_set_surrogate(None, None) == fspb.FSPB_ERR_INVALID
    assert L.fspb_surrogate_forward(None, None, 0, None, None) == fspb.FSPB_ERR_INVALID
    cfg = fspb.FspbTrainConfig(1, 64, 1e-3, 0.0, 0.9, 0.999, 1e-8, 0, 0)
    assert L.fspb_surrogate_train(None, None, None, 0, C.byref(cfg), None, None) == fspb.FSPB_ERR_INVALID
    L.fspb_surrogate_destroy(None)


def test_sparse_arguments_rejected(fspb):
    """Eq. 1 / transpose entry points: size query and argument checks, no device work."""
    L = fspb.lib()
    need = C.c_size_t(0)
    st = L.fspb_csr_transpose(None, None, None, 10, 1000, 5000, None, None, None, None, 0, C.byref(need), None)
    assert st == fspb.FSPB_ERR_CAPACITY and need.value >= 24 * 5000
    small = need.value
    L.fspb_csr_transpose(None, None, None, 10, 1000, 50000, None, None, None, None, 0, C.byref(need), None)
    assert need.value > small                                   # grows with nnz
    assert L.fspb_csr_transpose(None, None, None, 10, 0, 5, None, None, None, None, 0, C.byref(need),
                                None) == fspb.FSPB_ERR_INVALID
    assert L.fspb_csr_transpose(None, None, None, 10, 5, 1 << 32, None, None, None, None, 0, C.byref(need),
                                None) == fspb.FSPB_ERR_INVALID
    assert "2^32" in fspb.fspb_last_error()
    assert L.fspb_csr_transpose(None, None, None, 10, 5, 7, None, None, None, C.c_void_p(0x1000), 1,
                                C.byref(need), None) == fspb.FSPB_ERR_CAPACITY
    assert L.fspb_voxel_dose(None, None, None, 4, 2, None, None, None) == fspb.FSPB_ERR_INVALID
    assert L.fspb_fluence_dose(None, None, None, 1, 1, None, None, None) == fspb.FSPB_ERR_INVALID
    assert L.fspb_fluence_gradient(None, None, None, 1, 0, None, None, None) == fspb.FSPB_ERR_INVALID


def test_every_entry_point_has_a_binding(fspb):
    """Each exported C function is reachable from the package (wrapper or raw)."""
    missing = [n for n in fspb.EXPORTED if not hasattr(fspb, n)]
    assert not missing, missing


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "4"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""


def test_noalloc_transpose_size_limit(fspb):
    """The allocation-free transpose refuses sizes beyond its static scratch on the host,
    before any device work (so this runs without a GPU)."""
    st = fspb.fspb_csr_transpose_noalloc(1, 1, 1, 100, 1000, 3_000_000, 1, 1, 1, None)
    assert st == fspb.FSPB_ERR_CAPACITY and "scratch" in fspb.fspb_last_error()
    with pytest.raises(fspb.FspbError, match="nnz"):
        fspb.fspb_csr_transpose_noalloc(1, 1, 1, 100, 1000, -1, 1, 1, 1, None)
