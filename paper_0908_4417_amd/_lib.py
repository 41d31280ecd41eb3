"""ctypes declarations of the C ABI in ``include/fspb.h``.

Loading fails loudly if ``libfspb.so`` has not been built: there is no other
implementation behind these names.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libfspb.so")

FSPB_OK = 0
FSPB_ERR_INVALID = -1
FSPB_ERR_STATE = -2
FSPB_ERR_CAPACITY = -3
FSPB_ERR_HIP = -4
FSPB_ERR_NOMEM = -5
FSPB_ERR_OVERFLOW = -6
FSPB_DEPTH_TRILINEAR = 1       # fspb_kernel.flags: trilinear-sampled depth table
FSPB_ERF_COMPACT = 2           # fspb_kernel.flags: force the 8 KB erf table on [0, 4]
FSPB_ERF_MIRRORED = 4          # fspb_kernel.flags: force the 16 KB erf table mirrored onto [-4, 4]
FSPB_TILES_BLOCK = 8           # fspb_kernel.flags: fill every beamlet in tiles of its row block
FSPB_TILES_LIST = 16           # fspb_kernel.flags: fill every beamlet in tiles of its member-row list


class FspbError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{status_name(status)}: {message}")
        self.status = status


def status_name(s):
    return {0: "FSPB_OK", -1: "FSPB_ERR_INVALID", -2: "FSPB_ERR_STATE", -3: "FSPB_ERR_CAPACITY",
            -4: "FSPB_ERR_HIP", -5: "FSPB_ERR_NOMEM", -6: "FSPB_ERR_OVERFLOW"}.get(s, str(s))


class FspbGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("reserved", C.c_int32),
                ("spacing", C.c_double * 3), ("origin", C.c_double * 3),
                ("density", C.c_void_p)]


class FspbBeam(C.Structure):
    _fields_ = [("gantry_deg", C.c_double), ("isocenter", C.c_double * 3), ("sad", C.c_double),
                ("beamlet_a", C.c_double), ("beamlet_b", C.c_double),
                ("u0", C.c_double), ("v0", C.c_double), ("nu", C.c_int32), ("nv", C.c_int32)]


class FspbKernelTables(C.Structure):
    _fields_ = [("n_depth", C.c_int32), ("n_theta", C.c_int32), ("n_adepth", C.c_int32), ("reserved", C.c_int32),
                ("depth_step", C.c_double), ("theta_step", C.c_double), ("adepth_step", C.c_double),
                ("c1", C.POINTER(C.c_float)), ("c2", C.POINTER(C.c_float)), ("c3", C.POINTER(C.c_float)),
                ("A", C.POINTER(C.c_float))]


class FspbKernel(C.Structure):
    _fields_ = [("n_terms", C.c_int32), ("n_pdd", C.c_int32),
                ("weight", C.c_double * 4), ("sigma0", C.c_double * 4),
                ("sigma_slope", C.c_double * 4), ("width_scale", C.c_double * 4),
                ("pdd", C.POINTER(C.c_float)), ("pdd_step", C.c_double),
                ("cutoff_u", C.c_double), ("cutoff_v", C.c_double), ("table_step", C.c_double),
                ("rho_min", C.c_float), ("flags", C.c_uint32), ("tables", C.POINTER(FspbKernelTables))]


class FspbTiming(C.Structure):
    _fields_ = [("prep_ms", C.c_float), ("raytrace_ms", C.c_float), ("count_ms", C.c_float),
                ("scan_ms", C.c_float), ("fill_ms", C.c_float), ("valid", C.c_int32)]


class FspbBatchConfig(C.Structure):
    _fields_ = [("waves_per_group", C.c_int32), ("groups_per_cu", C.c_int32), ("order", C.c_int32),
                ("tuned", C.c_int32), ("fill_ms", C.c_float), ("tile_rows", C.c_int32),
                ("beamlets_per_item", C.c_int32), ("reserved", C.c_int32)]


class FspbTrainConfig(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr_max", C.c_float), ("lr_min", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float), ("reserved", C.c_int32),
                ("seed", C.c_uint64)]


SURROGATE_PARAMS = 4545


class FspbPlanDesc(C.Structure):
    _fields_ = [("n_beamlets", C.c_int32), ("n_voxels", C.c_int32), ("table_entries", C.c_int64),
                ("n_tiles", C.c_int64), ("max_table", C.c_int32), ("fill_lds_bytes", C.c_int32),
                ("fill_erf_mode", C.c_int32)]


# name -> (restype, argtypes); every symbol include/fspb.h declares
_SIGS = {
    "fspb_plan_create": (C.c_int32, [C.POINTER(FspbGrid), C.POINTER(FspbBeam), C.c_int32,
                                     C.POINTER(FspbKernel), C.c_void_p, C.c_size_t,
                                     C.POINTER(C.c_size_t), C.POINTER(C.c_void_p)]),
    "fspb_raytrace": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "fspb_dose_coeffs": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                     C.POINTER(C.c_int64), C.c_void_p]),
    "fspb_plan_destroy": (None, [C.c_void_p]),
    "fspb_plan_info": (C.c_int32, [C.c_void_p, C.POINTER(FspbPlanDesc)]),
    "fspb_plan_get_tables": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fspb_plan_set_timing": (C.c_int32, [C.c_void_p, C.c_int32]),
    "fspb_plan_get_timing": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "fspb_batch_create": (C.c_int32, [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_size_t,
                                      C.POINTER(C.c_size_t), C.c_void_p, C.POINTER(C.c_void_p)]),
    "fspb_batch_nnz": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64)]),
    "fspb_batch_bind": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_int64]),
    "fspb_batch_tune": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "fspb_batch_get_config": (C.c_int32, [C.c_void_p, C.POINTER(FspbBatchConfig)]),
    "fspb_batch_set_config": (C.c_int32, [C.c_void_p, C.POINTER(FspbBatchConfig)]),
    "fspb_batch_run": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "fspb_batch_check": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "fspb_batch_destroy": (None, [C.c_void_p]),
    "fspb_surrogate_create": (C.c_int32, [C.POINTER(FspbKernel), C.POINTER(C.c_float), C.c_int32,
                                          C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t),
                                          C.POINTER(C.c_void_p)]),
    "fspb_surrogate_targets": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                           C.c_void_p]),
    "fspb_surrogate_forward": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "fspb_surrogate_gradient": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                            C.POINTER(C.c_float), C.c_void_p]),
    "fspb_surrogate_train": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                         C.POINTER(FspbTrainConfig), C.POINTER(C.c_float), C.c_void_p]),
    "fspb_surrogate_get_params": (C.c_int32, [C.c_void_p, C.POINTER(C.c_float), C.c_void_p]),
    "fspb_surrogate_set_params": (C.c_int32, [C.c_void_p, C.POINTER(C.c_float)]),
    "fspb_plan_set_surrogate": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "fspb_surrogate_destroy": (None, [C.c_void_p]),
    "fspb_dose_coeffs_rows": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_int64, C.POINTER(C.c_int64), C.c_void_p]),
    "fspb_row_ranges": (C.c_int32, [C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32), C.c_int32, C.c_int64,
                                    C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)]),
    "fspb_fluence_dose": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                      C.c_void_p, C.c_void_p, C.c_void_p]),
    "fspb_fluence_gradient": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                          C.c_void_p, C.c_void_p, C.c_void_p]),
    "fspb_csr_transpose": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int64,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                       C.POINTER(C.c_size_t), C.c_void_p]),
    "fspb_csr_transpose_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                               C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fspb_voxel_dose": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                    C.c_void_p, C.c_void_p]),
    "fspb_status_string": (C.c_char_p, [C.c_int32]),
    "fspb_last_error": (C.c_char_p, []),
}
EXPORTED = tuple(_SIGS)

_lib = None


def library_path():
    return _LIB


def lib():
    """The loaded HIP library; raises if it was never built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise ImportError(f"{_LIB} is missing: build it with paper_0908_4417_amd.build.build() "
                              "(the HIP library is the only implementation)")
        L = C.CDLL(_LIB)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != FSPB_OK:
        raise FspbError(status, lib().fspb_last_error().decode())
    return status


def fspb_status_string(s):
    return lib().fspb_status_string(s).decode()


def fspb_last_error():
    return lib().fspb_last_error().decode()


def fspb_plan_create(grid, beams, n_beams, kernel, workspace, workspace_bytes):
    """Returns (status, plan handle or None, workspace bytes needed).  No exception on CAPACITY."""
    need = C.c_size_t(0)
    handle = C.c_void_p(None)
    st = lib().fspb_plan_create(C.byref(grid), beams, n_beams, C.byref(kernel), workspace,
                                workspace_bytes, C.byref(need), C.byref(handle))
    if st not in (FSPB_OK, FSPB_ERR_CAPACITY):
        _check(st)
    return st, (handle.value if st == FSPB_OK else None), need.value


def fspb_raytrace(plan, stream):
    return _check(lib().fspb_raytrace(plan, stream))


def fspb_dose_coeffs(plan, indptr, indices, values, capacity, stream):
    """Returns (status, nnz).  CAPACITY is returned, not raised (size query)."""
    nnz = C.c_int64(0)
    st = lib().fspb_dose_coeffs(plan, indptr, indices, values, capacity, C.byref(nnz), stream)
    if st not in (FSPB_OK, FSPB_ERR_CAPACITY):
        _check(st)
    return st, nnz.value


def fspb_plan_destroy(plan):
    lib().fspb_plan_destroy(plan)


def fspb_plan_info(plan):
    d = FspbPlanDesc()
    _check(lib().fspb_plan_info(plan, C.byref(d)))
    return d


def fspb_plan_get_tables(plan, tables_ptr, offsets_ptr, stream):
    return _check(lib().fspb_plan_get_tables(plan, tables_ptr, offsets_ptr, stream))


def fspb_plan_set_timing(plan, enable):
    return _check(lib().fspb_plan_set_timing(plan, int(enable)))


def fspb_plan_get_timing(plan):
    t = FspbTiming()
    _check(lib().fspb_plan_get_timing(plan, C.byref(t)))
    return t


def fspb_batch_create(plan_handles, workspace, workspace_bytes, stream):
    """Returns (status, batch handle or None, workspace bytes needed)."""
    arr = (C.c_void_p * len(plan_handles))(*plan_handles)
    need = C.c_size_t(0)
    handle = C.c_void_p(None)
    st = lib().fspb_batch_create(arr, len(plan_handles), workspace, workspace_bytes, C.byref(need),
                                 stream, C.byref(handle))
    if st not in (FSPB_OK, FSPB_ERR_CAPACITY):
        _check(st)
    return st, (handle.value if st == FSPB_OK else None), need.value


def fspb_batch_nnz(batch, plan):
    n = C.c_int64(0)
    _check(lib().fspb_batch_nnz(batch, plan, C.byref(n)))
    return n.value


def fspb_batch_bind(batch, plan, indptr, indices, values, capacity):
    return _check(lib().fspb_batch_bind(batch, plan, indptr, indices, values, capacity))


def fspb_batch_tune(batch, stream):
    return _check(lib().fspb_batch_tune(batch, stream))


def fspb_batch_get_config(batch):
    c = FspbBatchConfig()
    _check(lib().fspb_batch_get_config(batch, C.byref(c)))
    return c


def fspb_batch_set_config(batch, waves_per_group, groups_per_cu, order, tile_rows=64, beamlets_per_item=1):
    c = FspbBatchConfig(waves_per_group, groups_per_cu, order, 0, 0.0, tile_rows, beamlets_per_item, 0)
    return _check(lib().fspb_batch_set_config(batch, C.byref(c)))


def fspb_batch_run(batch, stream):
    return _check(lib().fspb_batch_run(batch, stream))


def fspb_batch_check(batch, stream):
    """Returns the status (OK or OVERFLOW) instead of raising on OVERFLOW."""
    st = lib().fspb_batch_check(batch, stream)
    if st not in (FSPB_OK, FSPB_ERR_OVERFLOW):
        _check(st)
    return st


def fspb_batch_destroy(batch):
    lib().fspb_batch_destroy(batch)


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def fspb_surrogate_create(kernel, init_params, max_batch, workspace, workspace_bytes):
    import numpy as np
    init = np.ascontiguousarray(init_params, dtype=np.float32)
    need = C.c_size_t(0)
    handle = C.c_void_p(None)
    st = lib().fspb_surrogate_create(C.byref(kernel), _fptr(init), max_batch, workspace, workspace_bytes,
                                     C.byref(need), C.byref(handle))
    if st not in (FSPB_OK, FSPB_ERR_CAPACITY):
        _check(st)
    return st, (handle.value if st == FSPB_OK else None), need.value


def fspb_surrogate_targets(sur, samples, n, features, targets, stream):
    return _check(lib().fspb_surrogate_targets(sur, samples, n, features, targets, stream))


def fspb_surrogate_forward(sur, features, n, out, stream):
    return _check(lib().fspb_surrogate_forward(sur, features, n, out, stream))


def fspb_surrogate_gradient(sur, features, targets, n, grad, stream):
    loss = C.c_float(0.0)
    _check(lib().fspb_surrogate_gradient(sur, features, targets, n, grad, C.byref(loss), stream))
    return loss.value


def fspb_surrogate_train(sur, features, targets, n, cfg, stream):
    import numpy as np
    losses = np.zeros(cfg.epochs, dtype=np.float32)
    _check(lib().fspb_surrogate_train(sur, features, targets, n, C.byref(cfg), _fptr(losses), stream))
    return losses


def fspb_surrogate_get_params(sur, stream):
    import numpy as np
    p = np.zeros(SURROGATE_PARAMS, dtype=np.float32)
    _check(lib().fspb_surrogate_get_params(sur, _fptr(p), stream))
    return p


def fspb_surrogate_set_params(sur, params):
    import numpy as np
    p = np.ascontiguousarray(params, dtype=np.float32)
    return _check(lib().fspb_surrogate_set_params(sur, _fptr(p)))


def fspb_plan_set_surrogate(plan, sur):
    return _check(lib().fspb_plan_set_surrogate(plan, sur))


def fspb_surrogate_destroy(sur):
    lib().fspb_surrogate_destroy(sur)


def fspb_dose_coeffs_rows(h, j0, j1, indptr, indices, values, capacity, stream):
    """Returns (status, nnz of the rows); CAPACITY is returned, not raised, with the size."""
    n = C.c_int64(0)
    st = lib().fspb_dose_coeffs_rows(h, j0, j1, indptr, indices, values, capacity, C.byref(n), stream)
    if st == FSPB_ERR_CAPACITY:
        return st, n.value
    return _check(st), n.value


def fspb_row_ranges(indptr, beam_rows, max_bytes):
    """Host row partition of a byte budget: list of (j0, j1); beam_rows None = by beamlet.
    Raises ValueError when a single row exceeds the budget."""
    import numpy as np
    ip = np.ascontiguousarray(indptr, dtype=np.int64)
    n_rows = len(ip) - 1
    br = None if beam_rows is None else np.ascontiguousarray(beam_rows, dtype=np.int32)
    brp = None if br is None else br.ctypes.data_as(C.POINTER(C.c_int32))
    nb = 0 if br is None else len(br)
    ipp = ip.ctypes.data_as(C.POINTER(C.c_int64))
    n = C.c_int32(0)
    st = lib().fspb_row_ranges(ipp, n_rows, brp, nb, int(max_bytes), None, 0, C.byref(n))
    if st == FSPB_ERR_INVALID:
        raise ValueError(lib().fspb_last_error().decode())
    if st != FSPB_ERR_CAPACITY:
        _check(st)
    bounds = np.zeros(n.value + 1, dtype=np.int32)
    _check(lib().fspb_row_ranges(ipp, n_rows, brp, nb, int(max_bytes), bounds.ctypes.data_as(C.POINTER(C.c_int32)),
                                 n.value, C.byref(n)))
    return [(int(bounds[k]), int(bounds[k + 1])) for k in range(n.value)]


def fspb_fluence_dose(indptr, indices, values, n_rows, n_voxels, w, dose, stream):
    return _check(lib().fspb_fluence_dose(indptr, indices, values, n_rows, n_voxels, w, dose, stream))


def fspb_fluence_gradient(indptr, indices, values, n_rows, n_voxels, r, g, stream):
    return _check(lib().fspb_fluence_gradient(indptr, indices, values, n_rows, n_voxels, r, g, stream))


def fspb_csr_transpose(indptr, indices, values, n_rows, n_voxels, nnz, t_indptr, t_indices, t_values,
                       workspace, workspace_bytes, stream):
    """Returns (status, bytes needed); a NULL workspace is the size query."""
    need = C.c_size_t(0)
    st = lib().fspb_csr_transpose(indptr, indices, values, n_rows, n_voxels, nnz, t_indptr, t_indices, t_values,
                                  workspace, workspace_bytes, C.byref(need), stream)
    if st == FSPB_ERR_CAPACITY and not workspace:
        return st, need.value
    return _check(st), need.value


NOALLOC_SCRATCH_BYTES = 64 << 20


def fspb_csr_transpose_noalloc(indptr, indices, values, n_rows, n_voxels, nnz, t_indptr, t_indices, t_values, stream):
    """The transpose into the library's static device scratch (no allocation).  Returns the
    status: CAPACITY (the sizes need more scratch) is returned, not raised."""
    st = lib().fspb_csr_transpose_noalloc(indptr, indices, values, n_rows, n_voxels, nnz, t_indptr, t_indices,
                                          t_values, stream)
    if st == FSPB_ERR_CAPACITY:
        return st
    return _check(st)


def fspb_voxel_dose(t_indptr, t_indices, t_values, n_voxels, n_beamlets, w, dose, stream):
    return _check(lib().fspb_voxel_dose(t_indptr, t_indices, t_values, n_voxels, n_beamlets, w, dose, stream))
