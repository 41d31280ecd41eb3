"""High-level plan object: torch-owned device buffers around the C ABI."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib as L


@dataclass
class CSR:
    """D_ij with rows = beamlets, columns = voxel linear indices (ascending per row)."""
    indptr: "torch.Tensor"      # int64 [n_beamlets + 1]
    indices: "torch.Tensor"     # int32 [nnz]
    values: "torch.Tensor"      # float32 [nnz]
    n_voxels: int

    @property
    def nnz(self):
        return int(self.indices.numel())

    def _s(self, stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.values.device)
        return C.c_void_p(s.cuda_stream)

    def dose(self, w, stream=None):
        """Eq. 1: dose of the beamlet weights w (device float32, one per row)."""
        import torch
        d = torch.empty(self.n_voxels, dtype=torch.float32, device=self.values.device)
        L.fspb_fluence_dose(self.indptr.data_ptr(), self.indices.data_ptr(), self.values.data_ptr(),
                            self.indptr.numel() - 1, self.n_voxels, w.data_ptr(), d.data_ptr(), self._s(stream))
        return d

    def gradient(self, r, stream=None):
        """g_j = sum_i D_ij r_i for a voxel vector r (device float32)."""
        import torch
        g = torch.empty(self.indptr.numel() - 1, dtype=torch.float32, device=self.values.device)
        L.fspb_fluence_gradient(self.indptr.data_ptr(), self.indices.data_ptr(), self.values.data_ptr(),
                                self.indptr.numel() - 1, self.n_voxels, r.data_ptr(), g.data_ptr(),
                                self._s(stream))
        return g

    def transpose(self, stream=None):
        """Voxel-row form of D (rows = voxels, beamlets ascending in each row)."""
        import torch
        dev = self.values.device
        n_rows, nnz = self.indptr.numel() - 1, self.nnz
        s = self._s(stream)
        _, need = L.fspb_csr_transpose(None, None, None, n_rows, self.n_voxels, nnz, None, None, None, None, 0, s)
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
        wsp = (ws.data_ptr() + 255) // 256 * 256
        t_indptr = torch.empty(self.n_voxels + 1, dtype=torch.int64, device=dev)
        t_indices = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)[:nnz]
        t_values = torch.empty(max(nnz, 1), dtype=torch.float32, device=dev)[:nnz]
        L.fspb_csr_transpose(self.indptr.data_ptr(), self.indices.data_ptr(), self.values.data_ptr(), n_rows,
                             self.n_voxels, nnz, t_indptr.data_ptr(), t_indices.data_ptr(), t_values.data_ptr(),
                             wsp, need, s)
        return VoxelCSR(t_indptr, t_indices, t_values, n_rows)


@dataclass
class VoxelCSR:
    """D_ij with rows = voxels, columns = beamlet ids (ascending per row)."""
    indptr: "torch.Tensor"      # int64 [n_voxels + 1]
    indices: "torch.Tensor"     # int32 [nnz]
    values: "torch.Tensor"      # float32 [nnz]
    n_beamlets: int

    @property
    def n_voxels(self):
        return int(self.indptr.numel() - 1)

    def dose(self, w, stream=None):
        """Eq. 1 by voxel rows: bit-reproducible dose of the beamlet weights w."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.values.device)
        d = torch.empty(self.n_voxels, dtype=torch.float32, device=self.values.device)
        L.fspb_voxel_dose(self.indptr.data_ptr(), self.indices.data_ptr(), self.values.data_ptr(), self.n_voxels,
                          self.n_beamlets, w.data_ptr(), d.data_ptr(), C.c_void_p(s.cuda_stream))
        return d


_ERF_FORMS = {None: 0, "compact": L.FSPB_ERF_COMPACT, "mirrored": L.FSPB_ERF_MIRRORED}
_TILES = {None: 0, "block": L.FSPB_TILES_BLOCK, "list": L.FSPB_TILES_LIST}


def _structs(problem, density_ptr, erf_form=None, tiles=None):
    g = problem.grid
    nz, ny, nx = g.density.shape
    grid = L.FspbGrid(nx, ny, nz, 0, (C.c_double * 3)(*g.spacing), (C.c_double * 3)(*g.origin),
                      C.c_void_p(density_ptr))
    beams = (L.FspbBeam * len(problem.beams))()
    for k, b in enumerate(problem.beams):
        beams[k] = L.FspbBeam(b.gantry_deg, (C.c_double * 3)(*b.isocenter), b.sad, b.beamlet_a,
                              b.beamlet_b, b.u0, b.v0, b.nu, b.nv)
    kp = problem.kernel
    pdd = np.ascontiguousarray(kp.pdd, dtype=np.float32)
    pad = lambda v: (C.c_double * 4)(*(list(v) + [0.0] * (4 - len(v))))
    kern = L.FspbKernel(kp.n_terms, len(pdd), pad(kp.weight), pad(kp.sigma0), pad(kp.sigma_slope),
                        pad(kp.width_scale), pdd.ctypes.data_as(C.POINTER(C.c_float)), kp.pdd_step,
                        kp.cutoff_u, kp.cutoff_v, kp.table_step, kp.rho_min,
                        (L.FSPB_DEPTH_TRILINEAR if kp.depth == "trilinear" else 0) | _ERF_FORMS[erf_form]
                        | _TILES[tiles])
    kt = getattr(kp, "tables", None)
    if kt is not None:
        arrs = [np.ascontiguousarray(x, dtype=np.float32) for x in (kt.c1, kt.c2, kt.c3, kt.A)]
        f = lambda a: a.ctypes.data_as(C.POINTER(C.c_float))
        tabs = L.FspbKernelTables(arrs[0].shape[1], arrs[3].shape[0], arrs[3].shape[1], 0, kt.depth_step,
                                  kt.theta_step, kt.adepth_step, f(arrs[0]), f(arrs[1]), f(arrs[2]), f(arrs[3]))
        tabs._keep = arrs                      # the host arrays must outlive the create call
        kern.tables = C.pointer(tabs)
        kern._keep = tabs
    return grid, beams, kern, pdd


def chunk_ranges(indptr, beam_rows, max_bytes, by_beam=True):
    """Beamlet ranges [j0, j1) covering all rows whose entries take at most
    ``max_bytes`` each (8 bytes per entry), given the host row pointers: the
    library's fspb_row_ranges.  With ``by_beam`` a range ends at a beam
    boundary where one fits (the paper computes a plan beam by beam on a small
    card); otherwise, or inside a beam too large for the budget, at a beamlet.
    A single row larger than the budget raises ValueError."""
    return L.fspb_row_ranges(indptr, beam_rows if by_beam else None, max_bytes)


class Plan:
    """One FSPB plan on a GPU.

    ``problem`` is a ``fspb_inputs.Problem`` (or anything with the same
    fields).  The density is copied to the device once; the plan borrows that
    tensor, and ``set_density`` may overwrite it in place (same shape) before
    the next ``raytrace``.  ``erf_form`` ("compact", "mirrored") forces the
    fill's erf table form; None lets plan creation choose it.  ``tiles``
    ("block", "list") forces how the fill walks every beamlet's VOI rows; None
    lets the count pass choose per beamlet.
    """

    def __init__(self, problem, device="cuda:0", density=None, erf_form=None, tiles=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        if density is None:
            density = torch.from_numpy(np.ascontiguousarray(problem.grid.density, dtype=np.float32))
        self.density = density.to(self.device, dtype=torch.float32).contiguous()
        grid, beams, kern, self._pdd = _structs(problem, self.density.data_ptr(), erf_form, tiles)
        st, _, need = L.fspb_plan_create(grid, beams, len(problem.beams), kern, None, 0)
        assert st == L.FSPB_ERR_CAPACITY
        self.workspace = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        st, handle, _ = L.fspb_plan_create(grid, beams, len(problem.beams), kern, aligned, need)
        self.handle = handle
        self.desc = L.fspb_plan_info(handle)
        self.n_beamlets = self.desc.n_beamlets
        self.n_voxels = self.desc.n_voxels
        self.indptr = torch.empty(self.n_beamlets + 1, dtype=torch.int64, device=self.device)
        self.indices = None
        self.values = None
        self.beam_rows = [int(b.nu) * int(b.nv) for b in problem.beams]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and L is not None and L.fspb_plan_destroy is not None:
            L.fspb_plan_destroy(h)
            self.handle = None

    def _stream(self, stream):
        s = stream if stream is not None else self.torch.cuda.current_stream(self.device)
        return C.c_void_p(s.cuda_stream)

    def set_density(self, density):
        self.density.copy_(density)

    def raytrace(self, stream=None):
        L.fspb_raytrace(self.handle, self._stream(stream))

    def dose_coeffs(self, stream=None):
        """Count, size the outputs (grown when needed) and fill; returns nnz."""
        s = self._stream(stream)
        cap = 0 if self.indices is None else self.indices.numel()
        st, nnz = L.fspb_dose_coeffs(self.handle, self.indptr.data_ptr(),
                                     self.indices.data_ptr() if cap else None,
                                     self.values.data_ptr() if cap else None, cap, s)
        if st == L.FSPB_ERR_CAPACITY:
            self.indices = self.torch.empty(max(nnz, 1), dtype=self.torch.int32, device=self.device)
            self.values = self.torch.empty(max(nnz, 1), dtype=self.torch.float32, device=self.device)
            st, nnz = L.fspb_dose_coeffs(self.handle, self.indptr.data_ptr(),
                                         self.indices.data_ptr(), self.values.data_ptr(),
                                         self.indices.numel(), s)
        self.nnz = nnz
        return nnz

    def compute(self, stream=None):
        self.raytrace(stream)
        nnz = self.dose_coeffs(stream)
        return CSR(self.indptr, self.indices[:nnz], self.values[:nnz], self.n_voxels)

    def count(self, stream=None):
        """Trace and count only: fills ``self.indptr`` (all rows) and returns nnz; no entries."""
        self.raytrace(stream)
        st, nnz = L.fspb_dose_coeffs(self.handle, self.indptr.data_ptr(), None, None, 0, self._stream(stream))
        self.nnz = nnz
        return nnz

    def compute_rows(self, j0, j1, indices=None, values=None, stream=None):
        """Rows j0..j1-1 of D after ``count``: a CSR whose columns are voxels and
        whose rows are those beamlets (row pointers start at 0).  ``indices`` /
        ``values`` may be caller buffers of at least the rows' nnz entries."""
        s = self._stream(stream)
        st, n = L.fspb_dose_coeffs_rows(self.handle, j0, j1, self.indptr.data_ptr(), None, None, 0, s)
        if indices is None or indices.numel() < n:
            indices = self.torch.empty(max(n, 1), dtype=self.torch.int32, device=self.device)
            values = self.torch.empty(max(n, 1), dtype=self.torch.float32, device=self.device)
        L.fspb_dose_coeffs_rows(self.handle, j0, j1, self.indptr.data_ptr(), indices.data_ptr(),
                                values.data_ptr(), indices.numel(), s)
        ip = self.indptr[j0:j1 + 1] - self.indptr[j0]
        return CSR(ip, indices[:n], values[:n], self.n_voxels)

    def row_chunks(self, max_bytes, by_beam=True):
        """Beamlet ranges of at most ``max_bytes`` of entries, after ``count``
        (see ``chunk_ranges``)."""
        return chunk_ranges(self.indptr.cpu().numpy(), self.beam_rows, max_bytes, by_beam)

    def chunks(self, max_bytes, by_beam=True, stream=None):
        """Yield (j0, j1, CSR) covering D in pieces of at most ``max_bytes`` of
        entries; the pieces share one buffer, so each is overwritten by the next."""
        self.count(stream)
        ranges = self.row_chunks(max_bytes, by_beam)
        per = self.indptr.cpu().numpy()
        biggest = max([per[b] - per[a] for a, b in ranges] + [1])
        idx = self.torch.empty(int(biggest), dtype=self.torch.int32, device=self.device)
        val = self.torch.empty(int(biggest), dtype=self.torch.float32, device=self.device)
        for a, b in ranges:
            yield a, b, self.compute_rows(a, b, idx, val, stream)

    def set_surrogate(self, sur):
        """Attach a trained ``Surrogate`` (None: analytic fill)."""
        L.fspb_plan_set_surrogate(self.handle, sur.handle if sur is not None else None)
        self._surrogate = sur

    def tables(self, stream=None):
        """Depth tables copied to host: (float32 values, int64 offsets)."""
        tab = np.zeros(max(int(self.desc.table_entries), 1), dtype=np.float32)
        off = np.zeros(self.n_beamlets + 1, dtype=np.int64)
        L.fspb_plan_get_tables(self.handle, tab.ctypes.data, off.ctypes.data, self._stream(stream))
        return tab[:int(self.desc.table_entries)], off


class Batch:
    """Many plans computed by one captured graph of persistent kernels.

    ``plans`` are ``Plan`` objects on the same device; they must outlive the
    batch.  Outputs are allocated from the sizing pass and bound at creation.
    """

    def __init__(self, plans, stream=None):
        torch = plans[0].torch
        self.torch = torch
        self.plans = list(plans)
        self.device = plans[0].device
        s = self._stream(stream)
        handles = [p.handle for p in self.plans]
        st, _, need = L.fspb_batch_create(handles, None, 0, s)
        assert st == L.FSPB_ERR_CAPACITY
        self.workspace = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        st, self.handle, _ = L.fspb_batch_create(handles, aligned, need, s)
        self.nnz = [L.fspb_batch_nnz(self.handle, i) for i in range(len(self.plans))]
        self.indptr, self.indices, self.values = [], [], []
        for i, p in enumerate(self.plans):
            ip = torch.empty(p.n_beamlets + 1, dtype=torch.int64, device=self.device)
            ix = torch.empty(max(self.nnz[i], 1), dtype=torch.int32, device=self.device)
            vv = torch.empty(max(self.nnz[i], 1), dtype=torch.float32, device=self.device)
            L.fspb_batch_bind(self.handle, i, ip.data_ptr(), ix.data_ptr(), vv.data_ptr(), ix.numel())
            self.indptr.append(ip)
            self.indices.append(ix)
            self.values.append(vv)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and L is not None and L.fspb_batch_destroy is not None:
            L.fspb_batch_destroy(h)
            self.handle = None

    def _stream(self, stream):
        s = stream if stream is not None else self.torch.cuda.current_stream(self.device)
        return C.c_void_p(s.cuda_stream)

    def tune(self, stream=None):
        L.fspb_batch_tune(self.handle, self._stream(stream))
        return self.config()

    def config(self):
        return L.fspb_batch_get_config(self.handle)

    def set_config(self, waves_per_group, groups_per_cu, order, tile_rows=64, beamlets_per_item=1):
        L.fspb_batch_set_config(self.handle, waves_per_group, groups_per_cu, order, tile_rows, beamlets_per_item)

    def run(self, stream=None):
        L.fspb_batch_run(self.handle, self._stream(stream))

    def check(self, stream=None):
        return L.fspb_batch_check(self.handle, self._stream(stream))

    def outputs(self):
        return [CSR(self.indptr[i], self.indices[i][:self.nnz[i]], self.values[i][:self.nnz[i]],
                    p.n_voxels) for i, p in enumerate(self.plans)]


def _kernel_struct(kp):
    pdd = np.ascontiguousarray(kp.pdd, dtype=np.float32)
    pad = lambda v: (C.c_double * 4)(*(list(v) + [0.0] * (4 - len(v))))
    k = L.FspbKernel(kp.n_terms, len(pdd), pad(kp.weight), pad(kp.sigma0), pad(kp.sigma_slope),
                     pad(kp.width_scale), pdd.ctypes.data_as(C.POINTER(C.c_float)), kp.pdd_step,
                     kp.cutoff_u, kp.cutoff_v, kp.table_step, kp.rho_min, 0)
    return k, pdd


class Surrogate:
    """Learned kernel surrogate on the GPU (4 -> 64 -> 64 -> 1 SiLU perceptron)."""

    def __init__(self, kernel_params, init_params, max_batch=16384, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        k, self._pdd = _kernel_struct(kernel_params)
        st, _, need = L.fspb_surrogate_create(k, init_params, max_batch, None, 0)
        self.workspace = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        st, self.handle, _ = L.fspb_surrogate_create(k, init_params, max_batch, aligned, need)
        self.max_batch = max_batch

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and L is not None and L.fspb_surrogate_destroy is not None:
            L.fspb_surrogate_destroy(h)
            self.handle = None

    def _stream(self, stream=None):
        s = stream if stream is not None else self.torch.cuda.current_stream(self.device)
        return C.c_void_p(s.cuda_stream)

    def targets(self, samples):
        """samples: device float32 [n, 4] (d, u, v, a) -> (features [n, 4], targets [n])."""
        n = samples.shape[0]
        f = self.torch.empty((n, 4), dtype=self.torch.float32, device=self.device)
        t = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        L.fspb_surrogate_targets(self.handle, samples.data_ptr(), n, f.data_ptr(), t.data_ptr(), self._stream())
        return f, t

    def forward(self, features):
        n = features.shape[0]
        out = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        L.fspb_surrogate_forward(self.handle, features.data_ptr(), n, out.data_ptr(), self._stream())
        return out

    def gradient(self, features, targets):
        g = self.torch.empty(L.SURROGATE_PARAMS, dtype=self.torch.float32, device=self.device)
        loss = L.fspb_surrogate_gradient(self.handle, features.data_ptr(), targets.data_ptr(),
                                         features.shape[0], g.data_ptr(), self._stream())
        return g, loss

    def train(self, features, targets, epochs, batch=8192, lr_max=3e-3, lr_min=1e-5, seed=0,
              beta1=0.9, beta2=0.999, eps=1e-8):
        cfg = L.FspbTrainConfig(epochs, batch, lr_max, lr_min, beta1, beta2, eps, 0, seed)
        return L.fspb_surrogate_train(self.handle, features.data_ptr(), targets.data_ptr(),
                                      features.shape[0], cfg, self._stream())

    def get_params(self):
        return L.fspb_surrogate_get_params(self.handle, self._stream())

    def set_params(self, params):
        L.fspb_surrogate_set_params(self.handle, params)
