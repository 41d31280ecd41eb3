"""Voxel-row transpose of D and the voxel-row dose (Eq. 1) on the GPU.

* seeded random CSR matrices: bit-exact against the oracle's transpose (one,
  two and three radix passes, several sort tiles with a ragged tail, empty
  rows and columns, nnz = 0, one column);
* entries with an out-of-range column are left out (both sort paths), the
  valid ones transposed exactly;
* the transpose runs without host synchronisation: captured in a HIP graph
  and replayed, interleaved with eager work, it gives the eager result;
* a plan's D: the voxel-row dose against the oracle's FP64 Eq. 1, and the
  transposed entries against the beamlet-row CSR they came from (same
  triples, beamlets ascending in every voxel row).
"""
import numpy as np
import pytest

import fspb_inputs as fi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _csr(torch, indptr, indices, values, n_cols):
    from paper_0908_4417_amd import CSR
    dev = "cuda:0"
    return CSR(torch.from_numpy(indptr).to(dev), torch.from_numpy(indices).to(dev),
               torch.from_numpy(values).to(dev), n_cols)


@pytest.mark.parametrize("seed,n_rows,n_cols,mean_row", [
    (1, 50, 200, 17.0),          # one pass, < one tile
    (2, 700, 5000, 90.0),        # two passes, ~16 tiles
    (3, 300, 70000, 400.0),      # three passes, ~30 tiles
    (4, 64, 1, 0.7),             # a single column
])
def test_random_matrix_matches_oracle(torch_gpu, oracle_lib, seed, n_rows, n_cols, mean_row):
    torch = torch_gpu
    indptr, indices, values = fi.random_csr(seed, n_rows, n_cols, mean_row)
    print(f"\n  case seed={seed} rows={n_rows} cols={n_cols} nnz={len(indices)}", flush=True)
    t = _csr(torch, indptr, indices, values, n_cols).transpose()
    torch.cuda.synchronize()
    ep, ei, ev = oracle_lib.csr_transpose(indptr, indices, values, n_cols)
    np.testing.assert_array_equal(t.indptr.cpu().numpy(), ep)
    np.testing.assert_array_equal(t.indices.cpu().numpy(), ei)
    np.testing.assert_array_equal(t.values.cpu().numpy(), ev)
    # voxel-row dose vs the definition in FP64
    w = np.random.default_rng(seed).uniform(size=n_rows).astype(np.float32)
    d = t.dose(torch.from_numpy(w).to("cuda:0")).cpu().numpy().astype(np.float64)
    vox = np.repeat(np.arange(n_cols), np.diff(ep))
    ref = np.bincount(vox, weights=ev.astype(np.float64) * w[ei].astype(np.float64), minlength=n_cols)
    assert np.max(np.abs(d - ref)) <= 4e-6 * max(ref.max(), 1e-30)


@pytest.mark.parametrize("seed,mode", [(6, "reversed runs"), (7, "repeated columns"), (8, "shuffled rows")])
def test_unsorted_rows_match_oracle(torch_gpu, oracle_lib, seed, mode):
    """Rows whose columns are not strictly ascending: the transpose is still the stable sort
    of the row-major entries by column.  Reversing each stretch of a row within one 32-column
    bucket keeps the stretches long (bucket placement for unsorted rows); shuffling whole rows
    makes them short (radix sort)."""
    torch = torch_gpu
    indptr, indices, values = fi.random_csr(seed, 400, 6000, 120.0)
    rng = np.random.default_rng(seed)
    for j in range(len(indptr) - 1):
        a, b = int(indptr[j]), int(indptr[j + 1])
        if mode == "shuffled rows":
            p = rng.permutation(b - a)
            indices[a:b] = indices[a:b][p]
            values[a:b] = values[a:b][p]
            continue
        cut = [a] + [e for e in range(a + 1, b) if indices[e] >> 5 != indices[e - 1] >> 5] + [b]
        for s0, s1 in zip(cut[:-1], cut[1:]):
            if mode == "reversed runs":
                indices[s0:s1] = indices[s0:s1][::-1].copy()
                values[s0:s1] = values[s0:s1][::-1].copy()
            elif s1 - s0 >= 2:
                indices[s0 + 1] = indices[s0]
    print(f"\n  {mode}: seed={seed} nnz={len(indices)}", flush=True)
    t = _csr(torch, indptr, indices, values, 6000).transpose()
    torch.cuda.synchronize()
    ep, ei, ev = oracle_lib.csr_transpose(indptr, indices, values, 6000)
    np.testing.assert_array_equal(t.indptr.cpu().numpy(), ep)
    np.testing.assert_array_equal(t.indices.cpu().numpy(), ei)
    np.testing.assert_array_equal(t.values.cpu().numpy(), ev)


def test_empty_and_invalid(torch_gpu):
    torch = torch_gpu
    indptr = np.zeros(6, dtype=np.int64)
    t = _csr(torch, indptr, np.zeros(0, np.int32), np.zeros(0, np.float32), 9).transpose()
    assert t.indptr.cpu().numpy().tolist() == [0] * 10 and t.indices.numel() == 0
    d = t.dose(torch.ones(5, device="cuda:0")).cpu().numpy()
    assert np.all(d == 0.0)
    bad = _csr(torch, np.array([0, 3], np.int64), np.array([1, 9, -4], np.int32),
               np.array([2.0, 3.0, 4.0], np.float32), 9).transpose()
    ip = bad.indptr.cpu().numpy()
    assert ip[-1] == 1 and ip[1] == 0 and ip[2] == 1                  # only column 1 is kept
    assert int(bad.indices[0]) == 0 and float(bad.values[0]) == 2.0


@pytest.mark.parametrize("seed,mean_row,mode", [(11, 120.0, "runs"), (12, 40.0, "entries")])
def test_invalid_columns_are_left_out(torch_gpu, oracle_lib, seed, mean_row, mode):
    """Columns outside [0, n_voxels) (negative or too large) sprinkled over a matrix whose
    stretches are long (run path) or short (rows shuffled: entry path): the result is the
    transpose of the valid entries."""
    torch = torch_gpu
    n_cols = 3000
    indptr, indices, values = fi.random_csr(seed, 300, n_cols, mean_row)
    rng = np.random.default_rng(seed)
    if mode == "entries":
        for j in range(len(indptr) - 1):
            a, b = int(indptr[j]), int(indptr[j + 1])
            p = rng.permutation(b - a)
            indices[a:b], values[a:b] = indices[a:b][p], values[a:b][p]
    bad = rng.uniform(size=len(indices)) < 0.03
    indices[bad] = np.where(rng.uniform(size=int(bad.sum())) < 0.5, -1 - rng.integers(0, 50, int(bad.sum())),
                            n_cols + rng.integers(0, 5000, int(bad.sum()))).astype(np.int32)
    print(f"\n  {mode}: nnz={len(indices)} invalid={int(bad.sum())}", flush=True)
    t = _csr(torch, indptr, indices, values, n_cols).transpose()
    torch.cuda.synchronize()
    keep = ~bad
    rows = np.repeat(np.arange(len(indptr) - 1), np.diff(indptr))[keep]
    vp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=len(indptr) - 1))]).astype(np.int64)
    ep, ei, ev = oracle_lib.csr_transpose(vp, indices[keep], values[keep], n_cols)
    np.testing.assert_array_equal(t.indptr.cpu().numpy(), ep)
    n = int(ep[-1])
    np.testing.assert_array_equal(t.indices[:n].cpu().numpy(), ei)
    np.testing.assert_array_equal(t.values[:n].cpu().numpy(), ev)


def test_graph_captured_transpose(torch_gpu, oracle_lib):
    """fspb_csr_transpose enqueues only kernels and reads no device value on the host, so it
    can be captured; replays interleaved with eager work equal the eager result each time."""
    torch = torch_gpu
    import ctypes as C
    import paper_0908_4417_amd as m
    n_cols = 20000
    indptr, indices, values = fi.random_csr(13, 500, n_cols, 300.0)
    csr = _csr(torch, indptr, indices, values, n_cols)
    ref = csr.transpose()
    torch.cuda.synchronize()
    nnz = len(indices)
    _, need = m.fspb_csr_transpose(None, None, None, 500, n_cols, nnz, None, None, None, None, 0, C.c_void_p(0))
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda:0")
    wsp = (ws.data_ptr() + 255) // 256 * 256
    tp = torch.full((n_cols + 1,), -1, dtype=torch.int64, device="cuda:0")
    ti = torch.full((nnz,), -1, dtype=torch.int32, device="cuda:0")
    tv = torch.full((nnz,), -1.0, dtype=torch.float32, device="cuda:0")
    side = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        m.fspb_csr_transpose(csr.indptr.data_ptr(), csr.indices.data_ptr(), csr.values.data_ptr(), 500, n_cols, nnz,
                             tp.data_ptr(), ti.data_ptr(), tv.data_ptr(), wsp, need,
                             C.c_void_p(side.cuda_stream))
    for rep in range(3):
        tp.fill_(-1)
        ti.fill_(-1)
        tv.fill_(-1.0)
        torch.randn(1 << 20, device="cuda:0").sum().item()            # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(tp, ref.indptr) and torch.equal(ti, ref.indices), rep
        assert torch.equal(tv.view(torch.int32), ref.values.view(torch.int32)), rep


def test_plan_voxel_rows(torch_gpu, oracle_lib):
    torch = torch_gpu
    from paper_0908_4417_amd import Plan
    g = fi.slab_phantom(21, n=(40, 38, 26), spacing=(0.5, 0.5, 0.5), lung_side=(3, 6), bone_side=(1, 2))
    prob = fi.Problem("vt", g, fi.coplanar_beams(4, (0.11, -0.05, 0.07), 100.0, 1.0, 1.0, 5, 4),
                      fi.default_kernel(21))
    plan = Plan(prob, "cuda:0")
    csr = plan.compute()
    t = csr.transpose()
    rng = np.random.default_rng(8)
    w = rng.uniform(0.0, 2.0, plan.n_beamlets).astype(np.float32)
    wd = torch.from_numpy(w).to("cuda:0")
    d = t.dose(wd).cpu().numpy().astype(np.float64)
    d_atomic = csr.dose(wd).cpu().numpy().astype(np.float64)
    ref = oracle_lib.OraclePlan(prob).fluence_dose(w.astype(np.float64))
    assert np.max(np.abs(d - ref)) <= 1e-5 * ref.max()
    assert np.max(np.abs(d - d_atomic)) <= 1e-6 * ref.max()
    np.testing.assert_array_equal(t.dose(wd).cpu().numpy(), d.astype(np.float32))   # bit-reproducible
    # the same (voxel, beamlet, value) triples, beamlets ascending per voxel row
    ip, ix, vv = csr.indptr.cpu().numpy(), csr.indices.cpu().numpy(), csr.values.cpu().numpy()
    tp, ti, tv = t.indptr.cpu().numpy(), t.indices.cpu().numpy(), t.values.cpu().numpy()
    rows = np.repeat(np.arange(plan.n_beamlets), np.diff(ip))
    vox = np.repeat(np.arange(plan.n_voxels), np.diff(tp))
    a = np.lexsort((rows, ix))
    np.testing.assert_array_equal(vox, ix[a])
    np.testing.assert_array_equal(ti, rows[a])
    np.testing.assert_array_equal(tv, vv[a])
