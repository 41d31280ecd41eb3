"""D computed in row ranges (the paper's beam-at-a-time mode for small cards).

* the pieces of ``Plan.chunks`` put together equal the one-shot CSR bit for bit,
  for whole-beam and beamlet-level budgets, and every piece's rows match the
  FP64 oracle (also on the full-size 128^3 slab under a one-beam budget);
* state and argument errors of fspb_dose_coeffs_rows.
"""
import os
import sys

import numpy as np
import pytest

import fspb_inputs as fi

sys.path.insert(0, os.path.dirname(__file__))
from parity import compare_plan  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _problem():
    g = fi.slab_phantom(61, n=(48, 44, 32), spacing=(0.5, 0.5, 0.5), lung_side=(3, 8), bone_side=(1, 3))
    return fi.Problem("chunks", g, fi.coplanar_beams(5, (0.11, -0.07, 0.13), 100.0, 1.0, 1.0, 6, 5),
                      fi.default_kernel(61))


def _piece_against_oracle(ora, plan, j0, j1, c):
    """Rows j0..j1-1 of a piece (row pointers from 0) against the oracle's rows."""
    from paper_0908_4417_amd import CSR
    ip = plan.torch.zeros(plan.n_beamlets + 1, dtype=plan.torch.int64, device=plan.device)
    ip[j0:j1 + 1] = c.indptr
    ip[j1 + 1:] = c.indptr[-1]
    return compare_plan(ora, CSR(ip, c.indices, c.values, plan.n_voxels), rows=np.arange(j0, j1))


@pytest.mark.parametrize("frac,by_beam", [(0.45, True), (0.1, True), (0.07, False)])
def test_chunks_equal_one_shot(torch_gpu, oracle_lib, frac, by_beam):
    torch = torch_gpu
    from paper_0908_4417_amd import Plan
    plan = Plan(_problem(), "cuda:0")
    full = plan.compute()
    ip, ix, vv = full.indptr.clone(), full.indices.clone(), full.values.clone()
    budget = int(8 * full.nnz * frac)
    ora = oracle_lib.OraclePlan(_problem())
    got_i, got_v, ranges = [], [], []
    for j0, j1, c in plan.chunks(budget, by_beam=by_beam):
        assert 8 * c.nnz <= budget
        torch.testing.assert_close(c.indptr, ip[j0:j1 + 1] - ip[j0], rtol=0, atol=0)
        r = _piece_against_oracle(ora, plan, j0, j1, c)
        assert r["rows"] == j1 - j0
        got_i.append(c.indices.clone())
        got_v.append(c.values.clone())
        ranges.append((j0, j1))
    print(f"\n  budget {budget} B: {len(ranges)} pieces {ranges}", flush=True)
    assert ranges[0][0] == 0 and ranges[-1][1] == plan.n_beamlets
    assert torch.equal(torch.cat(got_i), ix) and torch.equal(torch.cat(got_v), vv)
    if by_beam and frac > 0.3:
        assert all(b % 30 == 0 for _, b in ranges)          # whole beams of 30 beamlets


def test_rows_errors(torch_gpu):
    import paper_0908_4417_amd as m
    from paper_0908_4417_amd import Plan
    plan = Plan(_problem(), "cuda:0")
    plan.raytrace()
    with pytest.raises(m.FspbError, match="count"):
        plan.compute_rows(0, 3)
    nnz = plan.count()
    with pytest.raises(m.FspbError, match="range"):
        plan.compute_rows(5, 2)
    with pytest.raises(m.FspbError, match="range"):
        plan.compute_rows(0, plan.n_beamlets + 1)
    s = plan._stream(None)
    st, n = m.fspb_dose_coeffs_rows(plan.handle, 0, plan.n_beamlets, plan.indptr.data_ptr(), None, None, 0, s)
    assert st == m.FSPB_ERR_CAPACITY and n == nnz
    empty = plan.compute_rows(4, 4)
    assert empty.nnz == 0
    plan.raytrace()                                          # a new trace invalidates the counts
    with pytest.raises(m.FspbError, match="count"):
        plan.compute_rows(0, 1)


def test_full_size_slab_by_beam_against_oracle(torch_gpu, oracle_lib):
    """The 128^3 slab (9 beams) under a one-beam budget: ten pieces, every row of
    every piece against the oracle."""
    from paper_0908_4417_amd import Plan
    prob = fi.make_config(1)
    plan = Plan(prob, "cuda:0")
    nnz = plan.count()
    budget = int(8 * nnz / len(prob.beams) * 1.05)
    ora = oracle_lib.OraclePlan(prob)
    worst, rows, pieces = 0.0, 0, 0
    for j0, j1, c in plan.chunks(budget):
        r = _piece_against_oracle(ora, plan, j0, j1, c)
        worst = max(worst, r["max_rel"])
        rows += r["rows"]
        pieces += 1
    assert rows == plan.n_beamlets and pieces >= len(prob.beams)
    print(f"\n  {pieces} pieces of at most {budget} B, {rows} rows: max_rel {worst:.2e}", flush=True)
