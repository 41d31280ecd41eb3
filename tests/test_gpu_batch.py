"""Batched plans in one captured graph of persistent kernels (through the C ABI).

* every plan's CSR from the batch equals, bit for bit, the same plan computed
  on its own (each D_ij is computed independently, so tiling and scheduling
  must not change any bit);
* graph replays, interleaved with unrelated eager GPU work, give identical
  results each time;
* every launch shape (waves per group, groups per CU, queue order) and the
  tuner's choice give identical results;
* rows agree with the FP64 oracle (all rows of the small batch, at least 10 %
  of every plan's rows at full size);
* plans with a surrogate attached are refused, and a batched plan refuses one;
* a density change that adds nonzeros after sizing is reported as OVERFLOW.
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


def _say(msg):
    print(msg, flush=True)


def _equal(torch, a, b):
    return (torch.equal(a.indptr, b.indptr) and torch.equal(a.indices, b.indices)
            and torch.equal(a.values.view(torch.int32), b.values.view(torch.int32)))


def _single(prob):
    from paper_0908_4417_amd import Plan
    p = Plan(prob, "cuda:0")
    c = p.compute()
    return p, c


def test_small_batch_equals_single_plans(torch_gpu, oracle_lib):
    import torch
    from paper_0908_4417_amd import Plan, Batch
    probs = fi.batched_configs(n_plans=6, scale=0.3)
    _say("batch: 6 plans at 0.3 scale: " + ", ".join(p.name for p in probs))
    plans = [Plan(p, "cuda:0") for p in probs]
    batch = Batch(plans)
    batch.run()
    torch.cuda.synchronize()
    assert batch.check() == 0
    outs = [(o.indptr.clone(), o.indices.clone(), o.values.clone()) for o in batch.outputs()]
    # single-plan path on separate Plan objects (the batch's plans share workspaces with it)
    for k, prob in enumerate(probs):
        _, c = _single(prob)
        got = batch.outputs()[k]
        assert batch.nnz[k] == c.nnz
        assert _equal(torch, got, c), f"plan {k} differs from its single-plan result"
    # replays with eager work in between
    for rep in range(3):
        _single(probs[rep])                       # unrelated eager work on the device
        torch.randn(1 << 20, device="cuda:0").sum().item()
        batch.run()
        torch.cuda.synchronize()
        for k, o in enumerate(batch.outputs()):
            assert torch.equal(o.indices, outs[k][1]) and torch.equal(o.values, outs[k][2]), (rep, k)
    # every launch shape gives the same bits
    for w, g, order, rows, per in [(2, 1, 1, 64, 1), (8, 8, 0, 128, 2), (4, 2, 1, 256, 4), (4, 4, 0, 128, 1),
                                   (2, 4, 0, 64, 4)]:
        batch.set_config(w, g, order, rows, per)
        batch.run()
        torch.cuda.synchronize()
        for k, o in enumerate(batch.outputs()):
            assert torch.equal(o.indices, outs[k][1]), (w, g, order, rows, per, k)
            assert torch.equal(o.values, outs[k][2]), (w, g, order, rows, per, k)
    cfg = batch.tune()
    _say(f"  tuned: waves/group={cfg.waves_per_group} groups/CU={cfg.groups_per_cu} order={cfg.order} "
         f"tile rows={cfg.tile_rows} beamlets/item={cfg.beamlets_per_item} fill={cfg.fill_ms:.3f} ms")
    assert cfg.tile_rows in (64, 128, 256) and cfg.beamlets_per_item in (1, 2, 4)
    assert cfg.tuned == 1
    batch.run()
    torch.cuda.synchronize()
    for k, o in enumerate(batch.outputs()):
        assert torch.equal(o.values, outs[k][2])
    # every row of every plan against the oracle
    for k, prob in enumerate(probs):
        ora = oracle_lib.OraclePlan(prob)
        r = compare_plan(ora, batch.outputs()[k])
        _say(f"  plan {k}: nnz={batch.nnz[k]} rows={r['rows']} max_rel={r['max_rel']:.2e} "
             f"band={r['band_mismatches']}")


def test_full_size_batch_sampled(torch_gpu, oracle_lib):
    """32 plans of uneven size at full size, one graph launch; a seeded 10 % of
    every plan's rows (at least 8) against the oracle."""
    import torch
    from paper_0908_4417_amd import Plan, Batch
    probs = fi.batched_configs(n_plans=32)
    plans = [Plan(p, "cuda:0") for p in probs]
    batch = Batch(plans)
    total = sum(batch.nnz)
    _say(f"batch: 32 plans, {sum(p.n_beamlets for p in plans)} beamlets, {total} nonzeros")
    batch.run()
    batch.run()
    torch.cuda.synchronize()
    assert batch.check() == 0
    worst, rows_done, n_done, band = 0.0, 0, 0, 0
    for k, prob in enumerate(probs):
        ora = oracle_lib.OraclePlan(prob)
        rng = np.random.default_rng(1000 + k)
        n_pick = min(ora.n_beamlets, max(8, -(-ora.n_beamlets // 10)))
        rows = np.sort(rng.choice(ora.n_beamlets, n_pick, replace=False))
        r = compare_plan(ora, batch.outputs()[k], rows=rows)
        assert r["rows"] * 10 >= ora.n_beamlets
        worst = max(worst, r["max_rel"])
        rows_done += r["rows"]
        n_done += r["n"]
        band += r["band_mismatches"]
    _say(f"  {rows_done} rows, {n_done} entries compared: worst max_rel {worst:.2e}, band {band}")
    # two plans checked bit for bit against their single-plan runs
    for k in (0, 31):
        _, c = _single(probs[k])
        assert _equal(torch, batch.outputs()[k], c)


def test_batch_overflow_is_reported(torch_gpu):
    import torch
    from paper_0908_4417_amd import Plan, Batch
    g = fi.water_phantom((30, 30, 20), (0.5, 0.5, 0.5))
    g.density[:, :, ::2] = 0.0                       # half the voxels masked out at sizing time
    prob = fi.Problem("ovf", g, fi.coplanar_beams(2, (0.1, 0.0, 0.05), 100.0, 1.0, 1.0, 3, 3),
                      fi.default_kernel(1))
    plan = Plan(prob, "cuda:0")
    other = Plan(fi.Problem("ok", fi.water_phantom((20, 20, 20), (0.5, 0.5, 0.5)),
                            fi.coplanar_beams(1, (0.1, 0.0, 0.05), 100.0, 1.0, 1.0, 2, 2),
                            fi.default_kernel(1)), "cuda:0")
    batch = Batch([other, plan])
    batch.run()
    assert batch.check() == 0
    n0 = batch.nnz[1]
    plan.set_density(torch.ones_like(plan.density))  # now every voxel is a member
    batch.run()
    import paper_0908_4417_amd as m
    assert batch.check() == m.FSPB_ERR_OVERFLOW
    # entries up to the capacity are intact, the indptr reports the new count
    assert int(batch.indptr[1][-1]) > n0
    assert batch.check() == 0                          # flags were cleared


def test_batch_and_surrogate_exclude_each_other(torch_gpu):
    """A batch computes Eq. 2-3 analytically: a plan with a surrogate attached is
    refused at creation, and a plan held by a live batch refuses a surrogate."""
    import paper_0908_4417_amd as m
    from paper_0908_4417_amd import Plan, Batch, Surrogate
    prob = fi.Problem("bs", fi.water_phantom((20, 20, 16), (0.5, 0.5, 0.5)),
                      fi.coplanar_beams(1, (0.1, 0.0, 0.05), 100.0, 0.5, 0.5, 2, 2), fi.default_kernel(3))
    sur = Surrogate(prob.kernel, fi.surrogate_init(3), max_batch=1024)
    a, b = Plan(prob, "cuda:0"), Plan(prob, "cuda:0")
    a.set_surrogate(sur)
    with pytest.raises(m.FspbError, match="surrogate attached"):
        Batch([b, a])
    batch = Batch([b])
    with pytest.raises(m.FspbError, match="batch"):
        b.set_surrogate(sur)
    del batch                                         # the plan leaves its only batch
    import gc
    gc.collect()
    b.set_surrogate(sur)
    a.set_surrogate(None)
    Batch([a])
