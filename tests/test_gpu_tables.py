"""Eq. 2-3 in their general form on the GPU (depth-tabulated c1, c2, c3 and A(theta, d)).

* a seeded three-term kernel with depth-dependent c's and an off-axis A:
  full D against the FP64 oracle (the usual parity bar);
* the analytic kernel written as tables gives the analytic fill's D;
* plans with tables are refused by batches and by the surrogate.
"""
import dataclasses
import os
import sys

import numpy as np
import pytest

import fspb_inputs as fi

sys.path.insert(0, os.path.dirname(__file__))
from parity import compare_rows, gpu_rows_from_csr  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _grid(seed=71):
    return fi.slab_phantom(seed, n=(44, 40, 30), spacing=(0.5, 0.5, 0.5), lung_side=(3, 8), bone_side=(1, 3))


def _beams():
    # a wide field so that the beamlets span several rows of the A table (theta up to ~0.05 rad)
    return fi.coplanar_beams(3, (0.11, -0.07, 0.13), 100.0, 1.0, 1.0, 9, 7)


@pytest.mark.parametrize("depth", ["siddon", "trilinear"])
def test_tabulated_kernel_parity(torch_gpu, oracle_lib, depth):
    from paper_0908_4417_amd import Plan
    k = fi.default_kernel(71)
    kt = dataclasses.replace(k, weight=[0.0] * 3, sigma0=[1.0] * 3, sigma_slope=[0.0] * 3,
                             width_scale=[1.0] * 3, depth=depth, tables=fi.synthetic_tables(71, k))
    prob = fi.Problem("tab", _grid(), _beams(), kt)
    plan = Plan(prob, "cuda:0")
    csr = plan.compute()
    ora = oracle_lib.OraclePlan(prob)
    thetas = [b.theta for b in ora.beamlets]
    off, oidx, oval = ora.full()
    rows = list(range(ora.n_beamlets))
    r = compare_rows(ora, rows, gpu_rows_from_csr(csr, rows),
                     [(oidx[off[j]:off[j + 1]], oval[off[j]:off[j + 1]]) for j in rows])
    print(f"\n  {depth}: nnz={csr.nnz} theta max {max(thetas):.3f} rad max_rel={r['max_rel']:.2e} "
          f"eps={r['eps']:.2e} band={r['band_mismatches']}", flush=True)
    assert max(thetas) > 0.025                     # more than one interval of the A table is used


def test_analytic_tables_match_the_analytic_fill(torch_gpu):
    import torch
    from paper_0908_4417_amd import Plan
    k = fi.default_kernel(72)
    a = Plan(fi.Problem("a", _grid(72), _beams(), k), "cuda:0").compute()
    ai, av = a.indices.clone(), a.values.double().clone()
    kt = dataclasses.replace(k, tables=fi.analytic_tables(k, n_theta=2))
    b = Plan(fi.Problem("b", _grid(72), _beams(), kt), "cuda:0").compute()
    assert torch.equal(ai, b.indices)
    rel = ((b.values.double() - av).abs() / av.abs().max()).max().item()
    print(f"\n  analytic tables vs analytic fill: max |dD| = {rel:.2e} of max D", flush=True)
    assert rel < 2e-6


def test_tables_refused_by_batch_and_surrogate(torch_gpu):
    import paper_0908_4417_amd as m
    from paper_0908_4417_amd import Plan, Batch, Surrogate
    k = fi.default_kernel(73)
    kt = dataclasses.replace(k, tables=fi.analytic_tables(k))
    plan = Plan(fi.Problem("t", _grid(73), _beams(), kt), "cuda:0")
    with pytest.raises(m.FspbError, match="tables"):
        Batch([plan])
    sur = Surrogate(k, fi.surrogate_init(1), max_batch=1024)
    with pytest.raises(m.FspbError, match="tables"):
        plan.set_surrogate(sur)


@pytest.mark.parametrize("n_terms,n_theta,n_depth", [(1, 1, 2), (4, 3, 17)])
def test_tabulated_kernel_shapes(torch_gpu, oracle_lib, n_terms, n_theta, n_depth):
    """One and four terms, a single A row, the shortest c table."""
    from paper_0908_4417_amd import Plan
    k = fi.default_kernel(74)
    rng = np.random.default_rng(n_terms)
    d_end = 30.0
    step = d_end / (n_depth - 1)
    d = np.arange(n_depth) * step
    c1 = (rng.uniform(0.2, 1.0, (n_terms, 1)) * (1.0 + 0.01 * d[None, :])).astype(np.float32)
    c2 = np.full((n_terms, n_depth), 1.0, dtype=np.float32) + rng.uniform(0, 0.1, (n_terms, 1)).astype(np.float32)
    c3 = (rng.uniform(0.15, 1.0, (n_terms, 1)) + 0.02 * d[None, :]).astype(np.float32)
    A = np.repeat(np.asarray(k.pdd, dtype=np.float32)[None, :], n_theta, axis=0) * \
        np.linspace(1.0, 1.1, n_theta, dtype=np.float32)[:, None]
    tabs = fi.KernelTables(c1, c2, c3, step, A, 0.02, k.pdd_step)
    kt = dataclasses.replace(k, weight=[0.0] * n_terms, sigma0=[1.0] * n_terms, sigma_slope=[0.0] * n_terms,
                             width_scale=[1.0] * n_terms, tables=tabs)
    g = fi.slab_phantom(75, n=(31, 27, 19), spacing=(0.5, 0.5, 0.5), lung_side=(2, 5), bone_side=(1, 2))
    prob = fi.Problem("shapes", g, fi.coplanar_beams(2, (0.1, -0.05, 0.07), 100.0, 0.8, 0.6, 6, 4), kt)
    plan = Plan(prob, "cuda:0")
    csr = plan.compute()
    ora = oracle_lib.OraclePlan(prob)
    off, oidx, oval = ora.full()
    rows = list(range(ora.n_beamlets))
    r = compare_rows(ora, rows, gpu_rows_from_csr(csr, rows),
                     [(oidx[off[j]:off[j + 1]], oval[off[j]:off[j + 1]]) for j in rows])
    print(f"\n  K={n_terms} n_theta={n_theta} n_depth={n_depth}: nnz={csr.nnz} max_rel={r['max_rel']:.2e}",
          flush=True)


def test_tables_rejected_when_invalid(torch_gpu):
    import paper_0908_4417_amd as m
    from paper_0908_4417_amd import Plan
    k = fi.default_kernel(76)
    base = fi.analytic_tables(k)
    g = fi.water_phantom((12, 10, 8), (0.5, 0.5, 0.5))
    beams = fi.coplanar_beams(1, (0, 0, 0), 100.0, 1.0, 1.0, 2, 2)
    bad_c3 = base.c3.copy()
    bad_c3[1, 5] = 0.0
    for tabs, msg in [(dataclasses.replace(base, c3=bad_c3), "c3"),
                      (dataclasses.replace(base, depth_step=0.0), "steps"),
                      (dataclasses.replace(base, c1=base.c1[:, :1], c2=base.c2[:, :1], c3=base.c3[:, :1]),
                       "n_depth")]:
        with pytest.raises(m.FspbError, match=msg):
            Plan(fi.Problem("bad", g, beams, dataclasses.replace(k, tables=tabs)), "cuda:0")
