"""Eq. 1 on the full-size slab's D (653,399,552 nonzeros, the bench's plan).

* the atomic dose, the voxel-row dose and the adjoint of random weights against
  the oracle's FP64 Eq. 1 over every row (one full oracle pass each);
* the voxel-row transpose: its row pointers equal the column counts of the
  beamlet-row CSR, and on sampled voxels (random ones, the grid's first and last,
  and both sides of 32-column bucket boundaries) each voxel row equals, entry for
  entry, the beamlets whose rows hold that voxel with their values (bit-exact).
"""
import numpy as np
import pytest

import fspb_inputs as fi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slab(oracle_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0908_4417_amd import Plan
    prob = fi.make_config(1)
    plan = Plan(prob, "cuda:0")
    csr = plan.compute()
    torch.cuda.synchronize()
    print(f"\n  slab plan: nnz={csr.nnz}", flush=True)
    return prob, plan, csr


def test_full_size_dose_and_adjoint_match_oracle(slab, oracle_lib):
    import torch
    prob, plan, csr = slab
    rng = np.random.default_rng(31)
    w = rng.uniform(0.0, 2.0, plan.n_beamlets).astype(np.float32)
    w[::11] = 0.0
    r = rng.normal(size=plan.n_voxels).astype(np.float32)
    wd = torch.from_numpy(w).to("cuda:0")
    d_atomic = csr.dose(wd).cpu().numpy().astype(np.float64)
    t = csr.transpose()
    d_voxel = t.dose(wd).cpu().numpy().astype(np.float64)
    g = csr.gradient(torch.from_numpy(r).to("cuda:0")).cpu().numpy().astype(np.float64)
    del t
    ora = oracle_lib.OraclePlan(prob)
    dref = ora.fluence_dose(w.astype(np.float64))
    gref = ora.fluence_gradient(r.astype(np.float64))
    e_a = np.max(np.abs(d_atomic - dref)) / dref.max()
    e_v = np.max(np.abs(d_voxel - dref)) / dref.max()
    e_g = np.max(np.abs(g - gref)) / np.max(np.abs(gref))
    print(f"  dose: atomic {e_a:.2e}, voxel rows {e_v:.2e} of the maximum; adjoint {e_g:.2e}", flush=True)
    assert e_a <= 1e-5 and e_v <= 1e-5 and e_g <= 1e-5


def test_full_size_transpose_sampled_voxels(slab):
    import torch
    prob, plan, csr = slab
    nv = plan.n_voxels
    t = csr.transpose()
    torch.cuda.synchronize()
    ip = csr.indptr.cpu().numpy()
    ix = csr.indices.cpu().numpy()
    vv = csr.values.cpu().numpy()
    tp = t.indptr.cpu().numpy()
    # row pointers: the column counts of the beamlet-row CSR
    counts = np.bincount(ix, minlength=nv)
    np.testing.assert_array_equal(np.diff(tp), counts)
    assert tp[0] == 0 and tp[-1] == len(ix)
    # sampled voxel rows, entry for entry
    rng = np.random.default_rng(32)
    busy = np.flatnonzero(counts)
    edges = np.concatenate([b + np.array([-1, 0]) for b in rng.choice(np.arange(32, nv, 32), 200)])
    sample = np.unique(np.concatenate([rng.choice(busy, 2000, replace=False), edges, [0, nv - 1]]))
    sample = sample[(sample >= 0) & (sample < nv)]
    rows_of = [[] for _ in sample]
    vals_of = [[] for _ in sample]
    for j in range(plan.n_beamlets):
        a, b = int(ip[j]), int(ip[j + 1])
        cols = ix[a:b]
        pos = np.searchsorted(cols, sample)
        hit = np.flatnonzero((pos < b - a) & (cols[np.minimum(pos, b - a - 1)] == sample)) if b > a else []
        for h in hit:
            rows_of[h].append(j)
            vals_of[h].append(vv[a + pos[h]])
    ti = t.indices.cpu().numpy()
    tv = t.values.cpu().numpy()
    for k, i in enumerate(sample):
        a, b = int(tp[i]), int(tp[i + 1])
        np.testing.assert_array_equal(ti[a:b], np.array(rows_of[k], dtype=np.int32), err_msg=f"voxel {i}")
        np.testing.assert_array_equal(tv[a:b].view(np.int32), np.array(vals_of[k], dtype=np.float32).view(np.int32),
                                      err_msg=f"voxel {i}")
    print(f"  transpose: {len(sample)} voxel rows checked, "
          f"{sum(len(r) for r in rows_of)} entries", flush=True)
