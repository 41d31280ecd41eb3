"""Eq. 1 (dose of a fluence) and its adjoint on the GPU vs the FP64 oracle."""
import numpy as np
import pytest

import fspb_inputs as fi

pytestmark = pytest.mark.gpu


def test_fluence_dose_and_gradient_match_oracle(oracle_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0908_4417_amd import Plan
    g = fi.slab_phantom(12, n=(48, 44, 30), spacing=(0.5, 0.5, 0.5), lung_side=(3, 6), bone_side=(1, 2))
    prob = fi.Problem("flu", g, fi.coplanar_beams(5, (0.13, -0.07, 0.05), 100.0, 1.0, 1.0, 5, 4),
                      fi.default_kernel(12))
    plan = Plan(prob, "cuda:0")
    csr = plan.compute()
    rng = np.random.default_rng(3)
    w = rng.uniform(0.0, 2.0, plan.n_beamlets)
    w[::7] = 0.0
    r = rng.normal(size=plan.n_voxels)
    d = csr.dose(torch.from_numpy(w.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    gr = csr.gradient(torch.from_numpy(r.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    ora = oracle_lib.OraclePlan(prob)
    dref = ora.fluence_dose(w.astype(np.float32).astype(np.float64))
    gref = ora.fluence_gradient(r.astype(np.float32).astype(np.float64))
    assert np.max(np.abs(d - dref)) <= 1e-5 * dref.max()
    assert np.max(np.abs(gr - gref)) <= 1e-5 * np.max(np.abs(gref))
    # the gradient is deterministic
    g2 = csr.gradient(torch.from_numpy(r.astype(np.float32)).cuda()).cpu().numpy()
    np.testing.assert_array_equal(g2, gr.astype(np.float32))
