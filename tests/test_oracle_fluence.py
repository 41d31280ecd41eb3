"""Pins of the oracle's dose superposition (Eq. 1) and its adjoint.

* a unit weight on beamlet j reproduces row j of D;
* linearity in the weights;
* adjointness: sum_i r_i dose_i(w) = sum_j w_j g_j(r);
* Sec. 2.1's self-consistency: uniform weights over a tiled field with a far
  source give the broad beam's dose.
"""
import numpy as np

import fspb_inputs as fi


def _plan(oracle_lib, seed=3):
    g = fi.slab_phantom(seed, n=(20, 18, 14), spacing=(0.5, 0.5, 0.5), lung_side=(2, 4), bone_side=(1, 2))
    beams = fi.coplanar_beams(2, (0.13, -0.07, 0.05), 100.0, 0.8, 0.6, 3, 2)
    return oracle_lib.OraclePlan(fi.Problem("flu", g, beams, fi.default_kernel(seed)))


def test_unit_weight_reproduces_a_row(oracle_lib):
    p = _plan(oracle_lib)
    for j in (0, 5, 11):
        w = np.zeros(p.n_beamlets)
        w[j] = 1.0
        d = p.fluence_dose(w)
        idx, val = p.row(j)
        ref = np.zeros_like(d)
        ref[idx] = val
        np.testing.assert_array_equal(d, ref)


def test_linearity_and_adjointness(oracle_lib):
    p = _plan(oracle_lib)
    rng = np.random.default_rng(1)
    w1, w2 = rng.uniform(0, 1, p.n_beamlets), rng.uniform(0, 1, p.n_beamlets)
    d1, d2 = p.fluence_dose(w1), p.fluence_dose(w2)
    np.testing.assert_allclose(p.fluence_dose(2.0 * w1 - 0.5 * w2), 2.0 * d1 - 0.5 * d2, rtol=1e-12, atol=1e-14)
    r = rng.normal(size=d1.size)
    g = p.fluence_gradient(r)
    assert abs(r @ d1 - w1 @ g) <= 1e-12 * abs(r @ d1)


def test_tiled_field_dose_equals_broad_beam(oracle_lib):
    sad = 1e7
    g = fi.water_phantom((15, 11, 13), (0.5, 0.5, 0.5), centre=(0.1, 0.0, -0.05))
    k = fi.default_kernel(0)
    k.cutoff_u = k.cutoff_v = 50.0
    a, b, nu, nv = 0.5, 0.75, 5, 3
    tiled = oracle_lib.OraclePlan(fi.Problem("t", g, [fi.Beam(0.0, (0, 0, 0), sad, a, b, nu, nv,
                                                              -0.5 * (nu - 1) * a, -0.5 * (nv - 1) * b)], k))
    broad = oracle_lib.OraclePlan(fi.Problem("b", g, [fi.Beam(0.0, (0, 0, 0), sad, nu * a, nv * b, 1, 1,
                                                              0.0, 0.0)], k))
    dt = tiled.fluence_dose(np.ones(tiled.n_beamlets))
    db = broad.fluence_dose(np.ones(1))
    big = db > 1e-3 * db.max()
    np.testing.assert_allclose(dt[big], db[big], rtol=1e-6)
