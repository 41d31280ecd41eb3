"""Pins of the oracle's general kernel form (Eq. 2-3 with depth-tabulated c1, c2,
c3 and an angle-and-depth table A(theta, d)).

* the analytic kernel written as tables (constant c1, c2; linear c3; A = PDD)
  reproduces the analytic rows (linear interpolation of a linear function is
  exact);
* A linear in theta scales each beamlet's row by the factor at that beamlet's
  angle, computed here from the beamlet axis and the beam's central axis;
* at any depth, the plane integral of F is a b sum_k c1_k(d) c2_k(d)^2 and one
  term's bracket has variance (c2(d) a)^2 / 12 + c3(d)^2, with the c's
  interpolated here from the tables (depth handling of all three tables).
"""
import dataclasses

import numpy as np
import pytest

import fspb_inputs as fi


def _problem(kernel, gantries=(0.0, 140.0), n=(18, 16, 14)):
    g = fi.slab_phantom(7, n=n, spacing=(0.5, 0.5, 0.5), lung_side=(2, 3), bone_side=(1, 2))
    beams = []
    for gd in gantries:
        beams += fi.coplanar_beams(1, (0.11, -0.07, 0.05), 100.0, 0.8, 0.6, 5, 3, start_deg=gd)
    return fi.Problem("tab", g, beams, kernel)


def test_analytic_tables_reproduce_the_analytic_kernel(oracle_lib):
    k = fi.default_kernel(2)
    ka = oracle_lib.OraclePlan(_problem(k)).full()
    kt = dataclasses.replace(k, tables=fi.analytic_tables(k, n_theta=3))
    kb = oracle_lib.OraclePlan(_problem(kt)).full()
    np.testing.assert_array_equal(ka[0], kb[0])
    np.testing.assert_array_equal(ka[1], kb[1])
    np.testing.assert_allclose(kb[2], ka[2], rtol=1e-6, atol=1e-10 * ka[2].max())   # c3 stored as float32


def test_angle_factor_scales_each_row(oracle_lib):
    k = fi.default_kernel(2)
    kap = 0.9
    base = fi.analytic_tables(k, n_theta=5, theta_step=0.02)
    th = np.arange(5) * 0.02
    A = (base.A.astype(np.float64) * (1.0 + kap * th[:, None])).astype(np.float32)
    prob = _problem(dataclasses.replace(k, tables=dataclasses.replace(base, A=A)))
    plan = oracle_lib.OraclePlan(prob)
    off_t, idx_t, val_t = plan.full()
    # the same rows with A = PDD (theta-free), then the factor from geometry
    plain = oracle_lib.OraclePlan(_problem(dataclasses.replace(k, tables=base)))
    off_p, idx_p, val_p = plain.full()
    np.testing.assert_array_equal(idx_t, idx_p)
    rows = 0
    for j, b in enumerate(plan.beamlets):
        beam = prob.beams[b.beam]
        g = np.radians(beam.gantry_deg)
        S = np.array(beam.isocenter) + beam.sad * np.array([np.sin(g), -np.cos(g), 0.0])
        c0 = (np.array(beam.isocenter) - S) / beam.sad
        theta = np.arccos(np.clip(np.dot(c0, np.array(b.e)), -1.0, 1.0))
        assert theta < 4 * 0.02
        # A is stored in float32: the factor holds to float32 rounding of the table
        np.testing.assert_allclose(val_t[off_t[j]:off_t[j + 1]], val_p[off_p[j]:off_p[j + 1]] * (1.0 + kap * theta),
                                   rtol=3e-7, atol=1e-15)
        rows += off_t[j + 1] > off_t[j]
    assert rows > 10


def _simpson(n, R):
    x = np.linspace(-R, R, n)
    w = np.full(n, 2.0)
    w[0] = w[-1] = 1.0
    w[1:-1:2] = 4.0
    return x, w * (x[1] - x[0]) / 3.0


@pytest.mark.parametrize("d", [0.0, 3.3, 17.85, 39.0, 55.0])
def test_tabulated_normalisation_and_variance(oracle_lib, d):
    k = fi.default_kernel(4)
    tabs = fi.synthetic_tables(11, k)
    plan = oracle_lib.OraclePlan(_problem(dataclasses.replace(k, weight=[0, 0, 0], sigma0=[1, 1, 1],
                                                              sigma_slope=[0, 0, 0], width_scale=[1, 1, 1],
                                                              tables=tabs)))
    nodes = np.arange(tabs.c1.shape[1]) * tabs.depth_step
    c = [np.array([np.interp(d, nodes, t[i]) for i in range(3)]) for t in (tabs.c1, tabs.c2, tabs.c3)]
    a, b = 0.7, 0.45
    R = 0.6 + 9.0 * c[2].max()
    x, w = _simpson(1201, R)
    # separable per term: integrate u on a fine grid at v = 0 and v on the same grid at u = 0 is not
    # enough for a sum of terms, so integrate the full plane on a coarser v grid
    xv, wv = _simpson(301, R)
    F = np.array([[plan.lateral(u, v, a, b, d) for u in x] for v in xv])
    total = (F @ w) @ wv
    expect = a * b * np.sum(c[0] * c[1] ** 2)
    assert abs(total - expect) < 1e-5 * expect, (total, expect)
    # one term: variance of the u-profile at v = 0
    one = oracle_lib.OraclePlan(_problem(dataclasses.replace(
        k, weight=[0], sigma0=[1], sigma_slope=[0], width_scale=[1],
        tables=dataclasses.replace(tabs, c1=tabs.c1[:1], c2=tabs.c2[:1], c3=tabs.c3[:1]))))
    prof = np.array([one.lateral(u, 0.0, a, b, d) for u in x])
    var = (prof * x ** 2) @ w / (prof @ w)
    assert abs(var - ((c[1][0] * a) ** 2 / 12.0 + c[2][0] ** 2)) < 1e-6
