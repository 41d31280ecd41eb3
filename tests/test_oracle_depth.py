"""Pins of the oracle's radiological-depth table (Sec. 2.2; resolution study of Sec. 3.2).

* In water the radiological depth is the geometric depth, and the linear
  interpolation of a linear function is exact: d(O') = clamp(t' - tA, 0, |AB|).
* The paper's resolution study: element lengths of 1, 1/2, 1/3 and 1/4 voxel
  give the same coefficients in water.
* In a heterogeneous phantom the table (chords of the piecewise-linear path
  integral) stays within step * (rho_max - rho_min) / 4 of the exact integral.
"""
import dataclasses

import numpy as np
import pytest

import fspb_inputs as fi


def _water_problem(gantries, table_step=0.0, n=(40, 40, 40), spacing=(0.5, 0.5, 0.5)):
    g = fi.water_phantom(n, spacing, centre=(0.13, -0.21, 0.07))
    beams = []
    for gdeg in gantries:
        beams += fi.coplanar_beams(1, (0.3, -0.2, 0.1), 100.0, 1.0, 1.0, 5, 4,
                                   start_deg=gdeg)
    k = fi.default_kernel(0)
    k.table_step = table_step
    return fi.Problem("water", g, beams, k)


@pytest.mark.parametrize("gantries", [[0.0], [37.0, 90.0, 215.0]])
def test_water_depth_is_geometric(oracle_lib, gantries):
    p = _water_problem(gantries)
    plan = oracle_lib.OraclePlan(p)
    tab, off = plan.tables()
    for j in range(plan.n_beamlets):
        bl = plan.beamlets[j]
        t = tab[off[j]:off[j + 1]]
        L = bl.tB - bl.tA
        assert bl.n >= 2 and abs(bl.step * (bl.n - 1) - L) < 1e-12
        assert bl.step <= 0.25 * (1 + 1e-9)
        np.testing.assert_allclose(t, np.minimum(np.arange(bl.n) * bl.step, L), rtol=0, atol=1e-12)
        for tp in np.linspace(bl.tA - 3.0, bl.tB + 3.0, 17):
            d = plan.table_depth(j, t, tp)
            assert abs(d - min(max(tp - bl.tA, 0.0), L)) < 1e-12
            assert abs(plan.exact_depth(j, max(tp, bl.tA)) - min(max(tp - bl.tA, 0.0), L)) < 1e-12


def test_table_resolution_does_not_change_water_coefficients(oracle_lib):
    """Sec. 3.2: element lengths of one, 1/2, 1/3, 1/4 voxel."""
    rows = []
    for frac in (1.0, 0.5, 1.0 / 3.0, 0.25):
        p = _water_problem([0.0, 120.0], table_step=0.5 * frac)
        plan = oracle_lib.OraclePlan(p)
        rows.append(plan.rows([0, 7, 23]))
    for off, idx, val in rows[1:]:
        np.testing.assert_array_equal(off, rows[0][0])
        np.testing.assert_array_equal(idx, rows[0][1])
        np.testing.assert_allclose(val, rows[0][2], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("frac", [1.0, 0.5, 0.25])
def test_heterogeneous_table_error_is_bounded(oracle_lib, frac):
    g = fi.slab_phantom(21, n=(48, 48, 48), spacing=(0.5, 0.5, 0.5), lung_side=(3.0, 8.0),
                        bone_side=(1.0, 3.0))
    beams = fi.coplanar_beams(3, (0.17, 0.11, -0.09), 100.0, 1.0, 1.0, 4, 4)
    k = fi.default_kernel(0)
    k.table_step = 0.5 * frac
    plan = oracle_lib.OraclePlan(fi.Problem("slab", g, beams, k))
    tab, off = plan.tables()
    spread = float(g.density.max() - g.density.min())
    worst = 0.0
    for j in range(0, plan.n_beamlets, 5):
        bl = plan.beamlets[j]
        t = tab[off[j]:off[j + 1]]
        # nodes are exact
        for k_ in (0, bl.n // 3, bl.n - 1):
            tk = bl.tB if k_ == bl.n - 1 else bl.tA + k_ * bl.step
            assert abs(t[k_] - plan.exact_depth(j, tk)) < 1e-10
        # between nodes the chord stays within step * spread / 4
        for tp in np.linspace(bl.tA, bl.tB, 97):
            err = abs(plan.table_depth(j, t, tp) - plan.exact_depth(j, tp))
            worst = max(worst, err)
            assert err <= bl.step * spread / 4.0 + 1e-10
    assert worst > 0.0, "the phantom must actually exercise interpolation error"
