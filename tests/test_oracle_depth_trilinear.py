"""Pins of the oracle's trilinear depth table (Sec. 2.2 as the paper builds it).

* the density sampler equals scipy's linear RegularGridInterpolator on the
  voxel centres (a library routine), inside the centre hull and, with the
  position held at the outermost centre planes, outside it;
* uniform density: depth = rho * (t - tA) at every table point;
* a density that is linear along one axis and a ray along another: the
  sampled density is that linear function at the ray's fixed coordinate, so
  the table is exact (one case per axis, catching a wrong weight or index);
* with a fine table step the trapezoid table converges to a brute-force
  quadrature of the interpolated density along the ray.
"""
import dataclasses

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import fspb_inputs as fi


def _problem(density, spacing, origin, gantry, iso, table_step=0.0):
    g = fi.Grid(np.ascontiguousarray(density, dtype=np.float32), spacing, origin)
    k = fi.default_kernel(0)
    k.depth = "trilinear"
    k.table_step = table_step
    return fi.Problem("tri", g, [fi.Beam(gantry, iso, 100.0, 0.5, 0.5, 1, 1, 0.0, 0.0)], k)


def _rgi(density, spacing, origin):
    nz, ny, nx = density.shape
    axes = [origin[k] + spacing[k] * np.arange(n) for k, n in enumerate((nx, ny, nz))]
    f = RegularGridInterpolator(axes, np.transpose(density.astype(np.float64), (2, 1, 0)), method="linear")
    lo = np.array([a[0] for a in axes])
    hi = np.array([a[-1] for a in axes])
    return lambda p: f(np.clip(np.atleast_2d(p), lo, hi))


def test_sampler_matches_library_interpolator(oracle_lib):
    rng = np.random.default_rng(4)
    dens = rng.uniform(0.0, 2.0, (7, 9, 11))
    sp, org = (0.3, 0.4, 0.5), (-1.0, 0.5, 2.0)
    plan = oracle_lib.OraclePlan(_problem(dens, sp, org, 0.0, (0.5, 2.1, 3.4)))
    f = _rgi(dens.astype(np.float32), sp, org)
    pts = np.stack([rng.uniform(org[k] - 0.5 * sp[k] - 0.3, org[k] + (n - 0.5) * sp[k] + 0.3, 400)
                    for k, n in enumerate((11, 9, 7))], axis=1)
    got = np.array([plan.trilinear_density(p) for p in pts])
    np.testing.assert_allclose(got, f(pts), rtol=1e-12, atol=1e-12)


def test_uniform_density(oracle_lib):
    dens = np.full((12, 14, 16), 1.37)
    plan = oracle_lib.OraclePlan(_problem(dens, (0.5, 0.5, 0.5), (-3.7, -3.2, -2.9), 33.0, (0.1, 0.2, -0.1)))
    tab, off = plan.tables()
    bl = plan.beamlets[0]
    t = np.minimum(np.arange(bl.n) * bl.step, bl.tB - bl.tA)
    np.testing.assert_allclose(tab[off[0]:off[1]], np.float32(1.37) * t, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("axis,gantry", [(0, 0.0), (1, 90.0), (2, 90.0), (2, 0.0)])
def test_linear_density_across_the_ray(oracle_lib, axis, gantry):
    """gantry 0: the axis runs along y; gantry 90: along x."""
    n = (16, 18, 20)                                         # nz, ny, nx
    sp, org = (0.4, 0.5, 0.6), (-3.9, -4.1, -4.4)
    coords = np.meshgrid(*[org[k] + sp[k] * np.arange(m) for k, m in enumerate((n[2], n[1], n[0]))],
                         indexing="ij")                      # x, y, z
    lin = 0.8 + 0.07 * coords[axis]
    dens = np.transpose(lin, (2, 1, 0))                      # [z][y][x]
    iso = (0.237, -0.311, 0.143)
    plan = oracle_lib.OraclePlan(_problem(dens, sp, org, gantry, iso))
    tab, off = plan.tables()
    bl = plan.beamlets[0]
    assert abs(bl.e[axis]) < 1e-12                           # the ray keeps this coordinate
    rho = 0.8 + 0.07 * iso[axis]
    t = np.minimum(np.arange(bl.n) * bl.step, bl.tB - bl.tA)
    # float32 storage of the ramp: relative 6e-8 per sample
    np.testing.assert_allclose(tab[off[0]:off[1]], rho * t, rtol=2e-7, atol=1e-9)


def test_fine_table_converges_to_quadrature(oracle_lib):
    rng = np.random.default_rng(9)
    dens = rng.uniform(0.2, 1.8, (10, 12, 14)).astype(np.float32)
    sp, org = (0.5, 0.5, 0.5), (-3.2, -2.7, -2.3)
    plan = oracle_lib.OraclePlan(_problem(dens, sp, org, 27.0, (0.21, 0.13, 0.07), table_step=0.002))
    tab, off = plan.tables()
    bl = plan.beamlets[0]
    f = _rgi(dens, sp, org)
    S, e = np.array(bl.S), np.array(bl.e)
    for k in (bl.n // 3, 2 * bl.n // 3, bl.n - 1):
        t1 = bl.tB if k == bl.n - 1 else bl.tA + k * bl.step
        ts = np.linspace(bl.tA, t1, 200001)
        vals = f(S[None, :] + ts[:, None] * e[None, :])
        ref = np.trapezoid(vals, ts)
        assert abs(tab[off[0] + k] - ref) <= 1e-5 * max(ref, 1.0), (k, tab[off[0] + k], ref)
