"""Pins of the oracle's FSPB kernel (Eq. 1-3) and its VOI (Sec. 2.1).

Properties the model fixes, none of which re-types the oracle's formula:
* normalisation (Sec. 2.1 requires it): the double integral of F over the
  plane is a b sum_k c1_k c2_k^2;
* the lateral profile of one term is a box of width c2 a blurred by a
  Gaussian of standard deviation c3: its variance is (c2 a)^2 / 12 + c3^2;
* sigma -> 0 gives the sharp beamlet: sum c1 inside, 1/2 of it on an edge,
  1/4 on a corner, 0 outside;
* self-consistency (Sec. 2.1): summing a tiled field of beamlets equals one
  evaluation of the broad field (exact for parallel beamlets);
* mirror symmetry of a centred beamlet in water;
* the depth-dose table is reproduced at its nodes and the inverse-square law
  holds along a flat field.
"""
import dataclasses
import math

import numpy as np
import pytest

import fspb_inputs as fi


def _plan(oracle_lib, **kw):
    g = fi.water_phantom((9, 9, 9), (1.0, 1.0, 1.0))
    k = fi.default_kernel(0)
    for name, v in kw.items():
        setattr(k, name, v)
    return oracle_lib.OraclePlan(fi.Problem("k", g, fi.coplanar_beams(1, (0, 0, 0), 100.0, 1, 1, 1, 1), k))


@pytest.mark.parametrize("a,b,d", [(1.0, 1.0, 0.0), (0.25, 0.5, 12.0), (0.7, 0.3, 29.0)])
def test_lateral_profile_normalisation(oracle_lib, a, b, d):
    plan = _plan(oracle_lib, width_scale=[1.0, 1.3])
    K = plan.kernel
    sig_max = max(K.sigma0[i] + K.sigma_slope[i] * d for i in range(2))
    R = max(a, b) * 1.3 / 2 + 9.0 * sig_max
    n = 801
    x = np.linspace(-R, R, n)
    h = x[1] - x[0]
    w = np.full(n, 2.0)
    w[0] = w[-1] = 1.0
    w[1:-1:2] = 4.0
    w *= h / 3.0                                     # Simpson weights
    F = np.array([[plan.lateral(u, v, a, b, d) for u in x] for v in x[::8]])
    # integrate over u at every 8th v, then over v with the separable structure checked below
    Iu = F @ w
    # the profile is separable per term, so check the full 2D integral on a coarse v grid too
    v8 = x[::8]
    w8 = np.full(len(v8), 2.0)
    w8[0] = w8[-1] = 1.0
    w8[1:-1:2] = 4.0
    w8 *= (v8[1] - v8[0]) / 3.0
    total = Iu @ w8
    expect = a * b * sum(K.weight[i] * K.width_scale[i] ** 2 for i in range(2))
    assert abs(total - expect) < 2e-6 * expect


def test_edge_pair_variance_is_box_plus_gaussian(oracle_lib):
    """One bracket of Eq. 3 is a box of width w convolved with N(0, s^2), times 2."""
    lib = oracle_lib.lib()
    for w, s in ((1.0, 0.2), (0.25, 0.6), (2.0, 0.05)):
        R = w / 2 + 12 * s
        x = np.linspace(-R, R, 20001)
        f = np.array([lib.ofs_edge_pair(float(xx), w, s) for xx in x])
        m0 = np.trapezoid(f, x)
        m2 = np.trapezoid(f * x * x, x)
        assert abs(m0 - 2.0 * w) < 1e-7
        assert abs(m2 / m0 - (w * w / 12.0 + s * s)) < 1e-7


def test_sharp_beamlet_limit(oracle_lib):
    tiny = 1e-9
    plan = _plan(oracle_lib, sigma0=[tiny, tiny], sigma_slope=[0.0, 0.0])
    a, b = 1.0, 0.6
    total = sum(plan.kernel.weight[i] for i in range(2))
    cases = [((0.0, 0.0), 1.0), ((0.3, -0.2), 1.0), ((0.5, 0.0), 0.5), ((-0.5, 0.1), 0.5),
             ((0.2, 0.3), 0.5), ((0.5, 0.3), 0.25), ((-0.5, -0.3), 0.25), ((0.51, 0.0), 0.0),
             ((0.0, -0.31), 0.0), ((2.0, 2.0), 0.0)]
    for (u, v), frac in cases:
        assert abs(plan.lateral(u, v, a, b, 5.0) - frac * total) < 1e-12


def test_edge_pair_tail_keeps_relative_accuracy(oracle_lib):
    lib = oracle_lib.lib()
    # far tail: value ~1e-40; the two erf() terms would cancel to 0 in double
    v = lib.ofs_edge_pair(4.0, 1.0, 0.25)
    # asymptotic: erfc(z) ~ exp(-z^2)/(z sqrt(pi)), z = (x - w/2)/(sqrt2 s)
    z = 3.5 / (math.sqrt(2) * 0.25)
    approx = math.exp(-z * z) / (z * math.sqrt(math.pi)) * (1 - 1 / (2 * z * z))
    assert v > 0 and abs(v / approx - 1) < 2e-3


def test_pdd_table_nodes_and_hold(oracle_lib):
    plan = _plan(oracle_lib)
    pdd = plan.pdd
    step = plan.kernel.pdd_step
    for k in (0, 1, 15, 300, len(pdd) - 1):
        assert plan.pdd_at(k * step) == pytest.approx(float(pdd[k]), abs=1e-15)
    assert plan.pdd_at(1e4) == float(pdd[-1])
    mid = plan.pdd_at(15.5 * step)
    assert mid == pytest.approx(0.5 * (float(pdd[15]) + float(pdd[16])), abs=1e-15)


def test_inverse_square_along_flat_field(oracle_lib):
    """Flat depth dose and a very wide beamlet: D = (SAD/t')^2 sum c1 on the axis."""
    g = fi.water_phantom((7, 21, 7), (0.5, 0.5, 0.5))
    k = fi.default_kernel(0)
    k.pdd = np.ones(601, dtype=np.float32)
    k.cutoff_u = k.cutoff_v = 1.0
    beams = [fi.Beam(0.0, (0.0, 0.0, 0.0), 50.0, 60.0, 60.0, 1, 1, 0.0, 0.0)]
    plan = oracle_lib.OraclePlan(fi.Problem("flat", g, beams, k))
    idx, val = plan.row(0)
    nx, ny, nz = g.shape_xyz
    sel = (idx % nx == 3) & ((idx // (nx * ny)) == 3)        # the central axis voxels
    assert sel.sum() == ny
    iy = (idx[sel] // nx) % ny
    y = g.origin[1] + iy * g.spacing[1]
    tp = y + 50.0                                             # source at y = -50
    np.testing.assert_allclose(val[sel], (50.0 / tp) ** 2 * sum(k.weight), rtol=1e-12)


def test_centred_beamlet_mirror_symmetry(oracle_lib):
    n = 21
    g = fi.water_phantom((n, n, n), (0.5, 0.5, 0.5))
    k = fi.default_kernel(0)
    beams = [fi.Beam(0.0, (0.0, 0.0, 0.0), 100.0, 1.0, 1.0, 1, 1, 0.0, 0.0)]
    plan = oracle_lib.OraclePlan(fi.Problem("c", g, beams, k))
    idx, val = plan.row(0)
    D = np.zeros(n ** 3)
    D[idx] = val
    D = D.reshape(n, n, n)                                    # [z, y, x]
    assert D.max() > 0
    np.testing.assert_allclose(D, D[:, :, ::-1], rtol=1e-13, atol=1e-300)   # x -> -x
    np.testing.assert_allclose(D, D[::-1, :, :], rtol=1e-13, atol=1e-300)   # z -> -z
    np.testing.assert_allclose(D, D.transpose(2, 1, 0), rtol=1e-12, atol=1e-300)  # x <-> z


def test_tiled_field_equals_broad_field(oracle_lib):
    """Sec. 2.1 self-consistency: the beamlets of a field sum to the broad beam.

    With a far source the beamlets are parallel, every voxel sees the same
    depth from each of them, and the erf brackets telescope exactly.  (A
    beamlet tilted by theta moves O' along its axis by x theta, which changes
    the depth by ~1e-5 cm at SAD = 1e5; SAD = 1e7 makes that negligible.)
    """
    sad = 1e7
    g = fi.water_phantom((15, 11, 13), (0.5, 0.5, 0.5), centre=(0.1, 0.0, -0.05))
    iso = (0.0, sad * 0.0, 0.0)
    a, b, nu, nv = 0.5, 0.75, 5, 3
    k = fi.default_kernel(0)
    k.cutoff_u = k.cutoff_v = 50.0
    tiled = [fi.Beam(0.0, iso, sad, a, b, nu, nv, -0.5 * (nu - 1) * a, -0.5 * (nv - 1) * b)]
    broad = [fi.Beam(0.0, iso, sad, nu * a, nv * b, 1, 1, 0.0, 0.0)]
    pt = oracle_lib.OraclePlan(fi.Problem("t", g, tiled, k))
    pb = oracle_lib.OraclePlan(fi.Problem("b", g, broad, k))
    off, idx, val = pt.full()
    sumD = np.zeros(g.density.size)
    np.add.at(sumD, idx, val)
    ib, vb = pb.row(0)
    Db = np.zeros(g.density.size)
    Db[ib] = vb
    big = Db > 1e-3 * Db.max()
    assert big.sum() > 500
    np.testing.assert_allclose(sumD[big], Db[big], rtol=1e-6)


def test_tiled_field_deviation_at_clinical_sad_is_small(oracle_lib):
    """At SAD 100 cm the beamlets diverge; report that the sum stays within 1e-2."""
    g = fi.water_phantom((15, 11, 13), (0.5, 0.5, 0.5))
    a, nu = 0.5, 6
    k = fi.default_kernel(0)
    k.cutoff_u = k.cutoff_v = 50.0
    tiled = [fi.Beam(0.0, (0, 0, 0), 100.0, a, a, nu, nu, -0.5 * (nu - 1) * a, -0.5 * (nu - 1) * a)]
    broad = [fi.Beam(0.0, (0, 0, 0), 100.0, nu * a, nu * a, 1, 1, 0.0, 0.0)]
    off, idx, val = oracle_lib.OraclePlan(fi.Problem("t", g, tiled, k)).full()
    sumD = np.zeros(g.density.size)
    np.add.at(sumD, idx, val)
    ib, vb = oracle_lib.OraclePlan(fi.Problem("b", g, broad, k)).row(0)
    Db = np.zeros(g.density.size)
    Db[ib] = vb
    big = Db > 0.2 * Db.max()
    rel = np.abs(sumD[big] / Db[big] - 1.0)
    assert rel.max() < 1e-2


def test_central_axis_value(oracle_lib):
    """Axis voxels of a centred beamlet in water: u = v = 0, depth = t' - tA.

    Then each bracket of Eq. 3 is 2 erf(c2 a / (2 sqrt2 c3)) and the depth
    dose is read at the geometric depth.
    """
    n = 21
    g = fi.water_phantom((n, n, n), (0.5, 0.5, 0.5))
    k = fi.default_kernel(0)
    beams = [fi.Beam(0.0, (0.0, 0.0, 0.0), 100.0, 1.0, 0.5, 1, 1, 0.0, 0.0)]
    plan = oracle_lib.OraclePlan(fi.Problem("c", g, beams, k))
    bl = plan.beamlets[0]
    idx, val = plan.row(0)
    for iy in (0, 3, 10, 20):
        lin = (10 * n + iy) * n + 10
        v = val[np.searchsorted(idx, lin)]
        y = g.origin[1] + iy * 0.5
        tp = y + 100.0
        d = tp - bl.tA
        x = d / k.pdd_step
        i0 = int(math.floor(x))
        pdd = (1 - (x - i0)) * float(k.pdd[i0]) + (x - i0) * float(k.pdd[i0 + 1])
        F = 0.0
        for i in range(2):
            s = k.sigma0[i] + k.sigma_slope[i] * d
            F += k.weight[i] * math.erf(1.0 / (2 * math.sqrt(2) * s)) * math.erf(0.5 / (2 * math.sqrt(2) * s))
        assert v == pytest.approx(pdd * (100.0 / tp) ** 2 * F, rel=1e-13)
