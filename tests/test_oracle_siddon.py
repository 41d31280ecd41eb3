"""Pins of the oracle's ray trace (Siddon 1985, used for radiological depth in Sec. 2.2).

The oracle's sorted-merge Siddon is checked against brute-force fine sampling
of the same ray on tiny grids: per-voxel path lengths agree within two
sample steps and sum to |AB|.
"""
import numpy as np
import pytest

import fspb_inputs as fi


def _grid(rng, n, spacing=None):
    nx, ny, nz = n
    if spacing is None:
        spacing = tuple(rng.uniform(0.3, 1.2, 3))
    dens = rng.uniform(0.0, 2.0, (nz, ny, nx)).astype(np.float32)
    origin = tuple(rng.uniform(-2.0, 2.0, 3))
    return fi.Grid(dens, spacing, origin)


def _problem(g):
    b = fi.Beam(0.0, (0.0, 0.0, 0.0), 100.0, 1.0, 1.0, 1, 1, 0.0, 0.0)
    return fi.Problem("tiny", g, [b], fi.default_kernel(0))


def _clip(g, S, e):
    """Independent slab clip in numpy for the test's own rays."""
    nx, ny, nz = g.shape_xyz
    n = (nx, ny, nz)
    lo = np.array(g.origin) - 0.5 * np.array(g.spacing)
    hi = lo + np.array(n) * np.array(g.spacing)
    t0, t1 = 0.0, np.inf
    for k in range(3):
        if e[k] == 0.0:
            if not (lo[k] <= S[k] < hi[k]):
                return None
            continue
        a, b = sorted(((lo[k] - S[k]) / e[k], (hi[k] - S[k]) / e[k]))
        t0, t1 = max(t0, a), min(t1, b)
    return (t0, t1) if t1 > t0 else None


def _brute(g, S, e, tA, tB, nsamp=1_000_000):
    nx, ny, nz = g.shape_xyz
    h = (tB - tA) / nsamp
    t = tA + (np.arange(nsamp) + 0.5) * h
    lo = np.array(g.origin) - 0.5 * np.array(g.spacing)
    idx = []
    for k, n in enumerate((nx, ny, nz)):
        c = S[k] + t * e[k]
        idx.append(np.clip(np.floor((c - lo[k]) / g.spacing[k]).astype(np.int64), 0, n - 1))
    lin = (idx[2] * ny + idx[1]) * nx + idx[0]
    acc = np.bincount(lin, minlength=nx * ny * nz) * h
    return acc, h


def _rays(rng, g, count):
    nx, ny, nz = g.shape_xyz
    lo = np.array(g.origin) - 0.5 * np.array(g.spacing)
    hi = lo + np.array((nx, ny, nz)) * np.array(g.spacing)
    centre = 0.5 * (lo + hi)
    out = []
    while len(out) < count:
        target = lo + rng.uniform(0, 1, 3) * (hi - lo)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        S = target - 30.0 * d
        out.append((S, d))
    # axis-parallel rays (one and two zero direction components)
    for k in range(3):
        d = np.zeros(3)
        d[k] = 1.0
        S = centre.copy() + rng.uniform(-0.3, 0.3, 3) * (hi - lo)
        S[k] = lo[k] - 5.0
        out.append((S, d))
    # a ray lying in a voxel face plane (x = lo + 1 spacing) and a ray through a voxel edge
    d = np.array([0.0, 0.6, 0.8])
    S = np.array([lo[0] + g.spacing[0], lo[1] - 3.0, lo[2] - 4.0 + 0.37])
    out.append((S, d))
    d = np.array([1.0, 1.0, 0.0]) / np.sqrt(2.0)
    S = np.array([lo[0] - 2.0, lo[1] - 2.0, lo[2] + 1.5 * g.spacing[2]])
    out.append((S, d))
    return out


@pytest.mark.parametrize("n,seed", [((3, 4, 5), 11), ((5, 5, 5), 12), ((4, 3, 6), 13)])
def test_siddon_matches_fine_sampling(oracle_lib, n, seed):
    rng = np.random.default_rng(seed)
    g = _grid(rng, n)
    plan = oracle_lib.OraclePlan(_problem(g))
    checked = 0
    for S, e in _rays(rng, g, 12):
        c = _clip(g, S, e)
        if c is None:
            continue
        tA, tB = c
        vox, ln = oracle_lib.siddon(plan, S, e, tA, tB)
        assert abs(ln.sum() - (tB - tA)) <= 1e-12 * max(1.0, tB - tA)
        assert np.all(ln > 0.0)
        assert len(np.unique(vox)) == len(vox), "a straight ray visits each voxel once"
        got = np.zeros(np.prod(n))
        np.add.at(got, vox, ln)
        ref, h = _brute(g, S, e, tA, tB)
        assert np.max(np.abs(got - ref)) <= 2.0 * h + 1e-12
        checked += 1
    assert checked >= 10


def test_siddon_segments_are_ordered_along_the_ray(oracle_lib):
    rng = np.random.default_rng(5)
    g = _grid(rng, (5, 5, 5), spacing=(0.5, 0.5, 0.5))
    g.origin = (-1.0, -1.0, -1.0)
    plan = oracle_lib.OraclePlan(_problem(g))
    S = np.array([-10.0, -0.7, -1.1])
    e = np.array([1.0, 0.1, 0.05])
    e /= np.linalg.norm(e)
    tA, tB = _clip(g, S, e)
    vox, ln = oracle_lib.siddon(plan, S, e, tA, tB)
    nx, ny, nz = g.shape_xyz
    ix = vox % nx
    assert np.all(np.diff(ix) >= 0), "x index never decreases for a +x ray"
    # neighbouring segments share a face: indices differ by one step along one axis
    iy = (vox // nx) % ny
    iz = vox // (nx * ny)
    steps = np.abs(np.diff(ix)) + np.abs(np.diff(iy)) + np.abs(np.diff(iz))
    assert np.all((steps >= 1) & (steps <= 3))


def test_beamlet_entry_and_exit_lie_on_the_grid_boundary(oracle_lib):
    p = fi.make_config(0)
    plan = oracle_lib.OraclePlan(p)
    g = p.grid
    nx, ny, nz = g.shape_xyz
    lo = np.array(g.origin) - 0.5 * np.array(g.spacing)
    hi = lo + np.array((nx, ny, nz)) * np.array(g.spacing)
    for j in (0, 37, 99):
        bl = plan.beamlets[j]
        S, e = np.array(bl.S), np.array(bl.e)
        for t in (bl.tA, bl.tB):
            P = S + t * e
            assert np.all(P >= lo - 1e-9) and np.all(P <= hi + 1e-9)
            assert np.min(np.minimum(np.abs(P - lo), np.abs(P - hi))) < 1e-9
        ref = _clip(g, S, e)
        assert abs(ref[0] - bl.tA) < 1e-12 and abs(ref[1] - bl.tB) < 1e-12
