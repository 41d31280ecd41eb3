"""Seeded synthetic inputs for the FSPB dose-coefficient path.

This module only *draws* inputs: density grids, beam arrangements, a depth-dose
table and lateral-profile parameters.  It holds none of the method's
arithmetic (no ray tracing, no VOI test, no kernel evaluation), so both the
FP64 oracle and the HIP library can consume what it produces without sharing
any code with each other.

The paper's own inputs (a prostate CT and the fitted 6 MV kernel of Jiang 1998,
Sec. 2.1 and Sec. 3) are not available; every workload here is a seeded
stand-in with the shapes, sizes and density ranges of the paper's experiments
(Sec. 3.1 water phantom, Sec. 3.2 nine-field prostate plan).

Units: cm, g/cc relative to water, degrees.  Density arrays are float32 with
shape (nz, ny, nx), x fastest.  Voxel (0,0,0) is centred at ``origin``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

__all__ = [
    "Grid", "Beam", "KernelParams", "Problem",
    "pdd_table", "default_kernel", "water_phantom", "slab_phantom",
    "pelvis_phantom", "coplanar_beams", "make_config", "batched_configs",
    "surrogate_samples", "surrogate_init", "table1_case", "CONFIG_NAMES",
]


@dataclass
class Grid:
    density: np.ndarray            # float32 [nz, ny, nx]
    spacing: tuple                 # (sx, sy, sz) cm
    origin: tuple                  # centre of voxel (0,0,0), cm

    @property
    def shape_xyz(self):
        nz, ny, nx = self.density.shape
        return nx, ny, nz


@dataclass
class Beam:
    gantry_deg: float
    isocenter: tuple
    sad: float
    beamlet_a: float
    beamlet_b: float
    nu: int
    nv: int
    u0: float                      # centre of beamlet (0,0) on the iso plane
    v0: float


@dataclass
class KernelParams:
    weight: List[float]
    sigma0: List[float]
    sigma_slope: List[float]
    width_scale: List[float]
    pdd: np.ndarray                # float32 depth-dose table, node k at k*pdd_step
    pdd_step: float
    cutoff_u: float = 3.0          # VOI half-width at the iso plane (<=0: 3a)
    cutoff_v: float = 3.0
    table_step: float = 0.0        # <=0: half the smallest voxel spacing
    rho_min: float = 0.0
    depth: str = "siddon"          # depth table: "siddon" (exact path integral) or "trilinear"
    tables: "KernelTables | None" = None   # depth / angle tables of Eq. 2-3 (None: the analytic form)

    @property
    def n_terms(self):
        return len(self.weight) if self.tables is None else int(np.shape(self.tables.c1)[0])


@dataclass
class KernelTables:
    """Eq. 2-3 in their general form: per-term c1(d), c2(d), c3(d) on a depth grid
    and A(theta, d) on an (angle, depth) grid (theta in radians)."""
    c1: np.ndarray                 # float32 [n_terms][n_depth]
    c2: np.ndarray
    c3: np.ndarray
    depth_step: float
    A: np.ndarray                  # float32 [n_theta][n_adepth]
    theta_step: float
    adepth_step: float


@dataclass
class Problem:
    name: str
    grid: Grid
    beams: List[Beam]
    kernel: KernelParams
    meta: dict = field(default_factory=dict)

    @property
    def n_beamlets(self):
        return sum(b.nu * b.nv for b in self.beams)


# --------------------------------------------------------------------------
# Beam data
# --------------------------------------------------------------------------

def pdd_table(seed: int, step: float = 0.1, d_end: float = 60.0,
              s0: float = 0.25, beta: float = 2.498, mu: float = 0.045):
    """Seeded smooth build-up / exponential fall-off depth-dose table.

    Shape [s0 + (1-s0)(1-exp(-beta d))] exp(-mu d) (1 + r(d)) with a small
    seeded ripple r(d) = sum_m eps_m cos(2 pi d / lambda_m + phi_m),
    |eps_m| <= 0.002, lambda_m in [8, 25] cm; maximum near 1.5 cm for the
    default beta.  Normalised to a maximum of 1 and tabulated every ``step``.
    The paper's fitted 6 MV data are not printed, so this stands in for them.
    """
    rng = np.random.default_rng(seed)
    eps = rng.uniform(-0.002, 0.002, 3)
    lam = rng.uniform(8.0, 25.0, 3)
    phi = rng.uniform(0.0, 2 * np.pi, 3)
    n = int(round(d_end / step)) + 1
    d = np.arange(n, dtype=np.float64) * step
    shape = (s0 + (1 - s0) * (1 - np.exp(-beta * d))) * np.exp(-mu * d)
    ripple = sum(eps[m] * np.cos(2 * np.pi * d / lam[m] + phi[m]) for m in range(3))
    p = shape * (1.0 + ripple)
    p /= p.max()
    return p.astype(np.float32)


def default_kernel(seed: int, cutoff: float = 3.0, **kw) -> KernelParams:
    """Two-term erf lateral profile with sigma growing 0.2 -> 0.6 cm over 30 cm.

    weights (0.9, 0.1) sum to 1; sigma_2 = 2 sigma_1; width scale 1.  These
    replace the unprinted fitted parameters C of the paper's Eq. 3.
    """
    return KernelParams(
        weight=[0.9, 0.1],
        sigma0=[0.2, 0.4],
        sigma_slope=[0.4 / 30.0, 0.8 / 30.0],
        width_scale=[1.0, 1.0],
        pdd=pdd_table(seed), pdd_step=0.1,
        cutoff_u=cutoff, cutoff_v=cutoff, **kw)


def analytic_tables(kernel: KernelParams, depth_step: float | None = None, n_theta: int = 1,
                    theta_step: float = 0.05) -> KernelTables:
    """A kernel's analytic form written as tables: c1, c2 constant, c3 = sigma0 +
    slope d sampled at the nodes, A(theta, d) = the depth-dose table for every
    theta (nodes on the depth dose's own grid unless depth_step is given)."""
    step = kernel.pdd_step if depth_step is None else depth_step
    n_depth = int(round((len(kernel.pdd) - 1) * kernel.pdd_step / step)) + 1
    d = np.arange(n_depth) * step
    K = kernel.n_terms
    c1 = np.repeat(np.asarray(kernel.weight, dtype=np.float64)[:, None], n_depth, axis=1)
    c2 = np.repeat(np.asarray(kernel.width_scale, dtype=np.float64)[:, None], n_depth, axis=1)
    c3 = np.asarray(kernel.sigma0)[:, None] + np.asarray(kernel.sigma_slope)[:, None] * d[None, :]
    A = np.repeat(np.asarray(kernel.pdd, dtype=np.float32)[None, :], n_theta, axis=0)
    f32 = lambda x: np.ascontiguousarray(x, dtype=np.float32).reshape(K, n_depth)
    return KernelTables(f32(c1), f32(c2), f32(c3), step, A, theta_step, kernel.pdd_step)


def synthetic_tables(seed: int, kernel: KernelParams, n_terms: int = 3, depth_step: float = 0.5,
                     d_end: float = 40.0, n_theta: int = 9, theta_step: float = 0.025) -> KernelTables:
    """A three-term kernel in the paper's general form (Eq. 3 with depth-dependent
    c1, c2, c3 and an off-axis A(theta, d)): seeded smooth curves of plausible
    magnitude, c2 and c3 > 0.  Jiang's fitted values are not printed."""
    rng = np.random.default_rng(seed)
    n_depth = int(round(d_end / depth_step)) + 1
    d = np.arange(n_depth) * depth_step
    w = np.array([0.8, 0.15, 0.05][:n_terms])
    c1 = w[:, None] * (1.0 + rng.uniform(-0.15, 0.15, (n_terms, 1)) * np.tanh(d[None, :] / 10.0))
    c2 = 1.0 + rng.uniform(-0.03, 0.05, (n_terms, 1)) * d[None, :] / d_end
    s0 = np.array([0.15, 0.4, 1.2][:n_terms])[:, None]
    s1 = np.array([0.012, 0.03, 0.08][:n_terms])[:, None]
    c3 = s0 + s1 * d[None, :] + rng.uniform(0.0, 1e-4, (n_terms, 1)) * d[None, :] ** 2
    n_ad = len(kernel.pdd)
    ad = np.arange(n_ad) * kernel.pdd_step
    th = np.arange(n_theta) * theta_step
    horn = 1.0 + 0.8 * th[:, None] ** 2 * np.exp(-ad[None, :] / 15.0)     # off-axis "horns", fading with depth
    A = np.asarray(kernel.pdd, dtype=np.float64)[None, :] * horn
    f32 = lambda x: np.ascontiguousarray(x, dtype=np.float32)
    return KernelTables(f32(c1), f32(c2), f32(c3), depth_step, f32(A), theta_step, kernel.pdd_step)


def coplanar_beams(n_beams, iso, sad, a, b, nu, nv, start_deg=0.0, step_deg=None):
    """``n_beams`` coplanar beams, equally spaced unless ``step_deg`` is given.

    Each beam is an nu x nv grid of a x b beamlets centred on the beam axis.
    """
    if step_deg is None:
        step_deg = 360.0 / n_beams
    u0 = -0.5 * (nu - 1) * a
    v0 = -0.5 * (nv - 1) * b
    return [Beam(start_deg + k * step_deg, tuple(iso), sad, a, b, nu, nv, u0, v0)
            for k in range(n_beams)]


# --------------------------------------------------------------------------
# Phantoms
# --------------------------------------------------------------------------

def _centred_origin(shape_xyz, spacing, centre=(0.0, 0.0, 0.0)):
    return tuple(centre[k] - 0.5 * (shape_xyz[k] - 1) * spacing[k] for k in range(3))


def _coords(shape_xyz, spacing, origin):
    nx, ny, nz = shape_xyz
    x = origin[0] + spacing[0] * np.arange(nx)
    y = origin[1] + spacing[1] * np.arange(ny)
    z = origin[2] + spacing[2] * np.arange(nz)
    return x, y, z


def water_phantom(n, spacing, rho=1.0, centre=(0.0, 0.0, 0.0)):
    nx, ny, nz = n
    sp = tuple(spacing)
    dens = np.full((nz, ny, nx), rho, dtype=np.float32)
    return Grid(dens, sp, _centred_origin(n, sp, centre))


def slab_phantom(seed, n=(128, 128, 128), spacing=(0.25, 0.25, 0.25),
                 n_lung=4, n_bone=4, lung_side=(4.0, 10.0), bone_side=(1.0, 3.0),
                 rho_lung=0.25, rho_bone=1.8, background=1.0):
    """Water box with seeded axis-aligned lung blocks, then bone blocks on top."""
    rng = np.random.default_rng(seed)
    g = water_phantom(n, spacing, background)
    x, y, z = _coords(n, g.spacing, g.origin)
    ext = [c[-1] - c[0] for c in (x, y, z)]
    lo0 = [c[0] for c in (x, y, z)]

    def put(side_rng, rho):
        side = rng.uniform(side_rng[0], side_rng[1], 3)
        cen = [lo0[k] + rng.uniform(0, ext[k]) for k in range(3)]
        mx = np.abs(x - cen[0]) <= side[0] / 2
        my = np.abs(y - cen[1]) <= side[1] / 2
        mz = np.abs(z - cen[2]) <= side[2] / 2
        m = mz[:, None, None] & my[None, :, None] & mx[None, None, :]
        g.density[m] = rho

    for _ in range(n_lung):
        put(lung_side, rho_lung)
    for _ in range(n_bone):
        put(bone_side, rho_bone)
    return g


def pelvis_phantom(seed, n=(256, 256, 100), spacing=(0.2, 0.2, 0.3)):
    """Prostate-shaped synthetic patient (stand-in for the Sec. 3.2 CT).

    Elliptic body (semi-axes about 17 x 11 cm, +-5 %), density U[0.95, 1.05]
    per voxel; a pelvic ring and two femoral-head shells of bone
    (thickness 0.8-1.5 cm, density U[1.5, 1.9] per structure); a rectal air
    pocket (density 0.001) posterior to the isocentre; 0 outside the body.
    Gantry 0 looks along +y, so +y is posterior here.
    """
    rng = np.random.default_rng(seed)
    sp = tuple(spacing)
    origin = _centred_origin(n, sp)
    x, y, z = _coords(n, sp, origin)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    ax = 17.0 * rng.uniform(0.95, 1.05)
    ay = 11.0 * rng.uniform(0.95, 1.05)
    body = (X / ax) ** 2 + (Y / ay) ** 2 <= 1.0
    dens = rng.uniform(0.95, 1.05, X.shape).astype(np.float32)

    # pelvic ring: elliptic cylindrical shell
    t = rng.uniform(0.8, 1.5)
    rx, ry = 13.0 * rng.uniform(0.95, 1.05), 8.0 * rng.uniform(0.95, 1.05)
    r_out = np.sqrt((X / rx) ** 2 + (Y / ry) ** 2)
    r_in = np.sqrt((X / (rx - t)) ** 2 + (Y / (ry - t)) ** 2)
    ring = (r_out <= 1.0) & (r_in > 1.0)
    dens[ring] = rng.uniform(1.5, 1.9)
    # femoral heads: spherical shells left and right
    for side in (-1.0, 1.0):
        t = rng.uniform(0.8, 1.5)
        R = 2.5 * rng.uniform(0.9, 1.1)
        c = (side * 8.5 * rng.uniform(0.95, 1.05), rng.uniform(-1.0, 1.0), rng.uniform(-2.0, 2.0))
        rr = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
        dens[(rr <= R) & (rr > R - t)] = rng.uniform(1.5, 1.9)
    # rectal air pocket
    rc = 2.0 * rng.uniform(0.9, 1.1)
    cy = 3.5 * rng.uniform(0.9, 1.1)
    air = (X / rc) ** 2 + ((Y - cy) / rc) ** 2 + (Z / (1.5 * rc)) ** 2 <= 1.0
    dens[air] = 0.001
    dens[~body] = 0.0
    return Grid(np.ascontiguousarray(dens, dtype=np.float32), sp, origin)


def _ellipse_phantom(rng, n, spacing, lo, hi):
    sp = tuple(spacing)
    origin = _centred_origin(n, sp)
    x, y, z = _coords(n, sp, origin)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    ax = 0.4 * (x[-1] - x[0]) * rng.uniform(0.8, 1.0)
    ay = 0.4 * (y[-1] - y[0]) * rng.uniform(0.6, 1.0)
    dens = np.full(X.shape, rng.uniform(0.95, 1.05), dtype=np.float32)
    cx, cy = rng.uniform(-0.3, 0.3) * ax, rng.uniform(-0.3, 0.3) * ay
    inner = ((X - cx) / (0.35 * ax)) ** 2 + ((Y - cy) / (0.35 * ay)) ** 2 <= 1.0
    dens[inner] = rng.uniform(lo, hi)
    dens[(X / ax) ** 2 + (Y / ay) ** 2 > 1.0] = 0.0
    return Grid(dens, sp, origin)


def _slab_stack(rng, n, spacing, lo, hi):
    sp = tuple(spacing)
    origin = _centred_origin(n, sp)
    nx, ny, nz = n
    dens = np.empty((nz, ny, nx), dtype=np.float32)
    cuts = np.sort(rng.integers(1, ny, size=int(rng.integers(2, 6))))
    edges = np.concatenate([[0], cuts, [ny]])
    for i in range(len(edges) - 1):
        dens[:, edges[i]:edges[i + 1], :] = rng.uniform(lo, hi)
    return Grid(dens, sp, origin)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

CONFIG_NAMES = {
    0: "water64_1beam_100bl",
    1: "slab128_9beam_8100bl",
    2: "pelvis256x256x100_9beam_5184bl",
    3: "batch32_uneven",
    4: "surrogate_on_pelvis",
}


def make_config(k: int, seed: int | None = None) -> Problem:
    """The five workloads of the benchmark plan, seeded.

    0: 64^3 water at 4 mm, one beam at 0 deg, 10 x 10 beamlets of 1 cm.
    1: 128^3 slab phantom at 2.5 mm (lung 0.25, bone 1.8), 9 beams 40 deg
       apart, 30 x 30 beamlets of 0.5 cm.
    2: 256 x 256 x 100 pelvis at 2 x 2 x 3 mm, 9 beams, 24 x 24 beamlets of
       0.25 cm.
    4: the same patient as 2 (the surrogate's workload).
    Config 3 (32 plans) is produced by ``batched_configs``.
    """
    if seed is None:
        seed = {0: 1, 1: 2, 2: 3, 4: 5}[k]
    if k == 0:
        g = water_phantom((64, 64, 64), (0.4, 0.4, 0.4))
        beams = coplanar_beams(1, (0.0, 0.0, 0.0), 100.0, 1.0, 1.0, 10, 10)
        return Problem(CONFIG_NAMES[0], g, beams, default_kernel(seed), {"seed": seed})
    if k == 1:
        g = slab_phantom(seed)
        beams = coplanar_beams(9, (0.0, 0.0, 0.0), 100.0, 0.5, 0.5, 30, 30, step_deg=40.0)
        return Problem(CONFIG_NAMES[1], g, beams, default_kernel(seed), {"seed": seed})
    if k in (2, 4):
        g = pelvis_phantom(3 if k == 4 else seed)
        beams = coplanar_beams(9, (0.0, 0.0, 0.0), 100.0, 0.25, 0.25, 24, 24, step_deg=40.0)
        return Problem(CONFIG_NAMES[k], g, beams, default_kernel(3 if k == 4 else seed),
                       {"seed": seed})
    if k == 3:
        raise ValueError("config 3 is a batch: use batched_configs()")
    raise ValueError(f"unknown config {k}")


def batched_configs(n_plans: int = 32, base_seed: int = 4000, scale: float = 1.0):
    """Plans of uneven size for the batched launch.

    Grid points per axis from {64, ..., 256} (z <= 128), physical extent
    25-51 cm, 5-9 equally spaced beams, beamlet size from {0.25, 0.5, 1.0} cm
    over a 6 x 6 cm field, slab or ellipse densities in 0.001-1.9.  ``scale``
    < 1 shrinks every grid dimension (used for quick tests).
    """
    sizes = [64, 96, 128, 160, 192, 224, 256]
    plans = []
    for k in range(n_plans):
        rng = np.random.default_rng(base_seed + k)
        nx = int(rng.choice(sizes))
        ny = int(rng.choice(sizes))
        nz = int(rng.choice([s for s in sizes if s <= 128]))
        ext = rng.uniform(25.0, 51.0)
        if scale != 1.0:
            nx, ny, nz = (max(8, int(round(v * scale))) for v in (nx, ny, nz))
        h = ext / max(nx, ny)
        spacing = (h, h, min(0.5, ext * 0.6 / nz))
        n = (nx, ny, nz)
        if rng.uniform() < 0.5:
            g = _slab_stack(rng, n, spacing, 0.001, 1.9)
            kind = "slab"
        else:
            g = _ellipse_phantom(rng, n, spacing, 0.001, 1.9)
            kind = "ellipse"
        n_beams = int(rng.integers(5, 10))
        a = float(rng.choice([0.25, 0.5, 1.0]))
        nb = int(round(6.0 / a))
        start = rng.uniform(0.0, 360.0 / n_beams)
        beams = coplanar_beams(n_beams, (0.0, 0.0, 0.0), 100.0, a, a, nb, nb, start_deg=start)
        ker = default_kernel(base_seed + k)
        plans.append(Problem(f"batch{k:02d}_{kind}_{nx}x{ny}x{nz}_{n_beams}b_a{a}", g, beams, ker,
                             {"seed": base_seed + k}))
    return plans


def random_csr(seed: int, n_rows: int, n_cols: int, mean_row: float, empty_frac: float = 0.1):
    """A seeded sparse matrix in CSR form with ragged rows (input for transpose tests).

    Row lengths are Poisson(mean_row) (a fraction ``empty_frac`` of rows
    empty), capped at n_cols; each row's columns are distinct and ascending,
    drawn in a window around a random centre (like a beamlet's VOI) so that
    columns collide across rows.  Values are uniform in (0, 1].
    Returns (indptr int64, indices int32, values float32).
    """
    rng = np.random.default_rng(seed)
    lens = np.minimum(rng.poisson(mean_row, n_rows), n_cols)
    lens[rng.uniform(size=n_rows) < empty_frac] = 0
    indptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    indices = np.empty(int(indptr[-1]), dtype=np.int32)
    for j in range(n_rows):
        k = int(lens[j])
        if k == 0:
            continue
        width = min(n_cols, max(k, int(4 * k)))
        lo = int(rng.integers(0, n_cols - width + 1))
        indices[indptr[j]:indptr[j + 1]] = np.sort(rng.choice(width, size=k, replace=False)) + lo
    values = (1.0 - rng.uniform(size=int(indptr[-1]))).astype(np.float32)
    return indptr, indices, values


def surrogate_samples(n: int, seed: int, d_max: float = 30.0, uv_max: float = 3.0,
                      a_range=(0.25, 1.0), core: float = 0.0, core_uv: float = 1.0, core_d: float = 5.0,
                      log_a: bool = False, sqrt_uniform: bool = False, zero_depth: float = 0.0):
    """Training/evaluation points (d, |u|, |v|, a) for the kernel surrogate.

    float64 array [n, 4]; the profile is even in u and v, so only |u|, |v|
    are drawn.  A fraction ``1 - core`` is uniform over the whole box; the
    fraction ``core`` is uniform over the beamlet core |u|, |v| <= core_uv,
    half of it also restricted to the build-up region d <= core_d (where the
    kernel is largest and steepest).  With ``log_a`` the beamlet side is drawn
    log-uniformly (narrow beamlets, whose profiles are sharpest, get more
    samples).  With ``sqrt_uniform`` d, |u|, |v| are drawn as max * s^2 with s
    uniform, i.e. uniformly in the surrogate's square-root feature
    coordinates (dense near d = 0 and near the beamlet axis).  A fraction
    ``zero_depth`` of the points gets d = 0 exactly: every voxel whose
    projection on a beamlet axis lies before the entry point, or behind air
    only, has zero radiological depth, so the fill meets that value often.
    """
    rng = np.random.default_rng(seed)
    out = np.empty((n, 4), dtype=np.float64)
    if sqrt_uniform:
        out[:, 0] = d_max * rng.uniform(0.0, 1.0, n) ** 2
        out[:, 1] = uv_max * rng.uniform(0.0, 1.0, n) ** 2
        out[:, 2] = uv_max * rng.uniform(0.0, 1.0, n) ** 2
    else:
        out[:, 0] = rng.uniform(0.0, d_max, n)
        out[:, 1] = rng.uniform(0.0, uv_max, n)
        out[:, 2] = rng.uniform(0.0, uv_max, n)
    if log_a:
        out[:, 3] = np.exp(rng.uniform(np.log(a_range[0]), np.log(a_range[1]), n))
    else:
        out[:, 3] = rng.uniform(a_range[0], a_range[1], n)
    nz0 = int(round(zero_depth * n))
    if nz0:
        out[-nz0:, 0] = 0.0
    nc = int(round(core * n))
    if nc:
        out[:nc, 1] = rng.uniform(0.0, core_uv, nc)
        out[:nc, 2] = rng.uniform(0.0, core_uv, nc)
        out[:nc // 2, 0] = rng.uniform(0.0, core_d, nc // 2)
    if nc or nz0:
        rng.shuffle(out, axis=0)
    return out


# The training set and schedule used for the pelvis surrogate: 1e7 points drawn
# uniformly in the square-root feature coordinates, beamlet side log-uniform,
# 10 % of the points at zero depth; 800 epochs of Adam, batch 16384, cosine
# learning rate 3e-3 -> 1e-6.
SURROGATE_SAMPLES = 10_000_000
SURROGATE_RECIPE = {"sqrt_uniform": True, "log_a": True, "zero_depth": 0.1}
SURROGATE_TRAINING = {"batch": 16384, "lr_max": 3e-3, "lr_min": 1e-6}
SURROGATE_EPOCHS = 800


def surrogate_init(seed: int, hidden: int = 64, n_in: int = 4):
    """Seeded initial parameters of the 4 -> 64 -> 64 -> 1 surrogate (float32, 4545 values).

    Layout W1[64][4], b1[64], W2[64][64], b2[64], W3[64], b3; weights uniform
    in +-sqrt(6 / (fan_in + fan_out)), biases zero.
    """
    rng = np.random.default_rng(seed)
    lim = lambda fi, fo: np.sqrt(6.0 / (fi + fo))
    w1 = rng.uniform(-lim(n_in, hidden), lim(n_in, hidden), hidden * n_in)
    w2 = rng.uniform(-lim(hidden, hidden), lim(hidden, hidden), hidden * hidden)
    w3 = rng.uniform(-lim(hidden, 1), lim(hidden, 1), hidden)
    z = np.zeros(hidden)
    return np.concatenate([w1, z, w2, z, w3, [0.0]]).astype(np.float32)


def table1_case(case: int, seed: int = 6) -> Problem:
    """Geometry of the paper's water-phantom study (Table 1, cases 1-7).

    30 cm water cube, five coplanar beams 72 deg apart, 10 x 10 cm field,
    VOI side six times the beamlet side (Sec. 2.1).  Voxel and beamlet sizes
    follow Table 1 (case 2's voxel is read as 0.375 cm: 80^3 = 0.51 M).
    """
    vox = {1: 0.5, 2: 0.375, 3: 0.3, 4: 0.25, 5: 0.25, 6: 0.25, 7: 0.25}[case]
    bl = {1: 0.2, 2: 0.2, 3: 0.2, 4: 0.2, 5: 0.25, 6: 1.0 / 3.0, 7: 0.5}[case]
    n = int(round(30.0 / vox))
    g = water_phantom((n, n, n), (vox, vox, vox))
    nb = int(round(10.0 / bl))
    beams = coplanar_beams(5, (0.0, 0.0, 0.0), 100.0, bl, bl, nb, nb)
    ker = default_kernel(seed, cutoff=3.0 * bl)
    return Problem(f"table1_case{case}", g, beams, ker, {"seed": seed})
