"""Comparison of the HIP path's CSR rows with the FP64 oracle's.

Acceptance (per the project's tolerance for this method):
* values: |D_gpu - D_oracle| <= 1e-4 D_oracle for every entry with
  D_oracle > 1 % of the largest oracle entry among the rows compared;
* pattern: identical, except voxels whose |u| or |v| lies within 1e-4 cm of
  the VOI cutoff (there FP64 and FP32-rounded geometry may legitimately
  disagree);
* also reported: eps = mean |D_gpu - D_oracle| over common entries (the
  paper's error measure, Sec. 3.1), and the worst relative error.
"""
from __future__ import annotations

import numpy as np

REL_TOL = 1e-4
BAND_CM = 1e-4
FLOOR = 0.01


def compare_rows(ora, rows, gpu_rows, oracle_rows=None, vmax=None):
    """rows: beamlet ids; gpu_rows / oracle_rows: lists of (indices, values)."""
    if oracle_rows is None:
        off, oidx, oval = ora.rows(rows)
        oracle_rows = [(oidx[off[k]:off[k + 1]], oval[off[k]:off[k + 1]]) for k in range(len(rows))]
    if vmax is None:
        vmax = max([float(v.max()) for _, v in oracle_rows if len(v)] + [0.0])
    nx, ny = ora.grid.nx, ora.grid.ny
    worst = 0.0
    abs_sum = 0.0
    n_common = 0
    band_only = 0
    for j, (gi, gv), (oi, ov) in zip(rows, gpu_rows, oracle_rows):
        gi = np.asarray(gi)
        assert np.all(np.diff(gi) > 0), f"row {j}: GPU columns not strictly ascending"
        extra = np.setdiff1d(gi, oi, assume_unique=True)
        missing = np.setdiff1d(oi, gi, assume_unique=True)
        for v in np.concatenate([extra, missing]):
            ix, iy, iz = int(v % nx), int((v // nx) % ny), int(v // (nx * ny))
            _, t, u, vv = ora.voi_member(int(j), ix, iy, iz)
            bl = ora.beamlets[int(j)]
            near = min(abs(abs(u) - bl.cu), abs(abs(vv) - bl.cv)) <= BAND_CM
            assert near, (f"row {j}: voxel {v} differs outside the cutoff band "
                          f"(u={u:.6f}, v={vv:.6f}, cu={bl.cu}, cv={bl.cv}, "
                          f"{'extra' if v in extra else 'missing'})")
            band_only += 1
        common, ga, oa = np.intersect1d(gi, oi, assume_unique=True, return_indices=True)
        g = np.asarray(gv, dtype=np.float64)[ga]
        o = np.asarray(ov, dtype=np.float64)[oa]
        if len(o):
            abs_sum += float(np.abs(g - o).sum())
            n_common += len(o)
            big = o > FLOOR * vmax
            if big.any():
                rel = np.abs(g[big] - o[big]) / o[big]
                k = int(np.argmax(rel))
                worst = max(worst, float(rel[k]))
                assert rel[k] <= REL_TOL, (f"row {j}: voxel {common[big][k]} relative error "
                                           f"{rel[k]:.3e} (gpu {g[big][k]:.9g}, oracle {o[big][k]:.9g})")
    return {"max_rel": worst, "eps": abs_sum / max(n_common, 1), "n": n_common,
            "band_mismatches": band_only, "vmax": vmax}


def gpu_rows_from_csr(csr, rows):
    """Copy only the requested CSR rows to the host."""
    indptr = csr.indptr.cpu().numpy()
    out = []
    for j in rows:
        a, b = int(indptr[j]), int(indptr[j + 1])
        out.append((csr.indices[a:b].cpu().numpy(), csr.values[a:b].cpu().numpy()))
    return out
