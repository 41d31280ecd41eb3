"""The GPU-vs-oracle comparison itself, exercised on the CPU with the oracle's own
rows rounded to FP32 (what a correct HIP result looks like) and with planted
differences that the acceptance bar must reject."""
import os
import sys

import numpy as np
import pytest

import fspb_inputs as fi

sys.path.insert(0, os.path.dirname(__file__))
from parity import compare_plan  # noqa: E402


def _csr(off, idx, val, nv):
    import torch
    from paper_0908_4417_amd.plan import CSR
    return CSR(torch.from_numpy(off.astype(np.int64)), torch.from_numpy(idx.astype(np.int32)),
               torch.from_numpy(val.astype(np.float32)), nv)


@pytest.fixture(scope="module")
def small(oracle_lib):
    g = fi.slab_phantom(5, n=(30, 26, 20), spacing=(0.5, 0.5, 0.5), lung_side=(2, 5), bone_side=(1, 2))
    prob = fi.Problem("ph", g, fi.coplanar_beams(3, (0.11, -0.07, 0.13), 100.0, 1.0, 1.0, 4, 3),
                      fi.default_kernel(5))
    ora = oracle_lib.OraclePlan(prob)
    off, idx, val = ora.full()
    return ora, off, idx, val, 30 * 26 * 20


def test_fp32_rounded_oracle_passes(small):
    ora, off, idx, val, nv = small
    r = compare_plan(ora, _csr(off, idx, val, nv), chunk=5)
    assert r["rows"] == ora.n_beamlets and r["n"] == len(idx) and r["band_mismatches"] == 0
    assert r["max_rel"] <= 6e-8 and r["eps"] < 1e-8
    sub = compare_plan(ora, _csr(off, idx, val, nv), rows=[7, 3, 11], chunk=2)
    assert sub["rows"] == 3 and sub["n"] == sum(off[j + 1] - off[j] for j in (3, 7, 11))


def test_value_error_above_the_bar_fails(small):
    ora, off, idx, val, nv = small
    v = val.copy()
    k = int(np.argmax(v))
    v[k] *= 1 + 3e-4
    with pytest.raises(AssertionError, match="relative error|largest entry"):
        compare_plan(ora, _csr(off, idx, v, nv), chunk=7)
    v = val.copy()
    big = np.nonzero(v > 0.05 * v.max())[0]
    v[big[len(big) // 2]] *= 1 - 2e-4
    with pytest.raises(AssertionError, match="relative error"):
        compare_plan(ora, _csr(off, idx, v, nv), chunk=7)


def test_pattern_difference_outside_the_band_fails(small):
    ora, off, idx, val, nv = small
    j = 5
    a, b = off[j], off[j + 1]
    keep = np.ones(len(idx), dtype=bool)
    keep[(a + b) // 2] = False                        # a voxel in the middle of a row
    off2 = off.copy()
    off2[j + 1:] -= 1
    with pytest.raises(AssertionError, match="outside the cutoff band"):
        compare_plan(ora, _csr(off2, idx[keep], val[keep], nv), chunk=4)


def test_unsorted_columns_fail(small):
    ora, off, idx, val, nv = small
    i2 = idx.copy()
    a = off[2]
    i2[a], i2[a + 1] = i2[a + 1], i2[a]
    with pytest.raises(AssertionError, match="strictly ascending"):
        compare_plan(ora, _csr(off, i2, val, nv), chunk=4)
