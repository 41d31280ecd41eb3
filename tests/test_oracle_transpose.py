"""Pins of the oracle's voxel-row transpose (Eq. 1 read with rows = voxels).

* on a small matrix it equals the row-major nonzero list of the dense
  transpose (the textbook definition);
* transposing twice gives the input back;
* row/column sums are preserved (D w and D^T 1 computed both ways).
"""
import numpy as np

import fspb_inputs as fi
import oracle


def _csr_of_dense(a):
    r, c = np.nonzero(a)
    indptr = np.concatenate([[0], np.cumsum(np.bincount(r, minlength=a.shape[0]))])
    return indptr, c.astype(np.int32), a[r, c]


def test_matches_dense_transpose():
    rng = np.random.default_rng(0)
    a = rng.uniform(size=(13, 29)) * (rng.uniform(size=(13, 29)) < 0.3)
    a[4] = 0.0
    a[:, 7] = 0.0
    tp, ti, tv = oracle.csr_transpose(*_csr_of_dense(a), 29)
    ep, ei, ev = _csr_of_dense(a.T)
    np.testing.assert_array_equal(tp, ep)
    np.testing.assert_array_equal(ti, ei)
    np.testing.assert_array_equal(tv, ev)


def test_twice_is_identity_and_sums():
    indptr, indices, values = fi.random_csr(3, 40, 500, 30.0)
    tp, ti, tv = oracle.csr_transpose(indptr, indices, values, 500)
    assert tp[-1] == indptr[-1]
    bp, bi, bv = oracle.csr_transpose(tp, ti, tv, 40)
    np.testing.assert_array_equal(bp, indptr)
    np.testing.assert_array_equal(bi, indices)
    np.testing.assert_array_equal(bv, values)
    w = np.random.default_rng(1).uniform(size=40)
    rows = np.repeat(np.arange(40), np.diff(indptr))
    d1 = np.bincount(indices, weights=values.astype(np.float64) * w[rows], minlength=500)
    vox = np.repeat(np.arange(500), np.diff(tp))
    d2 = np.bincount(vox, weights=tv.astype(np.float64) * w[ti], minlength=500)
    np.testing.assert_allclose(d1, d2, rtol=1e-12, atol=0)


def test_random_csr_shape():
    indptr, indices, values = fi.random_csr(5, 200, 70000, 50.0, empty_frac=0.2)
    assert indptr[0] == 0 and np.all(np.diff(indptr) >= 0) and indptr[-1] == len(indices)
    for j in range(200):
        r = indices[indptr[j]:indptr[j + 1]]
        assert np.all(np.diff(r) > 0) and (len(r) == 0 or (r[0] >= 0 and r[-1] < 70000))
    assert np.all(values > 0) and np.all(values <= 1)
