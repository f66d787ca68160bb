"""Pins of the sparse-code parametrisation (Section 3.3): the kept weights are
scipy's softmax of the kept logits and sum to 1, the selection equals
numpy's stable descending argsort, K = L reduces to the plain softmax, and the
backward matches central finite differences of the forward."""
import numpy as np
import pytest
from scipy.special import softmax


def test_forward_against_library(orc):
    rng = np.random.default_rng(0)
    z = rng.normal(size=(50, 64))
    z[3, 10] = z[3, 20]                       # a tie: the smaller index comes first
    idx, w = orc.sparse_codes(z, 4)
    for r in range(50):
        order = np.argsort(-z[r], kind="stable")[:4]
        assert np.array_equal(idx[r], order)
        assert np.allclose(w[r], softmax(z[r, order]), rtol=1e-13)
    assert np.allclose(w.sum(1), 1.0)
    idx, w = orc.sparse_codes(z, 64)
    assert np.allclose(np.take_along_axis(softmax(z, axis=1), idx.astype(np.int64), 1), w)


@pytest.mark.parametrize("K", [1, 4, 8])
def test_backward_finite_differences(orc, K):
    rng = np.random.default_rng(K)
    z = rng.normal(size=(6, 16)) * 2
    dw = rng.normal(size=(6, K))
    dz = orc.sparse_codes_backward(z, K, dw)
    h = 1e-6
    num = np.zeros_like(z)
    for r in range(6):
        for j in range(16):
            zp, zm = z.copy(), z.copy()
            zp[r, j] += h
            zm[r, j] -= h
            ip, wp = orc.sparse_codes(zp, K)
            im, wm = orc.sparse_codes(zm, K)
            assert np.array_equal(ip, im)      # no selection change within +-h (random logits)
            num[r, j] = ((wp - wm) * dw).sum() / (2 * h)
    assert np.allclose(dz, num, rtol=1e-6, atol=1e-9)
