"""Pins of the oracle's relevancy post-processing against independent routines:
scipy's uniform filter (box mean, clipped window = filtered values over the
filtered indicator), numpy's argmax / min / max, and a brute-force mask."""
import numpy as np
import pytest
from scipy import ndimage


def _box_mean_scipy(M, k):
    out = np.zeros_like(M)
    for l in range(M.shape[0]):
        num = ndimage.uniform_filter(M[l], size=k, mode="constant", cval=0.0)
        den = ndimage.uniform_filter(np.ones_like(M[l]), size=k, mode="constant", cval=0.0)
        out[l] = num / den
    return out


@pytest.mark.parametrize("k", [1, 3, 5, 9])
def test_box_mean_matches_scipy(orc, k):
    rng = np.random.default_rng(k)
    M = rng.random((2, 13, 17))
    S, mask, res, stats = orc.postprocess(M, k)
    assert np.allclose(S, _box_mean_scipy(M, k), rtol=1e-12, atol=1e-12)
    S1, *_ = orc.postprocess(M, k, smooth_mode=1)
    assert np.allclose(S1, 0.5 * (M + S), rtol=1e-12, atol=1e-12)


def test_selection_argmax_and_mask(orc):
    rng = np.random.default_rng(3)
    M = rng.random((3, 20, 30)) * 0.2
    M[1, 7, 11] = 5.0                            # level 1 has the largest smoothed maximum
    S, mask, res, stats = orc.postprocess(M, 3, threshold=0.4)
    assert res[0] == 1
    y, x = np.unravel_index(np.argmax(S[1]), S[1].shape)
    assert (res[1], res[2], res[3]) == (x, y, y * 30 + x)
    assert np.allclose(stats[:, 0], S.reshape(3, -1).max(1)) and np.allclose(stats[:, 1], S.reshape(3, -1).min(1))
    norm = (S[1] - S[1].min()) / (S[1].max() - S[1].min())
    brute = np.array([[1 if norm[i, j] > 0.4 else 0 for j in range(30)] for i in range(20)], np.uint8)
    assert np.array_equal(mask, brute)
    assert stats[1, 3] == brute.sum() and np.isclose(stats[1, 2], S[1][brute == 1].mean())


def test_mask_mean_selection_and_degenerate(orc):
    M = np.zeros((2, 8, 8))
    M[0] += 0.3                                    # constant level: max == min, empty mask
    M[1, :4] = 0.9
    M[1, 4:] = 0.1
    S, mask, res, stats = orc.postprocess(M, 1, select_mode=1, threshold=0.5)
    assert stats[0, 3] == 0 and stats[0, 2] == -np.inf
    assert res[0] == 1 and mask.sum() == 32
    # ties: equal maxima select the first level and the first pixel
    S, mask, res, stats = orc.postprocess(np.ones((2, 4, 5)), 3)
    assert res[0] == 0 and res[3] == 0
