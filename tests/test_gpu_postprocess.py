"""GPU parity of the relevancy post-processing with the oracle (same inputs).

Smoothed maps: float32 against float64, 1e-6 absolute (sums of at most
kernel^2 terms in [0, 1]).  The selected level, the argmax and the mask are
discrete: inputs are drawn so that the decisions are far from ties, and mask
pixels whose normalised value lies within 1e-5 of the threshold are excluded
(counted).  Level statistics: 1e-5 relative."""
import numpy as np
import pytest
import torch

from gpu_common import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _run(rel, k, smooth, select, thr):
    import paper_2507_07136_amd as ls2
    levels, H, W = rel.shape
    t = torch.from_numpy(rel.astype(np.float32)).cuda()
    sm = torch.empty_like(t)
    mask = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    res = torch.empty((4,), dtype=torch.int32, device="cuda")
    stats = torch.empty((levels, 4), dtype=torch.float32, device="cuda")
    ws = torch.empty((ls2.ls2_postprocess_workspace(levels, H, W),), dtype=torch.uint8, device="cuda")
    ls2.ls2_postprocess(t, k, sm, mask, res, ws, smooth_mode=smooth, select_mode=select, threshold=thr,
                        level_stats=stats)
    torch.cuda.synchronize()
    return sm.cpu().numpy(), mask.cpu().numpy(), res.cpu().numpy(), stats.cpu().numpy()


def _smooth_field(rng, levels, H, W):
    yy, xx = np.mgrid[0:H, 0:W]
    out = np.zeros((levels, H, W))
    for l in range(levels):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        amp = 0.3 + 0.2 * l
        out[l] = 0.2 + amp * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * (0.15 * W) ** 2))
        out[l] += 0.05 * rng.random((H, W))
    return np.clip(out, 0.0, 1.0).astype(np.float32)


@pytest.mark.parametrize("smooth,select", [(0, 0), (1, 1), (1, 0), (0, 1)])
@pytest.mark.parametrize("k,H,W", [(5, 67, 91), (9, 135, 240), (1, 16, 17)])
def test_postprocess_parity(orc, smooth, select, k, H, W):
    rng = np.random.default_rng(k * 100 + H + smooth * 7 + select)
    rel = _smooth_field(rng, 3, H, W)
    thr = 0.5
    sm, mask, res, stats = _run(rel, k, smooth, select, thr)
    S, M, R, ST = orc.postprocess(rel.astype(np.float64), k, smooth_mode=smooth, select_mode=select, threshold=thr)
    assert np.abs(sm - S).max() <= 1e-6
    assert np.allclose(stats[:, 0], ST[:, 0], rtol=1e-6) and np.allclose(stats[:, 1], ST[:, 1], rtol=1e-6)
    assert res[0] == R[0]
    # argmax: the GPU's point is a maximum of the oracle's map to float32 rounding
    lv = R[0]
    assert S[lv].reshape(-1)[res[3]] >= S[lv].max() - 1e-6 and res[1] == res[3] % W and res[2] == res[3] // W
    mx, mn = S[lv].max(), S[lv].min()
    norm = (S[lv] - mn) / (mx - mn)
    near = np.abs(norm - thr) < 1e-5
    assert near.sum() <= max(2, 1e-3 * H * W)
    assert np.array_equal(mask[~near], M[~near])
    assert np.allclose(stats[:, 3], ST[:, 3], atol=near.sum() + 0.5)
    fin = np.isfinite(ST[:, 2])
    assert np.allclose(stats[fin, 2], ST[fin, 2], rtol=1e-5)
    assert np.all(np.isneginf(stats[~fin, 2]))


def test_postprocess_ties_and_constant(orc):
    rel = np.full((2, 10, 12), 0.4, np.float32)
    sm, mask, res, stats = _run(rel, 3, 0, 0, 0.5)
    assert res[0] == 0 and res[3] == 0 and mask.sum() == 0
    assert np.isneginf(stats[0, 2]) and stats[0, 3] == 0
