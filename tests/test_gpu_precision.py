"""Precision of the bf16 form at full size (1440x1080, 300k Gaussians, D=512),
codebook size L in {64, 128} and K in {4, 8}: the error of every output
against the FP64 oracle, with the float32 path beside it.

Per (L, K) the GPU renders the whole frame; 3000 random pixels are checked
against the oracle's compositing of the same (GPU-binned) lists, its FP64
decode and its relevancy.  Bars: float32 coefficients / features / relevancy
1e-5 absolute, bf16 features 1e-2 relative per pixel (L2), bf16 relevancy
3e-3 absolute (bf16 rounding of inputs and outputs); pixels within the
oracle's flip margin of a discrete decision are excluded and counted.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import gen
from gpu_common import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

MARGIN = 1e-5


@pytest.mark.parametrize("L,K", [(64, 4), (64, 8), (128, 4), (128, 8)])
def test_bf16_precision_full_size(orc, L, K):
    import paper_2507_07136_amd as ls2
    scene, cam = gen.config_scene("c4", L=L, K=K)
    t = ls2.to_device(scene)
    pipe = ls2.Pipeline(cam, scene.n, levels=1, K=K, L=L, D=scene.D)
    pipe.project(t["means"], t["scales"], t["quats"])
    pipe.bin_sort(sync=True)
    pipe.splat(t["opacity"], t["topk_idx"], t["topk_w"])
    pos, neg = gen.make_text(1004 + 7)
    tp, tn = torch.from_numpy(pos).cuda(), torch.from_numpy(neg).cuda()
    f32 = pipe.decode(t["dictionary"], ls2.LS2_F32, torch.float32).clone()
    r32 = pipe.query(tp, tn).clone()
    bf = pipe.decode(t["dictionary"], ls2.LS2_BF16, torch.bfloat16).clone()
    rbf = pipe.query(tp, tn).clone()
    rcoef = pipe.query_coef(t["dictionary"], tp, tn).clone()
    torch.cuda.synchronize()

    rng = np.random.default_rng(L + K)
    npx = cam.width * cam.height
    pix = rng.choice(npx, 3000, replace=False)
    ranges = pipe.tile_ranges.cpu().numpy().view(np.uint32)
    ids = pipe.ids[:pipe.num_pairs].cpu().numpy().view(np.uint32)
    coef64, _, _, margin, margin_T = orc.composite_pixels(
        cam, ranges, ids, pipe.mean2d.cpu().numpy().astype(np.float64), pipe.conic.cpu().numpy().astype(np.float64),
        scene.opacity, scene.topk_idx, scene.topk_w, L, pix, with_margin_T=True)
    ok = (margin >= MARGIN) & (margin_T >= MARGIN)
    F64 = orc.decode(coef64[:, 0], scene.dictionary)
    r64 = orc.query(F64, pos, neg)

    gcoef = pipe.coef[0].reshape(-1, L)[torch.from_numpy(pix).cuda()].cpu().numpy()
    g32 = f32[0].reshape(-1, scene.D)[torch.from_numpy(pix).cuda()].cpu().numpy()
    gbf = bf[0].reshape(-1, scene.D)[torch.from_numpy(pix).cuda()].float().cpu().numpy()
    sel = torch.from_numpy(pix).cuda()
    gr32 = r32[0].reshape(-1)[sel].cpu().numpy()
    grbf = rbf[0].reshape(-1)[sel].cpu().numpy()
    grc = rcoef[0].reshape(-1)[sel].cpu().numpy()

    nF = np.linalg.norm(F64, axis=1)
    live = ok & (nF > 1e-6)
    err = dict(
        coef_f32_abs=np.abs(gcoef - coef64[:, 0])[ok].max(),
        feat_f32_abs=np.abs(g32 - F64)[ok].max(),
        feat_bf16_rel_l2=(np.linalg.norm(gbf - F64, axis=1)[live] / nF[live]).max(),
        feat_bf16_abs=np.abs(gbf - F64)[ok].max(),
        rel_f32_abs=np.abs(gr32 - r64)[ok].max(),
        rel_bf16_abs=np.abs(grbf - r64)[ok].max(),
        rel_from_coef_abs=np.abs(grc - r64)[ok].max(),
    )
    print("\nprecision L=%d K=%d (P=%d, %d/%d sampled pixels inside the flip margins): %s" % (
        L, K, pipe.num_pairs, int(ok.sum()), len(pix), ", ".join("%s %.2e" % kv for kv in err.items())))
    assert (~ok).sum() <= max(2, 0.01 * len(pix))
    assert err["coef_f32_abs"] <= 2e-5
    assert err["feat_f32_abs"] <= 1e-5
    assert err["feat_bf16_rel_l2"] <= 1e-2
    assert err["rel_f32_abs"] <= 1e-5
    assert err["rel_from_coef_abs"] <= 1e-5
    assert err["rel_bf16_abs"] <= 3e-3


def test_one_pass_frame_full_size(orc):
    """The benchmarked frame at full size (1440x1080, 300k Gaussians, L=64,
    K=4, D=512) in the launch configuration bench.py times: splat_decode and
    splat_decode_query against the FP64 oracle on 3000 sampled pixels
    (features 1e-2 relative, relevancy 3e-3, T 2e-5, last exact, away from
    the flip margins), and bit for bit against the two-pass bf16 path on the
    whole frame."""
    import paper_2507_07136_amd as ls2
    scene, cam = gen.config_scene("c2")
    t = ls2.to_device(scene)
    p16 = ls2.Pipeline(cam, scene.n, levels=1, K=scene.K, L=scene.L, D=scene.D, coef_dtype=torch.bfloat16)
    p16.project(t["means"], t["scales"], t["quats"])
    p16.bin_sort(sync=True)
    pos, neg = gen.make_text(1002 + 7)
    tp, tn = torch.from_numpy(pos).cuda(), torch.from_numpy(neg).cuda()
    feat = p16.splat_decode(t["opacity"], t["topk_idx"], t["topk_w"], t["dictionary"]).clone()
    fT, last = p16.final_T.clone(), p16.last.clone()
    rel = p16.splat_decode_query(t["opacity"], t["topk_idx"], t["topk_w"], t["dictionary"], tp, tn,
                                 keep_feat=False).clone()
    # the two-pass path on the same lists
    p16.splat(t["opacity"], t["topk_idx"], t["topk_w"])
    feat2 = p16.decode(t["dictionary"], ls2.LS2_BF16, torch.bfloat16).clone()
    rel2 = p16.query(tp, tn).clone()
    torch.cuda.synchronize()
    assert torch.equal(feat, feat2) and torch.equal(rel, rel2)

    L, D = scene.L, scene.D
    rng = np.random.default_rng(2024)
    npx = cam.width * cam.height
    pix = rng.choice(npx, 3000, replace=False)
    ranges = p16.tile_ranges.cpu().numpy().view(np.uint32)
    ids = p16.ids[:p16.num_pairs].cpu().numpy().view(np.uint32)
    coef64, fT64, last64, margin, margin_T = orc.composite_pixels(
        cam, ranges, ids, p16.mean2d.cpu().numpy().astype(np.float64), p16.conic.cpu().numpy().astype(np.float64),
        scene.opacity, scene.topk_idx, scene.topk_w, L, pix, with_margin_T=True)
    ok = (margin >= MARGIN) & (margin_T >= MARGIN)
    F64 = orc.decode(coef64[:, 0], scene.dictionary)
    r64 = orc.query(F64, pos, neg)
    sel = torch.from_numpy(pix).cuda()
    gf = feat[0].reshape(-1, D)[sel].float().cpu().numpy()
    gr = rel[0].reshape(-1)[sel].cpu().numpy()
    gT = fT.reshape(-1)[sel].cpu().numpy()
    gl = last.reshape(-1)[sel].cpu().numpy()
    nF = np.linalg.norm(F64, axis=1)
    live = ok & (nF > 1e-6)
    e_feat = (np.linalg.norm(gf - F64, axis=1)[live] / nF[live]).max()
    e_rel = np.abs(gr - r64)[ok].max()
    e_T = np.abs(gT - fT64)[ok].max()
    print("\none-pass frame at full size (P=%d, %d/%d sampled pixels inside the flip margins): features %.2e "
          "relative, relevancy %.2e, T %.2e" % (p16.num_pairs, int(ok.sum()), len(pix), e_feat, e_rel, e_T))
    assert (~ok).sum() <= max(2, 0.01 * len(pix))
    assert e_feat <= 1e-2 and e_rel <= 3e-3 and e_T <= 2e-5
    assert np.array_equal(gl[ok], last64[ok])
