"""Precision of the bf16 form at full size (1440x1080, 300k Gaussians, D=512),
codebook size L in {64, 128} and K in {4, 8}: the error of every output
against the FP64 oracle, with the float32 path beside it.

Per (L, K) the GPU renders the whole frame; 3000 random pixels are checked
against the oracle's compositing of the same (GPU-binned) lists, its FP64
decode and its relevancy.  Bars: float32 coefficients / features / relevancy
1e-5 absolute, bf16 features 1e-2 relative per pixel (L2), bf16 relevancy
3e-3 absolute (bf16 rounding of inputs and outputs), final T 1e-5, last
exact.  Every sampled pixel is checked; one that misses the oracle's walk
passes if it meets every bar against the walk with some of its near
decisions taken the other way (tests/alt_check.py), and at most 0.1 % may
meet neither.  The reported maxima are over the pixels that match the plain
walk.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import gen
from alt_check import check_flips
from gpu_common import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

BARS = dict(coef_f32_abs=1e-5, feat_f32_abs=1e-5, feat_bf16_rel_l2=1e-2, rel_f32_abs=1e-5, rel_from_coef_abs=1e-5,
            rel_bf16_abs=3e-3, T_abs=1e-5)


def _rows(x, sel):
    return x[sel].float().cpu().numpy()


def _errors(orc, dictionary, pos, neg, got, sel, c, t, l):
    """Per-pixel errors of the GPU outputs (got: dict of per-pixel arrays in
    pix order) against one oracle outcome c [len(sel), 1, L], t, l."""
    F = orc.decode(c[:, 0], dictionary)
    r = orc.query(F, pos, neg)
    nF = np.linalg.norm(F, axis=1)
    e = dict(T_abs=np.abs(got["T"][sel] - t))
    if "coef" in got:
        e["coef_f32_abs"] = np.abs(got["coef"][sel] - c[:, 0]).max(axis=1)
    if "f32" in got:
        e["feat_f32_abs"] = np.abs(got["f32"][sel] - F).max(axis=1)
    if "bf" in got:
        e["feat_bf16_rel_l2"] = np.where(nF > 1e-6, np.linalg.norm(got["bf"][sel] - F, axis=1) / np.maximum(nF, 1e-6),
                                         0.0)
    for k, name in (("r32", "rel_f32_abs"), ("rbf", "rel_bf16_abs"), ("rc", "rel_from_coef_abs")):
        if k in got:
            e[name] = np.abs(got[k][sel] - r)
    return e, got["last"][sel] == l


def _flip_checked(orc, cam, scene, ranges, ids, mean2d, conic, pix, pos, neg, got, label):
    def close(sel, c, t, l):
        e, same_last = _errors(orc, scene.dictionary, pos, neg, got, sel, c, t, l)
        ok = same_last.copy()
        for k, v in e.items():
            ok &= v <= BARS[k]
        return ok

    res = check_flips(orc, cam, ranges, ids, mean2d, conic, scene.opacity, scene.topk_idx, scene.topk_w, scene.L,
                      pix, close, label=label)
    c, t, l = res["base"]
    e, _ = _errors(orc, scene.dictionary, pos, neg, got, np.arange(len(pix)), c, t, l)
    return res, {k: float(v[res["base_ok"]].max()) for k, v in e.items()}


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
    sel = torch.from_numpy(pix).cuda()
    got = dict(coef=_rows(pipe.coef[0].reshape(-1, L), sel), f32=_rows(f32[0].reshape(-1, scene.D), sel),
               bf=_rows(bf[0].reshape(-1, scene.D), sel), r32=_rows(r32[0].reshape(-1), sel),
               rbf=_rows(rbf[0].reshape(-1), sel), rc=_rows(rcoef[0].reshape(-1), sel),
               T=_rows(pipe.final_T.reshape(-1), sel), last=pipe.last.reshape(-1)[sel].cpu().numpy())
    res, err = _flip_checked(orc, cam, scene, ranges, ids, pipe.mean2d.cpu().numpy().astype(np.float64),
                             pipe.conic.cpu().numpy().astype(np.float64), pix, pos, neg, got,
                             "precision L=%d K=%d" % (L, K))
    print("precision L=%d K=%d (P=%d): %s" % (L, K, pipe.num_pairs, ", ".join("%s %.2e" % kv for kv in err.items())))
    for k, v in err.items():
        assert v <= BARS[k], k


def test_one_pass_frame_full_size(orc):
    """The benchmarked frame at full size (1440x1080, 300k Gaussians, L=64,
    K=4, D=512) in the launch configuration bench.py times: splat_decode and
    splat_decode_query against the FP64 oracle on 3000 sampled pixels
    (features 1e-2 relative, relevancy 3e-3, T 1e-5, last exact; every pixel
    checked, with the flipped outcomes of its near decisions), and bit for
    bit against the two-pass bf16 path on the whole frame."""
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
    sel = torch.from_numpy(pix).cuda()
    got = dict(bf=_rows(feat[0].reshape(-1, D), sel), rbf=_rows(rel[0].reshape(-1), sel),
               T=_rows(fT.reshape(-1), sel), last=last.reshape(-1)[sel].cpu().numpy())
    res, err = _flip_checked(orc, cam, scene, ranges, ids, p16.mean2d.cpu().numpy().astype(np.float64),
                             p16.conic.cpu().numpy().astype(np.float64), pix, pos, neg, got, "one-pass frame")
    print("one-pass frame at full size (P=%d): %s" % (p16.num_pairs, ", ".join("%s %.2e" % kv for kv in err.items())))
    for k, v in err.items():
        assert v <= BARS[k], k
