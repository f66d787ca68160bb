"""Full-form parity at full size, on sampled outputs: 1M Gaussians at
1920x1080, three semantic levels (L=64, K=4 each over one 64x512 codebook),
view 3 of the 8-view orbit, run through the same Trainer calls and launch
configuration as the benchmark's full-form training step.

The map has M = 3 x 1920 x 1080 rows of 512 features, 3.2e9 elements, past
2^31: these checks cover the 64-bit addressing of every kernel on the path.

HIP through the C ABI against the FP64 oracle, stage-isolated as in the small
parity tests (each stage consumes the GPU's own float32 upstream state):
  - projection of 2000 sampled Gaussians (independent per Gaussian): mean2d
    within 4 float32 ulps of max(|u - cx|, cx), depth 1e-6 relative, conic
    1e-4 relative, radius exact away from integer extents;
  - binning: ids and tile ranges bit-exact over all 48M pairs;
  - compositing of 3000 sampled pixels, all levels: |dW| <= 1e-5, |dT| <=
    1e-5, last exact; every sampled pixel checked, a pixel that misses the
    oracle's walk matching it with some near decisions flipped, at most
    0.1 % matching neither (tests/alt_check.py);
  - float32 decode fused with the L1 + cosine loss: feature rows |dF| <=
    1e-5 and dL/dF rows of 2000 sampled rows (the loss is a mean over rows,
    so a row's gradient is the oracle's gradient over the sampled rows times
    n_sampled / M) within 1e-5 of the row's max|dL/dF|, elements whose residual F - Y
    is within 1e-5 of zero (the sign of the L1 term may flip) excluded;
  - the training step's one-pass decode + loss + decode backward against
    the two-call chain on the whole map: bit for bit;
  - decode backward with dL/dF zero outside 2000 sampled rows: d_dict over
    the whole map against the oracle's over those rows, |dg| <= 1e-5 |A||B|;
    the sampled rows' d_coef likewise; every other row exactly zero;
  - splat backward with dL/dcoef zero outside 1500 sampled pixels: the
    gradient of every Gaussian against the oracle's pixel-list backward
    (1e-3 relative per tensor and element, 1e-3 max floor);
  - projection backward of 2000 sampled Gaussians (same bar);
  - softmax top-K codes of all 3M (Gaussian, level) rows: 3000 sampled rows,
    indices bit-exact, weights 1e-6.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import gen
from alt_check import coef_close
from gpu_common import compare_tile_lists, flip_check_gpu_lists, gpu_available, grad_close

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

MARGIN = 1e-5
VIEW, N_VIEWS = 3, 8


def _rows(x, idx):
    """Rows ``idx`` of a device tensor viewed as (rows, -1), as float64 numpy."""
    return x.index_select(0, torch.from_numpy(np.asarray(idx, np.int64)).cuda()).double().cpu().numpy()


@pytest.fixture(scope="module")
def c5(orc):
    import paper_2507_07136_amd as ls2
    cfg = gen.CONFIGS["c5"]
    scene, _ = gen.config_scene("c5")
    H, W, D, levels = cfg["height"], cfg["width"], cfg["D"], cfg["levels"]
    t = ls2.to_device(scene)
    tr = ls2.Trainer(gen.orbit_camera(W, H, 0, N_VIEWS), scene.n, levels=levels, K=scene.K, L=scene.L, D=D)
    cam = gen.orbit_camera(W, H, VIEW, N_VIEWS)
    tr.set_camera(cam)
    Y = torch.empty((levels, H, W, D), dtype=torch.float32, device="cuda")
    for lv in range(levels):
        zup, Pf = gen.make_target_factors(cfg["seed"] * 100 + 8 * lv + VIEW, H, W, D=D)
        Y[lv] = (torch.from_numpy(zup).cuda().reshape(-1, zup.shape[-1]) @ torch.from_numpy(Pf).cuda()).reshape(
            H, W, D)
    tr.forward_loss(t, Y, sync=True, keep_feat=True)
    torch.cuda.synchronize()
    P = tr.num_pairs
    g = dict(P=P, mean2d=tr.mean2d.cpu().numpy(), conic=tr.conic.cpu().numpy(), depth=tr.depth.cpu().numpy(),
             radius=tr.radius.cpu().numpy(), touched=tr.tiles_touched.cpu().numpy(),
             ranges=tr.tile_ranges.cpu().numpy().view(np.uint32), ids=tr.ids[:P].cpu().numpy().view(np.uint32))
    print("full form view %d: P = %d" % (VIEW, P))
    yield scene, cam, tr, t, Y, g
    del tr, t, Y
    torch.cuda.empty_cache()


def test_full_form_project_sampled(orc, c5):
    scene, cam, tr, t, Y, g = c5
    rng = np.random.default_rng(51)
    s = np.sort(rng.choice(scene.n, 2000, replace=False))
    pr = orc.project(cam, scene.means[s], scene.scales[s], scene.quats[s])
    near = np.abs(pr["extent"] - np.round(pr["extent"])) < 1e-4
    assert ((g["radius"][s] == pr["radius"]) | near).all()
    vis = (pr["radius"] > 0) & (g["radius"][s] > 0)
    assert vis.sum() > 1000
    # u = fx x / z + cx: the float32 sum's rounding is set by the larger of
    # |u - cx| and cx (about 6e-5 px per ulp at 1920 wide); 4 ulps of it
    pp = np.array([cam.cx, cam.cy])
    ulp = np.spacing(np.maximum(np.abs(pr["mean2d"] - pp), pp).astype(np.float32)).astype(np.float64)
    assert (np.abs(g["mean2d"][s] - pr["mean2d"]) <= 4 * ulp)[vis].all()
    np.testing.assert_allclose(g["depth"][s][vis], pr["depth"][vis], rtol=1e-6)
    np.testing.assert_allclose(g["conic"][s][vis], pr["conic"][vis], rtol=1e-4,
                               atol=1e-6 * np.abs(pr["conic"]).max())
    exact = vis & ~near
    assert np.array_equal(g["touched"][s][exact], pr["touched"][exact])


def test_full_form_bin_sort_bit_exact(orc, c5):
    scene, cam, tr, t, Y, g = c5
    keys, ids, ranges = orc.tile_lists(cam, g["mean2d"], g["radius"], g["depth"])
    assert g["P"] == len(ids) and g["P"] > 2 ** 25
    diff = compare_tile_lists(dict(g, keys=None), keys, ids, ranges, cam.tiles_x, cam.tiles_y)
    assert diff is None, diff


@pytest.fixture(scope="module")
def c5_pixels(orc, c5):
    """Oracle compositing of 3000 sampled pixels from the GPU's lists; ok
    marks those with no decision within 1e-5 of its threshold (the backward
    check draws its pixels from them)."""
    scene, cam, tr, t, Y, g = c5
    rng = np.random.default_rng(52)
    pix = rng.choice(cam.width * cam.height, 3000, replace=False)
    coef, fT, last, margin, margin_T = orc.composite_pixels(
        cam, g["ranges"], g["ids"], g["mean2d"].astype(np.float64), g["conic"].astype(np.float64), scene.opacity,
        scene.topk_idx, scene.topk_w, scene.L, pix, with_margin_T=True)
    ok = (margin >= MARGIN) & (margin_T >= MARGIN)
    print("pixels with a decision near its threshold: %d of %d" % ((~ok).sum(), ok.size))
    return pix, coef, fT, last, ok


def test_full_form_splat_sampled(orc, c5, c5_pixels):
    scene, cam, tr, t, Y, g = c5
    pix, coef, fT, last, ok = c5_pixels
    HW = cam.width * cam.height
    got = np.stack([_rows(tr.coef[lv].reshape(HW, scene.L), pix) for lv in range(scene.levels)], axis=1)
    err = np.abs(got - coef).reshape(len(pix), -1).max(axis=1)
    print("full-form coefficient max err %.3e" % err.max())
    close = coef_close(got, _rows(tr.final_T.reshape(HW, 1), pix)[:, 0],
                       _rows(tr.last.reshape(HW, 1), pix)[:, 0].astype(np.int64), 1e-5)
    flip_check_gpu_lists(orc, cam, scene, g, close, pix=pix, base=(coef, fT, last), label="full form")


def test_full_form_decode_loss_sampled(orc, c5):
    scene, cam, tr, t, Y, g = c5
    M = scene.levels * cam.width * cam.height
    rng = np.random.default_rng(53)
    rows = np.sort(rng.choice(M, 2000, replace=False))
    C = _rows(tr.coef.view(M, scene.L), rows)
    F64 = orc.decode(C, scene.dictionary)
    assert np.abs(_rows(tr.feat.view(M, scene.D), rows) - F64).max() <= 1e-5
    Ys = _rows(Y.view(M, scene.D), rows)
    _, dF = orc.loss_l1cos(F64, Ys)
    ref = dF * (len(rows) / M)
    got = _rows(tr.d_feat.view(M, scene.D), rows)
    flip = np.abs(F64 - Ys) < 1e-5
    assert flip.sum() <= 1e-3 * flip.size
    # per row: near-empty pixels (|F| -> 0) carry cosine gradients ~1/|F|, so
    # a global bound would hide the ordinary rows
    err = np.where(flip, 0.0, np.abs(got - ref)).max(axis=1) / np.abs(ref).max(axis=1)
    print("dL/dF sampled rows: worst per-row error %.3e of the row's max (global max %.3e; %d elements near a "
          "sign flip)" % (err.max(), np.abs(ref).max(), int(flip.sum())))
    assert err.max() <= 1e-5
    assert np.isfinite(tr.loss.item()) and tr.loss.item() > 0


def test_full_form_one_pass_loss_backward(c5):
    """The training step's one-pass decode + loss + decode backward at full
    size (3.2e9 feature elements, past 2^31) equals the two-call chain bit for
    bit: d_coef, d_dict and, with one workgroup per compute unit in both, the
    loss."""
    import paper_2507_07136_amd as ls2
    scene, cam, tr, t, Y, g = c5
    M, L, D = scene.levels * cam.height * cam.width, scene.L, scene.D
    loss_c = tr.decode_loss(t["dictionary"], Y).clone()
    dc_c = torch.empty((M, L), device="cuda")
    ds_c = torch.empty((L, D), device="cuda")
    ls2.ls2_dict_decode_backward(tr.coef.view(M, L), t["dictionary"], tr.d_feat.view(M, D), dc_c, ds_c, tr.dec_ws)
    loss_f = torch.zeros((1,), dtype=torch.float64, device="cuda")
    dc_f = torch.empty((M, L), device="cuda")
    ds_f = torch.empty((L, D), device="cuda")
    ls2.ls2_decode_loss_backward(tr.coef.view(M, L), t["dictionary"], Y.view(M, D), loss_f, dc_f, ds_f,
                                 tr.onepass_ws)
    torch.cuda.synchronize()
    assert torch.equal(dc_f, dc_c)
    assert torch.equal(ds_f, ds_c)
    assert loss_f.item() == loss_c.item()
    del dc_c, dc_f


def test_full_form_decode_backward_sparse_upstream(orc, c5):
    import paper_2507_07136_amd as ls2
    scene, cam, tr, t, Y, g = c5
    M, L, D = scene.levels * cam.width * cam.height, scene.L, scene.D
    rng = np.random.default_rng(54)
    rows = np.sort(rng.choice(M, 2000, replace=False))
    Gs = rng.standard_normal((len(rows), D)).astype(np.float32)
    G = torch.zeros((M, D), dtype=torch.float32, device="cuda")
    ridx = torch.from_numpy(rows).cuda()
    G.index_copy_(0, ridx, torch.from_numpy(Gs).cuda())
    d_coef = torch.empty((M, L), dtype=torch.float32, device="cuda")
    d_dict = torch.empty((L, D), dtype=torch.float32, device="cuda")
    ls2.ls2_dict_decode_backward(tr.coef.view(M, L), t["dictionary"], G, d_coef, d_dict, tr.dec_ws)
    torch.cuda.synchronize()
    del G
    C = _rows(tr.coef.view(M, L), rows)
    rc, rd = orc.decode_backward(C, scene.dictionary, Gs.astype(np.float64))
    Sd = scene.dictionary.astype(np.float64)
    assert (np.abs(d_dict.double().cpu().numpy() - rd) <= 1e-5 * (np.abs(C).T @ np.abs(Gs)) + 1e-30).all()
    got = _rows(d_coef, rows)
    assert (np.abs(got - rc) <= 1e-5 * (np.abs(Gs) @ np.abs(Sd).T) + 1e-30).all()
    nz = torch.nonzero(d_coef.abs().sum(dim=1)).flatten().cpu().numpy()
    assert np.isin(nz, rows).all(), "non-zero d_coef outside the sampled rows"


def test_full_form_splat_backward_sparse_upstream(orc, c5, c5_pixels):
    import paper_2507_07136_amd as ls2
    scene, cam, tr, t, Y, g = c5
    pix, _, _, _, ok = c5_pixels
    sel = np.sort(pix[ok][:1500])
    HW, lv, K, L, n = cam.width * cam.height, scene.levels, scene.K, scene.L, scene.n
    rng = np.random.default_rng(55)
    Gp = rng.standard_normal((len(sel), lv, L)).astype(np.float32)
    d_coef = torch.zeros((lv, HW, L), dtype=torch.float32, device="cuda")
    sidx = torch.from_numpy(sel).cuda()
    for l in range(lv):
        d_coef[l].index_copy_(0, sidx, torch.from_numpy(np.ascontiguousarray(Gp[:, l])).cuda())
    out = dict(mean2d=torch.empty((n, 2), device="cuda"), conic=torch.empty((n, 3), device="cuda"),
               opacity=torch.empty((n,), device="cuda"), topk_w=torch.empty((n, lv, K), device="cuda"))
    ls2.ls2_splat_sparse_backward(tr.cam, lv, K, L, tr.tile_ranges, tr.ids, tr.mean2d, tr.conic, t["opacity"],
                                  t["topk_idx"], t["topk_w"], tr.final_T, tr.last, d_coef, out["mean2d"],
                                  out["conic"], out["opacity"], out["topk_w"])
    torch.cuda.synchronize()
    del d_coef
    ref = orc.composite_backward_pixels(cam, g["ranges"], g["ids"], g["mean2d"].astype(np.float64),
                                        g["conic"].astype(np.float64), scene.opacity, scene.topk_idx,
                                        scene.topk_w, sel, Gp.astype(np.float64))
    touched = 0
    for name, r in zip(["mean2d", "conic", "opacity", "topk_w"], ref):
        o = out[name].cpu().numpy()
        touched = max(touched, int((np.abs(r).reshape(n, -1).max(axis=1) > 0).sum()))
        grad_close(o, r, "d_" + name)
    print("Gaussians with a gradient from the %d sampled pixels: %d" % (len(sel), touched))
    assert touched > 1000


def test_full_form_project_backward_sampled(orc, c5):
    import paper_2507_07136_amd as ls2
    scene, cam, tr, t, Y, g = c5
    n = scene.n
    rng = np.random.default_rng(56)
    dm = rng.standard_normal((n, 2)).astype(np.float32)
    dc = (rng.standard_normal((n, 3)) / (np.abs(g["conic"]).max(axis=1, keepdims=True) + 1e-6)).astype(np.float32)
    outs = [torch.empty((n, k), device="cuda") for k in (3, 3, 4)]
    ls2.ls2_project_backward(tr.cam, t["means"], t["scales"], t["quats"], tr.radius, torch.from_numpy(dm).cuda(),
                             torch.from_numpy(dc).cuda(), *outs)
    torch.cuda.synchronize()
    s = np.sort(rng.choice(n, 2000, replace=False))
    ref = orc.project_backward(cam, scene.means[s], scene.scales[s], scene.quats[s], g["radius"][s],
                               dm[s].astype(np.float64), dc[s].astype(np.float64))
    culled = g["radius"][s] == 0
    for name, o, r in zip(["means", "scales", "quats"], outs, ref):
        o = o.cpu().numpy()[s]
        assert np.all(o[culled] == 0.0), name
        grad_close(o, r, "d_" + name)


def test_full_form_sparse_codes_sampled(orc):
    import paper_2507_07136_amd as ls2
    cfg = gen.CONFIGS["c5"]
    rows, L, K = cfg["n"] * cfg["levels"], cfg["L"], cfg["K"]
    rng = np.random.default_rng(57)
    z = rng.standard_normal((rows, L), dtype=np.float32)
    tz = torch.from_numpy(z).cuda()
    idx = torch.empty((rows, K), dtype=torch.int32, device="cuda")
    w = torch.empty((rows, K), dtype=torch.float32, device="cuda")
    ls2.ls2_sparse_codes(tz, K, idx, w)
    torch.cuda.synchronize()
    s = np.sort(rng.choice(rows, 3000, replace=False))
    ridx, rw = orc.sparse_codes(z[s], K)
    assert np.array_equal(_rows(idx, s).astype(np.int32), ridx)
    assert np.abs(_rows(w, s) - rw).max() <= 1e-6
