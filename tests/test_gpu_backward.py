"""GPU parity of the backward pass (HIP through the C ABI vs the FP64 oracle).

Tolerances (float32 kernels against float64 references on identical inputs):
  - gradients of the splat and projection, and through the whole composed
    chain: per tensor |dg|_2 <= 1e-3 |g|_2 and per element
    |dg| <= 1e-3 max(|g|, 1e-3 max|g|);
  - the training step on the finite-difference scene (500 Gaussians, 64x64,
    D = 512) against central differences of the float64 oracle's whole
    forward, sampled parameters of every kind, the same bars;
  - decode backward (plain float32 products): per element
    |dg| <= 1e-5 (|A| |B|)  -- the product of absolute values bounds the
    float32 accumulation error;
  - loss value (compensated float32 sums on the GPU): relative 1e-6; dL/dF
    per element 1e-5 max|dF|;
  - query backward: per row |dg|_2 <= 1e-4 |g|_2 (rows whose two largest
    negative similarities are within 1e-4 are excluded: the minimum picks a
    different negative there).
Stage isolation: each backward consumes the GPU's own float32 forward state.
Discrete decisions of the splat (skip, clamp, stop) that are within the
oracle's margin of flipping are neutralised by zeroing dL/dcoef at those
pixels on both sides (a pixel with zero upstream gradient contributes nothing
to any Gaussian); the count is reported and bounded.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import gen
from gpu_common import grad_close as _grad_close
from gpu_common import compare_tile_lists, gpu_available, oracle_composite_from_gpu, run_forward, small_scene

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

MARGIN = 1e-5
CHAIN_FLOOR = 1e-3


def _risky_pixels(margin, margin_T):
    return (margin < MARGIN) | (margin_T < MARGIN)


def _splat_backward_gpu(g, scene, d_coef):
    import paper_2507_07136_amd as ls2
    pipe, t = g["pipe"], g["t"]
    n, lv, K = scene.topk_idx.shape
    dev = "cuda"
    out = dict(mean2d=torch.empty((n, 2), device=dev), conic=torch.empty((n, 3), device=dev),
               opacity=torch.empty((n,), device=dev), topk_w=torch.empty((n, lv, K), device=dev))
    ls2.ls2_splat_sparse_backward(pipe.cam, lv, K, scene.L, pipe.tile_ranges, pipe.ids, pipe.mean2d, pipe.conic,
                                  t["opacity"], t["topk_idx"], t["topk_w"], pipe.final_T, pipe.last,
                                  torch.from_numpy(np.ascontiguousarray(d_coef, np.float32)).cuda(),
                                  out["mean2d"], out["conic"], out["opacity"], out["topk_w"])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("cfg", [
    dict(seed=1100, n=500, w=64, h=64, L=64, K=4, levels=1),      # the FD scene
    dict(seed=1001, n=2000, w=128, h=128, L=64, K=4, levels=1),   # small parity scene
    dict(seed=77, n=3000, w=100, h=75, L=32, K=8, levels=2),      # ragged image, K = 8, 2 levels
    dict(seed=78, n=1500, w=90, h=70, L=64, K=3, levels=3),       # K < KMAX, 3 levels
    dict(seed=79, n=1200, w=80, h=48, L=128, K=5, levels=1),      # L = 128
])
def test_splat_backward_parity(orc, cfg):
    scene, cam = small_scene(cfg["seed"], cfg["n"], cfg["w"], cfg["h"], L=cfg["L"], K=cfg["K"],
                             levels=cfg["levels"], D=128)
    g = run_forward(cam, scene)
    coef, fT, last, margin, margin_T = oracle_composite_from_gpu(orc, cam, scene, g)
    rng = np.random.default_rng(cfg["seed"] + 5)
    d_coef = rng.standard_normal(coef.shape).astype(np.float32)
    risky = _risky_pixels(margin, margin_T)
    d_coef[:, risky, :] = 0.0
    assert risky.mean() <= 1e-2, risky.mean()
    got = _splat_backward_gpu(g, scene, d_coef)
    ref = orc.composite_backward(cam, g["ranges"], g["ids"], g["mean2d"].astype(np.float64),
                                 g["conic"].astype(np.float64), scene.opacity, scene.topk_idx, scene.topk_w,
                                 d_coef.astype(np.float64))
    print("splat backward: %d pixels neutralised of %d" % (int(risky.sum()), risky.size))
    for name, r in zip(["mean2d", "conic", "opacity", "topk_w"], ref):
        _grad_close(got[name], r, "d_" + name)


def test_splat_backward_forward_state(orc):
    """last and final_T that the backward consumes equal the oracle's walk."""
    scene, cam = small_scene(1100, 500, 64, 64, D=128)
    g = run_forward(cam, scene)
    coef, fT, last, margin, margin_T = oracle_composite_from_gpu(orc, cam, scene, g)
    ok = ~_risky_pixels(margin, margin_T)
    assert np.array_equal(g["last"][ok], last[ok])
    assert np.abs(g["final_T"][ok] - fT[ok]).max() <= 1e-5


def test_project_backward_parity(orc):
    import paper_2507_07136_amd as ls2
    for seed, n, w, h in [(1001, 2000, 128, 128), (1100, 500, 64, 64), (91, 5000, 200, 120)]:
        scene, cam = small_scene(seed, n, w, h, D=128)
        t = ls2.to_device(scene)
        pipe = ls2.Pipeline(cam, n)
        pipe.project(t["means"], t["scales"], t["quats"])
        rng = np.random.default_rng(seed + 9)
        dm = rng.standard_normal((n, 2)).astype(np.float32)
        # conic gradients scaled like the conic itself
        conic = pipe.conic.cpu().numpy()
        dc = (rng.standard_normal((n, 3)) * (1.0 / (np.abs(conic).max(axis=1, keepdims=True) + 1e-6))).astype(
            np.float32)
        outs = [torch.empty((n, k), device="cuda") for k in (3, 3, 4)]
        ls2.ls2_project_backward(pipe.cam, t["means"], t["scales"], t["quats"], pipe.radius,
                                 torch.from_numpy(dm).cuda(), torch.from_numpy(dc).cuda(), *outs)
        torch.cuda.synchronize()
        radius = pipe.radius.cpu().numpy()
        ref = orc.project_backward(cam, scene.means, scene.scales, scene.quats, radius, dm.astype(np.float64),
                                   dc.astype(np.float64))
        culled = radius == 0
        for name, o, r in zip(["means", "scales", "quats"], outs, ref):
            o = o.cpu().numpy()
            assert np.all(o[culled] == 0.0), name
            _grad_close(o, r, "d_" + name)


def _abs_bound(a, b):
    return np.abs(a) @ np.abs(b)


@pytest.mark.parametrize("m,L,D", [(4096, 64, 512), (1000, 64, 512), (777, 32, 256), (513, 128, 384),
                                   (300, 32, 1024), (64, 128, 128), (1, 64, 512), (33, 64, 1024),
                                   # many 32-pixel tiles per workgroup, ragged tails, 6 and 2 waves
                                   (100003, 64, 512), (40009, 64, 384), (9001, 32, 128)])
def test_decode_backward_parity(orc, m, L, D):
    import paper_2507_07136_amd as ls2
    rng = np.random.default_rng(m * 7 + L + D)
    coef = (rng.random((m, L)) * (rng.random((m, L)) < 0.2)).astype(np.float32)
    dct = rng.standard_normal((L, D)).astype(np.float32)
    gf = rng.standard_normal((m, D)).astype(np.float32)
    dc_ref, ds_ref = orc.decode_backward(coef, dct, gf)
    tc, td, tg = (torch.from_numpy(x).cuda() for x in (coef, dct, gf))
    d_coef = torch.empty((m, L), device="cuda")
    d_dict = torch.empty((L, D), device="cuda")
    ws = torch.empty((max(1, ls2.ls2_dict_decode_backward_workspace(m, L, D)),), dtype=torch.uint8, device="cuda")
    ls2.ls2_dict_decode_backward(tc, td, tg, d_coef, d_dict, ws)
    torch.cuda.synchronize()
    e1 = np.abs(d_coef.cpu().numpy() - dc_ref)
    assert (e1 <= 1e-5 * _abs_bound(gf.astype(np.float64), dct.T.astype(np.float64)) + 1e-12).all(), e1.max()
    e2 = np.abs(d_dict.cpu().numpy() - ds_ref)
    assert (e2 <= 1e-5 * _abs_bound(coef.T.astype(np.float64), gf.astype(np.float64)) + 1e-12).all(), e2.max()


def test_decode_backward_options(orc):
    """Either output alone; the empty product gives d_dict = 0; deterministic."""
    import paper_2507_07136_amd as ls2
    m, L, D = 2000, 64, 512
    rng = np.random.default_rng(3)
    coef = rng.random((m, L)).astype(np.float32)
    dct = rng.standard_normal((L, D)).astype(np.float32)
    gf = rng.standard_normal((m, D)).astype(np.float32)
    tc, td, tg = (torch.from_numpy(x).cuda() for x in (coef, dct, gf))
    ws = torch.empty((ls2.ls2_dict_decode_backward_workspace(m, L, D),), dtype=torch.uint8, device="cuda")
    a = torch.empty((m, L), device="cuda")
    ls2.ls2_dict_decode_backward(tc, td, tg, a, None, None)
    b1 = torch.empty((L, D), device="cuda")
    b2 = torch.empty((L, D), device="cuda")
    ls2.ls2_dict_decode_backward(tc, td, tg, None, b1, ws)
    ls2.ls2_dict_decode_backward(tc, td, tg, None, b2, ws)
    torch.cuda.synchronize()
    dc_ref, ds_ref = orc.decode_backward(coef, dct, gf)
    g64 = gf.astype(np.float64)
    assert (np.abs(a.cpu().numpy() - dc_ref) <= 1e-5 * _abs_bound(g64, dct.T.astype(np.float64))).all()
    assert torch.equal(b1, b2)
    assert (np.abs(b1.cpu().numpy() - ds_ref) <= 1e-5 * _abs_bound(coef.T.astype(np.float64), g64)).all()
    z = torch.full((L, D), 7.0, device="cuda")
    ls2.ls2_dict_decode_backward(tc[:0], td, tg[:0], None, z, None)
    torch.cuda.synchronize()
    assert torch.count_nonzero(z).item() == 0
    with pytest.raises(ls2.LS2Error):
        ls2.ls2_dict_decode_backward(tc, td, tg, None, b1, None)   # d_dict without workspace


@pytest.mark.parametrize("m,D", [(3000, 512), (257, 128), (100, 1024), (1, 64)])
def test_feature_loss_parity(orc, m, D):
    import paper_2507_07136_amd as ls2
    rng = np.random.default_rng(m + D)
    F = rng.standard_normal((m, D)).astype(np.float32) * 0.3
    Y = rng.standard_normal((m, D)).astype(np.float32) * 0.3
    F[0, : D // 2] = Y[0, : D // 2]          # exact zeros of F - Y: sign(0) = 0
    if m > 2:
        F[1] = 0.0                           # zero feature: cosine guard
    loss_ref, dF_ref = orc.loss_l1cos(F, Y)
    tF, tY = torch.from_numpy(F).cuda(), torch.from_numpy(Y).cuda()
    loss = torch.zeros((1,), dtype=torch.float64, device="cuda")
    dF = torch.empty_like(tF)
    ws = torch.empty((ls2.ls2_feature_loss_workspace(m),), dtype=torch.uint8, device="cuda")
    ls2.ls2_feature_loss(tF, tY, loss, dF, ws)
    loss2 = torch.zeros((1,), dtype=torch.float64, device="cuda")
    ls2.ls2_feature_loss(tF, tY, loss2, None, ws)
    torch.cuda.synchronize()
    assert abs(loss.item() - loss_ref) <= 1e-6 * abs(loss_ref), (loss.item(), loss_ref)
    assert loss.item() == loss2.item()
    err = np.abs(dF.cpu().numpy() - dF_ref)
    assert err.max() <= 1e-5 * np.abs(dF_ref).max(), err.max()


@pytest.mark.parametrize("m,L,D", [(3000, 64, 512), (1001, 32, 256), (33, 64, 128), (1, 32, 384)])
def test_decode_feature_loss_fused(orc, m, L, D):
    """The fused decode + loss equals decode then loss (float32 rounding) and
    the oracle's loss of the oracle's decode."""
    import paper_2507_07136_amd as ls2
    rng = np.random.default_rng(m + L + D)
    coef = (rng.random((m, L)) * (rng.random((m, L)) < 0.3)).astype(np.float32)
    dct = rng.standard_normal((L, D)).astype(np.float32)
    dct /= np.linalg.norm(dct, axis=1, keepdims=True)
    Y = (rng.standard_normal((m, D)) * 0.1).astype(np.float32)
    tc, td, tY = (torch.from_numpy(x).cuda() for x in (coef, dct, Y))
    loss_f = torch.zeros((1,), dtype=torch.float64, device="cuda")
    dF_f = torch.empty((m, D), device="cuda")
    F_f = torch.empty((m, D), device="cuda")
    ws = torch.empty((ls2.ls2_decode_feature_loss_workspace(m, D),), dtype=torch.uint8, device="cuda")
    ls2.ls2_decode_feature_loss(tc, td, tY, loss_f, dF_f, ws, feat=F_f)
    loss_n = torch.zeros((1,), dtype=torch.float64, device="cuda")
    dF_u = torch.empty((m, D), device="cuda")
    ls2.ls2_decode_feature_loss(tc, td, tY, loss_n, dF_u, ws)            # without the feature map
    F_u = torch.empty((m, D), device="cuda")
    ls2.ls2_dict_decode(tc, td, F_u, ls2.LS2_F32)
    loss_u = torch.zeros((1,), dtype=torch.float64, device="cuda")
    dF_uu = torch.empty((m, D), device="cuda")
    lws = torch.empty((ls2.ls2_feature_loss_workspace(m),), dtype=torch.uint8, device="cuda")
    ls2.ls2_feature_loss(F_u, tY, loss_u, dF_uu, lws)
    torch.cuda.synchronize()
    assert torch.equal(F_f, F_u)                                   # same matrix-core products
    assert torch.equal(dF_f, dF_u)
    gmax = dF_uu.abs().max().item()
    assert (dF_f - dF_uu).abs().max().item() <= 1e-6 * gmax
    # both sum the same float32 row terms with compensated float32 sums, in
    # different groupings: a few float32 roundings of the total apart
    assert abs(loss_f.item() - loss_u.item()) <= 1e-6 * abs(loss_u.item())
    assert loss_f.item() == loss_n.item()
    loss_ref, dF_ref = orc.loss_l1cos(orc.decode(coef, dct), Y)
    assert abs(loss_f.item() - loss_ref) <= 1e-5 * abs(loss_ref)
    assert np.abs(dF_f.cpu().numpy() - dF_ref).max() <= 1e-3 * np.abs(dF_ref).max()


@pytest.mark.parametrize("m,L,D", [(3000, 64, 512), (100003, 64, 512), (1001, 32, 256), (40009, 64, 384),
                                   (33, 64, 128), (1, 32, 512), (9001, 32, 128), (70001, 32, 512)])
def test_decode_loss_backward_fused(orc, m, L, D):
    """Decode + loss + both decode gradients in one pass equal the two-call
    chain (ls2_decode_feature_loss, then ls2_dict_decode_backward on its
    dL/dF) bit for bit, and the oracle's gradients of its own loss."""
    import paper_2507_07136_amd as ls2
    rng = np.random.default_rng(m + 3 * L + D)
    coef = (rng.random((m, L)) * (rng.random((m, L)) < 0.3)).astype(np.float32)
    dct = rng.standard_normal((L, D)).astype(np.float32)
    dct /= np.linalg.norm(dct, axis=1, keepdims=True)
    Y = (rng.standard_normal((m, D)) * 0.1).astype(np.float32)
    if m > 2:
        coef[1] = 0.0                        # zero feature: cosine guard
    tc, td, tY = (torch.from_numpy(x).cuda() for x in (coef, dct, Y))
    # the chain
    loss_c = torch.zeros((1,), dtype=torch.float64, device="cuda")
    dF = torch.empty((m, D), device="cuda")
    ws1 = torch.empty((ls2.ls2_decode_feature_loss_workspace(m, D),), dtype=torch.uint8, device="cuda")
    ls2.ls2_decode_feature_loss(tc, td, tY, loss_c, dF, ws1)
    dc_c = torch.empty((m, L), device="cuda")
    ds_c = torch.empty((L, D), device="cuda")
    ws2 = torch.empty((ls2.ls2_dict_decode_backward_workspace(m, L, D),), dtype=torch.uint8, device="cuda")
    ls2.ls2_dict_decode_backward(tc, td, dF, dc_c, ds_c, ws2)
    # one pass, twice (deterministic)
    ws = torch.empty((ls2.ls2_decode_loss_backward_workspace(m, L, D),), dtype=torch.uint8, device="cuda")
    outs = []
    for _ in range(2):
        loss_f = torch.zeros((1,), dtype=torch.float64, device="cuda")
        dc_f = torch.full((m, L), 7.0, device="cuda")
        ds_f = torch.full((L, D), 7.0, device="cuda")
        ls2.ls2_decode_loss_backward(tc, td, tY, loss_f, dc_f, ds_f, ws)
        outs.append((loss_f, dc_f, ds_f))
    torch.cuda.synchronize()
    (loss_f, dc_f, ds_f), (loss_g, dc_g, ds_g) = outs
    assert torch.equal(dc_f, dc_c)
    assert torch.equal(ds_f, ds_c)
    assert torch.equal(dc_f, dc_g) and torch.equal(ds_f, ds_g) and loss_f.item() == loss_g.item()
    # the loss partials follow the workgroups: equal to the chain's where the
    # two launch the same number (one per compute unit at D = 512), else a
    # few float32 roundings of the compensated total apart
    if D == 512:
        assert loss_f.item() == loss_c.item()
    else:
        assert abs(loss_f.item() - loss_c.item()) <= 1e-6 * abs(loss_c.item())
    loss_ref, dF_ref = orc.loss_l1cos(orc.decode(coef, dct), Y)
    assert abs(loss_f.item() - loss_ref) <= 1e-5 * abs(loss_ref)
    dc_ref, ds_ref = orc.decode_backward(coef, dct, dF_ref)
    for got, ref in ((dc_f, dc_ref), (ds_f, ds_ref)):
        g = got.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(g - ref) <= 1e-4 * np.linalg.norm(ref), (np.linalg.norm(g - ref), np.linalg.norm(ref))


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("m,D,n_neg,tau", [(5000, 512, 4, 1.0), (300, 128, 1, 10.0), (99, 1024, 8, 3.0)])
def test_query_backward_parity(orc, dtype, m, D, n_neg, tau):
    import paper_2507_07136_amd as ls2
    rng = np.random.default_rng(m + D + n_neg)
    F = rng.standard_normal((m, D)).astype(np.float32)
    F[0] = 0.0                                            # zero feature
    pos, neg = gen.make_text(m + 1, D=D, n_neg=n_neg)
    d_rel = rng.standard_normal(m).astype(np.float32)
    tF = torch.from_numpy(F).cuda().to(dtype)
    Fq = tF.float().cpu().numpy()                         # the values the kernel sees
    ref, margin = orc.query_backward(Fq, pos, neg, d_rel, tau)
    out = torch.empty((m, D), device="cuda")
    ls2.ls2_query_backward(tF, torch.from_numpy(pos).cuda(), torch.from_numpy(neg).cuda(),
                           torch.from_numpy(d_rel).cuda(), out, tau)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ok = margin >= 1e-4
    ok[0] = False                                         # the zero row is checked on its own below
    assert (~ok[1:]).sum() <= max(2, 0.03 * m), (~ok).sum()
    num = np.linalg.norm(got - ref, axis=1)[ok]
    den = np.maximum(np.linalg.norm(ref, axis=1)[ok], 1e-30)
    assert (num <= 1e-4 * den + 1e-30).all(), (num / den).max()
    # zero feature: every similarity is 0, both sides take the first negative,
    # and the guarded norm makes the score linear in F with slope e / (1e-12 |e|)
    assert np.linalg.norm(got[0] - ref[0]) <= 1e-4 * np.linalg.norm(ref[0])


def _oracle_chain(orc, cam, scene, g, dF, pix_zero=None):
    """Backward through the oracle from dL/dF, on the GPU's forward state."""
    dc, ds = orc.decode_backward(g["coef"].astype(np.float64), scene.dictionary, dF)
    dm, dcn, do, dw = orc.composite_backward(cam, g["ranges"], g["ids"], g["mean2d"].astype(np.float64),
                                             g["conic"].astype(np.float64), scene.opacity, scene.topk_idx,
                                             scene.topk_w, dc)
    dmu, dsc, dq = orc.project_backward(cam, scene.means, scene.scales, scene.quats, g["radius"], dm, dcn)
    return dict(means=dmu, scales=dsc, quats=dq, opacity=do, topk_w=dw, dictionary=ds)


def test_train_step_end_to_end(orc):
    """Trainer.step (loss + full backward) vs the oracle chain on the FD scene
    with a smooth random target; pixels near a decision flip get a zero
    upstream gradient on both sides."""
    import paper_2507_07136_amd as ls2
    c = gen.CONFIGS["fd"]
    scene, cam = small_scene(c["seed"], c["n"], c["width"], c["height"], D=c["D"])
    zup, P = gen.make_target_factors(c["seed"] + 1, c["height"], c["width"], D=c["D"])
    Y = gen.target_map(zup, P)
    tr = ls2.Trainer(cam, scene.n, D=c["D"])
    t = ls2.to_device(scene)
    tY = torch.from_numpy(Y).cuda().contiguous()
    loss = tr.forward_loss(t, tY, keep_feat=True)
    torch.cuda.synchronize()
    g = dict(coef=tr.coef.cpu().numpy(), ranges=tr.tile_ranges.cpu().numpy().view(np.uint32),
             ids=tr.ids[:tr.num_pairs].cpu().numpy().view(np.uint32), mean2d=tr.mean2d.cpu().numpy(),
             conic=tr.conic.cpu().numpy(), radius=tr.radius.cpu().numpy())
    F = tr.feat.cpu().numpy()
    loss_ref, dF_ref = orc.loss_l1cos(F, Y[None])
    assert abs(loss.item() - loss_ref) <= 1e-6 * abs(loss_ref)
    _, _, _, margin, margin_T = orc.composite(cam, g["ranges"], g["ids"], g["mean2d"].astype(np.float64),
                                              g["conic"].astype(np.float64), scene.opacity, scene.topk_idx,
                                              scene.topk_w, scene.L, with_margin_T=True)
    risky = _risky_pixels(margin, margin_T)
    dF = tr.d_feat.clone()
    dF[:, torch.from_numpy(risky).cuda()] = 0.0
    dF_np = dF.cpu().numpy().astype(np.float64)
    grads = tr.backward(t, dF)
    torch.cuda.synchronize()
    ref = _oracle_chain(orc, cam, scene, g, dF_np)
    print("train step: loss %.6f, %d risky pixels" % (loss.item(), int(risky.sum())))
    for name in ["means", "scales", "quats", "opacity", "topk_w", "dictionary"]:
        _grad_close(getattr(grads, name).cpu().numpy(), ref[name], "d_" + name, floor=CHAIN_FLOOR)


def test_autograd_function(orc):
    """torch.autograd through LS2Render equals the oracle chain for
    L = sum(F * R) (so dL/dF = R)."""
    import paper_2507_07136_amd as ls2
    scene, cam = small_scene(1100, 500, 64, 64, D=256)
    tr = ls2.Trainer(cam, scene.n, D=256)
    t = ls2.to_device(scene)
    params = {k: t[k].clone().requires_grad_(True) for k in ["means", "scales", "quats", "opacity", "topk_w",
                                                             "dictionary"]}
    F = ls2.LS2Render.apply(tr, params["means"], params["scales"], params["quats"], params["opacity"],
                            t["topk_idx"], params["topk_w"], params["dictionary"])
    torch.cuda.synchronize()
    g = dict(coef=tr.coef.cpu().numpy(), ranges=tr.tile_ranges.cpu().numpy().view(np.uint32),
             ids=tr.ids[:tr.num_pairs].cpu().numpy().view(np.uint32), mean2d=tr.mean2d.cpu().numpy(),
             conic=tr.conic.cpu().numpy(), radius=tr.radius.cpu().numpy())
    _, _, _, margin, margin_T = orc.composite(cam, g["ranges"], g["ids"], g["mean2d"].astype(np.float64),
                                              g["conic"].astype(np.float64), scene.opacity, scene.topk_idx,
                                              scene.topk_w, scene.L, with_margin_T=True)
    rng = np.random.default_rng(4)
    R = rng.standard_normal(F.shape).astype(np.float32)
    R[:, _risky_pixels(margin, margin_T)] = 0.0
    (F * torch.from_numpy(R).cuda()).sum().backward()
    torch.cuda.synchronize()
    ref = _oracle_chain(orc, cam, scene, g, R.astype(np.float64))
    for name in ["means", "scales", "quats", "opacity", "topk_w", "dictionary"]:
        _grad_close(params[name].grad.cpu().numpy(), ref[name], "d_" + name, floor=CHAIN_FLOOR)


@pytest.mark.parametrize("rows,L,K", [(5000, 64, 4), (777, 128, 8), (33, 32, 1), (1, 64, 8)])
def test_sparse_codes_parity(orc, rows, L, K):
    """Softmax / top-K / renormalise and its backward against the oracle:
    indices bit-exact (logits are distinct except one planted tie),
    weights and gradients within float32 rounding."""
    import paper_2507_07136_amd as ls2
    rng = np.random.default_rng(rows + L + K)
    z = (rng.normal(size=(rows, L)) * 2).astype(np.float32)
    z[0, 5] = z[0, 9] = z[0].max() + 1.0           # tie for the top: index 5 first
    dw = rng.normal(size=(rows, K)).astype(np.float32)
    tz = torch.from_numpy(z).cuda()
    idx = torch.empty((rows, K), dtype=torch.int32, device="cuda")
    w = torch.empty((rows, K), dtype=torch.float32, device="cuda")
    ls2.ls2_sparse_codes(tz, K, idx, w)
    dz = torch.empty((rows, L), dtype=torch.float32, device="cuda")
    ls2.ls2_sparse_codes_backward(idx, w, torch.from_numpy(dw).cuda(), dz)
    torch.cuda.synchronize()
    ridx, rw = orc.sparse_codes(z, K)
    assert np.array_equal(idx.cpu().numpy(), ridx)
    assert idx[0, 0].item() == 5 and (K == 1 or idx[0, 1].item() == 9)
    assert np.abs(w.cpu().numpy() - rw).max() <= 1e-6
    rdz = orc.sparse_codes_backward(z, K, dw)
    assert np.abs(dz.cpu().numpy() - rdz).max() <= 1e-5 * max(1.0, np.abs(rdz).max())


@pytest.mark.parametrize("n", [1, 3, 4, 4099, 1 << 22])
def test_accumulate_exact(n):
    """dst += src equals the float32 sum elementwise, bit for bit (one
    rounding per element), ragged tails included; two calls in a row."""
    import paper_2507_07136_amd as ls2
    rng = np.random.default_rng(n)
    a = rng.standard_normal(n).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    c = rng.standard_normal(n).astype(np.float32)
    dst = torch.from_numpy(a).cuda()
    ls2.ls2_accumulate(torch.from_numpy(b).cuda(), dst)
    ls2.ls2_accumulate(torch.from_numpy(c).cuda(), dst)
    torch.cuda.synchronize()
    assert np.array_equal(dst.cpu().numpy(), (a + b) + c)


def test_train_step_fd_config3(orc):
    """The GPU training step (Trainer.forward_loss + backward: loss, decode,
    splat and projection backward) on the finite-difference scene of the
    differentiation workload against central differences of the float64
    oracle's whole forward, for 16 sampled parameters of each kind (means,
    scales, quaternions, opacities, code weights, codebook); perturbations
    that change a decision are excluded and counted.  Pixels with a decision
    within 1e-5 of its threshold leave the loss on both sides."""
    import paper_2507_07136_amd as ls2
    from fd_chain import KINDS, Chain
    ch = Chain(orc)
    fw = ch.forward(ch.p0)
    risky = ((fw["margin"] < MARGIN) | (fw["margin_T"] < MARGIN)).reshape(-1)
    M = risky.size
    if risky.any():
        ch.mask = np.flatnonzero(~risky)
        fw = ch.forward(ch.p0)
    ref = ch.analytic(fw=fw)
    idx = ch.sample(ref, 16, 11)
    res = ch.fd(idx)
    sc, cam = ch.scene, ch.cam
    tr = ls2.Trainer(cam, sc.n, D=sc.D)
    t = ls2.to_device(sc)
    tY = torch.from_numpy(ch.Y.astype(np.float32).reshape(1, cam.height, cam.width, sc.D)).cuda()
    loss = tr.forward_loss(t, tY)
    dF = tr.d_feat.clone()
    if risky.any():
        dF.view(M, sc.D)[torch.from_numpy(risky).cuda()] = 0.0
        dF *= M / float(M - risky.sum())
    grads = tr.backward(t, dF)
    torch.cuda.synchronize()
    same_lists = compare_tile_lists(
        dict(P=tr.num_pairs, ranges=tr.tile_ranges.cpu().numpy().view(np.uint32),
             ids=tr.ids[:tr.num_pairs].cpu().numpy().view(np.uint32)),
        None, fw["ids"], fw["ranges"], cam.tiles_x, cam.tiles_y) is None
    print("fd scene: loss %.6f (oracle %.6f), %d risky pixels, GPU lists equal the oracle's: %s"
          % (loss.item(), fw["loss"], int(risky.sum()), same_lists))
    if not risky.any():
        assert abs(loss.item() - fw["loss"]) <= 1e-5 * abs(fw["loss"])
    for k in KINDS:
        vals, kept = res[k]
        assert kept.sum() >= 0.75 * len(kept), (k, int(kept.sum()))
        got = getattr(grads, k).cpu().numpy().astype(np.float64).flat[idx[k]][kept]
        v = vals[kept]
        gmax = np.abs(ref[k]).max()
        err = np.abs(got - v)
        print("%-10s %d/%d kept: |dg|/|g| %.2e, worst element %.2e of its bound" % (
            k, kept.sum(), len(kept), np.linalg.norm(got - v) / np.linalg.norm(v),
            (err / (1e-3 * np.maximum(np.abs(v), 1e-3 * gmax))).max()))
        assert np.linalg.norm(got - v) <= 1e-3 * np.linalg.norm(v), k
        assert np.all(err <= 1e-3 * np.maximum(np.abs(v), 1e-3 * gmax)), k


def _gpu_state(tr):
    return dict(coef=tr.coef.cpu().numpy(), ranges=tr.tile_ranges.cpu().numpy().view(np.uint32),
                ids=tr.ids[:tr.num_pairs].cpu().numpy().view(np.uint32), mean2d=tr.mean2d.cpu().numpy(),
                conic=tr.conic.cpu().numpy(), radius=tr.radius.cpu().numpy())


def test_autograd_two_views_one_trainer(orc):
    """Two views rendered through one trainer before a single backward of the
    summed loss: each LS2Render call differentiates its own frame (its own
    lists, maps and camera), so the gradients equal the sum of the oracle
    chains of the two views."""
    import paper_2507_07136_amd as ls2
    scene, _ = small_scene(1100, 500, 64, 64, D=256)
    cams = [gen.orbit_camera(64, 64, v, radius=3.0) for v in (0, 1)]
    tr = ls2.Trainer(cams[0], scene.n, D=256)
    t = ls2.to_device(scene)
    params = {k: t[k].clone().requires_grad_(True) for k in ["means", "scales", "quats", "opacity", "topk_w",
                                                             "dictionary"]}
    rng = np.random.default_rng(12)
    total = 0.0
    refs = []
    for cam in cams:
        tr.set_camera(cam)
        F = ls2.LS2Render.apply(tr, params["means"], params["scales"], params["quats"], params["opacity"],
                                t["topk_idx"], params["topk_w"], params["dictionary"])
        torch.cuda.synchronize()
        g = _gpu_state(tr)
        _, _, _, margin, margin_T = orc.composite(cam, g["ranges"], g["ids"], g["mean2d"].astype(np.float64),
                                                  g["conic"].astype(np.float64), scene.opacity, scene.topk_idx,
                                                  scene.topk_w, scene.L, with_margin_T=True)
        R = rng.standard_normal(F.shape).astype(np.float32)
        R[:, _risky_pixels(margin, margin_T)] = 0.0
        total = total + (F * torch.from_numpy(R).cuda()).sum()
        refs.append(_oracle_chain(orc, cam, scene, g, R.astype(np.float64)))
    assert not np.array_equal(refs[0]["means"], refs[1]["means"])
    total.backward()
    torch.cuda.synchronize()
    for name in ["means", "scales", "quats", "opacity", "topk_w", "dictionary"]:
        _grad_close(params[name].grad.cpu().numpy(), refs[0][name] + refs[1][name], "d_" + name, floor=CHAIN_FLOOR)


def test_autograd_logits_chain(orc):
    """Codes given as logits (Section 3.3: softmax, top K, renormalise)
    through LS2RenderLogits: the GPU codes equal the oracle's (indices bit
    for bit) and dL/dlogits equals the oracle's sparse-code backward of its
    composed chain."""
    import paper_2507_07136_amd as ls2
    scene, cam = small_scene(1100, 500, 64, 64, D=256)
    rng = np.random.default_rng(13)
    logits = (rng.standard_normal((scene.n, 1, scene.L)) * 2.0).astype(np.float32)
    ridx, rw = orc.sparse_codes(logits.reshape(scene.n, scene.L), scene.K)
    tr = ls2.Trainer(cam, scene.n, D=256)
    t = ls2.to_device(scene)
    params = {k: t[k].clone().requires_grad_(True) for k in ["means", "scales", "quats", "opacity", "dictionary"]}
    tl = torch.from_numpy(logits).cuda().requires_grad_(True)
    F = ls2.LS2RenderLogits.apply(tr, params["means"], params["scales"], params["quats"], params["opacity"], tl,
                                  params["dictionary"])
    torch.cuda.synchronize()
    assert np.array_equal(tr.topk_idx.cpu().numpy().reshape(scene.n, scene.K), ridx)
    assert np.abs(tr.topk_w.cpu().numpy().reshape(scene.n, scene.K) - rw).max() <= 1e-6
    g = _gpu_state(tr)
    codes = dict(topk_idx=ridx.reshape(scene.n, 1, scene.K).astype(np.int32),
                 topk_w=tr.topk_w.cpu().numpy())            # the weights the GPU rendered with
    _, _, _, margin, margin_T = orc.composite(cam, g["ranges"], g["ids"], g["mean2d"].astype(np.float64),
                                              g["conic"].astype(np.float64), scene.opacity, codes["topk_idx"],
                                              codes["topk_w"], scene.L, with_margin_T=True)
    R = rng.standard_normal(F.shape).astype(np.float32)
    R[:, _risky_pixels(margin, margin_T)] = 0.0
    (F * torch.from_numpy(R).cuda()).sum().backward()
    torch.cuda.synchronize()
    sc2 = gen.Scene(scene.means, scene.scales, scene.quats, scene.opacity, codes["topk_idx"], codes["topk_w"],
                    scene.dictionary)
    ref = _oracle_chain(orc, cam, sc2, g, R.astype(np.float64))
    d_logits = orc.sparse_codes_backward(logits.reshape(scene.n, scene.L), scene.K,
                                         ref["topk_w"].reshape(scene.n, scene.K))
    _grad_close(tl.grad.cpu().numpy().reshape(scene.n, scene.L), d_logits, "d_logits", floor=CHAIN_FLOOR)
    for name in ["means", "scales", "quats", "opacity", "dictionary"]:
        _grad_close(params[name].grad.cpu().numpy(), ref[name], "d_" + name, floor=CHAIN_FLOOR)


@pytest.mark.parametrize("levels,D", [(1, 512), (2, 256)])
def test_trainer_step_one_pass(levels, D):
    """Trainer.step (decode + loss + decode backward in one pass) against
    Trainer.forward_loss + backward (dL/dF through memory): the decode
    gradients bit for bit, the loss bit for bit where both launch the same
    workgroups (D = 512) and the rest of the chain, whose float atomics may
    add in another order, to float32 rounding."""
    import paper_2507_07136_amd as ls2
    scene, cam = small_scene(21 + levels, 3000, 200, 136, levels=levels, D=D)
    rng = np.random.default_rng(5)
    tY = torch.from_numpy((rng.standard_normal((levels, cam.height, cam.width, D)) * 0.1).astype(np.float32)).cuda()
    t = ls2.to_device(scene)
    tr = ls2.Trainer(cam, scene.n, levels=levels, D=D)
    loss_a = tr.forward_loss(t, tY).clone()
    ga = {k: getattr(tr.backward(t), k).clone() for k in ("coef", "dictionary", "means", "scales", "quats",
                                                          "opacity", "topk_w")}
    loss_b, gb = tr.step(t, tY)
    torch.cuda.synchronize()
    assert torch.equal(gb.coef, ga["coef"])
    assert torch.equal(gb.dictionary, ga["dictionary"])
    if D == 512:
        assert loss_b.item() == loss_a.item()
    else:
        assert abs(loss_b.item() - loss_a.item()) <= 1e-6 * abs(loss_a.item())
    for k in ("means", "scales", "quats", "opacity", "topk_w"):
        a, b = ga[k].double(), getattr(gb, k).double()
        assert torch.linalg.norm(a - b).item() <= 1e-5 * torch.linalg.norm(a).item() + 1e-30, k


def test_trainer_step_one_pass_logits():
    """The one-pass Trainer.step with codes given as logits: the codes are
    formed first and dL/dlogits closes the chain, as with forward_loss +
    backward (float atomics of the splat backward: float32 rounding)."""
    import paper_2507_07136_amd as ls2
    scene, cam = small_scene(41, 2000, 160, 104, D=512)
    rng = np.random.default_rng(9)
    tY = torch.from_numpy((rng.standard_normal((1, cam.height, cam.width, 512)) * 0.1).astype(np.float32)).cuda()
    t = ls2.to_device(scene)
    t["logits"] = torch.from_numpy((rng.standard_normal((scene.n, 1, scene.L)) * 2.0).astype(np.float32)).cuda()
    tr = ls2.Trainer(cam, scene.n, D=512)
    loss_a = tr.forward_loss(t, tY).clone()
    tr.backward(t)
    idx_a, dl_a = t["topk_idx"].clone(), tr.d_logits.clone()
    gd_a = tr.grad.dictionary.clone()
    loss_b, _ = tr.step(t, tY)
    torch.cuda.synchronize()
    assert torch.equal(t["topk_idx"], idx_a)
    assert loss_b.item() == loss_a.item()
    assert torch.equal(tr.grad.dictionary, gd_a)
    a, b = dl_a.double(), tr.d_logits.double()
    assert torch.linalg.norm(a - b).item() <= 1e-5 * torch.linalg.norm(a).item() + 1e-30
