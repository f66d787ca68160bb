"""Pins of the oracle's hand-derived backward pass against central finite
differences of its own forward functions (float64, h = 1e-6 relative).
Discrete decisions are held fixed: parameters whose +-h forward runs change
any decision (which Gaussians blend at which pixel) are excluded and counted."""
import numpy as np
import pytest

import gen


def fd(f, x, idx, h_rel=1e-6):
    """Central difference of scalar f at x along the flat indices idx."""
    out = np.zeros(len(idx))
    for j, i in enumerate(idx):
        h = h_rel * max(1.0, abs(x.flat[i]))
        xp = x.copy(); xp.flat[i] += h
        xm = x.copy(); xm.flat[i] -= h
        out[j] = (f(xp) - f(xm)) / (2 * h)
    return out


def test_loss_grad(orc):
    rng = np.random.default_rng(0)
    F = rng.normal(size=(9, 24))
    Y = rng.normal(size=(9, 24))
    F[3] = 0.0  # zero row: cosine guarded
    loss, dF = orc.loss_l1cos(F, Y)
    idx = rng.choice(F.size, 60, replace=False)
    idx = [i for i in idx if i // 24 != 3]  # |x| kink at 0 for the zero row
    num = fd(lambda x: orc.loss_l1cos(x, Y)[0], F, idx)
    np.testing.assert_allclose(dF.flat[idx], num, rtol=1e-6, atol=1e-9)
    # the loss itself: L1 and cosine parts by library routines
    cos = np.sum(F * Y, 1) / np.maximum(np.linalg.norm(F, axis=1), 1e-12) / np.linalg.norm(Y, axis=1)
    assert loss == pytest.approx(np.abs(F - Y).mean() + np.mean(1 - cos), rel=1e-12)


@pytest.mark.parametrize("tau", [1.0, 7.0])
def test_query_grad(orc, tau):
    rng = np.random.default_rng(1)
    pos, neg = gen.make_text(3, D=32)
    F = rng.normal(size=(12, 32))
    dr = rng.normal(size=12)
    g, margin = orc.query_backward(F, pos, neg, dr, tau)
    assert margin.min() > 1e-3
    idx = rng.choice(F.size, 80, replace=False)
    num = fd(lambda x: float(np.sum(dr * orc.query(x, pos, neg, tau))), F, idx)
    np.testing.assert_allclose(g.flat[idx], num, rtol=1e-6, atol=1e-10)


def test_decode_grad(orc):
    rng = np.random.default_rng(2)
    W = rng.random((17, 8))
    S = rng.normal(size=(8, 20))
    G = rng.normal(size=(17, 20))
    dW, dS = orc.decode_backward(W, S, G)
    f = lambda w, s: float(np.sum(G * orc.decode(w, s)))  # noqa: E731
    iw = rng.choice(W.size, 40, replace=False)
    np.testing.assert_allclose(dW.flat[iw], fd(lambda x: f(x, S), W, iw), rtol=1e-6, atol=1e-8)
    isd = rng.choice(S.size, 40, replace=False)
    np.testing.assert_allclose(dS.flat[isd], fd(lambda x: f(W, x), S, isd), rtol=1e-6, atol=1e-8)


def _small_splat_scene(seed=3, n=60, w=40, h=36, levels=2, K=3, L=16):
    scene = gen.make_scene(seed, n, L=L, K=K, D=8, levels=levels, log_scale_mu=-2.6, log_scale_sigma=0.3)
    scene.opacity[:] = np.minimum(scene.opacity, 0.9)  # keep alpha below the 0.99 clamp
    cam = gen.make_camera(w, h)
    return scene, cam


def test_composite_grad(orc):
    scene, cam = _small_splat_scene()
    pr = orc.project(cam, scene.means, scene.scales, scene.quats)
    keys, ids, ranges = orc.tile_lists(cam, pr["mean2d"].astype(np.float32), pr["radius"],
                                       pr["depth"].astype(np.float32))
    rng = np.random.default_rng(4)
    G = rng.normal(size=(scene.levels, cam.height, cam.width, scene.L))
    m2, cn = pr["mean2d"].copy(), pr["conic"].copy()
    op, w = scene.opacity.astype(np.float64), scene.topk_w.astype(np.float64)
    dm, dc, do, dw = orc.composite_backward(cam, ranges, ids, m2, cn, op, scene.topk_idx, w, G)

    def run(m2_, cn_, op_, w_):
        coef, fT, last, marg = orc.composite(cam, ranges, ids, m2_, cn_, op_, scene.topk_idx, w_, scene.L)
        return float(np.sum(G * coef)), last

    # decision signature: which Gaussians blend at which pixel (via a dense
    # one-hot render: e_i(v) > 0)
    eye = np.eye(scene.n)

    def signature(m2_, cn_, op_):
        return orc.composite_dense(cam, ranges, ids, m2_, cn_, op_, eye) > 0

    base_sig = signature(m2, cn, op)
    checked = skipped = 0
    for name, arr, grad in (("mean2d", m2, dm), ("conic", cn, dc), ("opacity", op, do), ("w", w, dw)):
        idx = rng.choice(arr.size, min(arr.size, 40), replace=False)
        for i in idx:
            h = 1e-6 * max(1.0, abs(arr.flat[i]))
            vals = []
            same = True
            for sgn in (1, -1):
                a2 = arr.copy()
                a2.flat[i] += sgn * h
                args = {"mean2d": m2, "conic": cn, "opacity": op, "w": w}
                args[name] = a2
                if name != "w":
                    same &= np.array_equal(signature(args["mean2d"], args["conic"], args["opacity"]), base_sig)
                vals.append(run(args["mean2d"], args["conic"], args["opacity"], args["w"])[0])
            if not same:
                skipped += 1
                continue
            num = (vals[0] - vals[1]) / (2 * h)
            assert grad.flat[i] == pytest.approx(num, rel=1e-5, abs=1e-7), (name, i)
            checked += 1
    assert checked >= 140 and skipped <= 10


def test_composite_backward_pixels_matches_masked(orc):
    """The pixel-list backward equals the full backward with dL/dcoef zeroed
    outside the listed pixels (an upstream-zero pixel adds nothing), in any
    list order (only the summation order differs)."""
    scene, cam = _small_splat_scene()
    pr = orc.project(cam, scene.means, scene.scales, scene.quats)
    keys, ids, ranges = orc.tile_lists(cam, pr["mean2d"].astype(np.float32), pr["radius"],
                                       pr["depth"].astype(np.float32))
    rng = np.random.default_rng(8)
    npx = cam.width * cam.height
    pix = rng.choice(npx, 300, replace=False)
    G = np.zeros((scene.levels, npx, scene.L))
    G[:, pix] = rng.normal(size=(scene.levels, len(pix), scene.L))
    args = (cam, ranges, ids, pr["mean2d"], pr["conic"], scene.opacity, scene.topk_idx, scene.topk_w)
    full = orc.composite_backward(*args, G.reshape(scene.levels, cam.height, cam.width, scene.L))
    part = orc.composite_backward_pixels(*args, pix, G[:, pix].transpose(1, 0, 2))
    for a, b in zip(full, part):
        assert np.abs(a).max() > 0
        np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-15 * np.abs(a).max())
    # every pixel listed: the full backward
    allpix = rng.permutation(npx)
    Gf = rng.normal(size=(scene.levels, npx, scene.L))
    full = orc.composite_backward(*args, Gf.reshape(scene.levels, cam.height, cam.width, scene.L))
    part = orc.composite_backward_pixels(*args, allpix, Gf[:, allpix].transpose(1, 0, 2))
    for a, b in zip(full, part):
        np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-14 * np.abs(a).max())


def test_composite_grad_weights_exact(orc):
    """For one Gaussian, dW/dw_k = alpha e_idx exactly (linear in w)."""
    scene, cam = _small_splat_scene(n=1, levels=1, K=4, L=16)
    scene.means[:] = 0.0
    pr = orc.project(cam, scene.means, scene.scales, scene.quats)
    keys, ids, ranges = orc.tile_lists(cam, pr["mean2d"].astype(np.float32), pr["radius"],
                                       pr["depth"].astype(np.float32))
    coef, fT, last, m = orc.composite(cam, ranges, ids, pr["mean2d"], pr["conic"], scene.opacity,
                                      scene.topk_idx, scene.topk_w, 16)
    alpha = 1.0 - fT  # single Gaussian: T = 1 - alpha where it blends
    G = np.zeros((1, cam.height, cam.width, 16))
    G[0, :, :, scene.topk_idx[0, 0, 2]] = 1.0
    dm, dc, do, dw = orc.composite_backward(cam, ranges, ids, pr["mean2d"], pr["conic"], scene.opacity,
                                            scene.topk_idx, scene.topk_w, G)
    assert dw[0, 0, 2] == pytest.approx(alpha.sum(), rel=1e-12)
    assert dw[0, 0, 0] == 0.0


@pytest.mark.parametrize("view", [0, 2])
def test_project_grad(orc, view):
    rng = np.random.default_rng(5 + view)
    cam = gen.orbit_camera(200, 160, view)
    n = 12
    means = rng.uniform(-0.5, 0.5, (n, 3))
    scales = np.exp(rng.normal(-3.0, 0.4, (n, 3)))
    quats = rng.normal(size=(n, 4))
    pr = orc.project(cam, means, scales, quats, f64=True)
    assert (pr["radius"] > 0).all()
    gm2 = rng.normal(size=(n, 2))
    gcn = rng.normal(size=(n, 3)) * 10.0
    dmu, ds, dq = orc.project_backward(cam, means, scales, quats, pr["radius"], gm2, gcn, f64=True)

    def f(mu, s, q):
        o = orc.project(cam, mu, s, q, f64=True)
        return float(np.sum(gm2 * o["mean2d"]) + np.sum(gcn * o["conic"]))

    for arr, grad, which in ((means, dmu, 0), (scales, ds, 1), (quats, dq, 2)):
        idx = np.arange(arr.size)

        def g(x, which=which):
            a = [means, scales, quats]
            a[which] = x
            return f(*a)
        num = fd(g, arr, idx, h_rel=1e-7)
        np.testing.assert_allclose(grad.flat[idx], num, rtol=2e-5, atol=1e-6 * np.abs(num).max())


def test_project_grad_quat_scale_invariance(orc):
    """d/dq is orthogonal to q (the projection depends on q / |q| only)."""
    rng = np.random.default_rng(9)
    cam = gen.make_camera(128, 128)
    n = 8
    means = rng.uniform(-0.3, 0.3, (n, 3))
    scales = np.exp(rng.normal(-3.0, 0.3, (n, 3)))
    quats = rng.normal(size=(n, 4)) * 3.0
    pr = orc.project(cam, means, scales, quats, f64=True)
    _, _, dq = orc.project_backward(cam, means, scales, quats, pr["radius"], rng.normal(size=(n, 2)),
                                    rng.normal(size=(n, 3)), f64=True)
    np.testing.assert_allclose(np.sum(dq * quats, 1), 0.0, atol=1e-10)


def test_chain_fd_config3_scene(orc):
    """The oracle's composed backward (loss -> decode -> splat -> project,
    Sections 3.1-3.4) against central differences of its whole float64
    forward on the finite-difference scene of the differentiation workload
    (500 Gaussians, 64x64, L = 64, K = 4, D = 512, L1 + cosine loss against
    a smooth random target), for sampled parameters of every kind: means,
    scales, quaternions, opacities, code weights and the codebook.
    Perturbations that change a decision are excluded and counted."""
    from fd_chain import KINDS, Chain
    ch = Chain(orc)
    fw = ch.forward(ch.p0)
    g = ch.analytic(fw=fw)
    idx = ch.sample(g, 12, 7)
    res = ch.fd(idx)
    for k in KINDS:
        vals, kept = res[k]
        assert kept.sum() >= 0.8 * len(kept), (k, int(kept.sum()))
        a = g[k].flat[idx[k]][kept]
        v = vals[kept]
        # float64 differences: truncation O(h^2) and term rounding, far below
        print("%-10s %d/%d kept, max rel err %.2e" % (k, kept.sum(), len(kept),
                                                      (np.abs(a - v) / np.abs(v)).max()))
        assert np.all(np.abs(a - v) <= 1e-5 * np.abs(v) + 1e-8 * np.abs(g[k]).max()), k
