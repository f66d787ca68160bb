"""Pins of the FP64 oracle against things other than itself.

Each test checks an oracle function against a library routine, a closed form
of the paper's model, an invariant, or a brute-force computation, chosen so
that a dropped term, wrong sign, wrong index or transposed operand fails.
Runs on the CPU only.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import gen

F32_099 = float(np.float32(0.99))
F32_1_255 = float(np.float32(1.0) / np.float32(255.0))
F32_1E4 = float(np.float32(1e-4))


def one_gaussian_scene(mu, s, q, o=0.8, L=64, K=4, idx=(3, 17, 40, 63), w=(0.1, 0.2, 0.3, 0.4)):
    n = len(mu)
    scene = gen.Scene(np.asarray(mu, np.float32).reshape(n, 3), np.asarray(s, np.float32).reshape(n, 3),
                      np.asarray(q, np.float32).reshape(n, 4), np.full(n, o, np.float32),
                      np.tile(np.asarray(idx, np.int32), (n, 1, 1)), np.tile(np.asarray(w, np.float32), (n, 1, 1)),
                      np.zeros((L, 8), np.float32))
    return scene


def run_oracle(orc, cam, scene, L=None):
    L = L or scene.L
    pr = orc.project(cam, scene.means, scene.scales, scene.quats)
    keys, ids, ranges = orc.tile_lists(cam, pr["mean2d"].astype(np.float32), pr["radius"],
                                       pr["depth"].astype(np.float32))
    coef, fT, last, mg = orc.composite(cam, ranges, ids, pr["mean2d"], pr["conic"], scene.opacity,
                                       scene.topk_idx, scene.topk_w, L)
    return pr, (keys, ids, ranges), (coef, fT, last, mg)


def sigma3d(s, q):
    """Eq. 2 via scipy's rotation (scipy takes x, y, z, w)."""
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    return R @ np.diag(np.asarray(s, float) ** 2) @ R.T


# ---------------------------------------------------------------- projection
def test_project_on_axis_isotropic(orc):
    cam = gen.make_camera(128, 128)
    s = 0.02
    q = Rotation.random(random_state=3).as_quat()  # isotropic: rotation must not matter
    pr = orc.project(cam, np.zeros((1, 3)), np.full((1, 3), s), [[q[3], q[0], q[1], q[2]]])
    f = cam.fx
    var = (f * float(np.float32(s)) / 3.0) ** 2 + float(np.float32(0.3))
    np.testing.assert_allclose(pr["cov2d"][0], [var, 0.0, var], rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(pr["conic"][0], [1 / var, 0.0, 1 / var], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(pr["mean2d"][0], [64.0, 64.0], atol=1e-12)
    assert pr["depth"][0] == pytest.approx(3.0)
    assert pr["radius"][0] == math.ceil(3 * math.sqrt(var))


def test_project_axis_aligned_and_swap(orc):
    cam = gen.make_camera(128, 128)
    s = np.array([[0.03, 0.01, 0.02]], np.float32)
    pr = orc.project(cam, np.zeros((1, 3)), s, [[1.0, 0, 0, 0]])
    d = float(np.float32(0.3))
    a = (cam.fx * float(s[0, 0]) / 3) ** 2 + d
    c = (cam.fy * float(s[0, 1]) / 3) ** 2 + d
    np.testing.assert_allclose(pr["cov2d"][0], [a, 0, c], rtol=1e-6, atol=1e-9)
    # 90 degrees about the optical axis swaps the screen axes
    h = math.sqrt(0.5)
    pr2 = orc.project(cam, np.zeros((1, 3)), s, [[h, 0, 0, h]])
    np.testing.assert_allclose(pr2["cov2d"][0], [c, 0, a], rtol=1e-6, atol=1e-6)


def test_project_fov_edge_pixel(orc):
    # 60 degree horizontal field of view: a point at x/z = tan 30 lands on the image edge u = W
    cam = gen.make_camera(1440, 1080)
    x = 3.0 * math.tan(math.radians(30.0))
    pr = orc.project(cam, [[x, 0.0, 0.0]], [[0.01] * 3], [[1.0, 0, 0, 0]])
    assert pr["mean2d"][0, 0] == pytest.approx(1440.0, abs=2e-4)
    assert pr["mean2d"][0, 1] == pytest.approx(540.0, abs=1e-9)


@pytest.mark.parametrize("view", [0, 1, 3])
def test_project_ewa_matches_numerical_jacobian(orc, view):
    """EWA: cov2d - 0.3 I equals Jn Sigma Jn^T with Jn the numerical Jacobian
    of the oracle's own mean2d with respect to the world-space mean."""
    cam = gen.orbit_camera(640, 480, view)
    rng = np.random.default_rng(view)
    for _ in range(5):
        mu = rng.uniform(-0.4, 0.4, 3)
        s = np.exp(rng.normal(-3.5, 0.4, 3)).astype(np.float32)
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        q = q.astype(np.float32)
        pr = orc.project(cam, mu[None].astype(np.float32), s[None], q[None])
        assert pr["radius"][0] > 0
        # numerical Jacobian via perturbed means (float32 inputs -> use larger steps, float64 center)
        h = 1e-3
        Jn = np.zeros((2, 3))
        for k in range(3):
            mp = mu.copy(); mp[k] += h
            mm = mu.copy(); mm[k] -= h
            up = orc.project(cam, mp[None].astype(np.float32), s[None], q[None])["mean2d"][0]
            um = orc.project(cam, mm[None].astype(np.float32), s[None], q[None])["mean2d"][0]
            dm = (np.float32(mp[k]) - np.float32(mm[k]))
            Jn[:, k] = (up - um) / float(dm)
        # evaluate at the float32 mean actually used
        sig = sigma3d(s.astype(float), q.astype(float))
        cov = Jn @ sig @ Jn.T
        d = float(np.float32(0.3))
        got = pr["cov2d"][0]
        np.testing.assert_allclose([got[0] - d, got[1], got[2] - d], [cov[0, 0], cov[0, 1], cov[1, 1]],
                                   rtol=2e-3, atol=1e-3 * max(1.0, abs(cov).max()))


def test_project_conic_radius_invariants(orc):
    scene, cam = gen.config_scene("c1")
    pr = orc.project(cam, scene.means, scene.scales, scene.quats)
    vis = pr["radius"] > 0
    a, b, c = pr["cov2d"][vis].T
    A, B, C = pr["conic"][vis].T
    # conic is the inverse of the dilated covariance
    np.testing.assert_allclose(a * A + b * B, 1.0, atol=1e-9)
    np.testing.assert_allclose(a * B + b * C, 0.0, atol=1e-9)
    np.testing.assert_allclose(b * B + c * C, 1.0, atol=1e-9)
    # radius from the largest eigenvalue (library eigen-solver)
    covs = np.stack([np.stack([a, b], -1), np.stack([b, c], -1)], -2)
    lam = np.linalg.eigvalsh(covs)[:, -1]
    np.testing.assert_allclose(pr["extent"][vis], 3 * np.sqrt(lam), rtol=1e-9)
    assert np.all(pr["radius"][vis] == np.ceil(3 * np.sqrt(lam)).astype(np.int32))


def test_project_culls_behind_and_nan(orc):
    cam = gen.make_camera(128, 128)
    means = np.array([[0, 0, -3.5], [0, 0, -2.85], [np.nan, 0, 0], [0, 0, 0], [50, 0, 0]], np.float32)
    pr = orc.project(cam, means, np.full((5, 3), 0.02, np.float32), np.tile([1.0, 0, 0, 0], (5, 1)))
    # behind the camera, closer than znear = 0.2, NaN, visible, off-screen
    assert list(pr["radius"] > 0) == [False, False, False, True, False]
    assert pr["touched"][3] > 0 and pr["touched"][4] == 0


def test_project_quaternion_sign_and_scale_invariance(orc):
    cam = gen.make_camera(128, 128)
    rng = np.random.default_rng(5)
    q = rng.normal(size=4)
    s = np.array([[0.03, 0.01, 0.02]], np.float32)
    mu = np.array([[0.1, -0.2, 0.3]], np.float32)
    p1 = orc.project(cam, mu, s, (q / np.linalg.norm(q))[None].astype(np.float32))
    p2 = orc.project(cam, mu, s, (-2.5 * q / np.linalg.norm(q))[None].astype(np.float32))
    np.testing.assert_allclose(p1["cov2d"], p2["cov2d"], rtol=1e-6)


# ---------------------------------------------------------------- binning
def test_tile_rect_is_exact_overlap(orc):
    """Tile rectangle = tiles whose pixel span [16t, 16t+16) overlaps
    [u - r, u + r], checked with exact rational arithmetic."""
    scene, cam = gen.config_scene("c1")
    pr = orc.project(cam, scene.means, scene.scales, scene.quats)
    m2 = pr["mean2d"].astype(np.float32)
    checked = 0
    for i in range(scene.n):
        r = int(pr["radius"][i])
        if r == 0:
            continue
        u, v = Fraction(float(m2[i, 0])), Fraction(float(m2[i, 1]))
        bounds = [u - r, u + r, v - r, v + r]
        if any(abs(float(x) / 16 - round(float(x) / 16)) < 1e-3 for x in bounds):
            continue
        xs = [t for t in range(cam.tiles_x) if 16 * t <= u + r and 16 * t + 16 > u - r]
        ys = [t for t in range(cam.tiles_y) if 16 * t <= v + r and 16 * t + 16 > v - r]
        x0, y0, x1, y1 = pr["rect"][i]
        assert xs == list(range(x0, x1 + 1)) and ys == list(range(y0, y1 + 1)), i
        checked += 1
    assert checked > 1500


def test_tile_lists_match_lexsort(orc):
    scene, cam = gen.config_scene("c1")
    pr = orc.project(cam, scene.means, scene.scales, scene.quats)
    m2 = pr["mean2d"].astype(np.float32)
    dep = pr["depth"].astype(np.float32)
    keys, ids, ranges = orc.tile_lists(cam, m2, pr["radius"], dep)
    tiles, dbits, gid = [], [], []
    for i in range(scene.n):
        if pr["radius"][i] == 0:
            continue
        x0, y0, x1, y1 = pr["rect"][i]
        for ty in range(y0, y1 + 1):
            for tx in range(x0, x1 + 1):
                tiles.append(ty * cam.tiles_x + tx)
                dbits.append(dep[i:i + 1].view(np.uint32)[0])
                gid.append(i)
    tiles, dbits, gid = map(np.array, (tiles, dbits, gid))
    order = np.lexsort((gid, dbits, tiles))
    assert np.array_equal(ids, gid[order].astype(np.uint32))
    exp_keys = (tiles[order].astype(np.uint64) << np.uint64(32)) | dbits[order].astype(np.uint64)
    assert np.array_equal(keys, exp_keys)
    counts = np.bincount(tiles, minlength=cam.tiles_x * cam.tiles_y)
    assert np.array_equal(ranges[:, 1] - ranges[:, 0], counts)
    assert np.array_equal(ranges[:, 0], np.concatenate([[0], np.cumsum(counts)[:-1]]))
    assert np.array_equal(ranges[:, 1], np.cumsum(counts))


def test_tile_lists_capacity_error(orc):
    scene, cam = gen.config_scene("c1")
    pr = orc.project(cam, scene.means, scene.scales, scene.quats)
    with pytest.raises(RuntimeError):
        orc.tile_lists(cam, pr["mean2d"].astype(np.float32), pr["radius"], pr["depth"].astype(np.float32),
                       cap=100)


def test_binned_equals_bruteforce(orc):
    scene, cam = gen.config_scene("c1", n=600)
    pr, lists, (coef, fT, last, mg) = run_oracle(orc, cam, scene)
    bcoef, bT = orc.composite_bruteforce(cam, pr["mean2d"].astype(np.float32), pr["radius"],
                                         pr["depth"].astype(np.float32), pr["mean2d"], pr["conic"],
                                         scene.opacity, scene.topk_idx, scene.topk_w, scene.L)
    np.testing.assert_allclose(coef, bcoef, rtol=0, atol=1e-14)
    np.testing.assert_allclose(fT, bT, rtol=0, atol=1e-14)


# ---------------------------------------------------------------- compositing
def unnormalised_gaussian(d, cov):
    """G(x) of Eq. 1 via scipy's normalised density times its normaliser."""
    from scipy.stats import multivariate_normal
    return multivariate_normal(mean=np.zeros(2), cov=cov).pdf(d) * 2 * np.pi * math.sqrt(np.linalg.det(cov))


def test_single_gaussian_closed_form(orc):
    cam = gen.make_camera(128, 128)
    sc = one_gaussian_scene([[0.05, -0.03, 0.1]], [[0.08, 0.04, 0.06]], [[0.9, 0.1, -0.3, 0.2]], o=0.7)
    sc.topk_w[:] = [0.1, 0.2, 0.3, 0.4]
    pr, _, (coef, fT, last, mg) = run_oracle(orc, cam, sc)
    a, b, c = pr["cov2d"][0]
    cov = np.array([[a, b], [b, c]])
    u, v = pr["mean2d"][0]
    x0, y0, x1, y1 = pr["rect"][0]
    hit = 0
    for py in range(cam.height):
        for px in range(cam.width):
            inside = x0 <= px // 16 <= x1 and y0 <= py // 16 <= y1
            alpha = min(F32_099, float(np.float32(0.7)) * unnormalised_gaussian([px + 0.5 - u, py + 0.5 - v], cov))
            if not inside or alpha < F32_1_255:
                assert np.all(coef[0, py, px] == 0.0) and fT[py, px] == 1.0
                continue
            hit += 1
            exp = np.zeros(64)
            exp[[3, 17, 40, 63]] = np.float32([0.1, 0.2, 0.3, 0.4]).astype(float) * alpha
            np.testing.assert_allclose(coef[0, py, px], exp, rtol=1e-10, atol=1e-15)
            assert fT[py, px] == pytest.approx(1 - alpha, rel=1e-12)
            assert last[py, px] == 1
    assert hit > 50


def test_two_gaussians_front_to_back(orc):
    cam = gen.make_camera(128, 128)
    # nearer Gaussian (smaller z) must be blended first, whatever its id
    mus = [[0.0, 0.0, 0.5], [0.01, 0.0, -0.5]]
    sc = one_gaussian_scene(mus, [[0.03] * 3] * 2, [[1, 0, 0, 0]] * 2, o=0.6)
    sc.topk_idx[1, 0] = [5, 6, 7, 8]
    pr, _, (coef, fT, last, mg) = run_oracle(orc, cam, sc)
    px, py = 64, 64
    e = []
    for i in range(2):
        a, b, c = pr["cov2d"][i]
        u, v = pr["mean2d"][i]
        e.append(min(F32_099, float(np.float32(0.6)) * unnormalised_gaussian([px + .5 - u, py + .5 - v],
                                                                            [[a, b], [b, c]])))
    w = np.float32([0.1, 0.2, 0.3, 0.4]).astype(float)
    exp = np.zeros(64)
    # Gaussian 1 is nearer (z = 2.5): it goes first
    exp[[5, 6, 7, 8]] += w * e[1]
    exp[[3, 17, 40, 63]] += w * e[0] * (1 - e[1])
    np.testing.assert_allclose(coef[0, py, px], exp, rtol=1e-10)
    assert fT[py, px] == pytest.approx((1 - e[0]) * (1 - e[1]), rel=1e-12)


def test_transmittance_stop_rule_closed_form(orc):
    """Fourteen Gaussians with alpha = 1/2 at the centre pixel, then six with
    alpha = 1/10 behind them: T halves each time; the 14th would take T to
    2^-14 < 1e-4, so compositing stops there (the weaker ones behind, which
    alone would keep T above 1e-4, are not blended either): W = w (1 - 2^-13)
    and T = 2^-13."""
    cam = gen.make_camera(128, 128)
    n = 20
    mus = [[0.0, 0.0, 0.01 * k] for k in range(n)]
    sc = one_gaussian_scene(mus, [[0.05] * 3] * n, [[1, 0, 0, 0]] * n, o=1.0)
    pr = orc.project(cam, sc.means, sc.scales, sc.quats)
    # place every mean exactly on pixel (64, 64)'s centre and set opacity so that alpha = 1/2
    mean2d = pr["mean2d"].copy()
    mean2d[:] = [64.5, 64.5]
    op = np.full(n, 0.5)
    op[14:] = 0.1
    keys, ids, ranges = orc.tile_lists(cam, mean2d.astype(np.float32), pr["radius"], pr["depth"].astype(np.float32))
    coef, fT, last, mg = orc.composite(cam, ranges, ids, mean2d, pr["conic"], op, sc.topk_idx, sc.topk_w, 64)
    w = np.float32([0.1, 0.2, 0.3, 0.4]).astype(float)
    assert fT[64, 64] == 2.0 ** -13
    assert last[64, 64] == 13
    np.testing.assert_allclose(coef[0, 64, 64, [3, 17, 40, 63]], w * (1 - 2.0 ** -13), rtol=1e-15)


def test_alpha_clamp(orc):
    """A single fully opaque Gaussian at the pixel centre: alpha = 0.99 (clamp)."""
    cam = gen.make_camera(128, 128)
    sc = one_gaussian_scene([[0, 0, 0]], [[0.05] * 3], [[1, 0, 0, 0]], o=1.0)
    pr = orc.project(cam, sc.means, sc.scales, sc.quats)
    mean2d = np.array([[64.5, 64.5]])
    keys, ids, ranges = orc.tile_lists(cam, mean2d.astype(np.float32), pr["radius"], pr["depth"].astype(np.float32))
    coef, fT, last, mg = orc.composite(cam, ranges, ids, mean2d, pr["conic"], np.ones(1), sc.topk_idx, sc.topk_w, 64)
    assert fT[64, 64] == pytest.approx(1 - F32_099, rel=1e-15)
    assert coef[0, 64, 64, 63] == pytest.approx(float(np.float32(0.4)) * F32_099, rel=1e-15)


def test_invariants_c1(orc):
    scene, cam = gen.config_scene("c1")
    # float64 weights that sum to one exactly (up to float64 rounding)
    w64 = scene.topk_w.astype(np.float64)
    w64 /= w64.sum(-1, keepdims=True)
    pr = orc.project(cam, scene.means, scene.scales, scene.quats)
    keys, ids, ranges = orc.tile_lists(cam, pr["mean2d"].astype(np.float32), pr["radius"],
                                       pr["depth"].astype(np.float32))
    coef, fT, last, mg = orc.composite(cam, ranges, ids, pr["mean2d"], pr["conic"], scene.opacity,
                                       scene.topk_idx, w64, scene.L)
    assert fT.min() >= F32_1E4 and fT.max() <= 1.0
    assert coef.min() >= 0.0
    np.testing.assert_allclose(coef.sum(-1)[0] + fT, 1.0, atol=1e-13)
    # list position of the last contributor lies inside the tile list
    lens = (ranges[:, 1] - ranges[:, 0]).reshape(cam.tiles_y, cam.tiles_x)
    tl = np.kron(lens, np.ones((16, 16), np.int64))[:cam.height, :cam.width]
    assert np.all(last <= tl) and np.all((last == 0) == (fT == 1.0))


def test_transmittance_non_increasing_along_list(orc):
    """Truncating every tile list (prefixes) can only raise T: T is
    non-increasing as Gaussians are added front to back."""
    scene, cam = gen.config_scene("c1")
    pr = orc.project(cam, scene.means, scene.scales, scene.quats)
    keys, ids, ranges = orc.tile_lists(cam, pr["mean2d"].astype(np.float32), pr["radius"],
                                       pr["depth"].astype(np.float32))
    prev = None
    for frac in (0.0, 0.25, 0.5, 0.75, 1.0):
        rr = ranges.copy()
        rr[:, 1] = rr[:, 0] + np.floor((ranges[:, 1] - ranges[:, 0]) * frac).astype(np.uint32)
        _, fT, _, _ = orc.composite(cam, rr, ids, pr["mean2d"], pr["conic"], scene.opacity, scene.topk_idx,
                                    scene.topk_w, scene.L)
        if prev is not None:
            assert np.all(fT <= prev)
        prev = fT


def test_sparse_equals_dense_L(orc):
    """Blending only the K non-zeros (Algorithm 1) equals blending the full
    L-vector with its zeros (Eq. 3 with c_i = w_i), bit for bit."""
    scene, cam = gen.config_scene("c1")
    pr, (keys, ids, ranges), (coef, fT, last, mg) = run_oracle(orc, cam, scene)
    dense = np.zeros((scene.n, scene.L))
    np.put_along_axis(dense, scene.topk_idx[:, 0, :].astype(np.int64), scene.topk_w[:, 0, :].astype(float), 1)
    out = orc.composite_dense(cam, ranges, ids, pr["mean2d"], pr["conic"], scene.opacity, dense)
    assert np.array_equal(out, coef[0])


def test_linearity_eq7(orc):
    """Eq. 7: rendering f_i = w_i S directly (Eq. 6) equals rendering the
    coefficients and multiplying by S."""
    scene, cam = gen.config_scene("c1")
    pr, (keys, ids, ranges), (coef, fT, last, mg) = run_oracle(orc, cam, scene)
    dense = np.zeros((scene.n, scene.L))
    np.put_along_axis(dense, scene.topk_idx[:, 0, :].astype(np.int64), scene.topk_w[:, 0, :].astype(float), 1)
    f = dense @ scene.dictionary.astype(np.float64)
    Sd = orc.composite_dense(cam, ranges, ids, pr["mean2d"], pr["conic"], scene.opacity, f)
    F = orc.decode(coef[0], scene.dictionary)
    np.testing.assert_allclose(F, Sd, rtol=0, atol=1e-13)
    assert np.abs(F).max() > 0.05


def test_levels_are_independent(orc):
    """Three levels share alpha and T; each level equals a one-level render
    with that level's codes."""
    scene = gen.make_scene(77, 800, levels=3)
    cam = gen.make_camera(96, 80)
    pr, (keys, ids, ranges), (coef, fT, last, mg) = run_oracle(orc, cam, scene)
    for lv in range(3):
        c1, t1, l1, _ = orc.composite(cam, ranges, ids, pr["mean2d"], pr["conic"], scene.opacity,
                                      scene.topk_idx[:, lv:lv + 1], scene.topk_w[:, lv:lv + 1], scene.L)
        assert np.array_equal(c1[0], coef[lv]) and np.array_equal(t1, fT)


def test_composite_pixels_matches_full(orc):
    scene, cam = gen.config_scene("c1")
    pr, (keys, ids, ranges), (coef, fT, last, mg) = run_oracle(orc, cam, scene)
    pix = np.random.default_rng(0).choice(cam.width * cam.height, 300, replace=False)
    c, t, l, m = orc.composite_pixels(cam, ranges, ids, pr["mean2d"], pr["conic"], scene.opacity,
                                      scene.topk_idx, scene.topk_w, scene.L, pix)
    assert np.array_equal(c[:, 0], coef[0].reshape(-1, scene.L)[pix])
    assert np.array_equal(t, fT.reshape(-1)[pix]) and np.array_equal(l, last.reshape(-1)[pix])


# ---------------------------------------------------------------- decode / query
def test_decode_matches_matmul(orc):
    rng = np.random.default_rng(1)
    W = rng.random((333, 64))
    S = rng.normal(size=(64, 512))
    np.testing.assert_allclose(orc.decode(W, S), W @ S, rtol=1e-12, atol=1e-12)
    # transposed operand would fail: non-square check
    W2 = rng.random((5, 32))
    S2 = rng.normal(size=(32, 48))
    np.testing.assert_allclose(orc.decode(W2, S2), W2 @ S2, rtol=1e-12, atol=1e-12)


def test_round_bf16_matches_torch():
    import torch
    from oracle import oracle as orc
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(size=20000).astype(np.float32) * 10.0 ** rng.integers(-8, 8, 20000),
                        np.float32([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -3.0e38, 1e-40])])
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    assert np.array_equal(orc.round_bf16(x), ref)


def test_decode_bf16_reduces_to_exact(orc):
    rng = np.random.default_rng(3)
    W = orc.round_bf16(rng.random((200, 64)).astype(np.float32))
    S = orc.round_bf16(rng.normal(size=(64, 512)).astype(np.float32))
    np.testing.assert_allclose(orc.decode_bf16(W, S), W.astype(float) @ S.astype(float), rtol=1e-13, atol=1e-13)
    Wf = rng.random((200, 64)).astype(np.float32)
    Sf = rng.normal(size=(64, 512)).astype(np.float32)
    ref = orc.round_bf16(Wf).astype(float) @ orc.round_bf16(Sf).astype(float)
    np.testing.assert_allclose(orc.decode_bf16(Wf, Sf), ref, rtol=1e-13, atol=1e-13)
    out_r = orc.decode_bf16(Wf, Sf, round_out=True)
    import torch
    exp = torch.from_numpy(ref.astype(np.float32)).to(torch.bfloat16).double().numpy()
    assert np.array_equal(out_r, exp)


def test_query_closed_form_and_special_cases(orc):
    rng = np.random.default_rng(4)
    pos, neg = gen.make_text(11, D=512)
    F = rng.normal(size=(500, 512)) * 0.05
    for tau in (1.0, 10.0):
        r = orc.query(F, pos, neg, tau)
        nrm = lambda a: a / np.linalg.norm(a, axis=-1, keepdims=True)  # noqa: E731
        sq = nrm(F) @ nrm(pos.astype(float))
        sj = nrm(F) @ nrm(neg.astype(float)).T
        exp = 1.0 / (1.0 + np.exp(-tau * (sq - sj.max(1))))
        np.testing.assert_allclose(r, exp, rtol=1e-12)
    # F parallel to the query: s_q = 1
    r = orc.query(3.0 * pos[None].astype(float), pos, neg, 1.0)
    n64, p64 = neg.astype(float), pos.astype(float)
    sj = (n64 @ p64) / np.linalg.norm(n64, axis=1) / np.linalg.norm(p64)
    assert r[0] == pytest.approx(1 / (1 + np.exp(-(1 - sj.max()))), rel=1e-12)
    # zero feature -> 0.5
    assert orc.query(np.zeros((1, 512)), pos, neg)[0] == 0.5
