"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances (float32 kernels vs float64 oracle):
  - binning and per-tile order (stage-isolated: the oracle sorts the GPU's
    own float32 projection): bit-exact keys, ids and ranges;
  - projection: mean2d and depth to a few float32 ulps, conic to 1e-4
    relative (the 2x2 inverse divides by det = ac - b^2), radius exact except
    where 3 sqrt(lambda_max) is within 1e-4 of an integer;
  - compositing (stage-isolated): every pixel is checked, |dW| <= 1e-5 and
    |dT| <= 1e-5 absolute, `last` exact.  A pixel that misses the oracle's
    walk passes if it matches the walk with some of its near decisions (a
    skip or the transmittance stop within 1e-5 of its threshold, relative,
    the stop's distance divided by the transmittance's condition number)
    taken the other way, as float32 may legitimately take them; pixels that
    match neither are counted and may be at most 0.1 % (tests/alt_check.py);
  - FP32 feature map: |dF| <= 1e-5 absolute (end to end);
  - BF16 decode: within 1e-5 of the bf16-emulated oracle (float32 output) /
    one bf16 ulp (bf16 output), and per-pixel ||dF|| / ||F|| <= 1e-2 against
    the exact float64 product;
  - relevancy: 1e-5 absolute (float32 features), 2e-3 (bfloat16 features,
    whose text embeddings are rounded to bf16 for the matrix cores).
"""
import numpy as np
import pytest
import torch

import gen
from alt_check import check_flips, coef_close
from gpu_common import (by_pixel, compare_tile_lists, flip_check_gpu_lists, oracle_composite_from_gpu,
                        oracle_lists_from_gpu, run_forward, small_scene)

pytestmark = pytest.mark.gpu

ATOL = 1e-5        # float32 coefficients, transmittance and features (absolute)


def _check_lists(orc, cam, g):
    keys, ids, ranges = oracle_lists_from_gpu(orc, cam, g)
    diff = compare_tile_lists(g, keys, ids, ranges, cam.tiles_x, cam.tiles_y)
    assert diff is None, diff


def _check_coef(orc, cam, scene, g, atol=ATOL):
    """Every pixel's coefficients, T and last against the oracle's walk of the
    GPU's lists, or one of its flipped outcomes."""
    coef, fT, last, margin, margin_T = oracle_composite_from_gpu(orc, cam, scene, g)
    err = np.abs(g["coef"] - coef).max(axis=(0, 3))
    print("coef max err %.3e (%d pixels above %.0e)" % (err.max(), int((err > atol).sum()), atol))
    close = coef_close(by_pixel(g["coef"]), g["final_T"].reshape(-1), g["last"].reshape(-1), atol)
    flip_check_gpu_lists(orc, cam, scene, g, close, base=(by_pixel(coef), fT.reshape(-1), last.reshape(-1)))
    return coef, fT, last


@pytest.fixture(scope="module")
def c1(orc):
    scene, cam = gen.config_scene("c1")
    g = run_forward(cam, scene)
    return scene, cam, g


def test_project_parity_c1(orc, c1):
    scene, cam, g = c1
    pr = orc.project(cam, scene.means, scene.scales, scene.quats)
    near = np.abs(pr["extent"] - np.round(pr["extent"])) < 1e-4
    same_r = (g["radius"] == pr["radius"]) | near
    assert same_r.all()
    vis = (pr["radius"] > 0) & (g["radius"] > 0)
    assert vis.sum() > 1900
    np.testing.assert_allclose(g["mean2d"][vis], pr["mean2d"][vis], rtol=2e-6, atol=2e-5)
    np.testing.assert_allclose(g["depth"][vis], pr["depth"][vis], rtol=1e-6)
    np.testing.assert_allclose(g["conic"][vis], pr["conic"][vis], rtol=1e-4, atol=1e-6 * np.abs(pr["conic"]).max())
    exact = vis & ~near
    assert np.array_equal(g["touched"][exact], pr["touched"][exact])


def test_bin_sort_bit_exact_c1(orc, c1):
    scene, cam, g = c1
    _check_lists(orc, cam, g)


def test_splat_parity_c1(orc, c1):
    scene, cam, g = c1
    _check_coef(orc, cam, scene, g)


def test_feature_map_end_to_end_c1(orc, c1):
    """Full FP64 oracle (its own projection, lists and compositing) against the
    GPU FP32 path: the 512-d feature map within 1e-5 absolute."""
    scene, cam, g = c1
    pr = orc.project(cam, scene.means, scene.scales, scene.quats)
    keys, ids, ranges = orc.tile_lists(cam, pr["mean2d"].astype(np.float32), pr["radius"],
                                       pr["depth"].astype(np.float32))
    coef, fT, last, margin, margin_T = orc.composite(cam, ranges, ids, pr["mean2d"], pr["conic"], scene.opacity,
                                                     scene.topk_idx, scene.topk_w, scene.L, with_margin_T=True)
    F = orc.decode(coef, scene.dictionary)
    err = np.abs(g["feat"] - F).max(axis=(0, 3))
    print("end-to-end feature max err %.3e (ref max %.3e)" % (err.max(), np.abs(F).max()))
    got = by_pixel(g["feat"])

    def close(sel, c, t, l):
        return np.abs(got[sel] - orc.decode(c, scene.dictionary)).reshape(len(sel), -1).max(axis=1) <= ATOL

    check_flips(orc, cam, ranges, ids, pr["mean2d"], pr["conic"], scene.opacity, scene.topk_idx, scene.topk_w,
                scene.L, np.arange(cam.width * cam.height), close,
                base=(by_pixel(coef), fT.reshape(-1), last.reshape(-1)), label="end to end")


def test_decode_f32_parity(orc, c1):
    scene, cam, g = c1
    F = orc.decode(g["coef"].astype(np.float64), scene.dictionary)
    err = np.abs(g["feat"] - F).max()
    print("decode f32 max err %.3e" % err)
    assert err <= 1e-5


@pytest.mark.parametrize("L,D", [(64, 512), (32, 256), (128, 1024), (64, 128)])
@pytest.mark.parametrize("out_bf16", [False, True])
def test_decode_bf16_parity(orc, L, D, out_bf16):
    import paper_2507_07136_amd as ls2
    rng = np.random.default_rng(L + D)
    m = 32 * 37 + 13  # ragged: not a multiple of the 32-row block
    W = (rng.random((m, L)) * (rng.random((m, 1)) < 0.9)).astype(np.float32)
    S = rng.normal(size=(L, D))
    S = (S / np.linalg.norm(S, axis=1, keepdims=True)).astype(np.float32)
    Wt, St = torch.from_numpy(W).cuda(), torch.from_numpy(S).cuda()
    out = torch.empty((m, D), dtype=torch.bfloat16 if out_bf16 else torch.float32, device="cuda")
    ls2.ls2_dict_decode(Wt, St, out, compute=ls2.LS2_BF16)
    got = out.float().cpu().numpy()
    emu = orc.decode_bf16(W, S, round_out=out_bf16)
    # float32 accumulation of L exact bf16 products: |error| <= L 2^-24 sum|terms|
    acc_bound = 1e-5 * orc.decode(np.abs(orc.round_bf16(W)), np.abs(orc.round_bf16(S))) + 1e-12
    if out_bf16:
        # the float32 accumulator may sit on the other side of a bf16 rounding
        # boundary than the exact sum: one bf16 ulp (<= 2^-7 relative) plus the
        # accumulation error
        assert np.all(np.abs(got - emu) <= 2.0 ** -7 * np.maximum(np.abs(emu), np.abs(got)) + acc_bound)
    else:
        assert np.all(np.abs(got - emu) <= acc_bound)
    exact = orc.decode(W.astype(np.float64), S)
    nrm = np.linalg.norm(exact, axis=1)
    rel = np.linalg.norm(got - exact, axis=1)[nrm > 1e-6] / nrm[nrm > 1e-6]
    print("bf16 decode L=%d D=%d rel err max %.3e" % (L, D, rel.max()))
    assert rel.max() <= 1e-2


@pytest.mark.parametrize("L,D", [(64, 512), (32, 128), (128, 1024)])
def test_decode_f32_shapes(orc, L, D):
    import paper_2507_07136_amd as ls2
    rng = np.random.default_rng(3 * L + D)
    m = 32 * 11 + 7
    W = rng.random((m, L)).astype(np.float32)
    S = rng.normal(size=(L, D)).astype(np.float32)
    out = torch.empty((m, D), dtype=torch.float32, device="cuda")
    ls2.ls2_dict_decode(torch.from_numpy(W).cuda(), torch.from_numpy(S).cuda(), out, compute=ls2.LS2_F32)
    ref = orc.decode(W.astype(np.float64), S.astype(np.float64))
    bound = 4e-7 * orc.decode(np.abs(W), np.abs(S)) * L ** 0.5 + 1e-7
    assert np.all(np.abs(out.cpu().numpy() - ref) <= bound)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("D,n_neg", [(512, 4), (256, 1), (1024, 8), (64, 3)])
def test_query_parity(orc, dtype, D, n_neg):
    import paper_2507_07136_amd as ls2
    rng = np.random.default_rng(D + n_neg)
    m = 16 * 53 + 5
    F = (rng.normal(size=(m, D)) * 0.05).astype(np.float32)
    F[3] = 0.0  # zero feature scores 0.5
    pos, neg = gen.make_text(5, D=D, n_neg=n_neg)
    F[4] = 2.0 * pos  # parallel to the query
    Ft = torch.from_numpy(F).cuda().to(dtype)
    out = torch.empty(m, dtype=torch.float32, device="cuda")
    for tau in (1.0, 10.0):
        ls2.ls2_query(Ft, torch.from_numpy(pos).cuda(), torch.from_numpy(neg).cuda(), out, tau)
        ref = orc.query(Ft.float().cpu().numpy().astype(np.float64), pos, neg, tau)
        err = np.abs(out.cpu().numpy() - ref).max()
        print("query %s D=%d tau=%g max err %.3e" % (dtype, D, tau, err))
        assert err <= (1e-5 if dtype == torch.float32 else 2e-3) * max(1.0, tau / 4)
        assert out[3].item() == 0.5


def test_query_end_to_end_c1(orc, c1):
    import paper_2507_07136_amd as ls2
    scene, cam, g = c1
    pos, neg = gen.make_text(9)
    pipe = g["pipe"]
    r = pipe.query(torch.from_numpy(pos).cuda(), torch.from_numpy(neg).cuda()).cpu().numpy()
    ref = orc.query(orc.decode(g["coef"].astype(np.float64), scene.dictionary), pos, neg)
    assert np.abs(r - ref).max() <= 1e-5


def test_forward_deterministic(c1):
    scene, cam, g = c1
    g2 = run_forward(cam, scene)
    for k in ("mean2d", "conic", "radius", "ranges", "ids", "coef", "final_T", "last", "feat"):
        assert np.array_equal(g[k], g2[k]), k


# ---------------------------------------------------------------- edge cases
@pytest.mark.parametrize("w,h", [(100, 75), (16, 16), (33, 17)])
def test_ragged_image(orc, w, h):
    scene, cam = small_scene(2024 + w, 700, w, h)
    g = run_forward(cam, scene)
    _check_lists(orc, cam, g)
    _check_coef(orc, cam, scene, g)


@pytest.mark.parametrize("L,K,levels", [(64, 4, 3), (128, 8, 1), (32, 2, 2), (128, 4, 1), (64, 8, 1), (64, 1, 1),
                                        (32, 8, 3)])
def test_shapes_levels(orc, L, K, levels):
    scene, cam = small_scene(7 + L + K + levels, 900, 96, 80, L=L, K=K, levels=levels, D=128)
    g = run_forward(cam, scene)
    _check_lists(orc, cam, g)
    _check_coef(orc, cam, scene, g)


def test_duplicate_indices_are_additive(orc):
    scene, cam = small_scene(99, 600, 64, 64)
    scene.topk_idx[:, :, 1] = scene.topk_idx[:, :, 0]
    g = run_forward(cam, scene)
    _check_coef(orc, cam, scene, g)


def test_empty_and_culled(orc):
    # no Gaussians at all
    scene, cam = small_scene(5, 0, 64, 48)
    g = run_forward(cam, scene)
    assert g["P"] == 0 and np.all(g["coef"] == 0) and np.all(g["final_T"] == 1) and np.all(g["last"] == 0)
    # every Gaussian behind the camera or NaN
    scene, cam = small_scene(6, 300, 64, 48)
    scene.means[:150, 2] = -5.0
    scene.means[150:, 0] = np.nan
    g = run_forward(cam, scene)
    assert g["P"] == 0 and np.all(g["radius"] == 0) and np.all(g["coef"] == 0)
    # the one-pass forms on an empty frame: zero features, relevancy 1/2
    import paper_2507_07136_amd as ls2
    t = g["t"]
    p16 = ls2.Pipeline(cam, scene.n, coef_dtype=torch.bfloat16)
    p16.project(t["means"], t["scales"], t["quats"])
    assert p16.bin_sort(sync=True) == 0
    feat = p16.splat_decode(t["opacity"], t["topk_idx"], t["topk_w"], t["dictionary"])
    pos, neg = gen.make_text(6)
    rel = p16.splat_decode_query(t["opacity"], t["topk_idx"], t["topk_w"], t["dictionary"],
                                 torch.from_numpy(pos).cuda(), torch.from_numpy(neg).cuda())
    torch.cuda.synchronize()
    assert torch.count_nonzero(feat).item() == 0
    assert bool((rel == 0.5).all()) and bool((p16.final_T == 1.0).all()) and bool((p16.last == 0).all())


def test_capacity_overflow(orc):
    import paper_2507_07136_amd as ls2
    scene, cam = gen.config_scene("c1")
    t = ls2.to_device(scene)
    pipe = ls2.Pipeline(cam, scene.n, max_pairs=100)
    pipe.project(t["means"], t["scales"], t["quats"])
    with pytest.raises(ls2.LS2Error) as e:
        ls2.ls2_bin_sort(pipe.cam, pipe.mean2d, pipe.radius, pipe.depth, 100, None, pipe.ids, pipe.tile_ranges,
                         pipe.workspace, sync=True)
    assert e.value.status == ls2.LS2_ERR_CAPACITY and e.value.num_pairs > 100
    # without sync: no error, every range empty, count readable afterwards
    ls2.ls2_bin_sort(pipe.cam, pipe.mean2d, pipe.radius, pipe.depth, 100, None, pipe.ids, pipe.tile_ranges,
                     pipe.workspace, sync=False)
    assert ls2.ls2_bin_sort_count(pipe.workspace) == e.value.num_pairs
    assert int(pipe.tile_ranges.abs().sum().item()) == 0
    # the pipeline grows its buffers and retries
    assert pipe.bin_sort(sync=True) == e.value.num_pairs


def test_long_tile_lists(orc):
    """Thousands of Gaussians piled onto one tile: a bucket beyond the LDS
    capacity is split over its depth range and sorted in LDS-sized runs, and
    with a pool of exactly P entries (no room for the split) it is sorted by
    the global-memory network; lists bit-exact."""
    rng = np.random.default_rng(12)
    n = 40000
    scene = gen.make_scene(12, n, D=128)
    scene.means[:] = rng.normal(0, 0.01, (n, 3)).astype(np.float32)
    scene.scales[:] = 0.004
    cam = gen.make_camera(64, 64)
    g = run_forward(cam, scene)
    lens = g["ranges"][:, 1] - g["ranges"][:, 0]
    assert lens.max() > 16384
    _check_lists(orc, cam, g)
    _check_coef(orc, cam, scene, g)
    # a pool of exactly P entries leaves no room for the split's scratch copy:
    # the global-memory network sorts the bucket instead
    g2 = run_forward(cam, scene, max_pairs=g["P"])
    assert g2["P"] == g["P"]
    _check_lists(orc, cam, g2)


@pytest.mark.parametrize("n,keep_keys,lo,hi", [(8500, False, 0, 9216), (9800, True, 9216, 10240),
                                               (9800, False, 9216, 10240), (12000, False, 10240, 16384),
                                               (20000, False, 16384, 1 << 30)])
def test_bucket_size_tiers(orc, n, keep_keys, lo, hi):
    """One superblock (a 64 x 64 image) holding every Gaussian, at bucket sizes
    that take each path of the sort kernel: up to 9216 keys (9 per thread,
    coverage masks sorted along), up to 10240 (16 per thread, masks along),
    up to 16384 (masks gathered from the rectangles) and beyond (the bucket is
    split over its depth range); with and without the keys output.  Lists
    bit-exact."""
    rng = np.random.default_rng(40 + n)
    scene = gen.make_scene(40 + n, n, D=128)
    scene.means[:] = rng.normal(0, 0.05, (n, 3)).astype(np.float32)
    scene.scales[:] = 0.004
    cam = gen.make_camera(64, 64)
    g = run_forward(cam, scene, keep_keys=keep_keys)
    vis = int((g["radius"] > 0).sum())
    assert lo < vis <= hi, vis  # every visible Gaussian is in the one bucket
    assert (g["keys"] is not None) == keep_keys
    _check_lists(orc, cam, g)


def test_large_bucket_depths_across_exponents(orc):
    """40000 Gaussians in one superblock with depths from 1.5 to 4.5, across
    three float exponents: the bucket is split into bins over its depth range
    (the float exponent alone would give three over-full bins) and each run of
    bins is sorted in LDS; lists bit-exact."""
    rng = np.random.default_rng(14)
    n = 40000
    scene = gen.make_scene(14, n, D=128)
    m = np.empty((n, 3))
    m[:, :2] = rng.normal(0, 0.01, (n, 2))
    m[:, 2] = rng.uniform(-1.5, 1.5, n)
    scene.means[:] = m.astype(np.float32)
    scene.scales[:] = 0.002
    cam = gen.make_camera(64, 64)
    g = run_forward(cam, scene)
    d = g["depth"][g["radius"] > 0]
    assert d.min() < 2.0 and d.max() > 4.0
    lens = g["ranges"][:, 1] - g["ranges"][:, 0]
    assert lens.max() > 16384
    _check_lists(orc, cam, g)


def test_bucket_with_one_heavy_depth_bin(orc):
    """20000 Gaussians at exactly one depth and one much nearer: the top
    digit of the bucket cannot split the pile, so it takes the global-memory
    network; lists stay bit-exact."""
    rng = np.random.default_rng(13)
    n = 20001
    scene = gen.make_scene(13, n, D=128)
    scene.means[:, :2] = rng.normal(0, 0.01, (n, 2)).astype(np.float32)
    scene.means[:, 2] = 0.0
    scene.means[0, 2] = -1.5
    scene.scales[:] = 0.004
    cam = gen.make_camera(64, 64)
    g = run_forward(cam, scene)
    assert len(np.unique(g["depth"][g["radius"] > 0])) == 2
    _check_lists(orc, cam, g)


# ---------------------------------------------------------------- full size, sampled
@pytest.mark.slow
def test_c2_full_size_sampled(orc):
    """1440x1080, 300k Gaussians (the benchmark workload): binning bit-exact
    at full size; compositing, decode and relevancy checked on sampled pixels."""
    scene, cam = gen.config_scene("c2")
    g = run_forward(cam, scene, keep_keys=True)
    print("P =", g["P"])
    _check_lists(orc, cam, g)
    rng = np.random.default_rng(0)
    pix = rng.choice(cam.width * cam.height, 4000, replace=False)
    gc = g["coef"][0].reshape(-1, scene.L)[pix]
    close = coef_close(gc[:, None], g["final_T"].reshape(-1)[pix], g["last"].reshape(-1)[pix], ATOL)
    flip_check_gpu_lists(orc, cam, scene, g, close, pix=pix, label="c2 sampled")
    F = orc.decode(gc.astype(np.float64), scene.dictionary)
    assert np.abs(g["feat"][0].reshape(-1, scene.D)[pix] - F).max() <= 1e-5


@pytest.mark.parametrize("L,D,n_neg,tau", [(64, 512, 4, 1.0), (32, 256, 1, 10.0), (128, 384, 8, 3.0)])
def test_query_coef_parity(orc, L, D, n_neg, tau):
    """Relevancy from the coefficient map equals the oracle's relevancy of the
    oracle-decoded feature map (Eq. 7), float32 tolerance."""
    import paper_2507_07136_amd as ls2
    rng = np.random.default_rng(L + D + n_neg)
    m = 3001
    coef = (rng.random((m, L)) * (rng.random((m, L)) < 0.3)).astype(np.float32)
    coef[0] = 0.0                                   # empty pixel: r = 0.5
    dct = rng.standard_normal((L, D)).astype(np.float32)
    dct /= np.linalg.norm(dct, axis=1, keepdims=True)
    pos, neg = gen.make_text(L + D, D=D, n_neg=n_neg)
    ref = orc.query(orc.decode(coef, dct), pos, neg, tau)
    out = torch.empty((m,), device="cuda")
    ws = torch.empty((ls2.ls2_query_coef_workspace(L, n_neg),), dtype=torch.uint8, device="cuda")
    ls2.ls2_query_coef(torch.from_numpy(coef).cuda(), torch.from_numpy(dct).cuda(), torch.from_numpy(pos).cuda(),
                       torch.from_numpy(neg).cuda(), out, ws, tau)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert got[0] == 0.5
    assert np.abs(got - ref).max() <= 1e-5 * max(1.0, tau / 4), np.abs(got - ref).max()


def test_query_coef_end_to_end_c1(orc, c1):
    """Score c1 from its rendered coefficients; equals the oracle's query of the
    oracle decode of the same coefficients (stage-isolated)."""
    scene, cam, g = c1
    pos, neg = gen.make_text(11)
    rel = g["pipe"].query_coef(g["t"]["dictionary"], torch.from_numpy(pos).cuda(), torch.from_numpy(neg).cuda())
    torch.cuda.synchronize()
    ref = orc.query(orc.decode(g["coef"].astype(np.float64), scene.dictionary), pos, neg)
    assert np.abs(rel.cpu().numpy() - ref).max() <= 1e-5


def _dense_weights(scene):
    n, lv, K = scene.topk_idx.shape
    W = np.zeros((n, lv, scene.L), np.float32)
    for k in range(K):   # in k order, as the sparse kernel merges repeated indices
        np.add.at(W, (np.arange(n)[:, None], np.arange(lv)[None, :], scene.topk_idx[:, :, k]), scene.topk_w[:, :, k])
    return W


@pytest.mark.parametrize("L,K,levels", [(64, 4, 1), (32, 8, 2), (64, 8, 2), (32, 4, 3), (64, 4, 3)])
def test_dense_splat_equals_sparse(L, K, levels):
    """Dense-L splat of the scattered codes equals the sparse splat bit for bit:
    both blend with one fused multiply-add per coefficient in list order (the
    dense one adds exact zeros for the atoms outside the K stored)."""
    import paper_2507_07136_amd as ls2
    scene, cam = small_scene(303 + L + K + levels, 3000, 120, 90, L=L, K=K, levels=levels, D=128)
    g = run_forward(cam, scene)
    pipe, t = g["pipe"], g["t"]
    Wd = torch.from_numpy(_dense_weights(scene)).cuda()
    pipe.splat_dense(t["opacity"], Wd)
    torch.cuda.synchronize()
    coef_d = pipe.coef.cpu().numpy()
    assert np.array_equal(pipe.last.cpu().numpy(), g["last"])
    assert np.array_equal(coef_d, g["coef"])
    assert np.array_equal(pipe.final_T.cpu().numpy(), g["final_T"])


@pytest.mark.parametrize("levels,w,h", [(1, 100, 75), (3, 100, 75), (3, 33, 47)])
def test_dense_splat_parity(orc, levels, w, h):
    """Table 9's dense baseline against the oracle's dense renderer (Eqs. 4
    and 6 with the L-vector of every level as the per-Gaussian channels):
    every weight non-zero, ragged image, the levels sharing alpha and T.  Each
    pixel's L-vectors of all levels, T and last within the float32 bar, or
    matching the walk with near decisions flipped (the flipped walk runs the
    sparse form with K = L, every atom stored)."""
    L = 64
    scene, cam = small_scene(707 + levels + w, 2500, w, h, L=L, K=4, levels=levels, D=128)
    g = run_forward(cam, scene)
    pipe, t = g["pipe"], g["t"]
    rng = np.random.default_rng(levels + w)
    z = rng.standard_normal((scene.n, levels, L))
    Wd = (np.exp(z) / np.exp(z).sum(-1, keepdims=True)).astype(np.float32)
    pipe.coef.fill_(5.0)
    pipe.splat_dense(t["opacity"], torch.from_numpy(Wd).cuda())
    torch.cuda.synchronize()
    got = by_pixel(pipe.coef.cpu().numpy())
    gT, gl = pipe.final_T.cpu().numpy().reshape(-1), pipe.last.cpu().numpy().reshape(-1)
    m2, cn = g["mean2d"].astype(np.float64), g["conic"].astype(np.float64)
    dense = orc.composite_dense(cam, g["ranges"], g["ids"], m2, cn, scene.opacity, Wd.reshape(scene.n, levels * L))
    base = dense.reshape(h * w, levels, L)
    # T and last of the same walk (they do not depend on the codes)
    _, fT, last, _ = orc.composite(cam, g["ranges"], g["ids"], m2, cn, scene.opacity, scene.topk_idx,
                                   scene.topk_w, scene.L)
    err = np.abs(got - base).max()
    print("dense splat %dx%d: max err %.3e against the dense oracle" % (levels, L, err))
    idx = np.broadcast_to(np.arange(L, dtype=np.int32), (scene.n, levels, L))
    check_flips(orc, cam, g["ranges"], g["ids"], m2, cn, scene.opacity, idx, Wd, L, np.arange(h * w),
                coef_close(got, gT, gl, ATOL), base=(base, fT.reshape(-1), last.reshape(-1)),
                label="dense %dx%d" % (levels, L))


@pytest.mark.parametrize("L,K,levels", [(64, 4, 1), (32, 8, 2), (128, 4, 1), (64, 4, 3)])
def test_bf16_coefficient_map(orc, L, K, levels):
    """The bf16 coefficient map is the float32 map rounded to nearest even (bit
    for bit), and decoding it gives the bf16-compute feature map of the float32
    map bit for bit (bf16 and float32 outputs)."""
    import paper_2507_07136_amd as ls2
    scene, cam = small_scene(404 + L + K + levels, 3000, 120, 90, L=L, K=K, levels=levels, D=256)
    g = run_forward(cam, scene)
    pipe, t = g["pipe"], g["t"]
    p16 = ls2.Pipeline(cam, scene.n, levels=levels, K=K, L=L, D=scene.D, coef_dtype=torch.bfloat16)
    p16.project(t["means"], t["scales"], t["quats"])
    p16.bin_sort(sync=True)
    p16.splat(t["opacity"], t["topk_idx"], t["topk_w"])
    torch.cuda.synchronize()
    c32 = torch.from_numpy(g["coef"]).cuda()
    assert torch.equal(p16.coef, c32.to(torch.bfloat16))
    assert np.array_equal(p16.last.cpu().numpy(), g["last"])
    assert np.array_equal(p16.final_T.cpu().numpy(), g["final_T"])
    for out_dtype in (torch.bfloat16, torch.float32):
        f16 = p16.decode(t["dictionary"], ls2.LS2_BF16, out_dtype).clone()
        f32 = pipe.decode(t["dictionary"], ls2.LS2_BF16, out_dtype).clone()
        torch.cuda.synchronize()
        assert torch.equal(f16, f32), out_dtype
    with pytest.raises(ls2.LS2Error):
        p16.decode(t["dictionary"], ls2.LS2_F32, torch.float32)


@pytest.mark.parametrize("L,K,levels,D,w,h", [(64, 4, 1, 512, 120, 90), (32, 8, 3, 256, 100, 76),
                                               (128, 4, 1, 384, 72, 56), (64, 8, 2, 128, 33, 47),
                                               (64, 3, 1, 1024, 64, 48)])
def test_splat_decode_fused(orc, L, K, levels, D, w, h):
    """The one-pass splat + decode writes the feature map of splat (bf16 map)
    followed by the bf16 decode bit for bit, and the same optional map,
    final_T and last; against the FP64 oracle (its compositing of the GPU's
    lists, exact decode) every clean pixel meets the bf16 decode bar.  Ragged
    image sizes leave partial quadrants at the right and bottom edges."""
    import paper_2507_07136_amd as ls2
    scene, cam = small_scene(505 + L + K + levels + D, 3000, w, h, L=L, K=K, levels=levels, D=D)
    g = run_forward(cam, scene)
    t = g["t"]
    p16 = ls2.Pipeline(cam, scene.n, levels=levels, K=K, L=L, D=D, coef_dtype=torch.bfloat16)
    p16.project(t["means"], t["scales"], t["quats"])
    p16.bin_sort(sync=True)
    p16.splat(t["opacity"], t["topk_idx"], t["topk_w"])
    ref_coef = p16.coef.clone()
    ref_T, ref_last = p16.final_T.clone(), p16.last.clone()
    ref_feat = p16.decode(t["dictionary"], ls2.LS2_BF16, torch.bfloat16).clone()
    # feature map only: stale values everywhere first
    p16.feat.fill_(7.0)
    p16.final_T.fill_(-1.0)
    p16.last.fill_(-5)
    feat = p16.splat_decode(t["opacity"], t["topk_idx"], t["topk_w"], t["dictionary"])
    torch.cuda.synchronize()
    assert torch.equal(feat, ref_feat)
    assert torch.equal(p16.final_T, ref_T) and torch.equal(p16.last, ref_last)
    # with the map kept
    p16.coef.fill_(3.0)
    p16.feat.fill_(-2.0)
    p16.splat_decode(t["opacity"], t["topk_idx"], t["topk_w"], t["dictionary"], keep_coef=True)
    torch.cuda.synchronize()
    assert torch.equal(p16.coef, ref_coef)
    assert torch.equal(p16.feat, ref_feat)
    # against the oracle: rows with ||F|| > 1e-3 within 1e-2 relative (L2),
    # pixels nothing reached decode to exact zeros
    coef64, fT, last = oracle_composite_from_gpu(orc, cam, scene, g)[:3]
    exact = orc.decode(coef64.reshape(-1, L), scene.dictionary).reshape(levels, h, w, D)
    nrm = np.linalg.norm(exact, axis=3)
    assert (nrm > 1e-3).sum() > 0.5 * nrm.size
    got = by_pixel(feat.float().cpu().numpy())

    def close(sel, c, t, l):
        F = orc.decode(c, scene.dictionary)
        n = np.linalg.norm(F, axis=2)
        rel = np.linalg.norm(got[sel] - F, axis=2) / np.maximum(n, 1e-6)
        zero = np.abs(got[sel]).max(axis=2) == 0.0
        return (((n <= 1e-3) | (rel <= 1e-2)) & ((n > 0.0) | zero)).all(axis=1)

    flip_check_gpu_lists(orc, cam, scene, g, close, base=(by_pixel(coef64), fT.reshape(-1), last.reshape(-1)),
                         label="fused splat+decode")


@pytest.mark.parametrize("L,K,levels,D,n_neg,w,h,keep", [(64, 4, 1, 512, 4, 120, 90, True),
                                                         (64, 4, 1, 512, 4, 120, 90, False),
                                                         (32, 8, 3, 256, 1, 100, 76, True),
                                                         (128, 4, 1, 384, 8, 72, 56, False),
                                                         (64, 3, 2, 128, 2, 33, 47, True)])
def test_splat_decode_query_fused(orc, L, K, levels, D, n_neg, w, h, keep):
    """The one-pass splat + decode + relevancy equals ls2_query on the
    one-pass bf16 feature map bit for bit (and writes that map only if asked);
    against the oracle (exact compositing of the GPU's lists, exact decode,
    LERF relevancy) every clean pixel meets the bf16 relevancy bar."""
    import paper_2507_07136_amd as ls2
    scene, cam = small_scene(606 + L + K + levels + D + n_neg, 3000, w, h, L=L, K=K, levels=levels, D=D)
    g = run_forward(cam, scene)
    t = g["t"]
    pos, neg = gen.make_text(L + D + n_neg, D=D, n_neg=n_neg)
    tp, tn = torch.from_numpy(pos).cuda(), torch.from_numpy(neg).cuda()
    p16 = ls2.Pipeline(cam, scene.n, levels=levels, K=K, L=L, D=D, coef_dtype=torch.bfloat16)
    p16.project(t["means"], t["scales"], t["quats"])
    p16.bin_sort(sync=True)
    ref_feat = p16.splat_decode(t["opacity"], t["topk_idx"], t["topk_w"], t["dictionary"]).clone()
    ref_T, ref_last = p16.final_T.clone(), p16.last.clone()
    ref_rel = torch.empty((levels, h, w), device="cuda")
    ls2.ls2_query(ref_feat, tp, tn, ref_rel)
    p16.feat.fill_(3.0)
    p16.final_T.fill_(-1.0)
    p16.last.fill_(-7)
    rel = p16.splat_decode_query(t["opacity"], t["topk_idx"], t["topk_w"], t["dictionary"], tp, tn,
                                 keep_feat=keep).clone()
    torch.cuda.synchronize()
    assert torch.equal(rel, ref_rel)
    assert torch.equal(p16.final_T, ref_T) and torch.equal(p16.last, ref_last)
    if keep:
        assert torch.equal(p16.feat, ref_feat)
    else:
        assert bool((p16.feat == 3.0).all())       # not written
    coef64, fT, last = oracle_composite_from_gpu(orc, cam, scene, g)[:3]
    got = rel.cpu().numpy().reshape(levels, -1).T

    def close(sel, c, t, l):
        r = orc.query(orc.decode(c, scene.dictionary), pos, neg)
        return (np.abs(got[sel] - r) <= 2e-3).all(axis=1)

    flip_check_gpu_lists(orc, cam, scene, g, close, base=(by_pixel(coef64), fT.reshape(-1), last.reshape(-1)),
                         label="one-pass relevancy")


@pytest.mark.parametrize("L,D,n_neg,coef_bf16,keep", [(64, 512, 4, True, True), (64, 512, 4, False, False),
                                                       (32, 256, 1, False, True), (128, 384, 8, True, False),
                                                       (64, 128, 2, False, True)])
def test_decode_query_epilogue(orc, L, D, n_neg, coef_bf16, keep):
    """Relevancy formed in the bf16 decode's epilogue equals ls2_query on the
    bf16 feature map bit for bit; the map itself equals the plain bf16 decode;
    against the oracle it meets the bf16 relevancy bar.  Ragged row count."""
    import paper_2507_07136_amd as ls2
    rng = np.random.default_rng(L + D + n_neg)
    m = 3001
    coef = (rng.random((m, L)) * (rng.random((m, L)) < 0.3)).astype(np.float32)
    coef[0] = 0.0                                   # empty pixel
    dct = rng.standard_normal((L, D)).astype(np.float32)
    dct /= np.linalg.norm(dct, axis=1, keepdims=True)
    pos, neg = gen.make_text(L + D + 1, D=D, n_neg=n_neg)
    tc = torch.from_numpy(coef).cuda()
    if coef_bf16:
        tc = tc.to(torch.bfloat16)
    td, tp, tn = (torch.from_numpy(x).cuda() for x in (dct, pos, neg))
    ref_feat = torch.empty((m, D), dtype=torch.bfloat16, device="cuda")
    ls2.ls2_dict_decode(tc, td, ref_feat, compute=ls2.LS2_BF16)
    ref_rel = torch.empty((m,), device="cuda")
    ls2.ls2_query(ref_feat, tp, tn, ref_rel)
    rel = torch.empty((m,), device="cuda")
    feat = torch.empty((m, D), dtype=torch.bfloat16, device="cuda") if keep else None
    ls2.ls2_dict_decode_query(tc, td, tp, tn, rel, feat=feat)
    torch.cuda.synchronize()
    assert torch.equal(rel, ref_rel)
    if keep:
        assert torch.equal(feat, ref_feat)
    r64 = orc.query(orc.decode(coef.astype(np.float64), dct), pos, neg)
    assert np.abs(rel.cpu().numpy() - r64).max() <= 2e-3
    assert rel[0].item() == 0.5


def test_equal_depth_runs_in_id_order(orc):
    """Short runs of equal float32 depth (ordered by id inside their depth
    bin by the insertion sort) and one run of 300 equal depths (a depth bin
    beyond 16 keys: sorted by the LDS bitonic network): lists bit-exact."""
    rng = np.random.default_rng(21)
    n = 3000
    scene = gen.make_scene(21, n, D=128)
    scene.means[:] = rng.uniform(-0.15, 0.15, (n, 3)).astype(np.float32)
    scene.means[1:200:2, 2] = scene.means[0:199:2, 2]   # 100 pairs of equal depth
    scene.means[500:800, 2] = 0.05                      # one run of 300
    scene.scales[:] = 0.01
    cam = gen.make_camera(96, 80)
    g = run_forward(cam, scene)
    d = g["depth"][g["radius"] > 0]
    assert len(d) - len(np.unique(d)) >= 300
    _check_lists(orc, cam, g)
    _check_coef(orc, cam, scene, g)


def test_many_equal_depth_runs_across_buckets(orc):
    """Depths on a coarse grid across 12 superblocks: buckets hold many runs
    of 2-16 equal depths (ordered by id inside their depth bins by the
    insertion sort) and, where 40 Gaussians share one depth in one place,
    bins beyond 16 keys (sorted by the LDS bitonic network): lists
    bit-exact."""
    rng = np.random.default_rng(31)
    n_base, n_a, n_b = 20000, 30 * 12, 3 * 40
    n = n_base + n_a + n_b
    scene = gen.make_scene(31, n, D=128)
    m = rng.uniform(-1.0, 1.0, (n, 3))
    m[:n_base, 2] = np.round(rng.uniform(-1.0, 1.0, n_base) * 1000.0) / 1000.0  # 2001 depth levels
    off = n_base
    for size, groups in ((12, 30), (40, 3)):
        for _ in range(groups):
            c = rng.uniform(-0.8, 0.8, 2)
            m[off:off + size, :2] = c + rng.normal(0.0, 0.03, (size, 2))
            m[off:off + size, 2] = rng.uniform(-1.0, 1.0)
            off += size
    scene.means[:] = m.astype(np.float32)
    scene.scales[:] = 0.02
    cam = gen.make_camera(256, 192)
    g = run_forward(cam, scene, keep_keys=True)
    _, mult = np.unique(g["depth"][g["radius"] > 0], return_counts=True)
    assert ((mult >= 2) & (mult <= 16)).sum() >= 1000 and mult.max() >= 40
    _check_lists(orc, cam, g)


def test_index_check_mode(orc):
    """With the code-index check on, an index outside [0, L) makes the
    splat, the one-pass splat + decode and the splat backward return
    LS2_ERR_ARG before any launch; valid indices pass and render as without
    the check.  With the check off the index is taken modulo L."""
    import paper_2507_07136_amd as ls2
    scene, cam = small_scene(808, 600, 64, 48)
    g = run_forward(cam, scene)
    pipe, t = g["pipe"], g["t"]
    bad = t["topk_idx"].clone()
    bad[17, 0, 2] = scene.L + 3
    prev = ls2.set_check(True)
    try:
        pipe.coef.fill_(2.0)
        pipe.splat(t["opacity"], t["topk_idx"], t["topk_w"])        # valid: renders
        torch.cuda.synchronize()
        assert np.array_equal(pipe.coef.cpu().numpy(), g["coef"])
        with pytest.raises(ls2.LS2Error) as e:
            pipe.splat(t["opacity"], bad, t["topk_w"])
        assert e.value.status == ls2.LS2_ERR_ARG
        bad2 = t["topk_idx"].clone()
        bad2[5, 0, 0] = -1
        with pytest.raises(ls2.LS2Error):
            pipe.splat(t["opacity"], bad2, t["topk_w"])
        p16 = ls2.Pipeline(cam, scene.n, coef_dtype=torch.bfloat16, D=scene.D)
        p16.project(t["means"], t["scales"], t["quats"])
        p16.bin_sort(sync=True)
        with pytest.raises(ls2.LS2Error):
            p16.splat_decode(t["opacity"], bad, t["topk_w"], t["dictionary"])
        n, lv, K = scene.topk_idx.shape
        outs = [torch.empty(s, device="cuda") for s in ((n, 2), (n, 3), (n,), (n, lv, K))]
        with pytest.raises(ls2.LS2Error):
            ls2.ls2_splat_sparse_backward(pipe.cam, lv, K, scene.L, pipe.tile_ranges, pipe.ids, pipe.mean2d,
                                          pipe.conic, t["opacity"], bad, t["topk_w"], pipe.final_T, pipe.last,
                                          torch.zeros_like(pipe.coef), *outs)
    finally:
        ls2.set_check(prev)
    # check off: index L + 3 composites into atom 3
    wrapped = t["topk_idx"].clone()
    wrapped[17, 0, 2] = 3
    pipe.splat(t["opacity"], bad, t["topk_w"])
    c_bad = pipe.coef.clone()
    pipe.splat(t["opacity"], wrapped, t["topk_w"])
    torch.cuda.synchronize()
    assert torch.equal(c_bad, pipe.coef)


def test_large_image_superblock_geometry(orc):
    """An image above 4096 x 4096 (4160 x 4160: 260 x 260 tiles) bins by
    superblocks of 8 x 8 tiles, each filled as four blocks of 4 x 4 tiles:
    lists bit-exact over the whole image; 3000 sampled pixels (most
    of them in covered tiles) composited against the oracle."""
    import paper_2507_07136_amd as ls2
    W = H = 4160
    scene, cam = small_scene(4160, 3000, W, H, L=32, K=4, D=64)
    t = ls2.to_device(scene)
    pipe = ls2.Pipeline(cam, scene.n, L=32, K=4, D=64, keep_keys=True)
    pipe.project(t["means"], t["scales"], t["quats"])
    P = pipe.bin_sort(sync=True)
    pipe.splat(t["opacity"], t["topk_idx"], t["topk_w"])
    torch.cuda.synchronize()
    g = dict(P=P, mean2d=pipe.mean2d.cpu().numpy(), conic=pipe.conic.cpu().numpy(), depth=pipe.depth.cpu().numpy(),
             radius=pipe.radius.cpu().numpy(), ranges=pipe.tile_ranges.cpu().numpy().view(np.uint32),
             ids=pipe.ids[:P].cpu().numpy().view(np.uint32),
             keys=pipe.keys[:P].cpu().numpy().view(np.uint64))
    print("P = %d over %d tiles" % (P, len(g["ranges"])))
    assert P > 10000
    _check_lists(orc, cam, g)
    tiles = np.flatnonzero(g["ranges"][:, 1] > g["ranges"][:, 0])
    rng = np.random.default_rng(3)
    tsel = rng.choice(tiles, 2500)
    txs, tys = tsel % cam.tiles_x, tsel // cam.tiles_x
    px = np.minimum(txs * 16 + rng.integers(0, 16, 2500), W - 1)
    py = np.minimum(tys * 16 + rng.integers(0, 16, 2500), H - 1)
    pix = np.unique(np.concatenate([py * W + px, rng.choice(W * H, 500, replace=False)]))
    sel = torch.from_numpy(pix).cuda()
    gc = pipe.coef[0].reshape(-1, 32).index_select(0, sel).cpu().numpy()[:, None]
    gT = pipe.final_T.reshape(-1).index_select(0, sel).cpu().numpy()
    gl = pipe.last.reshape(-1).index_select(0, sel).cpu().numpy()
    flip_check_gpu_lists(orc, cam, scene, g, coef_close(gc, gT, gl, ATOL), pix=pix, label="4160x4160 sampled")


@pytest.mark.parametrize("case", ["c1", "c2", "ragged", "culled", "empty", "overflow", "large_image"])
def test_project_bin_sort_fused(orc, case):
    """ls2_project_bin_sort (the binning's first pass projects) equals
    ls2_project followed by ls2_bin_sort bit for bit: every projection output,
    P, the keys, ids and tile ranges, the overflow path included; and its
    lists equal the oracle's."""
    import paper_2507_07136_amd as ls2
    max_pairs = None
    if case in ("c1", "c2"):
        scene, cam = gen.config_scene(case)
    elif case == "ragged":
        scene, cam = small_scene(31, 4000, 203, 117)
    elif case == "culled":
        scene, cam = small_scene(32, 3000, 160, 96)
        scene.means[:500, 2] = -5.0
        scene.means[500:700, 0] = np.nan
    elif case == "empty":
        scene, cam = small_scene(33, 0, 64, 48)
    elif case == "overflow":
        scene, cam = gen.config_scene("c1")
        max_pairs = 100
    else:  # beyond 4096 superblocks of 4x4 tiles: 8x8-tile superblocks
        scene, cam = small_scene(34, 2000, 4200, 4200)
    t = ls2.to_device(scene)
    pa = ls2.Pipeline(cam, scene.n, keep_keys=True, max_pairs=max_pairs)
    pb = ls2.Pipeline(cam, scene.n, keep_keys=True, max_pairs=max_pairs)
    for p_ in (pa, pb):  # garbage in every output, so nothing unwritten passes
        for buf in (p_.mean2d, p_.conic, p_.depth):
            buf.fill_(-7.0)
        for buf in (p_.radius, p_.tiles_touched, p_.ids, p_.tile_ranges, p_.keys):
            buf.fill_(-7)
    pa.project(t["means"], t["scales"], t["quats"])
    if case == "overflow":
        Pa = ls2.ls2_bin_sort(pa.cam, pa.mean2d, pa.radius, pa.depth, 100, pa.keys, pa.ids, pa.tile_ranges,
                              pa.workspace, sync=False)
        Pb = ls2.ls2_project_bin_sort(pb.cam, t["means"], t["scales"], t["quats"], pb.mean2d, pb.conic, pb.depth,
                                      pb.radius, 100, pb.keys, pb.ids, pb.tile_ranges, pb.workspace,
                                      tiles_touched=pb.tiles_touched, sync=False)
        with pytest.raises(ls2.LS2Error) as e:
            ls2.ls2_project_bin_sort(pb.cam, t["means"], t["scales"], t["quats"], pb.mean2d, pb.conic, pb.depth,
                                     pb.radius, 100, pb.keys, pb.ids, pb.tile_ranges, pb.workspace,
                                     tiles_touched=pb.tiles_touched, sync=True)
        assert e.value.status == ls2.LS2_ERR_CAPACITY
        Pa = Pb = ls2.ls2_bin_sort_count(pa.workspace)
        assert ls2.ls2_bin_sort_count(pb.workspace) == Pa == e.value.num_pairs > 100
    else:
        Pa = pa.bin_sort(sync=True)
        Pb = pb.project_bin_sort(t["means"], t["scales"], t["quats"], sync=True)
    torch.cuda.synchronize()
    assert Pa == Pb
    for name in ("mean2d", "conic", "depth", "radius", "tiles_touched", "tile_ranges"):
        a, b = getattr(pa, name), getattr(pb, name)
        assert torch.equal(a.view(torch.int32), b.view(torch.int32)), name   # bits, NaN-safe
    if case != "overflow":
        assert torch.equal(pa.ids[:Pa], pb.ids[:Pb]) and torch.equal(pa.keys[:Pa], pb.keys[:Pb])
    else:
        assert int(pb.tile_ranges.abs().sum().item()) == 0
    if case == "ragged":  # tiles_touched is optional: the same lists without it
        ids_b = pb.ids[:Pb].clone()
        pb.ids.fill_(-7)
        Pc = ls2.ls2_project_bin_sort(pb.cam, t["means"], t["scales"], t["quats"], pb.mean2d, pb.conic, pb.depth,
                                      pb.radius, pb.max_pairs, pb.keys, pb.ids, pb.tile_ranges, pb.workspace,
                                      tiles_touched=None, sync=True)
        assert Pc == Pb and torch.equal(pb.ids[:Pc], ids_b)
    if case in ("c1", "ragged", "culled", "large_image"):
        g = dict(P=Pb, mean2d=pb.mean2d.cpu().numpy(), radius=pb.radius.cpu().numpy(),
                 depth=pb.depth.cpu().numpy(), ranges=pb.tile_ranges.cpu().numpy().view(np.uint32),
                 ids=pb.ids[:Pb].cpu().numpy().view(np.uint32), keys=pb.keys[:Pb].cpu().numpy().view(np.uint64))
        keys, ids, ranges = orc.tile_lists(cam, g["mean2d"], g["radius"], g["depth"])
        diff = compare_tile_lists(g, keys, ids, ranges, cam.tiles_x, cam.tiles_y)
        assert diff is None, diff


@pytest.mark.parametrize("mix", [False, True])
def test_emission_staging_overflow(orc, mix):
    """Large Gaussians (about 6 superblocks each): the emission workgroups
    hold more entries than they stage in LDS (12.7k against 10240) and write
    them in place; with mix, only the first workgroup's Gaussians are large,
    so one workgroup writes in place and the other stages.  The lists stay
    bit-exact against the oracle."""
    scene, cam = small_scene(51, 4096, 640, 480)
    scene.scales[: 2048 if mix else 4096] *= 3.0
    g = run_forward(cam, scene, keep_keys=True)
    _check_lists(orc, cam, g)


@pytest.mark.parametrize("n", [1, 2048, 2049, 10240, 10241, 16384, 16385])
def test_single_superblock_bucket_sizes(orc, n):
    """A 64 x 64 image is one superblock of 4 x 4 tiles, and every Gaussian of
    the scene projects inside it (means within [-1, 1]^3 seen from z = -3
    with a 60 degree field of view), so the superblock's bucket holds exactly
    n keys.  The sizes sit on both sides of each change of method in the
    sort kernel: the per-tile list fill (at most 2048 keys), the slice fill
    with the coverage masks sorted along (at most 10240), the fill from the
    stored rectangles, and the split of buckets beyond 16384 keys.  Lists,
    keys and ranges bit-exact against the oracle."""
    scene, cam = small_scene(57, n, 64, 64)
    g = run_forward(cam, scene, keep_keys=True)
    assert int((g["radius"] > 0).sum()) == n
    _check_lists(orc, cam, g)
