"""Pins of the oracle walk with near decisions flipped (Eq. 3, Algorithm 1),
which the parity checks use where a float32 decision may legitimately come
out the other way.

Each flipped outcome is pinned to the plain walk on an input nudged just
across the threshold (or with the entry removed), so that taking a decision
"the other way" means what the compositing rule itself would compute there.
Runs on the CPU only.
"""
import math

import numpy as np
import pytest

import gen
from alt_check import check_flips, coef_close

F32_1_255 = float(np.float32(1.0) / np.float32(255.0))
F32_1E4 = float(np.float32(1e-4))
L = 8
PX, PY = 8, 8                      # the pixel whose centre is (8.5, 8.5)
PIX = np.array([PY * 16 + PX])
E = math.exp(-0.05)                # exp(power) at offset dx = 1 for conic A = 0.1


def hand_scene(offsets, opacity):
    """Gaussians on one 16x16 tile, in list order, with isotropic conic 0.1
    and mean offset (dx, 0) from the pixel centre; level 0 codes: Gaussian i
    puts weight 1 on atom i % L."""
    n = len(offsets)
    mean2d = np.array([[PX + 0.5 + d, PY + 0.5] for d in offsets], np.float64)
    conic = np.tile([0.1, 0.0, 0.1], (n, 1)).astype(np.float64)
    idx = (np.arange(n) % L).astype(np.int32).reshape(n, 1, 1)
    w = np.ones((n, 1, 1))
    ranges = np.array([[0, n]], np.uint32)
    ids = np.arange(n, dtype=np.uint32)
    return ranges, ids, mean2d, conic, np.asarray(opacity, np.float64), idx, w


def walk(orc, sc, flips=0, pix=PIX):
    cam = gen.make_camera(16, 16)
    ranges, ids, mean2d, conic, op, idx, w = sc
    return orc.composite_pixels_alt(cam, ranges, ids, mean2d, conic, op, idx, w, L, pix, flips)


def plain(orc, sc, pix=PIX):
    cam = gen.make_camera(16, 16)
    ranges, ids, mean2d, conic, op, idx, w = sc
    c, t, l, _ = orc.composite_pixels(cam, ranges, ids, mean2d, conic, op, idx, w, L, pix)
    return c, t, l


def same(a, b, rtol=0.0):
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_allclose(x, y, rtol=rtol, atol=0)


def test_no_flip_equals_plain_walk(orc):
    """flips = 0 is the plain walk, bit for bit, on a whole seeded image."""
    scene, cam = gen.config_scene("c1")
    pr = orc.project(cam, scene.means, scene.scales, scene.quats)
    _, ids, ranges = orc.tile_lists(cam, pr["mean2d"].astype(np.float32), pr["radius"],
                                    pr["depth"].astype(np.float32))
    pix = np.arange(cam.width * cam.height)
    args = (cam, ranges, ids, pr["mean2d"], pr["conic"], scene.opacity, scene.topk_idx, scene.topk_w, scene.L, pix)
    c0, t0, l0, _ = orc.composite_pixels(*args)
    c1, t1, l1, nn = orc.composite_pixels_alt(*args, 0)
    assert np.array_equal(c0, c1) and np.array_equal(t0, t1) and np.array_equal(l0, l1)
    # near decisions are rare on a random scene
    assert nn.sum() < 0.01 * pix.size


@pytest.mark.parametrize("above", [True, False])
def test_alpha_skip_flip(orc, above):
    """A faint Gaussian with alpha within 2e-6 of 1/255, then an alpha = 1/2
    one: flipping its skip equals the plain walk with its opacity moved to
    the other side of the threshold."""
    rel = 2e-6 if above else -2e-6
    o0 = F32_1_255 * (1 + rel) / E
    sc = hand_scene([1.0, 1.0], [o0, 0.5 / E])
    base = walk(orc, sc)
    assert base[3][0] == 1
    same(base, plain(orc, sc))
    flipped = walk(orc, sc, 1)
    nudged = hand_scene([1.0, 1.0], [F32_1_255 * (1 - rel) / E, 0.5 / E])
    ref = plain(orc, nudged)
    # skipping is exact; blending the nudged one differs by its 4e-6 in alpha
    same(flipped, ref, rtol=0 if above else 1e-5)
    assert flipped[2][0] != base[2][0] or not np.array_equal(flipped[0], base[0])
    # the faint one blends in exactly one of the two walks
    blended = base if above else flipped
    assert blended[0][0, 0, 0] == pytest.approx(F32_1_255, rel=1e-5)
    assert (flipped if above else base)[0][0, 0, 0] == 0.0


def test_stop_flip(orc):
    """Thirteen alpha = 1/2 Gaussians, then one whose T (1 - alpha) is 1e-4
    (1 + 1e-6): it is blended; flipping the stop equals the plain walk where
    its opacity is raised so that T (1 - alpha) = 1e-4 (1 - 1e-6), which
    stops there."""
    offs = [1.0] * 14
    op = [0.5 / E] * 13
    T13 = plain(orc, hand_scene(offs[:13], op))[1][0]
    assert T13 == pytest.approx(2.0 ** -13, rel=1e-12)
    a_blend = 1 - F32_1E4 * (1 + 1e-6) / T13
    a_stop = 1 - F32_1E4 * (1 - 1e-6) / T13
    sc = hand_scene(offs, op + [a_blend / E])
    base = walk(orc, sc)
    same(base, plain(orc, sc))
    assert base[2][0] == 14 and base[3][0] == 1
    flipped = walk(orc, sc, 1)
    ref = plain(orc, hand_scene(offs, op + [a_stop / E]))
    same(flipped, ref)
    assert flipped[2][0] == 13 and flipped[1][0] == pytest.approx(T13, rel=1e-15)
    # and the other way round: a stopping walk flipped blends it
    sc2 = hand_scene(offs, op + [a_stop / E])
    f2 = walk(orc, sc2, 1)
    same(f2, plain(orc, sc), rtol=1e-5)


def test_positive_exponent_flip(orc):
    """A Gaussian centred exactly on the pixel centre has exponent 0, at the
    threshold of the skip of a positive exponent: flipping it equals the plain
    walk of the list without that Gaussian."""
    sc = hand_scene([0.0, 1.0], [0.3, 0.5 / E])
    base = walk(orc, sc)
    assert base[3][0] == 1
    same(base, plain(orc, sc))
    assert base[0][0, 0, 0] == pytest.approx(0.3, rel=1e-15)
    flipped = walk(orc, sc, 1)
    ranges, ids, mean2d, conic, op, idx, w = sc
    without = (np.array([[0, 1]], np.uint32), np.array([1], np.uint32), mean2d, conic, op, idx, w)
    ref = plain(orc, without)
    same(flipped[:2], ref[:2])
    assert flipped[2][0] == ref[2][0] + 1   # list positions count the skipped entry


def test_two_independent_flips(orc):
    """Two faint Gaussians near 1/255 (one above, one below) and an opaque
    one: the four flip masks give the four plain walks with the opacities
    nudged across the threshold independently."""
    lo, hi = F32_1_255 * (1 - 3e-6) / E, F32_1_255 * (1 + 3e-6) / E
    offs = [1.0, 1.0, 1.0]
    sc = hand_scene(offs, [hi, lo, 0.5 / E])
    seen = set()
    for mask in range(4):
        got = walk(orc, sc, mask)
        assert got[3][0] == 2
        o0 = lo if mask & 1 else hi
        o1 = hi if mask & 2 else lo
        same(got, plain(orc, hand_scene(offs, [o0, o1, 0.5 / E])), rtol=1e-5)
        seen.add(tuple(np.round(got[0][0, 0, :3], 12)))
    assert len(seen) == 4


def test_pixel_without_near_decision_ignores_flips(orc):
    sc = hand_scene([1.0, 2.0], [0.4, 0.5])
    base = walk(orc, sc)
    assert base[3][0] == 0
    for mask in (1, 2, 255):
        same(walk(orc, sc, mask), base)


def test_check_flips_matches_flipped_and_catches_mistakes(orc):
    """The parity helper accepts a kernel result that took a near decision
    the other way, and reports a planted error (an oracle output moved by
    1e-3 at one pixel) as matching no outcome."""
    cam = gen.make_camera(16, 16)
    o0 = F32_1_255 * (1 + 2e-6) / E
    ranges, ids, mean2d, conic, op, idx, w = hand_scene([1.0, 1.0], [o0, 0.5 / E])
    pix = np.arange(256)
    args = (cam, ranges, ids, mean2d, conic, op, idx, w, L)
    c, t, l, nn = orc.composite_pixels_alt(*args, pix, 0)
    cf, tf, lf, _ = orc.composite_pixels_alt(*args, PIX, 1)
    got_c, got_t, got_l = c.copy(), t.copy(), l.copy()
    got_c[PIX], got_t[PIX], got_l[PIX] = cf, tf, lf
    res = check_flips(orc, *args, pix, coef_close(got_c, got_t, got_l, 1e-5))
    assert res["base_mismatch"] == 1 and res["matched_flip"] == 1 and res["unmatched"] == 0
    got_c[PIX[0] + 1, 0, 1] += 1e-3
    with pytest.raises(AssertionError, match="match no outcome"):
        check_flips(orc, *args, pix, coef_close(got_c, got_t, got_l, 1e-5))
