"""ctypes shim over the FP64 CPU oracle (``ls2_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It marshals
numpy arrays; all arithmetic happens in the C file (plus the numpy loss and
finite-difference helpers that the tests define themselves).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ls2_oracle.c")
_CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-fopenmp"]
# LS2_ORACLE_SANITIZE=1: a separate build with AddressSanitizer and
# UndefinedBehaviorSanitizer (host code only; the process must preload the
# gcc sanitizer runtimes), used by the sanitizer test
_SANITIZE = os.environ.get("LS2_ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "libls2_oracle_san.so" if _SANITIZE else "libls2_oracle.so")
if _SANITIZE:
    _CFLAGS = [f for f in _CFLAGS if f != "-O2"] + ["-O1", "-g", "-fno-omit-frame-pointer",
                                                   "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA
    contraction, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        _declare(_lib)
    return _lib


_P = ctypes.c_void_p


def _declare(L):
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.orc_num_threads.restype = ctypes.c_int
    L.orc_project.argtypes = [_P, ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.orc_project.restype = None
    L.orc_project_f64.argtypes = [_P, ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.orc_project_f64.restype = None
    L.orc_tile_lists.argtypes = [_P, ctypes.c_int, _P, _P, _P, i64, _P, _P, _P, _P]
    L.orc_tile_lists.restype = ctypes.c_int
    L.orc_composite.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P, _P, _P, _P, _P,
                                _P, _P, _P, _P, _P]
    L.orc_composite.restype = None
    L.orc_composite_dense.argtypes = [_P, ctypes.c_int, _P, _P, _P, _P, _P, _P, _P]
    L.orc_composite_dense.restype = None
    L.orc_composite_pixels.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P, _P, _P,
                                       _P, _P, i64, _P, _P, _P, _P, _P, _P]
    L.orc_composite_pixels.restype = None
    L.orc_composite_pixels_alt.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P, _P, _P,
                                           _P, _P, i64, _P, _P, f64, _P, _P, _P, _P]
    L.orc_composite_pixels_alt.restype = None
    L.orc_composite_bruteforce.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.orc_composite_bruteforce.restype = None
    L.orc_decode.argtypes = [i64, ctypes.c_int, ctypes.c_int, _P, _P, _P]
    L.orc_decode.restype = None
    L.orc_decode_bf16.argtypes = [i64, ctypes.c_int, ctypes.c_int, _P, _P, ctypes.c_int, _P]
    L.orc_decode_bf16.restype = None
    L.orc_round_bf16.argtypes = [i64, _P, _P]
    L.orc_round_bf16.restype = None
    L.orc_query.argtypes = [i64, ctypes.c_int, _P, _P, ctypes.c_int, _P, f64, _P]
    L.orc_query.restype = None
    for name, args in _BACKWARD_DECLS.items():
        if hasattr(L, name):
            getattr(L, name).argtypes = args
            getattr(L, name).restype = None
    del i32


_P_ = ctypes.c_void_p
_BACKWARD_DECLS: dict = {
    "orc_loss_l1cos": [ctypes.c_int64, ctypes.c_int, _P_, _P_, _P_, _P_],
    "orc_query_backward": [ctypes.c_int64, ctypes.c_int, _P_, _P_, ctypes.c_int, _P_, ctypes.c_double, _P_, _P_, _P_],
    "orc_decode_backward": [ctypes.c_int64, ctypes.c_int, ctypes.c_int, _P_, _P_, _P_, _P_, _P_],
    "orc_composite_backward": [_P_, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P_, _P_, _P_, _P_, _P_,
                               _P_, _P_, _P_, _P_, _P_, _P_, _P_],
    "orc_composite_backward_pixels": [_P_, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P_, _P_, _P_,
                                      _P_, _P_, _P_, _P_, ctypes.c_int64, _P_, _P_, _P_, _P_, _P_, _P_],
    "orc_project_backward": [_P_, ctypes.c_int, _P_, _P_, _P_, _P_, _P_, _P_, _P_, _P_, _P_],
    "orc_project_backward_f64": [_P_, ctypes.c_int, _P_, _P_, _P_, _P_, _P_, _P_, _P_, _P_, _P_],
}


def _c(a, dtype):
    """Contiguous array of dtype (copy only if needed)."""
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def cam_array(cam) -> np.ndarray:
    return _c(cam.as_array() if hasattr(cam, "as_array") else cam, np.float64)


# --------------------------------------------------------------------------
def project(cam, means, scales, quats, f64=False):
    """Projection of every Gaussian (Eqs. 1-2, EWA reading).  Returns a dict
    of float64/int32 arrays: mean2d (N,2), cov2d (N,3), conic (N,3), depth,
    extent, radius, rect (N,4), touched.  Inputs are taken as float32 (the
    kernels' input type) unless f64 is set."""
    dt = np.float64 if f64 else np.float32
    means, scales, quats = _c(means, dt), _c(scales, dt), _c(quats, dt)
    n = means.shape[0]
    out = dict(mean2d=np.zeros((n, 2)), cov2d=np.zeros((n, 3)), conic=np.zeros((n, 3)),
               depth=np.zeros(n), extent=np.zeros(n), radius=np.zeros(n, np.int32),
               rect=np.zeros((n, 4), np.int32), touched=np.zeros(n, np.int32))
    ca = cam_array(cam)
    fn = lib().orc_project_f64 if f64 else lib().orc_project
    fn(_p(ca), n, _p(means), _p(scales), _p(quats), _p(out["mean2d"]), _p(out["cov2d"]),
                      _p(out["conic"]), _p(out["depth"]), _p(out["extent"]), _p(out["radius"]),
                      _p(out["rect"]), _p(out["touched"]))
    return out


def tile_lists(cam, mean2d_f32, radius, depth_f32, cap=None):
    """Per-tile depth-ordered lists from float32 mean2d/depth and int radius.
    Returns (keys u64 [P], ids u32 [P], ranges u32 [tiles, 2])."""
    n = radius.shape[0]
    m2 = _c(mean2d_f32, np.float32)
    rd = _c(radius, np.int32)
    dp = _c(depth_f32, np.float32)
    ca = cam_array(cam)
    ntiles = cam.tiles_x * cam.tiles_y
    P = ctypes.c_int64(0)
    ranges = np.zeros((ntiles, 2), np.uint32)
    if cap is None:
        st = lib().orc_tile_lists(_p(ca), n, _p(m2), _p(rd), _p(dp), 0, None, None, _p(ranges),
                                  ctypes.byref(P))
        cap = P.value
    keys = np.zeros(max(cap, 1), np.uint64)
    ids = np.zeros(max(cap, 1), np.uint32)
    st = lib().orc_tile_lists(_p(ca), n, _p(m2), _p(rd), _p(dp), cap, _p(keys), _p(ids), _p(ranges),
                              ctypes.byref(P))
    if st != 0:
        raise RuntimeError("tile_lists capacity %d < %d" % (cap, P.value))
    return keys[:P.value], ids[:P.value], ranges


def composite(cam, ranges, ids, mean2d, conic, opacity, topk_idx, topk_w, L, with_margin_T=False):
    """Sparse coefficient splatting (Algorithm 1).  topk_idx/topk_w: (N, levels, K).
    Returns coef (levels, H, W, L), final_T (H, W), last (H, W), margin (H, W)
    and, if with_margin_T, margin_T (H, W): the relative distances of the
    alpha decisions (clamp, skip) and of the stop decision to their thresholds."""
    n, levels, K = topk_idx.shape
    H, W = cam.height, cam.width
    coef = np.zeros((levels, H, W, L))
    fT = np.zeros((H, W))
    last = np.zeros((H, W), np.int32)
    margin = np.zeros((H, W))
    margin_T = np.zeros((H, W))
    ids = _c(ids, np.uint32)
    args = [_c(ranges, np.uint32), ids if ids.size else np.zeros(1, np.uint32), _c(mean2d, np.float64),
            _c(conic, np.float64), _c(opacity, np.float64), _c(topk_idx, np.int32), _c(topk_w, np.float64)]
    lib().orc_composite(_p(cam_array(cam)), levels, K, L, *[_p(a) for a in args], _p(coef), _p(fT),
                        _p(last), _p(margin), _p(margin_T))
    if with_margin_T:
        return coef, fT, last, margin, margin_T
    return coef, fT, last, margin


def composite_pixels(cam, ranges, ids, mean2d, conic, opacity, topk_idx, topk_w, L, pix, with_margin_T=False):
    """Composite only the flat pixel indices ``pix``.  Returns coef
    (npix, levels, L), final_T, last, margin (npix,) [, margin_T]."""
    n, levels, K = topk_idx.shape
    pix = _c(pix, np.int64)
    npix = pix.shape[0]
    coef = np.zeros((npix, levels, L))
    fT = np.zeros(npix)
    last = np.zeros(npix, np.int32)
    margin = np.zeros(npix)
    margin_T = np.zeros(npix)
    ids = _c(ids, np.uint32)
    args = [_c(ranges, np.uint32), ids if ids.size else np.zeros(1, np.uint32), _c(mean2d, np.float64),
            _c(conic, np.float64), _c(opacity, np.float64), _c(topk_idx, np.int32), _c(topk_w, np.float64)]
    lib().orc_composite_pixels(_p(cam_array(cam)), levels, K, L, *[_p(a) for a in args], npix, _p(pix),
                               _p(coef), _p(fT), _p(last), _p(margin), _p(margin_T))
    if with_margin_T:
        return coef, fT, last, margin, margin_T
    return coef, fT, last, margin


def composite_pixels_alt(cam, ranges, ids, mean2d, conic, opacity, topk_idx, topk_w, L, pix, flips, thr=1e-5):
    """``composite_pixels`` with the near decisions of Eq. 3 (a skip of a
    positive exponent, a skip below alpha = 1/255, the transmittance stop;
    near = within ``thr`` of the threshold, relative, the stop's margin
    divided by the transmittance's condition number) taken the other way
    where bit b of ``flips[q]`` is set, b counting the near decisions met
    along pixel q's walk.  Returns coef (npix, levels, L), final_T, last and
    n_near (npix,): the number of near decisions each walk met."""
    n, levels, K = topk_idx.shape
    pix = _c(pix, np.int64)
    npix = pix.shape[0]
    fl = _c(np.broadcast_to(np.asarray(flips, np.uint32), (npix,)), np.uint32)
    coef = np.zeros((npix, levels, L))
    fT = np.zeros(npix)
    last = np.zeros(npix, np.int32)
    n_near = np.zeros(npix, np.int32)
    ids = _c(ids, np.uint32)
    args = [_c(ranges, np.uint32), ids if ids.size else np.zeros(1, np.uint32), _c(mean2d, np.float64),
            _c(conic, np.float64), _c(opacity, np.float64), _c(topk_idx, np.int32), _c(topk_w, np.float64)]
    lib().orc_composite_pixels_alt(_p(cam_array(cam)), levels, K, L, *[_p(a) for a in args], npix, _p(pix),
                                   _p(fl), float(thr), _p(coef), _p(fT), _p(last), _p(n_near))
    return coef, fT, last, n_near


def composite_dense(cam, ranges, ids, mean2d, conic, opacity, feat):
    """Dense renderer (Eqs. 4/6): feat (N, C) -> (H, W, C)."""
    feat = _c(feat, np.float64)
    C = feat.shape[1]
    out = np.zeros((cam.height, cam.width, C))
    ids = _c(ids, np.uint32)
    args = [_c(ranges, np.uint32), ids if ids.size else np.zeros(1, np.uint32), _c(mean2d, np.float64),
            _c(conic, np.float64), _c(opacity, np.float64), feat]
    lib().orc_composite_dense(_p(cam_array(cam)), C, *[_p(a) for a in args], _p(out))
    return out


def composite_bruteforce(cam, mean2d_f32, radius, depth_f32, mean2d, conic, opacity, topk_idx, topk_w, L):
    """Brute-force per-pixel renderer (no tile lists).  Returns (coef, final_T)."""
    n, levels, K = topk_idx.shape
    coef = np.zeros((levels, cam.height, cam.width, L))
    fT = np.zeros((cam.height, cam.width))
    args = [_c(mean2d_f32, np.float32), _c(radius, np.int32), _c(depth_f32, np.float32),
            _c(mean2d, np.float64), _c(conic, np.float64), _c(opacity, np.float64), _c(topk_idx, np.int32),
            _c(topk_w, np.float64)]
    lib().orc_composite_bruteforce(_p(cam_array(cam)), n, levels, K, L, *[_p(a) for a in args], _p(coef),
                                   _p(fT))
    return coef, fT


def decode(coef, dictionary):
    """F = W S in float64.  coef (..., L), dictionary (L, D) -> (..., D)."""
    L, D = dictionary.shape
    c = _c(coef, np.float64).reshape(-1, L)
    s = _c(dictionary, np.float64)
    out = np.zeros((c.shape[0], D))
    lib().orc_decode(c.shape[0], L, D, _p(c), _p(s), _p(out))
    return out.reshape(*coef.shape[:-1], D)


def decode_bf16(coef_f32, dictionary_f32, round_out=False):
    """Decode with bf16-rounded operands, float64 accumulation; optionally
    bf16-rounded output.  Inputs float32."""
    L, D = dictionary_f32.shape
    c = _c(coef_f32, np.float32).reshape(-1, L)
    s = _c(dictionary_f32, np.float32)
    out = np.zeros((c.shape[0], D))
    lib().orc_decode_bf16(c.shape[0], L, D, _p(c), _p(s), int(bool(round_out)), _p(out))
    return out.reshape(*coef_f32.shape[:-1], D)


def round_bf16(x):
    x = _c(x, np.float32)
    out = np.empty_like(x)
    lib().orc_round_bf16(x.size, _p(x), _p(out))
    return out


def query(feat, pos, neg, tau=1.0):
    """LERF relevancy per pixel.  feat (..., D) float64; pos (D,), neg (J, D)."""
    D = feat.shape[-1]
    f = _c(feat, np.float64).reshape(-1, D)
    pos = _c(pos, np.float32)
    neg = _c(neg, np.float32).reshape(-1, D)
    out = np.zeros(f.shape[0])
    lib().orc_query(f.shape[0], D, _p(f), _p(pos), neg.shape[0], _p(neg), float(tau), _p(out))
    return out.reshape(feat.shape[:-1])


# -------------------------------------------------------------------------- backward
def loss_l1cos(F, Y):
    """loss = mean|F - Y| + mean_rows (1 - cos(F_row, Y_row)); returns (loss, dF)."""
    D = F.shape[-1]
    f = _c(F, np.float64).reshape(-1, D)
    y = _c(Y, np.float64).reshape(-1, D)
    dF = np.zeros_like(f)
    loss = ctypes.c_double(0.0)
    lib().orc_loss_l1cos(f.shape[0], D, _p(f), _p(y), ctypes.byref(loss), _p(dF))
    return loss.value, dF.reshape(F.shape)


def query_backward(feat, pos, neg, d_rel, tau=1.0):
    """dL/dF of the relevancy given dL/dr.  Returns (d_feat, margin) where
    margin is the gap between the two most similar negatives per row."""
    D = feat.shape[-1]
    f = _c(feat, np.float64).reshape(-1, D)
    pos = _c(pos, np.float32)
    neg = _c(neg, np.float32).reshape(-1, D)
    dr = _c(d_rel, np.float64).reshape(-1)
    out = np.zeros_like(f)
    margin = np.zeros(f.shape[0])
    lib().orc_query_backward(f.shape[0], D, _p(f), _p(pos), neg.shape[0], _p(neg), float(tau), _p(dr), _p(out),
                             _p(margin))
    return out.reshape(feat.shape), margin.reshape(feat.shape[:-1])


def decode_backward(coef, dictionary, d_feat):
    """(d_coef, d_dict) of F = W S."""
    L, D = dictionary.shape
    c = _c(coef, np.float64).reshape(-1, L)
    s = _c(dictionary, np.float64)
    g = _c(d_feat, np.float64).reshape(-1, D)
    dc = np.zeros_like(c)
    ds = np.zeros_like(s)
    lib().orc_decode_backward(c.shape[0], L, D, _p(c), _p(s), _p(g), _p(dc), _p(ds))
    return dc.reshape(coef.shape), ds


def composite_backward(cam, ranges, ids, mean2d, conic, opacity, topk_idx, topk_w, d_coef):
    """Gradients of the sparse splat w.r.t. mean2d (N,2), conic (N,3),
    opacity (N,), topk_w (N, levels, K) given d_coef (levels, H, W, L)."""
    n, levels, K = topk_idx.shape
    L = d_coef.shape[-1]
    dm = np.zeros((n, 2))
    dcn = np.zeros((n, 3))
    do = np.zeros(n)
    dw = np.zeros((n, levels, K))
    ids = _c(ids, np.uint32)
    args = [_c(ranges, np.uint32), ids if ids.size else np.zeros(1, np.uint32), _c(mean2d, np.float64),
            _c(conic, np.float64), _c(opacity, np.float64), _c(topk_idx, np.int32), _c(topk_w, np.float64),
            _c(d_coef, np.float64)]
    lib().orc_composite_backward(_p(cam_array(cam)), n, levels, K, L, *[_p(a) for a in args], _p(dm), _p(dcn),
                                 _p(do), _p(dw))
    return dm, dcn, do, dw


def composite_backward_pixels(cam, ranges, ids, mean2d, conic, opacity, topk_idx, topk_w, pix, d_coef_pix):
    """``composite_backward`` for an upstream gradient that is zero outside the
    flat pixel indices ``pix`` (each listed once); d_coef_pix (npix, levels, L)
    holds the gradient of those pixels.  Same outputs."""
    n, levels, K = topk_idx.shape
    pix = _c(pix, np.int64)
    g = _c(d_coef_pix, np.float64)
    assert g.shape[:2] == (pix.shape[0], levels) and len(np.unique(pix)) == pix.shape[0]
    L = g.shape[-1]
    dm = np.zeros((n, 2))
    dcn = np.zeros((n, 3))
    do = np.zeros(n)
    dw = np.zeros((n, levels, K))
    ids = _c(ids, np.uint32)
    args = [_c(ranges, np.uint32), ids if ids.size else np.zeros(1, np.uint32), _c(mean2d, np.float64),
            _c(conic, np.float64), _c(opacity, np.float64), _c(topk_idx, np.int32), _c(topk_w, np.float64)]
    lib().orc_composite_backward_pixels(_p(cam_array(cam)), n, levels, K, L, *[_p(a) for a in args], pix.shape[0],
                                        _p(pix), _p(g), _p(dm), _p(dcn), _p(do), _p(dw))
    return dm, dcn, do, dw


def project_backward(cam, means, scales, quats, radius, d_mean2d, d_conic, f64=False):
    """(d_means, d_scales, d_quats) of the projection."""
    dt = np.float64 if f64 else np.float32
    means, scales, quats = _c(means, dt), _c(scales, dt), _c(quats, dt)
    n = means.shape[0]
    dmu = np.zeros((n, 3))
    ds = np.zeros((n, 3))
    dq = np.zeros((n, 4))
    fn = lib().orc_project_backward_f64 if f64 else lib().orc_project_backward
    fn(_p(cam_array(cam)), n, _p(means), _p(scales), _p(quats), _p(_c(radius, np.int32)),
                               _p(_c(d_mean2d, np.float64)), _p(_c(d_conic, np.float64)), _p(dmu), _p(ds), _p(dq))
    return dmu, ds, dq


# -------------------------------------------------------------------------- post-processing
def postprocess(relevancy, kernel, smooth_mode=0, select_mode=0, threshold=0.5):
    """Relevancy post-processing (Section 3.2: a mean filter over each level's
    relevancy map, then one level is selected; the evaluation appendix gives
    the localization point as the argmax of the smoothed map, the mask as the
    normalised smoothed map above a threshold, and two selection rules).

    relevancy: [levels, H, W].  kernel: odd box size.  smooth_mode 0: Avg(M),
    1: 0.5 (M + Avg(M)).  select_mode 0: the level with the largest smoothed
    maximum; 1: the level with the largest mean of the smoothed map inside its
    own mask.  Readings: the box mean runs over the window clipped to the
    image; ties (argmax, level) go to the smallest index; normalisation is
    (s - min) / (max - min) per level (zero when max == min); the mask is
    normalised > threshold; a level with an empty mask has mean -inf.

    Plain float64 loops over the definitions.  Returns (smoothed, mask,
    result=[level, x, y, flat index], stats [levels, 4] = max, min,
    mask mean, mask count)."""
    M = np.asarray(relevancy, np.float64)
    lv, H, W = M.shape
    r = kernel // 2
    S = np.zeros_like(M)
    for l in range(lv):
        for y in range(H):
            y0, y1 = max(0, y - r), min(H - 1, y + r)
            for x in range(W):
                x0, x1 = max(0, x - r), min(W - 1, x + r)
                S[l, y, x] = M[l, y0:y1 + 1, x0:x1 + 1].sum() / ((y1 - y0 + 1) * (x1 - x0 + 1))
    if smooth_mode == 1:
        S = 0.5 * (M + S)
    stats = np.zeros((lv, 4))
    masks = np.zeros((lv, H, W), bool)
    argmax = np.zeros(lv, np.int64)
    for l in range(lv):
        flat = S[l].reshape(-1)
        argmax[l] = int(np.argmax(flat))       # first maximum in row-major order
        mx, mn = flat.max(), flat.min()
        norm = (S[l] - mn) / (mx - mn) if mx > mn else np.zeros_like(S[l])
        masks[l] = norm > threshold
        cnt = masks[l].sum()
        stats[l] = (mx, mn, S[l][masks[l]].mean() if cnt else -np.inf, cnt)
    key = stats[:, 0] if select_mode == 0 else stats[:, 2]
    sel = int(np.argmax(key))                  # first level on ties
    idx = int(argmax[sel])
    result = np.array([sel, idx % W, idx // W, idx], np.int64)
    return S, masks[sel].astype(np.uint8), result, stats


# -------------------------------------------------------------------------- sparse code parametrisation
def sparse_codes(logits, K):
    """Section 3.3: the L-dimensional parameter of a Gaussian is normalised by a
    softmax, the top-K values are kept and renormalised to sum 1.  Returns
    (idx [rows, K] int32, w [rows, K]) with indices in descending order of the
    logit (ties: smaller index first).  Since every softmax value shares the
    same denominator, the renormalised weights are the softmax of the K kept
    logits; computed here from the definition (softmax, select, divide)."""
    z = np.asarray(logits, np.float64)
    rows, L = z.shape
    idx = np.zeros((rows, K), np.int32)
    w = np.zeros((rows, K))
    for r in range(rows):
        p = np.exp(z[r] - z[r].max())
        p /= p.sum()
        order = sorted(range(L), key=lambda j: (-z[r, j], j))[:K]
        idx[r] = order
        kept = p[order]
        w[r] = kept / kept.sum()
    return idx, w


def sparse_codes_backward(logits, K, d_w):
    """d logits of sparse_codes given dL/dw (the selection is piecewise
    constant): for kept j, dz_j = w_j (dw_j - sum_k w_k dw_k); 0 elsewhere."""
    idx, w = sparse_codes(logits, K)
    d_w = np.asarray(d_w, np.float64)
    dz = np.zeros(np.asarray(logits).shape)
    for r in range(dz.shape[0]):
        s = float((w[r] * d_w[r]).sum())
        for k in range(K):
            dz[r, idx[r, k]] = w[r, k] * (d_w[r, k] - s)
    return dz
