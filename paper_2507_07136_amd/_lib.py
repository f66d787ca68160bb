"""ctypes binding of libls2 (include/ls2.h).

Argument marshalling only: tensors are checked for device, dtype, shape and
contiguity, converted to raw device pointers, and handed to the C ABI together
with the current HIP stream.  Every step of the path runs in the HIP library;
there is no CPU or PyTorch fallback.  If the library is missing the import
fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# LS2_LIB_SANITIZED=1 loads the host-sanitized build instead (a debugging
# build of the same sources; the process must preload the sanitizer runtimes)
LIB_PATH = os.path.join(_HERE, "libls2_san.so" if os.environ.get("LS2_LIB_SANITIZED") == "1" else "libls2.so")

LS2_OK, LS2_ERR_ARG, LS2_ERR_CAPACITY, LS2_ERR_UNSUPPORTED, LS2_ERR_DEVICE = 0, -1, -2, -3, -4
LS2_F32, LS2_BF16 = 0, 1
LS2_SMOOTH_AVG, LS2_SMOOTH_HALF = 0, 1
LS2_SELECT_MAX, LS2_SELECT_MASK_MEAN = 0, 1
TILE = 16


class LS2Error(RuntimeError):
    def __init__(self, fn, status):
        super().__init__("%s failed: %s (%d)" % (fn, status_string(status), status))
        self.status = status


class ls2_camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("world_to_cam", ctypes.c_float * 12), ("znear", ctypes.c_float)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libls2.so not built at %s: run `python paper_2507_07136_amd/build.py` "
                          "(or __graft_entry__.build())" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    cam = ctypes.POINTER(ls2_camera)
    sig = {
        "ls2_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "ls2_version": ([], ctypes.c_int),
        "ls2_source_hash": ([], ctypes.c_char_p),
        "ls2_set_check": ([ctypes.c_int], ctypes.c_int),
        "ls2_project": ([cam, i32, P, P, P, P, P, P, P, P, P], ctypes.c_int),
        "ls2_bin_sort_workspace": ([cam, i32, i64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ls2_bin_sort": ([cam, i32, P, P, P, i64, P, P, P, ctypes.POINTER(ctypes.c_int64), P, ctypes.c_size_t, P],
                         ctypes.c_int),
        "ls2_bin_sort_count": ([P, ctypes.POINTER(ctypes.c_int64), P], ctypes.c_int),
        "ls2_project_bin_sort": ([cam, i32] + [P] * 8 + [i64, P, P, P, ctypes.POINTER(ctypes.c_int64), P,
                                                       ctypes.c_size_t, P], ctypes.c_int),
        "ls2_splat_sparse": ([cam, i32, i32, i32, i32, P, P, P, P, P, P, P, P, i32, P, P, P], ctypes.c_int),
        "ls2_splat_decode_workspace": ([i32, i32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ls2_splat_decode": ([cam, i32, i32, i32, i32, i32] + [P] * 13 + [ctypes.c_size_t, P], ctypes.c_int),
        "ls2_splat_decode_query_workspace": ([i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ls2_splat_decode_query": ([cam, i32, i32, i32, i32, i32] + [P] * 9 + [i32, P, ctypes.c_float] + [P] * 6
                                   + [ctypes.c_size_t, P], ctypes.c_int),
        "ls2_splat_decode_query_noalloc": ([cam, i32, i32, i32, i32, i32] + [P] * 9 + [i32, P, ctypes.c_float]
                                           + [P] * 5, ctypes.c_int),
        "ls2_dict_decode": ([i64, i32, i32, P, i32, P, i32, i32, P, P], ctypes.c_int),
        "ls2_dict_decode_query": ([i64, i32, i32, P, i32, P, P, P, i32, P, ctypes.c_float, P, P], ctypes.c_int),
        "ls2_splat_dense": ([cam, i32, i32, i32, P, P, P, P, P, P, P, P, P, P], ctypes.c_int),
        "ls2_query": ([i64, i32, P, i32, P, i32, P, ctypes.c_float, P, P], ctypes.c_int),
        "ls2_query_coef_workspace": ([i32, i32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ls2_query_coef": ([i64, i32, i32, P, P, P, i32, P, ctypes.c_float, P, P, ctypes.c_size_t, P], ctypes.c_int),
        "ls2_postprocess_workspace": ([i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ls2_postprocess": ([i32, i32, i32, P, i32, i32, i32, ctypes.c_float, P, P, P, P, P, ctypes.c_size_t, P],
                            ctypes.c_int),
        "ls2_feature_loss_workspace": ([i64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ls2_feature_loss": ([i64, i32, P, P, P, P, P, ctypes.c_size_t, P], ctypes.c_int),
        "ls2_query_backward": ([i64, i32, P, i32, P, i32, P, ctypes.c_float, P, P, P], ctypes.c_int),
        "ls2_decode_feature_loss_workspace": ([i64, i32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ls2_decode_feature_loss": ([i64, i32, i32, P, P, P, P, P, P, P, ctypes.c_size_t, P], ctypes.c_int),
        "ls2_decode_loss_backward_workspace": ([i64, i32, i32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ls2_decode_loss_backward": ([i64, i32, i32, P, P, P, P, P, P, P, ctypes.c_size_t, P], ctypes.c_int),
        "ls2_dict_decode_backward_workspace": ([i64, i32, i32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ls2_dict_decode_backward": ([i64, i32, i32, P, P, i32, P, P, P, P, ctypes.c_size_t, P], ctypes.c_int),
        "ls2_splat_sparse_backward": ([cam, i32, i32, i32, i32] + [P] * 15, ctypes.c_int),
        "ls2_project_backward": ([cam, i32] + [P] * 9 + [P], ctypes.c_int),
        "ls2_sparse_codes": ([i64, i32, i32, P, P, P, P], ctypes.c_int),
        "ls2_accumulate": ([i64, P, P, P], ctypes.c_int),
        "ls2_sparse_codes_backward": ([i64, i32, i32, P, P, P, P, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


def _check_fresh():
    """A library built from other sources than the ones beside it (a
    forgotten rebuild) is refused."""
    from ._srchash import source_hash
    want = source_hash()
    got = _lib.ls2_source_hash().decode()
    if want is not None and got != want:
        raise ImportError("libls2.so was built from other sources (fingerprint %s) than csrc/ holds (%s): rebuild it "
                          "with `python paper_2507_07136_amd/build.py` or __graft_entry__.build()" % (got, want))


_check_fresh()


def lib():
    return _lib


def status_string(status: int) -> str:
    return _lib.ls2_status_string(int(status)).decode()


def version() -> int:
    return int(_lib.ls2_version())


def set_check(enabled: bool) -> bool:
    """Code-index check on or off for the process (LS2_CHECK); returns the
    previous setting."""
    return bool(_lib.ls2_set_check(int(bool(enabled))))


def _check(fn, status):
    if status != LS2_OK:
        raise LS2Error(fn, status)


def make_camera(cam) -> ls2_camera:
    """ctypes camera from an object with width, height, fx, fy, cx, cy,
    world_to_cam (3x4) and znear (e.g. ``gen.Camera``)."""
    c = ls2_camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    w2c = [float(x) for x in torch.as_tensor(cam.world_to_cam, dtype=torch.float64).reshape(-1).tolist()]
    for i in range(12):
        c.world_to_cam[i] = w2c[i]
    c.znear = float(getattr(cam, "znear", 0.2))
    return c


def _ptr(t, dtype=None, name="tensor", numel=None, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError("%s is required" % name)
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor (the library has no CPU path)" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() < numel:
        raise ValueError("%s has %d elements, needs %d" % (name, t.numel(), numel))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------ C ABI, one wrapper per entry point
def ls2_project(cam, means, scales, quats, mean2d, conic, depth, radius, tiles_touched=None, stream=None):
    n = means.shape[0]
    c = make_camera(cam) if not isinstance(cam, ls2_camera) else cam
    f32, i32 = torch.float32, torch.int32
    st = _lib.ls2_project(ctypes.byref(c), n, _ptr(means, f32, "means", 3 * n), _ptr(scales, f32, "scales", 3 * n),
                          _ptr(quats, f32, "quats", 4 * n), _ptr(mean2d, f32, "mean2d", 2 * n),
                          _ptr(conic, f32, "conic", 3 * n), _ptr(depth, f32, "depth", n),
                          _ptr(radius, i32, "radius", n),
                          _ptr(tiles_touched, i32, "tiles_touched", n, allow_none=True), _stream(stream))
    _check("ls2_project", st)


def ls2_bin_sort_workspace(cam, n, max_pairs) -> int:
    c = make_camera(cam) if not isinstance(cam, ls2_camera) else cam
    b = ctypes.c_size_t(0)
    _check("ls2_bin_sort_workspace", _lib.ls2_bin_sort_workspace(ctypes.byref(c), int(n), int(max_pairs),
                                                                 ctypes.byref(b)))
    return int(b.value)


def ls2_bin_sort(cam, mean2d, radius, depth, max_pairs, keys, ids, tile_ranges, workspace, sync=True, stream=None):
    """Returns P (synchronising once) if sync, else None.  Raises LS2Error
    with status LS2_ERR_CAPACITY when P > max_pairs (sync mode)."""
    n = radius.shape[0]
    c = make_camera(cam) if not isinstance(cam, ls2_camera) else cam
    P = ctypes.c_int64(-1)
    ntiles = ((c.width + TILE - 1) // TILE) * ((c.height + TILE - 1) // TILE)
    st = _lib.ls2_bin_sort(ctypes.byref(c), n, _ptr(mean2d, torch.float32, "mean2d", 2 * n),
                           _ptr(radius, torch.int32, "radius", n), _ptr(depth, torch.float32, "depth", n),
                           int(max_pairs), _ptr(keys, torch.int64, "keys", int(max_pairs), allow_none=True),
                           _ptr(ids, torch.int32, "ids", int(max_pairs)),
                           _ptr(tile_ranges, torch.int32, "tile_ranges", 2 * ntiles),
                           ctypes.byref(P) if sync else None, _ptr(workspace, torch.uint8, "workspace"),
                           workspace.numel(), _stream(stream))
    if st == LS2_ERR_CAPACITY:
        err = LS2Error("ls2_bin_sort", st)
        err.num_pairs = int(P.value)
        raise err
    _check("ls2_bin_sort", st)
    return int(P.value) if sync else None


def ls2_project_bin_sort(cam, means, scales, quats, mean2d, conic, depth, radius, max_pairs, keys, ids, tile_ranges,
                         workspace, tiles_touched=None, sync=True, stream=None):
    """ls2_project then ls2_bin_sort in one call (one launch fewer); returns
    P if sync, else None, as ls2_bin_sort."""
    n = means.shape[0]
    c = make_camera(cam) if not isinstance(cam, ls2_camera) else cam
    f32, i32 = torch.float32, torch.int32
    P = ctypes.c_int64(-1)
    ntiles = ((c.width + TILE - 1) // TILE) * ((c.height + TILE - 1) // TILE)
    st = _lib.ls2_project_bin_sort(
        ctypes.byref(c), n, _ptr(means, f32, "means", 3 * n), _ptr(scales, f32, "scales", 3 * n),
        _ptr(quats, f32, "quats", 4 * n), _ptr(mean2d, f32, "mean2d", 2 * n), _ptr(conic, f32, "conic", 3 * n),
        _ptr(depth, f32, "depth", n), _ptr(radius, i32, "radius", n),
        _ptr(tiles_touched, i32, "tiles_touched", n, allow_none=True), int(max_pairs),
        _ptr(keys, torch.int64, "keys", int(max_pairs), allow_none=True), _ptr(ids, i32, "ids", int(max_pairs)),
        _ptr(tile_ranges, i32, "tile_ranges", 2 * ntiles), ctypes.byref(P) if sync else None,
        _ptr(workspace, torch.uint8, "workspace"), workspace.numel(), _stream(stream))
    if st == LS2_ERR_CAPACITY:
        err = LS2Error("ls2_project_bin_sort", st)
        err.num_pairs = int(P.value)
        raise err
    _check("ls2_project_bin_sort", st)
    return int(P.value) if sync else None


def ls2_bin_sort_count(workspace, stream=None) -> int:
    P = ctypes.c_int64(-1)
    _check("ls2_bin_sort_count", _lib.ls2_bin_sort_count(_ptr(workspace, torch.uint8, "workspace"),
                                                         ctypes.byref(P), _stream(stream)))
    return int(P.value)


def ls2_splat_sparse(cam, levels, K, L, tile_ranges, ids, mean2d, conic, opacity, topk_idx, topk_w, coef,
                     final_T=None, last=None, stream=None):
    n = opacity.shape[0]
    c = make_camera(cam) if not isinstance(cam, ls2_camera) else cam
    HW = c.width * c.height
    f32, i32 = torch.float32, torch.int32
    st = _lib.ls2_splat_sparse(ctypes.byref(c), n, int(levels), int(K), int(L), _ptr(tile_ranges, i32, "tile_ranges"),
                               _ptr(ids, i32, "ids"), _ptr(mean2d, f32, "mean2d", 2 * n),
                               _ptr(conic, f32, "conic", 3 * n), _ptr(opacity, f32, "opacity", n),
                               _ptr(topk_idx, i32, "topk_idx", n * levels * K),
                               _ptr(topk_w, f32, "topk_w", n * levels * K),
                               _ptr(coef, None, "coef", levels * HW * L), _dtype_code(coef),
                               _ptr(final_T, f32, "final_T", HW, allow_none=True),
                               _ptr(last, i32, "last", HW, allow_none=True), _stream(stream))
    _check("ls2_splat_sparse", st)


def ls2_splat_decode_workspace(L, D) -> int:
    b = ctypes.c_size_t(0)
    _check("ls2_splat_decode_workspace", _lib.ls2_splat_decode_workspace(int(L), int(D), ctypes.byref(b)))
    return int(b.value)


def ls2_splat_decode(cam, levels, K, L, tile_ranges, ids, mean2d, conic, opacity, topk_idx, topk_w, dictionary, feat,
                     workspace, coef=None, final_T=None, last=None, stream=None):
    n = opacity.shape[0]
    c = make_camera(cam) if not isinstance(cam, ls2_camera) else cam
    HW = c.width * c.height
    D = dictionary.shape[1]
    f32, i32, b16 = torch.float32, torch.int32, torch.bfloat16
    st = _lib.ls2_splat_decode(ctypes.byref(c), n, int(levels), int(K), int(L), int(D),
                               _ptr(tile_ranges, i32, "tile_ranges"), _ptr(ids, i32, "ids"),
                               _ptr(mean2d, f32, "mean2d", 2 * n), _ptr(conic, f32, "conic", 3 * n),
                               _ptr(opacity, f32, "opacity", n), _ptr(topk_idx, i32, "topk_idx", n * levels * K),
                               _ptr(topk_w, f32, "topk_w", n * levels * K), _ptr(dictionary, f32, "dict", L * D),
                               _ptr(feat, b16, "feat", levels * HW * D),
                               _ptr(coef, b16, "coef", levels * HW * L, allow_none=True),
                               _ptr(final_T, f32, "final_T", HW, allow_none=True),
                               _ptr(last, i32, "last", HW, allow_none=True),
                               _ptr(workspace, torch.uint8, "workspace"), workspace.numel(), _stream(stream))
    _check("ls2_splat_decode", st)


def ls2_splat_decode_query_workspace(L, D, n_neg) -> int:
    b = ctypes.c_size_t(0)
    _check("ls2_splat_decode_query_workspace",
           _lib.ls2_splat_decode_query_workspace(int(L), int(D), int(n_neg), ctypes.byref(b)))
    return int(b.value)


def ls2_splat_decode_query(cam, levels, K, L, tile_ranges, ids, mean2d, conic, opacity, topk_idx, topk_w, dictionary,
                           pos, neg, relevancy, workspace, feat=None, coef=None, final_T=None, last=None, tau=1.0,
                           stream=None):
    n = opacity.shape[0]
    c = make_camera(cam) if not isinstance(cam, ls2_camera) else cam
    HW = c.width * c.height
    D = dictionary.shape[1]
    n_neg = neg.numel() // D
    f32, i32, b16 = torch.float32, torch.int32, torch.bfloat16
    st = _lib.ls2_splat_decode_query(ctypes.byref(c), n, int(levels), int(K), int(L), int(D),
                                     _ptr(tile_ranges, i32, "tile_ranges"), _ptr(ids, i32, "ids"),
                                     _ptr(mean2d, f32, "mean2d", 2 * n), _ptr(conic, f32, "conic", 3 * n),
                                     _ptr(opacity, f32, "opacity", n),
                                     _ptr(topk_idx, i32, "topk_idx", n * levels * K),
                                     _ptr(topk_w, f32, "topk_w", n * levels * K), _ptr(dictionary, f32, "dict", L * D),
                                     _ptr(pos, f32, "pos", D), n_neg, _ptr(neg, f32, "neg", n_neg * D), float(tau),
                                     _ptr(relevancy, f32, "relevancy", levels * HW),
                                     _ptr(feat, b16, "feat", levels * HW * D, allow_none=True),
                                     _ptr(coef, b16, "coef", levels * HW * L, allow_none=True),
                                     _ptr(final_T, f32, "final_T", HW, allow_none=True),
                                     _ptr(last, i32, "last", HW, allow_none=True),
                                     _ptr(workspace, torch.uint8, "workspace"), workspace.numel(), _stream(stream))
    _check("ls2_splat_decode_query", st)


def ls2_splat_decode_query_noalloc(cam, levels, K, L, tile_ranges, ids, mean2d, conic, opacity, topk_idx, topk_w,
                                   dictionary, pos, neg, relevancy, feat=None, coef=None, final_T=None, last=None,
                                   tau=1.0, stream=None):
    """ls2_splat_decode_query with the library's own fixed scratch (no
    workspace argument, nothing allocated)."""
    n = opacity.shape[0]
    c = make_camera(cam) if not isinstance(cam, ls2_camera) else cam
    HW = c.width * c.height
    D = dictionary.shape[1]
    n_neg = neg.numel() // D
    f32, i32, b16 = torch.float32, torch.int32, torch.bfloat16
    st = _lib.ls2_splat_decode_query_noalloc(ctypes.byref(c), n, int(levels), int(K), int(L), int(D),
                                             _ptr(tile_ranges, i32, "tile_ranges"), _ptr(ids, i32, "ids"),
                                             _ptr(mean2d, f32, "mean2d", 2 * n), _ptr(conic, f32, "conic", 3 * n),
                                             _ptr(opacity, f32, "opacity", n),
                                             _ptr(topk_idx, i32, "topk_idx", n * levels * K),
                                             _ptr(topk_w, f32, "topk_w", n * levels * K),
                                             _ptr(dictionary, f32, "dict", L * D),
                                             _ptr(pos, f32, "pos", D), n_neg, _ptr(neg, f32, "neg", n_neg * D),
                                             float(tau), _ptr(relevancy, f32, "relevancy", levels * HW),
                                             _ptr(feat, b16, "feat", levels * HW * D, allow_none=True),
                                             _ptr(coef, b16, "coef", levels * HW * L, allow_none=True),
                                             _ptr(final_T, f32, "final_T", HW, allow_none=True),
                                             _ptr(last, i32, "last", HW, allow_none=True), _stream(stream))
    _check("ls2_splat_decode_query_noalloc", st)


def ls2_splat_dense(cam, levels, L, tile_ranges, ids, mean2d, conic, opacity, weights, coef, final_T=None, last=None,
                    stream=None):
    n = opacity.shape[0]
    c = make_camera(cam) if not isinstance(cam, ls2_camera) else cam
    HW = c.width * c.height
    f32, i32 = torch.float32, torch.int32
    st = _lib.ls2_splat_dense(ctypes.byref(c), n, int(levels), int(L), _ptr(tile_ranges, i32, "tile_ranges"),
                              _ptr(ids, i32, "ids"), _ptr(mean2d, f32, "mean2d", 2 * n),
                              _ptr(conic, f32, "conic", 3 * n), _ptr(opacity, f32, "opacity", n),
                              _ptr(weights, f32, "weights", n * levels * L), _ptr(coef, f32, "coef", levels * HW * L),
                              _ptr(final_T, f32, "final_T", HW, allow_none=True),
                              _ptr(last, i32, "last", HW, allow_none=True), _stream(stream))
    _check("ls2_splat_dense", st)


def _dtype_code(t):
    if t.dtype == torch.float32:
        return LS2_F32
    if t.dtype == torch.bfloat16:
        return LS2_BF16
    raise TypeError("expected float32 or bfloat16, got %s" % t.dtype)


def ls2_dict_decode(coef, dictionary, feat, compute=LS2_F32, stream=None):
    L, D = dictionary.shape
    m = coef.numel() // L
    st = _lib.ls2_dict_decode(m, L, D, _ptr(coef, None, "coef", m * L), _dtype_code(coef),
                              _ptr(dictionary, torch.float32, "dict", L * D), int(compute), _dtype_code(feat),
                              _ptr(feat, None, "feat", m * D), _stream(stream))
    _check("ls2_dict_decode", st)


def ls2_dict_decode_query(coef, dictionary, pos, neg, relevancy, feat=None, tau=1.0, stream=None):
    """bf16 decode with the relevancy formed in its epilogue; feat (bf16) optional."""
    L, D = dictionary.shape
    m = coef.numel() // L
    n_neg = neg.numel() // D
    if feat is not None and feat.dtype != torch.bfloat16:
        raise TypeError("feat must be bfloat16")
    st = _lib.ls2_dict_decode_query(m, L, D, _ptr(coef, None, "coef", m * L), _dtype_code(coef),
                                    _ptr(dictionary, torch.float32, "dict", L * D),
                                    _ptr(feat, torch.bfloat16, "feat", m * D, allow_none=True),
                                    _ptr(pos, torch.float32, "pos", D), n_neg, _ptr(neg, torch.float32, "neg", n_neg * D),
                                    float(tau), _ptr(relevancy, torch.float32, "relevancy", m), _stream(stream))
    _check("ls2_dict_decode_query", st)


def ls2_query(feat, pos, neg, relevancy, tau=1.0, stream=None):
    D = pos.shape[-1]
    m = feat.numel() // D
    n_neg = neg.numel() // D
    st = _lib.ls2_query(m, D, _ptr(feat, None, "feat", m * D), _dtype_code(feat), _ptr(pos, torch.float32, "pos", D),
                        n_neg, _ptr(neg, torch.float32, "neg", n_neg * D), float(tau),
                        _ptr(relevancy, torch.float32, "relevancy", m), _stream(stream))
    _check("ls2_query", st)


def ls2_query_coef_workspace(L, n_neg) -> int:
    b = ctypes.c_size_t(0)
    _check("ls2_query_coef_workspace", _lib.ls2_query_coef_workspace(int(L), int(n_neg), ctypes.byref(b)))
    return int(b.value)


def ls2_query_coef(coef, dictionary, pos, neg, relevancy, workspace, tau=1.0, stream=None):
    L, D = dictionary.shape
    m = coef.numel() // L
    n_neg = neg.numel() // D
    f32 = torch.float32
    st = _lib.ls2_query_coef(m, L, D, _ptr(coef, f32, "coef", m * L), _ptr(dictionary, f32, "dict", L * D),
                             _ptr(pos, f32, "pos", D), n_neg, _ptr(neg, f32, "neg", n_neg * D), float(tau),
                             _ptr(relevancy, f32, "relevancy", m), _ptr(workspace, torch.uint8, "workspace"),
                             workspace.numel(), _stream(stream))
    _check("ls2_query_coef", st)


def ls2_postprocess_workspace(levels, H, W) -> int:
    b = ctypes.c_size_t(0)
    _check("ls2_postprocess_workspace", _lib.ls2_postprocess_workspace(int(levels), int(H), int(W), ctypes.byref(b)))
    return int(b.value)


def ls2_postprocess(relevancy, kernel, smoothed, mask, result, workspace, smooth_mode=LS2_SMOOTH_AVG,
                    select_mode=LS2_SELECT_MAX, threshold=0.5, level_stats=None, stream=None):
    """relevancy [levels, H, W] f32 -> smoothed (same shape), mask [H, W] uint8,
    result [4] int32 (level, x, y, flat index), level_stats [levels, 4] (optional)."""
    levels, H, W = relevancy.shape
    n = levels * H * W
    st = _lib.ls2_postprocess(int(levels), int(H), int(W), _ptr(relevancy, torch.float32, "relevancy", n), int(kernel),
                              int(smooth_mode), int(select_mode), float(threshold),
                              _ptr(smoothed, torch.float32, "smoothed", n), _ptr(mask, torch.uint8, "mask", H * W),
                              _ptr(result, torch.int32, "result", 4),
                              _ptr(level_stats, torch.float32, "level_stats", 4 * levels, allow_none=True),
                              _ptr(workspace, torch.uint8, "workspace"), workspace.numel(), _stream(stream))
    _check("ls2_postprocess", st)


# ------------------------------------------------------------------ backward
def ls2_feature_loss_workspace(m) -> int:
    b = ctypes.c_size_t(0)
    _check("ls2_feature_loss_workspace", _lib.ls2_feature_loss_workspace(int(m), ctypes.byref(b)))
    return int(b.value)


def ls2_feature_loss(feat, target, loss, d_feat, workspace, stream=None):
    """loss: float64 device tensor with one element; d_feat may be None."""
    D = feat.shape[-1]
    m = feat.numel() // D
    f32 = torch.float32
    st = _lib.ls2_feature_loss(m, D, _ptr(feat, f32, "feat", m * D), _ptr(target, f32, "target", m * D),
                               _ptr(loss, torch.float64, "loss", 1),
                               _ptr(d_feat, f32, "d_feat", m * D, allow_none=True),
                               _ptr(workspace, torch.uint8, "workspace"), workspace.numel(), _stream(stream))
    _check("ls2_feature_loss", st)


def ls2_decode_feature_loss_workspace(m, D) -> int:
    b = ctypes.c_size_t(0)
    _check("ls2_decode_feature_loss_workspace", _lib.ls2_decode_feature_loss_workspace(int(m), int(D),
                                                                                       ctypes.byref(b)))
    return int(b.value)


def ls2_decode_feature_loss(coef, dictionary, target, loss, d_feat, workspace, feat=None, stream=None):
    L, D = dictionary.shape
    m = coef.numel() // L
    f32 = torch.float32
    st = _lib.ls2_decode_feature_loss(m, L, D, _ptr(coef, f32, "coef", m * L), _ptr(dictionary, f32, "dict", L * D),
                                      _ptr(target, f32, "target", m * D), _ptr(loss, torch.float64, "loss", 1),
                                      _ptr(d_feat, f32, "d_feat", m * D), _ptr(feat, f32, "feat", m * D, allow_none=True),
                                      _ptr(workspace, torch.uint8, "workspace"), workspace.numel(), _stream(stream))
    _check("ls2_decode_feature_loss", st)


def ls2_decode_loss_backward_workspace(m, L, D) -> int:
    b = ctypes.c_size_t(0)
    _check("ls2_decode_loss_backward_workspace",
           _lib.ls2_decode_loss_backward_workspace(int(m), int(L), int(D), ctypes.byref(b)))
    return int(b.value)


def ls2_decode_loss_backward(coef, dictionary, target, loss, d_coef, d_dict, workspace, stream=None):
    L, D = dictionary.shape
    m = coef.numel() // L
    f32 = torch.float32
    st = _lib.ls2_decode_loss_backward(m, L, D, _ptr(coef, f32, "coef", m * L), _ptr(dictionary, f32, "dict", L * D),
                                       _ptr(target, f32, "target", m * D), _ptr(loss, torch.float64, "loss", 1),
                                       _ptr(d_coef, f32, "d_coef", m * L), _ptr(d_dict, f32, "d_dict", L * D),
                                       _ptr(workspace, torch.uint8, "workspace"), workspace.numel(), _stream(stream))
    _check("ls2_decode_loss_backward", st)


def ls2_query_backward(feat, pos, neg, d_rel, d_feat, tau=1.0, stream=None):
    D = pos.shape[-1]
    m = feat.numel() // D
    n_neg = neg.numel() // D
    st = _lib.ls2_query_backward(m, D, _ptr(feat, None, "feat", m * D), _dtype_code(feat),
                                 _ptr(pos, torch.float32, "pos", D), n_neg,
                                 _ptr(neg, torch.float32, "neg", n_neg * D), float(tau),
                                 _ptr(d_rel, torch.float32, "d_rel", m), _ptr(d_feat, torch.float32, "d_feat", m * D),
                                 _stream(stream))
    _check("ls2_query_backward", st)


def ls2_dict_decode_backward_workspace(m, L, D) -> int:
    b = ctypes.c_size_t(0)
    _check("ls2_dict_decode_backward_workspace",
           _lib.ls2_dict_decode_backward_workspace(int(m), int(L), int(D), ctypes.byref(b)))
    return int(b.value)


def ls2_dict_decode_backward(coef, dictionary, d_feat, d_coef, d_dict, workspace=None, compute=LS2_F32,
                             stream=None):
    L, D = dictionary.shape
    m = d_feat.numel() // D
    f32 = torch.float32
    st = _lib.ls2_dict_decode_backward(
        m, L, D, _ptr(coef, f32, "coef", m * L, allow_none=True), _ptr(dictionary, f32, "dict", L * D),
        int(compute), _ptr(d_feat, f32, "d_feat", m * D), _ptr(d_coef, f32, "d_coef", m * L, allow_none=True),
        _ptr(d_dict, f32, "d_dict", L * D, allow_none=True),
        _ptr(workspace, torch.uint8, "workspace", allow_none=True),
        0 if workspace is None else workspace.numel(), _stream(stream))
    _check("ls2_dict_decode_backward", st)


def ls2_splat_sparse_backward(cam, levels, K, L, tile_ranges, ids, mean2d, conic, opacity, topk_idx, topk_w,
                              final_T, last, d_coef, d_mean2d, d_conic, d_opacity, d_topk_w, stream=None):
    n = opacity.shape[0]
    c = make_camera(cam) if not isinstance(cam, ls2_camera) else cam
    HW = c.width * c.height
    f32, i32 = torch.float32, torch.int32
    st = _lib.ls2_splat_sparse_backward(
        ctypes.byref(c), n, int(levels), int(K), int(L), _ptr(tile_ranges, i32, "tile_ranges"),
        _ptr(ids, i32, "ids"), _ptr(mean2d, f32, "mean2d", 2 * n), _ptr(conic, f32, "conic", 3 * n),
        _ptr(opacity, f32, "opacity", n), _ptr(topk_idx, i32, "topk_idx", n * levels * K),
        _ptr(topk_w, f32, "topk_w", n * levels * K), _ptr(final_T, f32, "final_T", HW),
        _ptr(last, i32, "last", HW), _ptr(d_coef, f32, "d_coef", levels * HW * L),
        _ptr(d_mean2d, f32, "d_mean2d", 2 * n), _ptr(d_conic, f32, "d_conic", 3 * n),
        _ptr(d_opacity, f32, "d_opacity", n), _ptr(d_topk_w, f32, "d_topk_w", n * levels * K), _stream(stream))
    _check("ls2_splat_sparse_backward", st)


def ls2_project_backward(cam, means, scales, quats, radius, d_mean2d, d_conic, d_means, d_scales, d_quats,
                         stream=None):
    n = means.shape[0]
    c = make_camera(cam) if not isinstance(cam, ls2_camera) else cam
    f32 = torch.float32
    st = _lib.ls2_project_backward(
        ctypes.byref(c), n, _ptr(means, f32, "means", 3 * n), _ptr(scales, f32, "scales", 3 * n),
        _ptr(quats, f32, "quats", 4 * n), _ptr(radius, torch.int32, "radius", n),
        _ptr(d_mean2d, f32, "d_mean2d", 2 * n), _ptr(d_conic, f32, "d_conic", 3 * n),
        _ptr(d_means, f32, "d_means", 3 * n), _ptr(d_scales, f32, "d_scales", 3 * n),
        _ptr(d_quats, f32, "d_quats", 4 * n), _stream(stream))
    _check("ls2_project_backward", st)


def ls2_sparse_codes(logits, K, topk_idx, topk_w, stream=None):
    """logits [..., L] -> topk_idx [..., K] int32, topk_w [..., K] f32."""
    L = logits.shape[-1]
    rows = logits.numel() // L
    st = _lib.ls2_sparse_codes(rows, L, int(K), _ptr(logits, torch.float32, "logits", rows * L),
                               _ptr(topk_idx, torch.int32, "topk_idx", rows * K),
                               _ptr(topk_w, torch.float32, "topk_w", rows * K), _stream(stream))
    _check("ls2_sparse_codes", st)


def ls2_sparse_codes_backward(topk_idx, topk_w, d_topk_w, d_logits, stream=None):
    L = d_logits.shape[-1]
    rows = d_logits.numel() // L
    K = topk_idx.shape[-1]
    st = _lib.ls2_sparse_codes_backward(rows, L, int(K), _ptr(topk_idx, torch.int32, "topk_idx", rows * K),
                                        _ptr(topk_w, torch.float32, "topk_w", rows * K),
                                        _ptr(d_topk_w, torch.float32, "d_topk_w", rows * K),
                                        _ptr(d_logits, torch.float32, "d_logits", rows * L), _stream(stream))
    _check("ls2_sparse_codes_backward", st)


def ls2_accumulate(src, dst, stream=None):
    """dst += src (float32, same number of elements)."""
    n = src.numel()
    _check("ls2_accumulate", _lib.ls2_accumulate(n, _ptr(src, torch.float32, "src", n),
                                                 _ptr(dst, torch.float32, "dst", n), _stream(stream)))
