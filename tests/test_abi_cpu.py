"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/ls2.h declares, and rejects invalid arguments before touching
the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ls2.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ls2_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2507_07136_amd import _lib
    return _lib.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["ls2_project", "ls2_bin_sort", "ls2_splat_sparse", "ls2_dict_decode", "ls2_query",
              "ls2_feature_loss", "ls2_query_backward", "ls2_dict_decode_backward", "ls2_splat_sparse_backward",
              "ls2_project_backward"]:
        assert n in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings(L):
    from paper_2507_07136_amd import _lib
    assert _lib.status_string(0) == "ok"
    assert "capacity" in _lib.status_string(-2)
    assert _lib.version() >= 100


def _cam(w=128, h=128):
    import gen
    from paper_2507_07136_amd import _lib
    return _lib.make_camera(gen.make_camera(w, h))


def test_argument_validation_without_device(L):
    c = _cam()
    V = ctypes.c_void_p
    # negative n, bad camera
    assert L.ls2_project(ctypes.byref(c), -1, None, None, None, None, None, None, None, None, None) == -1
    bad = _cam()
    bad.width = 0
    assert L.ls2_project(ctypes.byref(bad), 1, V(16), V(16), V(16), V(16), V(16), V(16), V(16), None, None) == -1
    # n = 0 is a no-op
    assert L.ls2_project(ctypes.byref(c), 0, None, None, None, None, None, None, None, None, None) == 0
    # splat: K > L, unsupported L, too many levels, null outputs, bad or
    # misaligned coefficient map
    args = [V(16)] * 8 + [0] + [V(16)] * 3
    assert L.ls2_splat_sparse(ctypes.byref(c), 10, 1, 9, 8, *args) == -1
    assert L.ls2_splat_sparse(ctypes.byref(c), 10, 1, 4, 48, *args) == -3
    assert L.ls2_splat_sparse(ctypes.byref(c), 10, 1, 9, 64, *args) == -3
    assert L.ls2_splat_sparse(ctypes.byref(c), 10, 4, 4, 64, *args) == -3
    assert L.ls2_splat_sparse(ctypes.byref(c), 10, 3, 4, 128, *args) == -3
    assert L.ls2_splat_sparse(ctypes.byref(c), 10, 1, 4, 64, None, *args[1:]) == -1
    assert L.ls2_splat_sparse(ctypes.byref(c), 10, 1, 4, 64, *args[:8], 5, *args[9:]) == -1
    assert L.ls2_splat_sparse(ctypes.byref(c), 10, 1, 4, 64, *args[:7], V(24), 1, *args[9:]) == -1
    # decode: bad dtype codes, unsupported D / L, bf16 map with f32 compute, misaligned map
    assert L.ls2_dict_decode(10, 64, 512, V(16), 0, V(16), 7, 0, V(16), None) == -1
    assert L.ls2_dict_decode(10, 64, 512, V(16), 3, V(16), 0, 0, V(16), None) == -1
    assert L.ls2_dict_decode(10, 64, 500, V(16), 0, V(16), 0, 0, V(16), None) == -3
    assert L.ls2_dict_decode(10, 48, 512, V(16), 0, V(16), 0, 0, V(16), None) == -3
    assert L.ls2_dict_decode(10, 64, 512, V(16), 1, V(16), 0, 0, V(16), None) == -3
    assert L.ls2_dict_decode(10, 64, 512, V(24), 0, V(16), 1, 0, V(16), None) == -1
    assert L.ls2_dict_decode(-1, 64, 512, V(16), 0, V(16), 0, 0, V(16), None) == -1
    assert L.ls2_dict_decode(0, 64, 512, V(16), 0, V(16), 0, 0, V(16), None) == 0
    # query: bad n_neg, unsupported D
    assert L.ls2_query(10, 512, V(16), 0, V(16), 0, V(16), ctypes.c_float(1.0), V(16), None) == -1
    assert L.ls2_query(10, 500, V(16), 0, V(16), 4, V(16), ctypes.c_float(1.0), V(16), None) == -3
    assert L.ls2_query(10, 512, V(16), 0, V(16), 9, V(16), ctypes.c_float(1.0), V(16), None) == -3


def test_camera_validation_without_device(L):
    """A near plane that is not finite and positive, or non-finite
    intrinsics, is rejected before any launch (sort keys are the bits of a
    positive depth)."""
    V = ctypes.c_void_p
    args = [V(16)] * 7 + [None]
    for field, value in (("znear", 0.0), ("znear", -0.2), ("znear", float("nan")), ("znear", float("inf")),
                         ("fx", float("inf")), ("cy", float("nan"))):
        c = _cam()
        setattr(c, field, value)
        assert L.ls2_project(ctypes.byref(c), 1, *args, None) == -1, (field, value)
    c = _cam()
    c.world_to_cam[3] = float("nan")
    assert L.ls2_project(ctypes.byref(c), 1, *args, None) == -1
    c = _cam()
    c.znear = 1e-3
    assert L.ls2_project(ctypes.byref(c), 0, *args, None) == 0


def test_set_check_toggles(L):
    prev = L.ls2_set_check(1)
    assert L.ls2_set_check(0) == 1
    assert L.ls2_set_check(prev) == 0


def test_bin_sort_workspace_and_validation(L):
    c = _cam()
    b = ctypes.c_size_t(0)
    assert L.ls2_bin_sort_workspace(ctypes.byref(c), 100, 1000, ctypes.byref(b)) == 0
    assert b.value >= 1000 * 8
    assert L.ls2_bin_sort_workspace(ctypes.byref(c), 100, -1, ctypes.byref(b)) == -1
    assert L.ls2_bin_sort_workspace(ctypes.byref(c), 100, 1 << 33, ctypes.byref(b)) == -3
    P = ctypes.c_int64(0)
    V = ctypes.c_void_p
    # misaligned workspace, too small workspace
    assert L.ls2_bin_sort(ctypes.byref(c), 10, V(256), V(256), V(256), 1000, None, V(256), V(256), ctypes.byref(P),
                          V(257), b.value, None) == -1
    assert L.ls2_bin_sort(ctypes.byref(c), 10, V(256), V(256), V(256), 1000, None, V(256), V(256), ctypes.byref(P),
                          V(256), 16, None) == -1
    # the projecting form: missing projection inputs, then the same workspace checks
    pb = [V(256)] * 8
    assert L.ls2_project_bin_sort(ctypes.byref(c), 10, None, *pb[1:], 1000, None, V(256), V(256), ctypes.byref(P),
                                  V(256), b.value, None) == -1
    assert L.ls2_project_bin_sort(ctypes.byref(c), 10, *pb[:6], None, V(256), 1000, None, V(256), V(256),
                                  ctypes.byref(P), V(256), b.value, None) == -1
    assert L.ls2_project_bin_sort(ctypes.byref(c), 10, *pb, 1000, None, V(256), V(256), ctypes.byref(P),
                                  V(257), b.value, None) == -1
    assert L.ls2_project_bin_sort(ctypes.byref(c), 10, *pb, 1000, None, V(256), V(256), ctypes.byref(P),
                                  V(256), 16, None) == -1
    assert L.ls2_project_bin_sort(None, 10, *pb, 1000, None, V(256), V(256), ctypes.byref(P), V(256), b.value,
                                  None) == -1


def test_backward_argument_validation_without_device(L):
    c = _cam()
    V = ctypes.c_void_p
    f1 = ctypes.c_float(1.0)
    # splat backward: null tile_ranges, K > L, unsupported L / levels
    args = [V(16)] * 15
    assert L.ls2_splat_sparse_backward(ctypes.byref(c), 10, 1, 4, 64, None, *args[1:]) == -1
    assert L.ls2_splat_sparse_backward(ctypes.byref(c), 10, 1, 9, 8, *args) == -1
    assert L.ls2_splat_sparse_backward(ctypes.byref(c), 10, 1, 4, 48, *args) == -3
    assert L.ls2_splat_sparse_backward(ctypes.byref(c), 10, 4, 4, 64, *args) == -3
    assert L.ls2_splat_sparse_backward(ctypes.byref(c), 10, 1, 4, 64, *args[:7], None, *args[8:]) == -1  # final_T
    # project backward: negative n, null output, n = 0 no-op
    assert L.ls2_project_backward(ctypes.byref(c), -1, *([V(16)] * 9), None) == -1
    assert L.ls2_project_backward(ctypes.byref(c), 5, *([V(16)] * 8), None, None) == -1
    assert L.ls2_project_backward(ctypes.byref(c), 0, *([None] * 9), None) == 0
    # decode backward: workspace query, bad compute, unsupported L, no output, BF16 not built, small workspace
    b = ctypes.c_size_t(0)
    assert L.ls2_dict_decode_backward_workspace(1000, 64, 512, ctypes.byref(b)) == 0 and b.value >= 64 * 512 * 4
    assert L.ls2_dict_decode_backward_workspace(1000, 48, 512, ctypes.byref(b)) == -3
    assert L.ls2_dict_decode_backward_workspace(0, 64, 512, ctypes.byref(b)) == 0 and b.value == 0
    assert L.ls2_dict_decode_backward(10, 64, 512, V(16), V(16), 7, V(16), V(16), V(16), V(16), 1 << 30, None) == -1
    assert L.ls2_dict_decode_backward(10, 48, 512, V(16), V(16), 0, V(16), V(16), V(16), V(16), 1 << 30, None) == -3
    assert L.ls2_dict_decode_backward(10, 64, 512, V(16), V(16), 0, V(16), None, None, V(16), 1 << 30, None) == -1
    assert L.ls2_dict_decode_backward(10, 64, 512, V(16), V(16), 1, V(16), V(16), V(16), V(16), 1 << 30, None) == -3
    assert L.ls2_dict_decode_backward(10, 64, 512, V(16), V(16), 0, V(16), V(16), V(16), V(16), 16, None) == -1
    assert L.ls2_dict_decode_backward(-1, 64, 512, V(16), V(16), 0, V(16), V(16), V(16), V(16), 1 << 30, None) == -1
    # query backward: no negatives, tau <= 0, bad dtype, unsupported D / n_neg
    qa = [V(16), 0, V(16)]
    assert L.ls2_query_backward(10, 512, *qa, 0, V(16), f1, V(16), V(16), None) == -1
    assert L.ls2_query_backward(10, 512, *qa, 4, V(16), ctypes.c_float(0.0), V(16), V(16), None) == -1
    assert L.ls2_query_backward(10, 512, V(16), 5, V(16), 4, V(16), f1, V(16), V(16), None) == -1
    assert L.ls2_query_backward(10, 500, *qa, 4, V(16), f1, V(16), V(16), None) == -3
    assert L.ls2_query_backward(10, 512, *qa, 9, V(16), f1, V(16), V(16), None) == -3
    assert L.ls2_query_backward(0, 512, None, 0, V(16), 4, V(16), f1, None, None, None) == 0
    # fused decode + loss: unsupported L / D, null output, small workspace
    assert L.ls2_decode_feature_loss_workspace(1000, 512, ctypes.byref(b)) == 0 and b.value >= 16
    fa = [V(16)] * 5
    assert L.ls2_decode_feature_loss(10, 128, 512, *fa, None, V(16), 1 << 20, None) == -3
    assert L.ls2_decode_feature_loss(10, 64, 1024, *fa, None, V(16), 1 << 20, None) == -3
    assert L.ls2_decode_feature_loss(10, 64, 512, V(16), V(16), V(16), V(16), None, None, V(16), 1 << 20,
                                     None) == -1
    assert L.ls2_decode_feature_loss(10, 64, 512, *fa, None, V(16), 8, None) == -1
    # decode + loss + decode backward in one pass: unsupported L / D, null
    # output, empty input, misalignment, small workspace
    assert L.ls2_decode_loss_backward_workspace(1000, 64, 512, ctypes.byref(b)) == 0 and b.value >= 64 * 512 * 4
    assert L.ls2_decode_loss_backward_workspace(1000, 128, 512, ctypes.byref(b)) == -3
    assert L.ls2_decode_loss_backward_workspace(0, 64, 512, ctypes.byref(b)) == -1
    # the dS partials: one [L, D] slice per workgroup, at most one per 32 pixels
    # and at most 512, plus 512 pairs of compensated loss partials (8 bytes each)
    for m_, parts in ((1, 1), (32, 1), (33, 2), (32 * 300, 300), (32 * 512 + 1, 512), (10 ** 8, 512)):
        assert L.ls2_decode_loss_backward_workspace(m_, 64, 512, ctypes.byref(b)) == 0
        assert b.value == parts * 64 * 512 * 4 + 512 * 2 * 8, (m_, b.value)
    la = [V(16)] * 6
    assert L.ls2_decode_loss_backward(10, 128, 512, *la, V(16), 1 << 24, None) == -3
    assert L.ls2_decode_loss_backward(10, 64, 1024, *la, V(16), 1 << 24, None) == -3
    assert L.ls2_decode_loss_backward(10, 64, 64, *la, V(16), 1 << 24, None) == -3
    assert L.ls2_decode_loss_backward(10, 64, 512, *la[:5], None, V(16), 1 << 24, None) == -1
    assert L.ls2_decode_loss_backward(0, 64, 512, *la, V(16), 1 << 24, None) == -1
    assert L.ls2_decode_loss_backward(10, 64, 512, V(4), *la[1:], V(16), 1 << 24, None) == -1
    assert L.ls2_decode_loss_backward(10, 64, 512, *la, V(16), 64, None) == -1
    # feature loss: empty input, unsupported D, small workspace
    assert L.ls2_feature_loss_workspace(1000, ctypes.byref(b)) == 0 and b.value >= 16
    assert L.ls2_feature_loss(0, 512, V(16), V(16), V(16), None, V(16), 1 << 20, None) == -1
    assert L.ls2_feature_loss(10, 500, V(16), V(16), V(16), None, V(16), 1 << 20, None) == -3
    assert L.ls2_feature_loss(10, 512, V(16), V(16), V(16), None, V(16), 8, None) == -1


def test_codes_and_accumulate_validation_without_device(L):
    V = ctypes.c_void_p
    # sparse codes: K > L, K = 0, null output, unsupported K / L, rows = 0 no-op
    assert L.ls2_sparse_codes(10, 4, 8, V(16), V(16), V(16), None) == -1
    assert L.ls2_sparse_codes(10, 64, 0, V(16), V(16), V(16), None) == -1
    assert L.ls2_sparse_codes(10, 64, 4, V(16), None, V(16), None) == -1
    assert L.ls2_sparse_codes(10, 64, 9, V(16), V(16), V(16), None) == -3
    assert L.ls2_sparse_codes(10, 30, 4, V(16), V(16), V(16), None) == -3
    assert L.ls2_sparse_codes(0, 64, 4, None, None, None, None) == 0
    assert L.ls2_sparse_codes_backward(10, 64, 4, V(16), V(16), V(16), None, None) == -1
    assert L.ls2_sparse_codes_backward(-1, 64, 4, V(16), V(16), V(16), V(16), None) == -1
    assert L.ls2_sparse_codes_backward(0, 64, 4, None, None, None, None, None) == 0
    # accumulate: negative n, null or misaligned pointers, n = 0 no-op
    assert L.ls2_accumulate(-1, V(16), V(16), None) == -1
    assert L.ls2_accumulate(8, None, V(16), None) == -1
    assert L.ls2_accumulate(8, V(16), V(20), None) == -1
    assert L.ls2_accumulate(0, None, None, None) == 0


def test_decode_query_validation_without_device(L):
    V = ctypes.c_void_p
    f1 = ctypes.c_float(1.0)
    # null text, no negatives, too many negatives, D beyond one chunk, bad coef dtype, misaligned map
    assert L.ls2_dict_decode_query(10, 64, 512, V(16), 0, V(16), None, None, 4, V(16), f1, V(16), None) == -1
    assert L.ls2_dict_decode_query(10, 64, 512, V(16), 0, V(16), None, V(16), 0, V(16), f1, V(16), None) == -1
    assert L.ls2_dict_decode_query(10, 64, 512, V(16), 0, V(16), None, V(16), 9, V(16), f1, V(16), None) == -3
    assert L.ls2_dict_decode_query(10, 64, 1024, V(16), 0, V(16), None, V(16), 4, V(16), f1, V(16), None) == -3
    assert L.ls2_dict_decode_query(10, 64, 512, V(16), 2, V(16), None, V(16), 4, V(16), f1, V(16), None) == -1
    assert L.ls2_dict_decode_query(10, 64, 512, V(16), 0, V(16), V(8), V(16), 4, V(16), f1, V(16), None) == -1
    assert L.ls2_dict_decode_query(0, 64, 512, V(16), 0, V(16), None, V(16), 4, V(16), f1, V(16), None) == 0


def test_splat_decode_validation_without_device(L):
    c = _cam()
    V = ctypes.c_void_p
    b = ctypes.c_size_t(0)
    assert L.ls2_splat_decode_workspace(64, 512, ctypes.byref(b)) == 0 and b.value == 64 * 512 * 2
    assert L.ls2_splat_decode_workspace(64, 500, ctypes.byref(b)) == -3
    assert L.ls2_splat_decode_workspace(48, 512, ctypes.byref(b)) == -3
    assert L.ls2_splat_decode_workspace(64, 512, None) == -1
    ws = 64 * 512 * 2
    inp = [V(16)] * 7                     # tile_ranges .. topk_w

    def call(n=10, levels=1, K=4, Lc=64, D=512, dct=V(16), feat=V(16), coef=None, wsp=V(16), wsb=ws):
        return L.ls2_splat_decode(ctypes.byref(c), n, levels, K, Lc, D, *inp, dct, feat, coef, None, None, wsp,
                                  wsb, None)
    # every case is rejected before any launch
    assert call(D=500) == -3              # D not a multiple of 64
    assert call(D=2048, wsb=64 * 2048 * 2) == -3
    assert call(Lc=48) == -3
    assert call(levels=3, Lc=128) == -3
    assert call(K=9) == -3
    assert call(K=80) == -1               # K > L
    assert call(feat=None) == -1
    assert call(feat=V(24)) == -1         # misaligned feature map
    assert call(coef=V(24)) == -1         # misaligned optional map
    assert call(dct=None) == -1
    assert call(wsp=None) == -1
    assert call(wsp=V(24)) == -1
    assert call(wsb=ws - 1) == -1         # workspace too small
    assert call(n=-1) == -1


def test_splat_decode_query_validation_without_device(L):
    c = _cam()
    V = ctypes.c_void_p
    b = ctypes.c_size_t(0)
    assert L.ls2_splat_decode_query_workspace(64, 512, 4, ctypes.byref(b)) == 0 and b.value >= 64 * 512 * 2 + 5 * 1024
    assert L.ls2_splat_decode_query_workspace(64, 512, 9, ctypes.byref(b)) == -3
    assert L.ls2_splat_decode_query_workspace(64, 512, 0, ctypes.byref(b)) == -1
    L.ls2_splat_decode_query_workspace(64, 512, 4, ctypes.byref(b))
    ws = b.value
    inp = [V(16)] * 7
    f1 = ctypes.c_float(1.0)

    def call(n_neg=4, D=512, pos=V(16), neg=V(16), rel=V(16), feat=None, wsp=V(16), wsb=ws):
        return L.ls2_splat_decode_query(ctypes.byref(c), 10, 1, 4, 64, D, *inp, V(16), pos, n_neg, neg, f1, rel,
                                        feat, None, None, None, wsp, wsb, None)
    # every case is rejected before any launch
    assert call(n_neg=9) == -3
    assert call(n_neg=0) == -1
    assert call(pos=None) == -1
    assert call(rel=None) == -1
    assert call(feat=V(24)) == -1          # misaligned optional feature map
    assert call(wsb=ws - 1) == -1
    assert call(D=500) == -3


def test_splat_decode_query_noalloc_validation_without_device(L):
    """The no-allocation query frame rejects bad texts and shapes, and shapes
    whose repacked dictionary and texts exceed its fixed scratch, before any
    device call."""
    c = _cam()
    V = ctypes.c_void_p
    inp = [V(16)] * 7
    f1 = ctypes.c_float(1.0)

    def call(n_neg=4, Lc=64, D=512, pos=V(16), neg=V(16), rel=V(16)):
        return L.ls2_splat_decode_query_noalloc(ctypes.byref(c), 10, 1, 4, Lc, D, *inp, V(16), pos, n_neg, neg, f1,
                                                rel, None, None, None, None, None)
    assert call(n_neg=9) == -3
    assert call(n_neg=0) == -1
    assert call(pos=None) == -1
    assert call(neg=None) == -1
    assert call(rel=None) == -1
    assert call(D=500) == -3
    assert call(Lc=48) == -3
    assert call(Lc=128, D=1024, n_neg=8) == -2   # 288 KB of scratch needed, 160 KiB held


def test_library_built_from_these_sources():
    """The loaded library's source fingerprint is the one of csrc/ and
    include/ls2.h beside it (the binding refuses a stale build)."""
    import paper_2507_07136_amd._lib as lib
    from paper_2507_07136_amd._srchash import source_hash
    assert lib._lib.ls2_source_hash().decode() == source_hash()


def test_list_layout_reference():
    """The test helper that places oracle tile lists in the library's layout
    (superblocks of S x S tiles row-major, tiles row-major inside each),
    against a direct walk over superblocks and tiles."""
    import numpy as np
    from gpu_common import superblock_list_ranges
    rng = np.random.default_rng(5)
    for tx, ty, S in ((9, 7, 4), (90, 68, 4), (260, 260, 8)):
        lens = rng.integers(0, 5, tx * ty)
        lens[rng.random(tx * ty) < 0.3] = 0
        row_major = np.concatenate([[0], np.cumsum(lens)])
        ranges = np.stack([row_major[:-1], row_major[1:]], axis=1)
        want = np.zeros((tx * ty, 2), np.int64)
        pos = 0
        for sy in range(0, ty, S):
            for sx in range(0, tx, S):
                for y in range(sy, min(sy + S, ty)):
                    for x in range(sx, min(sx + S, tx)):
                        t = y * tx + x
                        want[t] = (pos, pos + lens[t])
                        pos += lens[t]
        assert np.array_equal(superblock_list_ranges(ranges, tx, ty), want)
