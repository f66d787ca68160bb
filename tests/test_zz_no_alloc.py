"""ls2_splat_decode_query_noalloc (the query frame with the library's fixed
scratch instead of a caller workspace) against ls2_splat_decode_query, the
entry point it is a variant of: both run the same kernels, so every output
must be bit-identical.  Two no-allocation calls run back to back, the second
on a smaller frame with smaller L, D and text count, before either is
compared, so what the first call leaves in the shared scratch must not leak
into the second."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import gen
from gpu_common import gpu_available, small_scene

pytestmark = pytest.mark.gpu


def _lists(cam, scene):
    import paper_2507_07136_amd as ls2
    t = ls2.to_device(scene)
    pipe = ls2.Pipeline(cam, scene.n, levels=scene.levels, K=scene.K, L=scene.L, D=scene.D)
    pipe.project(t["means"], t["scales"], t["quats"])
    pipe.bin_sort(sync=True)
    return pipe, t


def _frame(fn, cam, scene, pipe, t, tp, tn, keep_feat, keep_coef, tau, **kw):
    lv, H, W = scene.levels, cam.height, cam.width
    out = dict(rel=torch.full((lv, H, W), -5.0, device="cuda"),
               feat=torch.full((lv, H, W, scene.D), 7.0, dtype=torch.bfloat16, device="cuda") if keep_feat else None,
               coef=torch.full((lv, H, W, scene.L), 9.0, dtype=torch.bfloat16, device="cuda") if keep_coef else None,
               final_T=torch.full((H, W), -1.0, device="cuda"),
               last=torch.full((H, W), -3, dtype=torch.int32, device="cuda"))
    fn(cam, lv, scene.K, scene.L, pipe.tile_ranges, pipe.ids, pipe.mean2d, pipe.conic, t["opacity"], t["topk_idx"],
       t["topk_w"], t["dictionary"], tp, tn, out["rel"], feat=out["feat"], coef=out["coef"], final_T=out["final_T"],
       last=out["last"], tau=tau, **kw)
    return out


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_noalloc_query_frame_matches_workspace_form():
    import paper_2507_07136_amd as ls2
    cases = [
        # (seed, n, w, h, L, K, levels, D, n_neg, keep_feat, keep_coef, tau)
        (5101, 3000, 120, 90, 64, 4, 1, 512, 4, True, True, 1.0),
        (5102, 500, 40, 24, 32, 8, 2, 256, 1, False, True, 10.0),   # smaller in every size
    ]
    runs = []
    for seed, n, w, h, L, K, levels, D, n_neg, kf, kc, tau in cases:
        scene, cam = small_scene(seed, n, w, h, L=L, K=K, levels=levels, D=D)
        pipe, t = _lists(cam, scene)
        pos, neg = gen.make_text(seed, D=D, n_neg=n_neg)
        tp, tn = torch.from_numpy(pos).cuda(), torch.from_numpy(neg).cuda()
        got = _frame(ls2.ls2_splat_decode_query_noalloc, cam, scene, pipe, t, tp, tn, kf, kc, tau)
        runs.append((scene, cam, pipe, t, tp, tn, kf, kc, tau, got))
    torch.cuda.synchronize()
    for scene, cam, pipe, t, tp, tn, kf, kc, tau, got in runs:
        n_neg = tn.numel() // scene.D
        ws = torch.empty((ls2.ls2_splat_decode_query_workspace(scene.L, scene.D, n_neg),), dtype=torch.uint8,
                         device="cuda")
        ref = _frame(ls2.ls2_splat_decode_query, cam, scene, pipe, t, tp, tn, kf, kc, tau, workspace=ws)
        torch.cuda.synchronize()
        assert bool((ref["rel"] >= 0).all())  # every pixel written
        for k in ("rel", "final_T", "last", "feat", "coef"):
            if ref[k] is None:
                assert got[k] is None
                continue
            assert torch.equal(got[k], ref[k]), k


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_noalloc_rejects_shapes_beyond_its_scratch():
    import paper_2507_07136_amd as ls2
    scene, cam = small_scene(5103, 200, 32, 32, L=128, K=4, levels=1, D=1024)
    pipe, t = _lists(cam, scene)
    pos, neg = gen.make_text(5103, D=1024, n_neg=8)
    tp, tn = torch.from_numpy(pos).cuda(), torch.from_numpy(neg).cuda()
    with pytest.raises(ls2.LS2Error) as e:
        _frame(ls2.ls2_splat_decode_query_noalloc, cam, scene, pipe, t, tp, tn, False, False, 1.0)
    assert e.value.status == ls2.LS2_ERR_CAPACITY
    # the largest shape that fits still runs and matches the workspace form
    scene, cam = small_scene(5104, 400, 48, 40, L=128, K=4, levels=1, D=512)
    pipe, t = _lists(cam, scene)
    pos, neg = gen.make_text(5104, D=512, n_neg=8)
    tp, tn = torch.from_numpy(pos).cuda(), torch.from_numpy(neg).cuda()
    got = _frame(ls2.ls2_splat_decode_query_noalloc, cam, scene, pipe, t, tp, tn, True, False, 1.0)
    ws = torch.empty((ls2.ls2_splat_decode_query_workspace(128, 512, 8),), dtype=torch.uint8, device="cuda")
    ref = _frame(ls2.ls2_splat_decode_query, cam, scene, pipe, t, tp, tn, True, False, 1.0, workspace=ws)
    torch.cuda.synchronize()
    for k in ("rel", "final_T", "last", "feat"):
        assert torch.equal(got[k], ref[k]), k
    assert np.isfinite(got["rel"].cpu().numpy()).all()
