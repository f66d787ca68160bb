"""Shared helpers for the GPU parity tests (the HIP path through the C ABI on
one side, the FP64 oracle on the other, on the same seeded inputs)."""
from __future__ import annotations

import numpy as np
import torch

import gen

F32_099 = float(np.float32(0.99))


def gpu_available() -> bool:
    return torch.cuda.is_available()


def run_forward(cam, scene, compute=None, out_dtype=torch.float32, keep_keys=True, sync=True, max_pairs=None):
    """Run project -> bin_sort -> splat -> decode on the GPU; return numpy copies."""
    import paper_2507_07136_amd as ls2
    compute = ls2.LS2_F32 if compute is None else compute
    t = ls2.to_device(scene)
    pipe = ls2.Pipeline(cam, scene.n, levels=scene.levels, K=scene.K, L=scene.L, D=scene.D, keep_keys=keep_keys,
                        max_pairs=max_pairs)
    pipe.project(t["means"], t["scales"], t["quats"])
    P = pipe.bin_sort(sync=sync)
    pipe.splat(t["opacity"], t["topk_idx"], t["topk_w"])
    feat = pipe.decode(t["dictionary"], compute, out_dtype)
    torch.cuda.synchronize()
    P = pipe.num_pairs if P is None else P
    out = dict(pipe=pipe, t=t, P=P,
               mean2d=pipe.mean2d.cpu().numpy(), conic=pipe.conic.cpu().numpy(), depth=pipe.depth.cpu().numpy(),
               radius=pipe.radius.cpu().numpy(), touched=pipe.tiles_touched.cpu().numpy(),
               ranges=pipe.tile_ranges.cpu().numpy().view(np.uint32),
               ids=pipe.ids[:P].cpu().numpy().view(np.uint32) if P else np.zeros(0, np.uint32),
               keys=pipe.keys[:P].cpu().numpy().view(np.uint64) if (keep_keys and P) else None,
               coef=pipe.coef.cpu().numpy(), final_T=pipe.final_T.cpu().numpy(), last=pipe.last.cpu().numpy(),
               feat=feat.float().cpu().numpy())
    return out


def oracle_lists_from_gpu(orc, cam, g):
    """Stage-isolated binning: the oracle sorts the GPU's own float32 projection."""
    return orc.tile_lists(cam, g["mean2d"], g["radius"], g["depth"])


def oracle_composite_from_gpu(orc, cam, scene, g):
    """Stage-isolated splat: the oracle composites the GPU's lists and float32
    projected Gaussians in float64."""
    return orc.composite(cam, g["ranges"], g["ids"], g["mean2d"].astype(np.float64),
                         g["conic"].astype(np.float64), scene.opacity, scene.topk_idx, scene.topk_w, scene.L,
                         with_margin_T=True)


def by_pixel(a):
    """[levels, H, W, C] -> [H W, levels, C] (pixel-major, as the flip check
    takes outcomes)."""
    lv, H, W, C = a.shape
    return np.ascontiguousarray(a.transpose(1, 2, 0, 3)).reshape(H * W, lv, C)


def flip_check_gpu_lists(orc, cam, scene, g, close, pix=None, base=None, label=""):
    """check_flips on the GPU's own lists and float32 projection (stage
    isolation); pix defaults to every pixel."""
    from alt_check import check_flips
    if pix is None:
        pix = np.arange(cam.width * cam.height)
    return check_flips(orc, cam, g["ranges"], g["ids"], g["mean2d"].astype(np.float64),
                       g["conic"].astype(np.float64), scene.opacity, scene.topk_idx, scene.topk_w, scene.L, pix,
                       close, base=base, label=label)


def small_scene(seed, n, w, h, L=64, K=4, levels=1, D=512):
    scene = gen.make_scene(seed, n, L=L, K=K, D=D, levels=levels)
    cam = gen.make_camera(w, h)
    return scene, cam


def grad_close(got, ref, name, rtol=1e-3, floor=1e-3):
    """Per tensor |got - ref|_2 <= rtol |ref|_2 and per element
    |got - ref| <= rtol max(|ref|, floor max|ref|)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    assert got.shape == ref.shape, (name, got.shape, ref.shape)
    nref = np.linalg.norm(ref)
    err = np.linalg.norm(got - ref)
    assert err <= rtol * max(nref, 1e-30), "%s: |d|/|g| = %.3e" % (name, err / max(nref, 1e-30))
    gmax = np.abs(ref).max() if ref.size else 0.0
    bound = rtol * np.maximum(np.abs(ref), floor * gmax)
    bad = np.abs(got - ref) > bound + 1e-30
    assert not bad.any(), "%s: %d elements out of bound, worst %.3e vs %.3e" % (
        name, int(bad.sum()), float(np.abs(got - ref)[bad].max()), float(bound[bad].max()))
