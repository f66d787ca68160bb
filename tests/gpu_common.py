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


def superblock_list_ranges(ranges, tiles_x, tiles_y):
    """The library's placement of the tile lists (include/ls2.h, ls2_bin_sort):
    superblocks of S x S tiles (S = 4, doubled while there are more than 4096
    superblocks) in row-major order, tiles row-major inside each.  Given the
    per-tile list lengths of `ranges` (any placement), returns the [start, end)
    ranges of that layout."""
    ranges = np.asarray(ranges, np.int64)
    lens = ranges[:, 1] - ranges[:, 0]
    S = 4
    while ((tiles_x + S - 1) // S) * ((tiles_y + S - 1) // S) > 4096:
        S *= 2
    t = np.arange(tiles_x * tiles_y)
    x, y = t % tiles_x, t // tiles_x
    sb = (y // S) * ((tiles_x + S - 1) // S) + x // S
    order = np.lexsort(((y % S) * S + x % S, sb))
    start = np.empty_like(lens)
    start[order] = np.concatenate([[0], np.cumsum(lens[order])[:-1]])
    return np.stack([start, start + lens], axis=1)


def compare_tile_lists(g, keys, ids, ranges, tiles_x, tiles_y):
    """The GPU lists g (P, ranges, ids, optional keys) against the oracle's
    (keys, ids, ranges in row-major tile order): the same pair count, the
    documented placement of every tile's list, and every list bit for bit.
    Returns None if equal, else what differs."""
    if g["P"] != len(ids):
        return "P %d, oracle %d" % (g["P"], len(ids))
    exp = superblock_list_ranges(ranges, tiles_x, tiles_y)
    if not np.array_equal(np.asarray(g["ranges"], np.int64), exp):
        return "tile ranges differ at %d tiles" % int((np.asarray(g["ranges"], np.int64) != exp).any(axis=1).sum())
    ranges = np.asarray(ranges, np.int64)
    lens = ranges[:, 1] - ranges[:, 0]
    # oracle position p of tile t sits at exp[t, 0] + (p - ranges[t, 0]) in the GPU lists
    gpos = np.arange(len(ids), dtype=np.int64) + np.repeat(exp[:, 0] - ranges[:, 0], lens)
    if not np.array_equal(g["ids"][gpos], ids):
        return "ids differ at %d positions" % int((g["ids"][gpos] != ids).sum())
    if g.get("keys") is not None and not np.array_equal(g["keys"][gpos], keys):
        return "keys differ at %d positions" % int((g["keys"][gpos] != keys).sum())
    return None


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
