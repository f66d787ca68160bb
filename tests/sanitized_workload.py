"""Every C entry point of the FP64 oracle on a small scene, for the
sanitizer test (run in a child process with the ASan / UBSan build of the
oracle and the gcc sanitizer runtimes preloaded).  Prints "sanitized
workload ok" at the end."""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
from oracle import oracle as orc  # noqa: E402


def main():
    if os.environ.get("LS2_WORKLOAD_ANY_BUILD") != "1":
        assert orc._SANITIZE, "run with LS2_ORACLE_SANITIZE=1"
    scene = gen.make_scene(77, 300, L=32, K=4, D=64, levels=2)
    cam = gen.make_camera(72, 40)
    pr = orc.project(cam, scene.means, scene.scales, scene.quats)
    m32, d32 = pr["mean2d"].astype(np.float32), pr["depth"].astype(np.float32)
    keys, ids, ranges = orc.tile_lists(cam, m32, pr["radius"], d32)
    args = (cam, ranges, ids, pr["mean2d"], pr["conic"], scene.opacity, scene.topk_idx, scene.topk_w)
    coef, fT, last, margin, margin_T = orc.composite(*args, scene.L, with_margin_T=True)
    pix = np.array([0, 5, 71, 72 * 20 + 33, 72 * 40 - 1], np.int64)
    orc.composite_pixels(*args, scene.L, pix, with_margin_T=True)
    orc.composite_pixels_alt(*args, scene.L, pix, np.array([0, 1, 2, 3, 0xffffffff], np.uint32))
    dense = np.zeros((scene.n, scene.levels * scene.L))
    orc.composite_dense(cam, ranges, ids, pr["mean2d"], pr["conic"], scene.opacity, dense)
    orc.composite_bruteforce(cam, m32, pr["radius"], d32, pr["mean2d"], pr["conic"], scene.opacity, scene.topk_idx,
                             scene.topk_w, scene.L)
    F = orc.decode(coef, scene.dictionary)
    orc.decode_bf16(coef.astype(np.float32), scene.dictionary)
    orc.round_bf16(np.linspace(-3, 3, 101).astype(np.float32))
    pos, neg = gen.make_text(3, D=scene.D)
    rel = orc.query(F, pos, neg)
    orc.query_backward(F, pos, neg, np.ones_like(rel))
    d_coef = orc.decode_backward(coef, scene.dictionary, np.ones_like(F))[0]
    orc.composite_backward(*args, d_coef)
    lv, H, W, L = d_coef.shape
    orc.composite_backward_pixels(*args, pix, d_coef.reshape(lv, H * W, L)[:, pix].transpose(1, 0, 2))
    orc.project_backward(cam, scene.means, scene.scales, scene.quats, pr["radius"],
                         np.ones_like(pr["mean2d"]), np.ones_like(pr["conic"]))
    orc.postprocess(rel, 5, smooth_mode=1, select_mode=1)
    print("sanitized workload ok", flush=True)


if __name__ == "__main__":
    main()
