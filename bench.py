#!/usr/bin/env python3
"""Feature-map benchmark of the sparse-coefficient splatting path on one GPU.

One step = one feature-map frame of the whole forward hot path over the
synthetic 1440x1080 scene (300k Gaussians, L=64, K=4, D=512, one level):
project -> bin_sort -> splat_decode (float32 compositing of the K sparse
coefficients, then each pixel's coefficients rounded to bf16 and decoded on
the matrix cores in the same kernel, bf16 output), with the scene already
resident in HBM.  Prints one JSON line.

Also reported: the same frame in two passes (splat writing a bf16
coefficient map, then dict_decode), per-stage times (HIP events on the launch
stream), the query rate (frame + relevancy), the plain FP32 path's rate, the
roofline of the dominant kernel and the FP64 CPU oracle timed on a bounded
sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
BF16_PEAK_TFLOPS = 2500.0      # dense MFMA bf16
F32_MFMA_PEAK_TFLOPS = 157.3   # MFMA fp32
METRIC = "feature-map FPS at 1440x1080, L=64 K=4 D=512; fwd+bwd ms; % HBM/MFMA peak"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(stage, n, P, H, W, L, D, K, levels, feat_bytes, coef_bytes=4):
    """HBM bytes the method itself must move per launch of each stage
    (coef_bytes: element size of the stored coefficient map)."""
    M = levels * H * W
    if stage == "project":
        return n * (12 + 12 + 16) + n * (8 + 12 + 4 + 4 + 4)
    if stage == "bin_sort":
        # count + emit read the projection (mean2d, radius, depth); emit writes
        # 8-byte keys; the sort reads them and writes 4-byte ids
        return n * (8 + 4) * 2 + n * 4 + P * 8 + P * 8 + P * 4
    if stage == "splat":
        rec = 8 + 12 + 4 + levels * K * 8
        return M * L * coef_bytes + H * W * 8 + P * 4 + n * rec
    if stage == "decode":
        return M * L * coef_bytes + L * D * 4 + M * D * feat_bytes
    if stage == "splat_decode":
        # the splat's reads, final_T and last, the dictionary and the feature
        # map; the coefficient map stays on chip
        rec = 8 + 12 + 4 + levels * K * 8
        return H * W * 8 + P * 4 + n * rec + L * D * 4 + M * D * feat_bytes
    if stage == "query":
        return M * D * feat_bytes + M * 4
    return 0


def _source_sha(hip):
    """sha256 prefix of a kernel source and the library's headers."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2507_07136_amd", "csrc")
    h = hashlib.sha256()
    for f in [os.path.join(csrc, hip)] + sorted(os.path.join(csrc, x) for x in os.listdir(csrc) if x.endswith(".h")):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(stage, config):
    """HBM bytes per launch of a stage from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE counters, scaled by the copy-kernel calibration; None when no
    counters exist for this workload or the kernel changed since they were
    taken."""
    path = os.path.join(ROOT, "profiles", "%s_hbm_counters.txt" % config)
    if not os.path.exists(path):
        return None
    kv = {}
    entry = None
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            fields = dict(t.split("=", 1) for t in line.split())
            if "stage" in fields:
                if fields["stage"] == stage:
                    entry = fields
            else:
                kv.update(fields)
    if entry is None or _source_sha(entry["source"]) != entry["source_sha"]:
        return None
    return (float(entry["fetch_kib"]) * 1024.0 * float(kv["copy_fetch_factor"]) +
            float(entry["write_kib"]) * 1024.0 * float(kv["copy_write_factor"]))


def cpu_baseline(cam, scene, frac):
    """The FP64 oracle, untuned, on the same frame: projection and binning of
    the full scene, then compositing + decode of every pixel (frac < 1: of a
    random fraction of the pixels, the frame time extrapolated)."""
    import numpy as np
    from oracle import oracle as orc
    orc.build()
    t0 = time.perf_counter()
    pr = orc.project(cam, scene.means, scene.scales, scene.quats)
    t1 = time.perf_counter()
    keys, ids, ranges = orc.tile_lists(cam, pr["mean2d"].astype(np.float32), pr["radius"],
                                       pr["depth"].astype(np.float32))
    t2 = time.perf_counter()
    npx = cam.width * cam.height
    pix = (np.arange(npx) if frac >= 1.0 else
           np.random.default_rng(0).choice(npx, max(1, int(frac * npx)), replace=False))
    coef, fT, last, margin = orc.composite_pixels(cam, ranges, ids, pr["mean2d"], pr["conic"], scene.opacity,
                                                  scene.topk_idx, scene.topk_w, scene.L, pix)
    t3 = time.perf_counter()
    orc.decode(coef.reshape(-1, scene.L), scene.dictionary)
    t4 = time.perf_counter()
    scale = npx / len(pix)
    frame_s = (t1 - t0) + (t2 - t1) + ((t3 - t2) + (t4 - t3)) * scale
    if len(pix) == npx:
        sample = ("the whole frame: projection, binning, compositing and decode of all %d pixels, not "
                  "extrapolated; %.2f s wall on %d threads" % (npx, t4 - t0, orc.num_threads()))
    else:
        sample = ("full-scene projection + binning; compositing + decode of %d random pixels (%.1f%% of the "
                  "frame), extrapolated; %.2f s wall on %d threads" % (len(pix), 100.0 * len(pix) / npx, t4 - t0,
                                                                      orc.num_threads()))
    return dict(value=1.0 / frame_s, unit="FPS", cores=orc.num_threads(), kind="oracle", sample=sample,
                frame_s=frame_s, stages_s=dict(project=t1 - t0, bin_sort=t2 - t1, composite=(t3 - t2) * scale,
                                               decode=(t4 - t3) * scale))


def cpu_model():
    """The host CPU's model name and logical core count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, os.cpu_count()


def cpu_baseline_one_core(config, frac):
    """The same oracle frame on one host thread (OpenMP limited to 1 in a
    child process), on a pixel fraction `frac` (extrapolated)."""
    import subprocess
    code = ("import json, sys; sys.path.insert(0, %r); import gen, bench; s, c = gen.config_scene(%r); "
            "r = bench.cpu_baseline(c, s, %r); print(json.dumps(r))" % (ROOT, config, frac))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        log("one-core oracle run failed: %s" % r.stderr[-2000:])
        return None
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return dict(value=d["value"], cores=d["cores"], frame_s=round(d["frame_s"], 3),
                stages_s={k: round(v, 3) for k, v in d["stages_s"].items()}, sample=d["sample"])


def c4_oracle_errors(samples):
    """Maximum error of every output of the precision workload against the
    FP64 oracle, on the sampled pixels each (L, K) run kept: the oracle
    composites those pixels from the GPU's lists and projection (stage
    isolated), decodes them in FP64 and forms their relevancy.  Pixels with a
    compositing decision within 1e-5 of its threshold are left out of the
    maxima and counted."""
    import numpy as np
    from oracle import oracle as orc
    out = {}
    for key, s in samples.items():
        sc = s["scene"]
        c, fT, last, margin, margin_T = orc.composite_pixels(s["cam"], s["ranges"], s["ids"], s["mean2d"], s["conic"],
                                                             sc.opacity, sc.topk_idx, sc.topk_w, sc.L, s["pix"],
                                                             with_margin_T=True)
        c = c.reshape(len(s["pix"]), -1)
        F = orc.decode(c, sc.dictionary)
        r = orc.query(F, s["pos"], s["neg"])
        ok = (margin.reshape(-1) >= 1e-5) & (margin_T.reshape(-1) >= 1e-5)
        nF = np.linalg.norm(F, axis=1)
        okn = ok & (nF > 1e-6)
        e = dict(coef_f32_abs=np.abs(s["coef"] - c).max(axis=1)[ok].max(),
                 feat_f32_abs=np.abs(s["f32"] - F).max(axis=1)[ok].max(),
                 feat_bf16_rel_l2=(np.linalg.norm(s["bf"] - F, axis=1)[okn] / nF[okn]).max(),
                 relevancy_f32_abs=np.abs(s["r32"] - r)[ok].max(),
                 relevancy_bf16_abs=np.abs(s["rbf"] - r)[ok].max(),
                 T_abs=np.abs(s["T"] - fT.reshape(-1))[ok].max())
        out[key] = {k: float("%.3e" % v) for k, v in e.items()}
        out[key]["pixels"] = int(len(s["pix"]))
        out[key]["near_threshold_left_out"] = int((~ok).sum())
    return out


def train_step_timing(args, torch, np, gen, ls2, onepass=True):
    """Forward + backward of the feature-map objective on the differentiation
    workload (float32 throughout): project, bin_sort, splat, then decode +
    loss + decode backward in one pass (dL/dF kept on chip), splat and
    projection backward; with onepass=False the decode + loss and the decode
    backward run as two kernels with dL/dF through HBM.  Per-stage HIP
    events."""
    cfg = gen.CONFIGS[args.train_config]
    scene, cam = gen.config_scene(args.train_config)
    zup, Pf = gen.make_target_factors(cfg["seed"] * 100, cfg["height"], cfg["width"], D=cfg["D"])
    # the target map Y = Zup P is materialised on the device (input preparation, outside the timed region)
    Y = (torch.from_numpy(zup).cuda().reshape(-1, zup.shape[-1]) @ torch.from_numpy(Pf).cuda()).reshape(
        cfg["levels"], cfg["height"], cfg["width"], cfg["D"]).contiguous()
    t = ls2.to_device(scene)
    tr = ls2.Trainer(cam, scene.n, levels=scene.levels, K=scene.K, L=scene.L, D=scene.D)
    tr.forward_loss(t, Y, sync=True)          # sizes the pair buffers
    onepass = onepass and tr.fused_loss
    names = ["project", "bin_sort", "splat"] + (["decode_loss_bw"] if onepass else ["decode_loss", "decode_bw"]) + [
        "splat_bw", "project_bw"]

    def step(ev=None):
        def mark(i):
            if ev is not None:
                ev[i].record()
        mark(0)
        tr.project(t["means"], t["scales"], t["quats"])
        mark(1)
        tr.bin_sort(sync=False)
        mark(2)
        tr.splat(t["opacity"], t["topk_idx"], t["topk_w"])
        mark(3)
        g = tr.grad
        m = tr.levels * tr.H * tr.W
        if onepass:
            ls2.ls2_decode_loss_backward(tr.coef.view(m, tr.L), t["dictionary"], Y.view(m, tr.D), tr.loss,
                                         g.coef.view(m, tr.L), g.dictionary, tr.onepass_ws)
            k = 4
        else:
            tr.decode_loss(t["dictionary"], Y)      # float32 decode fused with the loss (F stays on chip)
            mark(4)
            ls2.ls2_dict_decode_backward(tr.coef.view(m, tr.L), t["dictionary"], tr.d_feat.view(m, tr.D),
                                         g.coef.view(m, tr.L), g.dictionary, tr.dec_ws)
            k = 5
        mark(k)
        ls2.ls2_splat_sparse_backward(tr.cam, tr.levels, tr.K, tr.L, tr.tile_ranges, tr.ids, tr.mean2d, tr.conic,
                                      t["opacity"], t["topk_idx"], t["topk_w"], tr.final_T, tr.last, g.coef,
                                      g.mean2d, g.conic, g.opacity, g.topk_w)
        mark(k + 1)
        ls2.ls2_project_backward(tr.cam, t["means"], t["scales"], t["quats"], tr.radius, g.mean2d, g.conic,
                                 g.means, g.scales, g.quats)
        mark(k + 2)

    steps = max(5, args.steps // 2)
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for _ in range(steps)]
    t0 = time.perf_counter()
    for s_ in range(steps):
        step(evs[s_])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = {names[i]: round(float(np.mean([evs[s_][i].elapsed_time(evs[s_][i + 1]) for s_ in range(steps)])), 4)
           for i in range(len(names))}
    ms = 1000.0 * wall / steps
    m = scene.levels * cam.height * cam.width
    # matrix-core work of the decode stages: 2 m L D flops per product
    stage, prods = ("decode_loss_bw", 3.0) if onepass else ("decode_bw", 2.0)
    dec_flops = prods * 2.0 * m * scene.L * scene.D
    tf = dec_flops / (per[stage] * 1e-3) / 1e12
    log("fwd+bwd (%s): %.3f ms/step, stages %s, loss %.6f" % ("one pass" if onepass else "two pass", ms, per,
                                                              tr.loss.item()))
    return dict(ms=ms, steps=steps, workload="%s: %d Gaussians, %dx%d, L=%d, K=%d, D=%d, L1+cosine loss vs a smooth "
                "random 512-D target, float32" % (args.train_config, scene.n, cam.width, cam.height, scene.L,
                                                   scene.K, scene.D),
                decode=("decode + loss + decode backward in one pass (dL/dF on chip)" if onepass else
                        "decode + loss, then decode backward (dL/dF through HBM)"),
                stages_ms=per, loss=tr.loss.item(),
                **{stage + "_tflops": round(tf, 2), stage + "_frac_f32_peak": round(tf / F32_MFMA_PEAK_TFLOPS, 4)})


def full_form(args, torch, np, gen, ls2, steps=2):
    """The full form: 1M Gaussians at 1920x1080, three semantic levels (each
    with its own K=4 codes over one shared 64x512 codebook), a batch of 8
    views on a radius-3 circle.  One step = for every view: project, bin,
    splat, float32 decode fused with the L1 + cosine loss against that view's
    per-level targets, decode / splat / projection backward, and the
    accumulation of the per-Gaussian and codebook gradients over the views."""
    cfg = gen.CONFIGS["c5"]
    scene, _ = gen.config_scene("c5")
    H, W, D, levels = cfg["height"], cfg["width"], cfg["D"], cfg["levels"]
    cams = [gen.orbit_camera(W, H, j, 8) for j in range(8)]
    t = ls2.to_device(scene)
    # per (view, level) targets, materialised on the device (input preparation)
    targets = []
    for j in range(8):
        Y = torch.empty((levels, H, W, D), dtype=torch.float32, device="cuda")
        for lv in range(levels):
            zup, Pf = gen.make_target_factors(1005 * 100 + 8 * lv + j, H, W, D=D)
            Y[lv] = (torch.from_numpy(zup).cuda().reshape(-1, zup.shape[-1]) @ torch.from_numpy(Pf).cuda()).reshape(
                H, W, D)
        targets.append(Y)
    tr = ls2.Trainer(cams[0], scene.n, levels=levels, K=scene.K, L=scene.L, D=D)
    total = ls2.Gradients(scene.n, levels, scene.K, scene.L, D, H, W, "cuda")
    pairs = []
    for j in range(8):                                  # size the pair buffers for every view
        tr.set_camera(cams[j])
        tr.project(t["means"], t["scales"], t["quats"])
        pairs.append(tr.bin_sort(sync=True))
    torch.cuda.synchronize()

    def step():
        for name in ("dictionary", "means", "scales", "quats", "opacity", "topk_w"):
            getattr(total, name).zero_()
        for j in range(8):
            tr.set_camera(cams[j])
            tr.step(t, targets[j], sync=False)   # one-pass decode + loss + decode backward
            tr.accumulate_into(total)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / steps
    # algorithmic HBM bytes of one step (per view: projection, lists, splat,
    # one-pass decode + loss + decode backward, splat / projection backward)
    n, L, K, M = scene.n, scene.L, scene.K, levels * H * W
    per_view = []
    for P in pairs:
        b = algorithmic_bytes("project", n, P, H, W, L, D, K, levels, 4)
        b += algorithmic_bytes("bin_sort", n, P, H, W, L, D, K, levels, 4)
        b += algorithmic_bytes("splat", n, P, H, W, L, D, K, levels, 4)
        b += 2 * M * L * 4 + M * D * 4                      # decode + loss + decode backward: W in, Y in, dW out
        b += M * L * 4 + H * W * 8 + P * 4 + n * (8 + 12 + 4 + levels * K * 8) + n * levels * K * 4 + n * 24
        b += n * (40 + 20 + 40)                             # projection backward
        per_view.append(b)
    gb = sum(per_view) / 1e9
    out = dict(workload="c5: %d Gaussians, %dx%d, %d levels (L=%d, K=%d each, shared %dx%d codebook), 8 orbit views; "
                        "float32 forward + loss + backward per view, gradients accumulated over the views"
                        % (n, W, H, levels, L, K, L, D),
               ms_per_step=round(ms, 3), ms_per_view=round(ms / 8, 3), pairs_per_view=[int(P) for P in pairs],
               algorithmic_GB_per_step=round(gb, 2), hbm_GBs=round(gb / (ms * 1e-3), 1),
               hbm_frac=round(gb / (ms * 1e-3) / HBM_PEAK_GBS, 4), loss_last_view=tr.loss.item())
    log("full form: %s" % out)
    del targets, tr, total, t
    torch.cuda.empty_cache()
    return out


def precision_form(args, torch, np, gen, ls2, n_pix=400):
    """The precision workload (1440x1080, 300k Gaussians, D=512) at L in
    {64, 128} and K in {4, 8}: the bf16 one-pass frame (project, bin_sort,
    splat_decode) and the plain float32 path (project, bin_sort, float32
    splat, float32 decode) timed on the same scene.  Keeps every output at
    n_pix random pixels for the FP64 comparison of the oracle leg."""
    out, samples = {}, {}
    steps = max(5, args.steps // 2)
    for L, K in ((64, 4), (64, 8), (128, 4), (128, 8)):
        scene, cam = gen.config_scene("c4", L=L, K=K)
        t = ls2.to_device(scene)
        n, D = scene.n, scene.D
        p16 = ls2.Pipeline(cam, n, levels=1, K=K, L=L, D=D, coef_dtype=torch.bfloat16)
        p32 = ls2.Pipeline(cam, n, levels=1, K=K, L=L, D=D)
        for p_ in (p16, p32):
            p_.project(t["means"], t["scales"], t["quats"])
            p_.bin_sort(sync=True)

        def f16():
            p16.project(t["means"], t["scales"], t["quats"])
            p16.bin_sort(sync=False)
            p16.splat_decode(t["opacity"], t["topk_idx"], t["topk_w"], t["dictionary"])

        def f32():
            p32.project(t["means"], t["scales"], t["quats"])
            p32.bin_sort(sync=False)
            p32.splat(t["opacity"], t["topk_idx"], t["topk_w"])
            p32.decode(t["dictionary"], ls2.LS2_F32, torch.float32)

        row = {}
        for name, fn in (("bf16_one_pass_fps", f16), ("f32_path_fps", f32)):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                fn()
            torch.cuda.synchronize()
            row[name] = round(steps / (time.perf_counter() - t0), 2)
        out["L%d_K%d" % (L, K)] = row
        log("precision form L=%d K=%d: %s" % (L, K, row))
        # sampled outputs of both paths (outside the timed frames)
        pos, neg = gen.make_text(1004 + 7, D=D)
        tp, tn = torch.from_numpy(pos).cuda(), torch.from_numpy(neg).cuda()
        pix = np.random.default_rng(L + K).choice(cam.width * cam.height, n_pix, replace=False)
        sel = torch.from_numpy(pix).cuda()
        rbf = p16.splat_decode_query(t["opacity"], t["topk_idx"], t["topk_w"], t["dictionary"], tp, tn)
        bf = p16.feat
        r32 = p32.query(tp, tn)
        torch.cuda.synchronize()

        def rows(x, w):
            return x.reshape(-1, w)[sel].double().cpu().numpy()
        samples["L%d_K%d" % (L, K)] = dict(
            scene=scene, cam=cam, pix=pix, pos=pos, neg=neg,
            ranges=p32.tile_ranges.cpu().numpy().view(np.uint32),
            ids=p32.ids[:p32.num_pairs].cpu().numpy().view(np.uint32),
            mean2d=p32.mean2d.double().cpu().numpy(), conic=p32.conic.double().cpu().numpy(),
            coef=rows(p32.coef, L), f32=rows(p32.feat, D), bf=rows(bf, D), r32=rows(r32, 1)[:, 0],
            rbf=rows(rbf, 1)[:, 0], T=rows(p32.final_T, 1)[:, 0])
        del p16, p32, t
        torch.cuda.empty_cache()
    return out, samples


def query_post_frames(args, torch, np, gen, ls2, kernel=29):
    """Query frames with the relevancy post-processing of Section 3.2 and
    the evaluation appendix: project, bin_sort, splat + bf16 decode +
    relevancy in one pass (the feature map not written), then the box mean
    over each level's map, the level selection, the argmax point and the
    mask (ls2_postprocess, a kernel x kernel window).  On the 1440x1080
    scene (one level) and on a 1920x1080 view of the 1M-Gaussian, 3-level
    scene."""
    out = {}
    steps = max(5, args.steps // 2)
    for name, cfg, levels in (("c2_1level", "c2", 1), ("c5_view0_3levels", "c5", 3)):
        scene, cam = gen.config_scene(cfg)
        if cfg == "c5":
            cam = gen.orbit_camera(cam.width, cam.height, 0, 8)
        t = ls2.to_device(scene)
        pos, neg = gen.make_text(gen.CONFIGS[cfg]["seed"] + 7, D=scene.D)
        tp, tn = torch.from_numpy(pos).cuda(), torch.from_numpy(neg).cuda()
        p = ls2.Pipeline(cam, scene.n, levels=levels, K=scene.K, L=scene.L, D=scene.D, coef_dtype=torch.bfloat16)
        p.project(t["means"], t["scales"], t["quats"])
        p.bin_sort(sync=True)
        H, W = cam.height, cam.width
        sm = torch.empty((levels, H, W), dtype=torch.float32, device="cuda")
        mask = torch.empty((H, W), dtype=torch.uint8, device="cuda")
        res = torch.empty((4,), dtype=torch.int32, device="cuda")
        ws = torch.empty((ls2.ls2_postprocess_workspace(levels, H, W),), dtype=torch.uint8, device="cuda")

        def frame(ev=None):
            if ev is not None:
                ev[0].record()
            p.project(t["means"], t["scales"], t["quats"])
            p.bin_sort(sync=False)
            rel = p.splat_decode_query(t["opacity"], t["topk_idx"], t["topk_w"], t["dictionary"], tp, tn,
                                       keep_feat=False)
            if ev is not None:
                ev[1].record()
            ls2.ls2_postprocess(rel, kernel, sm, mask, res, ws)
            if ev is not None:
                ev[2].record()
        for _ in range(3):
            frame()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            frame()
        torch.cuda.synchronize()
        fps = steps / (time.perf_counter() - t0)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        for i in range(steps):
            frame(evs[i])
        torch.cuda.synchronize()
        out[name] = dict(fps=round(fps, 2), workload="%d Gaussians, %dx%d, %d level(s)" % (scene.n, W, H, levels),
                         render_decode_relevancy_ms=round(float(np.mean([e[0].elapsed_time(e[1]) for e in evs])), 4),
                         postprocess_ms=round(float(np.mean([e[1].elapsed_time(e[2]) for e in evs])), 4),
                         window=kernel)
        log("query + post-processing %s: %s" % (name, out[name]))
        del p, t, sm, mask, ws
        torch.cuda.empty_cache()
    out["paper_table1_context"] = "384.6 FPS querying (A100, its own scenes and resolution): context, not a target"
    return out


def dense_ablation(args, torch, np, gen, ls2):
    """Sparse (K of L blended) against dense (all L blended) splatting on the
    1440x1080 scene with one level (L = 64) and three levels (3 x 64 = 192,
    the rendering dimension Table 9 times); same lists, HIP events around the
    splat kernel only."""
    out = {}
    for levels in (1, 3):
        scene, cam = gen.config_scene(args.config, levels=levels)
        t = ls2.to_device(scene)
        pipe = ls2.Pipeline(cam, scene.n, levels=levels, K=scene.K, L=scene.L, D=scene.D)
        pipe.project(t["means"], t["scales"], t["quats"])
        pipe.bin_sort(sync=True)
        n, L = scene.n, scene.L
        Wd = torch.zeros((n, levels, L), dtype=torch.float32, device="cuda")
        Wd.scatter_add_(2, t["topk_idx"].long(), t["topk_w"])    # input preparation
        times = {}
        for name, fn in (("sparse", lambda: pipe.splat(t["opacity"], t["topk_idx"], t["topk_w"])),
                         ("dense", lambda: pipe.splat_dense(t["opacity"], Wd))):
            for _ in range(2):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 5
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            times[name + "_ms"] = round(e0.elapsed_time(e1) / reps, 4)
        times["dense_over_sparse"] = round(times["dense_ms"] / times["sparse_ms"], 2)
        out["%dx%d" % (levels, L)] = times
        del pipe, t, Wd
        torch.cuda.empty_cache()
    log("sparse vs dense splat: %s" % out)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed frames before each timed run (the clocks settle within about 100 frames)")
    ap.add_argument("--config", default="c2")
    ap.add_argument("--cpu-frac", type=float, default=1.0,
                    help="pixel fraction the CPU oracle composites and decodes (default: the whole frame, a few "
                         "seconds on 16 host threads; below 1 the frame time is extrapolated)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true", help="skip the plain FP32 path measurement")
    ap.add_argument("--no-train", action="store_true", help="skip the forward+backward (training step) timing")
    ap.add_argument("--train-config", default="c3")
    ap.add_argument("--no-ablation", action="store_true", help="skip the sparse-vs-dense splat timing")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the L in {64,128} x K in {4,8} timings and their FP64 comparison")
    ap.add_argument("--no-query-post", action="store_true", help="skip the query + post-processing frames")
    ap.add_argument("--cpu-frac-one-core", type=float, default=0.05,
                    help="pixel fraction of the one-thread oracle run (extrapolated to the frame)")
    ap.add_argument("--no-full-form", action="store_true",
                    help="skip the 1M-Gaussian, 3-level, 8-view training step")
    ap.add_argument("--full-form-only", action="store_true",
                    help="only run the full-form training step and print its JSON (for profiling it alone)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES bytes five times (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the splatting path runs on a single MI355X here "
              "(multi-GPU sharding is not run); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4, "launches": 5}), flush=True)
        return

    import gen
    import paper_2507_07136_amd as ls2

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.full_form_only:
        print(json.dumps({"full_form": full_form(args, torch, np, gen, ls2, steps=max(1, args.steps))}), flush=True)
        return
    cfg = gen.CONFIGS[args.config]
    log("generating scene", args.config, cfg)
    scene, cam = gen.config_scene(args.config)
    pos, neg = gen.make_text(cfg["seed"] + 7, D=cfg["D"])
    t = ls2.to_device(scene)
    post, negt = torch.from_numpy(pos).cuda(), torch.from_numpy(neg).cuda()
    n, H, W, L, D, K, levels = scene.n, cam.height, cam.width, scene.L, scene.D, scene.K, scene.levels

    # float32 coefficient map: the float32 path and the coefficient-space query
    pipe = ls2.Pipeline(cam, n, levels=levels, K=K, L=L, D=D)
    # bf16 coefficient map (the values the bf16 decode rounds to): the bf16 path
    pipe16 = ls2.Pipeline(cam, n, levels=levels, K=K, L=L, D=D, coef_dtype=torch.bfloat16)
    # first frame sizes the pair buffers (one host sync); later frames run without host syncs
    for p_ in (pipe, pipe16):
        p_.project(t["means"], t["scales"], t["quats"])
        P = p_.bin_sort(sync=True)
    log("P =", P, "pairs")

    def frame(p_, compute, out_dtype, ev=None, query=False, fused=False, one_pass=False, keep_feat=True,
              sync=False, pb=False):
        k = [0]

        def mark():
            if ev is not None:
                ev[k[0]].record()
            k[0] += 1
        mark()
        if pb:  # projection and binning in one call (the binning's first pass projects)
            p_.project_bin_sort(t["means"], t["scales"], t["quats"], sync=sync)
            mark()
        else:
            p_.project(t["means"], t["scales"], t["quats"])
            mark()
            p_.bin_sort(sync=sync)  # sync: the pair count is read back to the host (one round trip)
            mark()
        if one_pass:  # splat and bf16 decode in one kernel: the coefficient map stays on chip
            if query:  # and the relevancy formed in the same pass
                p_.splat_decode_query(t["opacity"], t["topk_idx"], t["topk_w"], t["dictionary"], post, negt,
                                      keep_feat=keep_feat)
            else:
                p_.splat_decode(t["opacity"], t["topk_idx"], t["topk_w"], t["dictionary"])
            mark()
            return
        p_.splat(t["opacity"], t["topk_idx"], t["topk_w"])
        mark()
        if fused:  # bf16 decode with the relevancy formed in its epilogue
            p_.decode_query(t["dictionary"], post, negt)
            mark()
            return
        p_.decode(t["dictionary"], compute, out_dtype)
        mark()
        if query:
            p_.query(post, negt)
            mark()

    stages = ["project", "bin_sort", "splat", "decode", "query"]

    def run(p_, compute, out_dtype, steps, warmup, query=False, fused=False, one_pass=False, keep_feat=True,
            sync=False):
        """Wall-clock rate over `steps` uninstrumented frames, then the same
        number of frames with HIP events between the stages (per-stage
        times; these frames are not part of the rate).  One-pass frames
        project and bin in one call (ls2_project_bin_sort)."""
        kw = dict(query=query, fused=fused, one_pass=one_pass, keep_feat=keep_feat, sync=sync, pb=one_pass)
        for _ in range(warmup):
            frame(p_, compute, out_dtype, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            frame(p_, compute, out_dtype, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
        for s in range(steps):
            frame(p_, compute, out_dtype, evs[s], **kw)
        torch.cuda.synchronize()
        names = (["project_bin_sort", "splat_decode_query" if query else "splat_decode"] if one_pass
                 else stages[:5 if (query and not fused) else 4])
        per = {names[i]: float(np.mean([evs[s][i].elapsed_time(evs[s][i + 1]) for s in range(steps)]))
               for i in range(len(names))}
        # per-frame times of the instrumented frames: p10 / median / p90
        totals = [evs[s][0].elapsed_time(evs[s][len(names)]) for s in range(steps)]
        pct = [round(float(np.percentile(totals, q)), 4) for q in (10, 50, 90)]
        return wall, per, pct

    # headline: float32 splat accumulation, the coefficients rounded to bf16 and
    # decoded on the matrix cores inside the splat (bf16 feature map)
    wall, per, per_pct = run(pipe16, ls2.LS2_BF16, torch.bfloat16, args.steps, args.warmup, one_pass=True)
    assert ls2.ls2_bin_sort_count(pipe16.workspace) == P
    fps = args.steps / wall
    ms = 1000.0 * wall / args.steps
    log("one-pass bf16 frame: %.1f FPS, %.3f ms/frame, stages %s" % (fps, ms, per))
    # the same frames with bin_sort's host synchronisation (the pair count read
    # back every frame, as a caller that sizes its buffers per frame would)
    swall, sper, sper_pct = run(pipe16, ls2.LS2_BF16, torch.bfloat16, args.steps, args.warmup, one_pass=True,
                                sync=True)
    sync_frame = dict(fps=round(args.steps / swall, 2), ms_per_frame=round(1000.0 * swall / args.steps, 4),
                      frame_ms_p10_p50_p90=sper_pct)
    log("one-pass bf16 frame with the host sync: %s" % sync_frame)
    # the same feature map in two passes: bf16 coefficient map written by the
    # splat, read back by the decode
    twall, tper, tper_pct = run(pipe16, ls2.LS2_BF16, torch.bfloat16, args.steps, args.warmup)
    two_pass = dict(fps=round(args.steps / twall, 2), ms_per_frame=round(1000.0 * twall / args.steps, 4),
                    stages_ms={k: round(v, 4) for k, v in tper.items()}, frame_ms_p10_p50_p90=tper_pct)
    log("two-pass bf16 frame: %s" % two_pass)

    # successive views on two streams (default priority), each with its own
    # buffers: one view's binning overlaps the previous view's splat tail.
    # Reported beside the headline, which is the one-stream rate above.
    pipe_b = ls2.Pipeline(cam, n, levels=levels, K=K, L=L, D=D, coef_dtype=torch.bfloat16)
    pipe_b.project(t["means"], t["scales"], t["quats"])
    pipe_b.bin_sort(sync=True)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    pipes2 = [pipe16, pipe_b]

    def two_stream_frames(k):
        for i in range(k):
            with torch.cuda.stream(streams[i & 1]):
                frame(pipes2[i & 1], ls2.LS2_BF16, torch.bfloat16, one_pass=True)
    two_stream_frames(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    two_stream_frames(args.steps)
    torch.cuda.synchronize()
    two_stream_fps = args.steps / (time.perf_counter() - t0)
    log("one-pass frames on two streams: %.1f FPS" % two_stream_fps)
    del pipe_b

    # query frame, two passes: decode writes the feature map, ls2_query reads it back
    qwall, qper, qper_pct = run(pipe16, ls2.LS2_BF16, torch.bfloat16, max(5, args.steps // 2), 3, query=True)
    query_fps_two_pass = max(5, args.steps // 2) / qwall
    # query frame, relevancy in the decode's epilogue (splat, then decode + relevancy)
    nqs = max(5, args.steps // 2)
    fqwall, fqper, fqper_pct = run(pipe16, ls2.LS2_BF16, torch.bfloat16, nqs, 3, query=True, fused=True)
    query_fps_epilogue = nqs / fqwall
    # query frame in one pass: splat, decode and relevancy in one kernel (feature map written)
    oqwall, oqper, oqper_pct = run(pipe16, ls2.LS2_BF16, torch.bfloat16, nqs, 3, query=True, one_pass=True)
    query_fps = nqs / oqwall
    # ... and without writing the feature map at all
    nqwall, nqper, nqper_pct = run(pipe16, ls2.LS2_BF16, torch.bfloat16, nqs, 3, query=True, one_pass=True,
                                   keep_feat=False)
    query_fps_no_feat = nqs / nqwall
    log("query frames: one pass %.1f FPS (splat+decode+relevancy %.4f ms), without the feature map %.1f FPS, "
        "decode epilogue %.1f FPS, two-pass %.1f FPS" % (query_fps, oqper["splat_decode_query"], query_fps_no_feat,
                                                         query_fps_epilogue, query_fps_two_pass))

    # relevancy straight from the coefficient map (Eq. 7): project, bin, splat, query_coef
    def coef_query_frame():
        pipe.project(t["means"], t["scales"], t["quats"])
        pipe.bin_sort(sync=False)
        pipe.splat(t["opacity"], t["topk_idx"], t["topk_w"])
        pipe.query_coef(t["dictionary"], post, negt)
    nq = max(5, args.steps // 2)
    for _ in range(3):
        coef_query_frame()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    for _ in range(nq):
        coef_query_frame()
    e0.record()
    pipe.query_coef(t["dictionary"], post, negt)
    e1.record()
    torch.cuda.synchronize()
    cq_wall = time.perf_counter() - t0
    query_coef = dict(fps=round(nq / cq_wall, 2), query_coef_ms=round(e0.elapsed_time(e1), 4))
    log("coefficient-space query: %s" % query_coef)

    f32 = None
    if not args.no_f32:
        fwall, fper, fper_pct = run(pipe, ls2.LS2_F32, torch.float32, max(5, args.steps // 2), 3)
        f32 = dict(fps=max(5, args.steps // 2) / fwall, stages_ms=fper)
        log("f32 path: %.1f FPS" % f32["fps"])

    # roofline per stage (bf16 path); the dominant kernel is the slowest stage
    roof_all = {}
    for st, tms in qper.items():
        fb = 2
        b = algorithmic_bytes(st, n, P, H, W, L, D, K, levels, fb, coef_bytes=2)
        gbs = b / (tms * 1e-3) / 1e9
        roof_all[st] = dict(ms=tms, bytes=b, gbs=gbs, frac_hbm=gbs / HBM_PEAK_GBS)
    for st in ("splat_decode",):
        b = algorithmic_bytes(st, n, P, H, W, L, D, K, levels, 2)
        gbs = b / (per[st] * 1e-3) / 1e9
        roof_all[st] = dict(ms=per[st], bytes=b, gbs=gbs, frac_hbm=gbs / HBM_PEAK_GBS)
    dom = max(per, key=per.get)
    b = algorithmic_bytes(dom, n, P, H, W, L, D, K, levels, 2, coef_bytes=2)
    ach = b / (per[dom] * 1e-3) / 1e9
    traffic = counter_traffic(dom, args.config)
    roofline = dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 4),
                    traffic=None if traffic is None else int(traffic), kernel=dom, kernel_ms=round(per[dom], 4),
                    algorithmic_bytes=int(b))
    M = levels * H * W
    decode_flops = 2.0 * M * L * D
    mfma = dict(decode_tflops=decode_flops / (tper["decode"] * 1e-3) / 1e12,
                decode_frac_bf16_peak=decode_flops / (tper["decode"] * 1e-3) / 1e12 / BF16_PEAK_TFLOPS)

    train = None
    if not args.no_train:
        del pipe, pipe16
        torch.cuda.empty_cache()
        train = train_step_timing(args, torch, np, gen, ls2)
        train_two_pass = train_step_timing(args, torch, np, gen, ls2, onepass=False)
        train["two_pass_ms"] = round(train_two_pass["ms"], 4)
        train["two_pass_stages_ms"] = train_two_pass["stages_ms"]

    ablation = None if args.no_ablation else dense_ablation(args, torch, np, gen, ls2)
    precision, prec_samples = (None, None) if args.no_precision else precision_form(args, torch, np, gen, ls2)
    query_post = None if args.no_query_post else query_post_frames(args, torch, np, gen, ls2)
    full = None if args.no_full_form else full_form(args, torch, np, gen, ls2)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample ...")
        cpu = cpu_baseline(cam, scene, args.cpu_frac)
        log("cpu oracle: %.4f FPS (%d threads)" % (cpu["value"], cpu["cores"]))
        cpu["cpu_model"], cpu["logical_cpus"] = cpu_model()
        cpu["stages_s"] = {k: round(v, 3) for k, v in cpu["stages_s"].items()}
        cpu["one_core"] = cpu_baseline_one_core(args.config, args.cpu_frac_one_core)
        log("cpu oracle, one thread: %s" % cpu["one_core"])
        if prec_samples is not None:
            precision["max_error_vs_fp64_oracle"] = c4_oracle_errors(prec_samples)
            log("precision form errors: %s" % precision["max_error_vs_fp64_oracle"])

    out = {
        "metric": METRIC,
        "value": round(fps, 2),
        "unit": "FPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 splat accumulation, bf16 decode operands (fp32 accumulate), bf16 feature map",
        "data": "synthetic",
        "config": {"workload": "%s: %d Gaussians, %dx%d, L=%d, K=%d, D=%d, %d level(s), 16x16 tiles"
                               % (args.config, n, W, H, L, K, D, levels),
                   "pairs": P},
        "stages_ms": {k: round(v, 4) for k, v in per.items()},
        "frame_ms_p10_p50_p90": per_pct,
        "with_host_sync": sync_frame,
        "two_pass_frame": two_pass,
        "two_stream_fps": round(two_stream_fps, 2),
        "query_fps": round(query_fps, 2),
        "query_fps_without_feature_map": round(query_fps_no_feat, 2),
        "query_fps_decode_epilogue": round(query_fps_epilogue, 2),
        "query_fps_two_pass": round(query_fps_two_pass, 2),
        "splat_decode_query_ms": round(oqper["splat_decode_query"], 4),
        "query_from_coefficients": query_coef,
        "fp32_path": None if f32 is None else {"fps": round(f32["fps"], 2),
                                               "stages_ms": {k: round(v, 4) for k, v in f32["stages_ms"].items()}},
        "sparse_vs_dense_splat": ablation,
        "precision_form": precision,
        "query_postprocess": query_post,
        "full_form": full,
        "fwd_bwd_ms": None if train is None else round(train["ms"], 4),
        "fwd_bwd": train,
        "roofline": roofline,
        "roofline_stages": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                            for k, v in roof_all.items()},
        "mfma": {k: round(v, 4) for k, v in mfma.items()},
        "cpu_baseline": None if cpu is None else {k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample",
                                                                     "cpu_model", "logical_cpus", "stages_s",
                                                                     "one_core")},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
