"""Central finite differences of the whole float64 oracle chain
(projection -> binning -> sparse compositing -> decode -> L1 + cosine loss,
Sections 3.1-3.4, Eqs. 1-7) on the finite-difference scene: 500 Gaussians at
64x64, L = 64, K = 4, D = 512, against a seeded smooth 512-d target.

Test infrastructure: the parameters are perturbed one at a time by
h = 1e-6 max(1, |theta|) in float64.  A perturbation that changes any
discrete decision is excluded and counted: the integer radius of any
Gaussian, the tile lists, any pixel's last contributor (the stop), or where
the perturbed Gaussian is skipped or clamped at 0.99 (its alpha at T = 1,
from the oracle's own renderer of that Gaussian alone).
"""
from __future__ import annotations

import math

import numpy as np

import gen

KINDS = ("means", "scales", "quats", "opacity", "topk_w", "dictionary")
F32_099 = float(np.float32(0.99))


def _cos(F, Y):
    nf = np.maximum(np.linalg.norm(F, axis=1), 1e-12)
    ny = np.maximum(np.linalg.norm(Y, axis=1), 1e-12)
    return np.einsum("ij,ij->i", F, Y) / (nf * ny)


def loss_difference(Fp, Fm, Y):
    """loss(Fp) - loss(Fm) for the oracle's L1 + cosine loss (mean |F - Y|
    over elements plus mean (1 - cos) over rows, norms guarded below by
    1e-12), summed term by term with exactly rounded sums: the difference of
    two rounded losses of about 1.5 would carry an error of an ulp of 1.5,
    1e-10 of a gradient after division by 2h = 2e-6.  Unchanged terms cancel
    exactly."""
    d = np.abs(Fp - Y) - np.abs(Fm - Y)
    dc = _cos(Fm, Y) - _cos(Fp, Y)
    return math.fsum(d[d != 0].tolist()) / Fp.size + math.fsum(dc[dc != 0].tolist()) / Fp.shape[0]


class Chain:
    def __init__(self, orc, cfg="fd", mask=None):
        c = gen.CONFIGS[cfg]
        self.orc = orc
        self.scene, self.cam = gen.config_scene(cfg)
        zup, P = gen.make_target_factors(c["seed"] + 1, c["height"], c["width"], D=c["D"])
        self.Y = gen.target_map(zup, P).astype(np.float64).reshape(-1, c["D"])
        sc = self.scene
        self.p0 = dict(means=sc.means.astype(np.float64), scales=sc.scales.astype(np.float64),
                       quats=sc.quats.astype(np.float64), opacity=sc.opacity.astype(np.float64),
                       topk_w=sc.topk_w.astype(np.float64), dictionary=sc.dictionary.astype(np.float64))
        self.mask = mask     # flat pixel indices that enter the loss (None: every pixel)

    def rows(self):
        return np.arange(self.Y.shape[0]) if self.mask is None else np.asarray(self.mask)

    def forward(self, p):
        """Loss and everything the backward and the decision signature need."""
        orc, cam, sc = self.orc, self.cam, self.scene
        pr = orc.project(cam, p["means"], p["scales"], p["quats"], f64=True)
        _, ids, ranges = orc.tile_lists(cam, pr["mean2d"].astype(np.float32), pr["radius"],
                                        pr["depth"].astype(np.float32))
        coef, fT, last, margin, margin_T = orc.composite(cam, ranges, ids, pr["mean2d"], pr["conic"], p["opacity"],
                                                         sc.topk_idx, p["topk_w"], sc.L, with_margin_T=True)
        F = orc.decode(coef, p["dictionary"]).reshape(-1, sc.D)
        r = self.rows()
        loss, dFr = orc.loss_l1cos(F[r], self.Y[r])
        return dict(loss=loss, F=F[r], dFr=dFr, pr=pr, ids=ids, ranges=ranges, coef=coef, last=last, margin=margin,
                    margin_T=margin_T)

    def analytic(self, p=None, fw=None):
        """The oracle's hand-derived gradient of the loss (every kind)."""
        orc, cam, sc = self.orc, self.cam, self.scene
        p = self.p0 if p is None else p
        fw = self.forward(p) if fw is None else fw
        dF = np.zeros((self.Y.shape[0], sc.D))
        dF[self.rows()] = fw["dFr"]
        dc, ds = orc.decode_backward(fw["coef"], p["dictionary"], dF.reshape(fw["coef"].shape[:-1] + (sc.D,)))
        pr = fw["pr"]
        dm, dcn, do, dw = orc.composite_backward(cam, fw["ranges"], fw["ids"], pr["mean2d"], pr["conic"],
                                                 p["opacity"], sc.topk_idx, p["topk_w"], dc)
        dmu, dsc, dq = orc.project_backward(cam, p["means"], p["scales"], p["quats"], pr["radius"], dm, dcn, f64=True)
        return dict(means=dmu, scales=dsc, quats=dq, opacity=do, topk_w=dw, dictionary=ds)

    def _alpha_alone(self, fw, p, g):
        """alpha of Gaussian g at every pixel of its tiles, composited alone."""
        ids, ranges = fw["ids"], fw["ranges"]
        one = np.zeros_like(ranges)
        for t in range(ranges.shape[0]):
            if np.any(ids[ranges[t, 0]:ranges[t, 1]] == g):
                one[t] = (0, 1)
        pr = fw["pr"]
        return self.orc.composite_dense(self.cam, one, np.array([g], np.uint32), pr["mean2d"], pr["conic"],
                                        p["opacity"], np.ones((self.scene.n, 1)))[..., 0]

    def signature(self, fw, p, g):
        a = self._alpha_alone(fw, p, g) if g is not None else None
        return (fw["pr"]["radius"].tobytes(), fw["ids"].tobytes(), fw["ranges"].tobytes(), fw["last"].tobytes(),
                None if a is None else ((a > 0).tobytes(), (a == F32_099).tobytes()))

    def sample(self, grad, per_kind, seed):
        """per_kind flat indices of each kind, drawn among the elements with a
        non-zero analytic gradient."""
        rng = np.random.default_rng(seed)
        out = {}
        for k in KINDS:
            live = np.flatnonzero(np.abs(grad[k]) > 0)
            out[k] = np.sort(rng.choice(live, min(per_kind, live.size), replace=False))
        return out

    def fd(self, idx, h_rel=1e-6):
        """{kind: (values, kept mask)} of central differences at the flat
        indices idx[kind]; kept is False where a decision changed."""
        base = self.forward(self.p0)
        res = {}
        for k, ii in idx.items():
            per = self.p0[k][0].size if k != "dictionary" else None
            vals = np.zeros(len(ii))
            kept = np.ones(len(ii), bool)
            for j, i in enumerate(ii):
                g = int(i // per) if per is not None and k != "topk_w" else None
                sig0 = self.signature(base, self.p0, g)
                x0 = self.p0[k].flat[i]
                h = h_rel * max(1.0, abs(x0))
                Fs = []
                for sgn in (1.0, -1.0):
                    p = dict(self.p0)
                    p[k] = self.p0[k].copy()
                    p[k].flat[i] = x0 + sgn * h
                    fw = self.forward(p)
                    if self.signature(fw, p, g) != sig0:
                        kept[j] = False
                    Fs.append(fw["F"])
                vals[j] = loss_difference(Fs[0], Fs[1], self.Y[self.rows()]) / (2 * h)
            res[k] = (vals, kept)
        return res
