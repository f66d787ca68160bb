"""Feature-map pipeline over the libls2 C ABI.

``Pipeline`` owns the device buffers of one camera / scene size and chains the
ABI calls of the inference path of Section 3 (Table 1's rendering and
decoding stages, then the relevancy of the post-processing stage):
project -> bin_sort -> splat_sparse -> dict_decode -> query.  PyTorch supplies
device memory and the stream; every step runs in the HIP library.
"""
from __future__ import annotations

import torch

from . import _lib
from ._lib import LS2_BF16, LS2_F32, LS2Error

_TILE = _lib.TILE


class Pipeline:
    def __init__(self, cam, n: int, levels: int = 1, K: int = 4, L: int = 64, D: int = 512,
                 max_pairs: int | None = None, device="cuda", keep_keys: bool = False,
                 coef_dtype=torch.float32):
        """``coef_dtype`` torch.bfloat16 stores the coefficient map in bf16 (the
        values the bf16 decode rounds a float32 map to): half the map traffic
        for the bf16 feature-map path; the float32 decode, the coefficient
        query and training need the float32 map."""
        self.cam = _lib.make_camera(cam)
        self.n, self.levels, self.K, self.L, self.D = n, levels, K, L, D
        self.H, self.W = self.cam.height, self.cam.width
        self.tiles_x = (self.W + _TILE - 1) // _TILE
        self.tiles_y = (self.H + _TILE - 1) // _TILE
        self.device = torch.device(device)
        dev = self.device
        f32, i32 = torch.float32, torch.int32
        self.mean2d = torch.empty((n, 2), dtype=f32, device=dev)
        self.conic = torch.empty((n, 3), dtype=f32, device=dev)
        self.depth = torch.empty((n,), dtype=f32, device=dev)
        self.radius = torch.empty((n,), dtype=i32, device=dev)
        self.tiles_touched = torch.empty((n,), dtype=i32, device=dev)
        self.tile_ranges = torch.empty((self.tiles_x * self.tiles_y, 2), dtype=i32, device=dev)
        self.keep_keys = keep_keys
        self.num_pairs = None
        self._alloc_pairs(max_pairs if max_pairs is not None else max(1024, 64 * n))
        self.coef = torch.empty((levels, self.H, self.W, L), dtype=coef_dtype, device=dev)
        self.final_T = torch.empty((self.H, self.W), dtype=f32, device=dev)
        self.last = torch.empty((self.H, self.W), dtype=i32, device=dev)
        self.feat = None
        self.relevancy = None

    def _alloc_pairs(self, cap: int):
        dev = self.device
        self.max_pairs = int(cap)
        self.ids = torch.empty((self.max_pairs,), dtype=torch.int32, device=dev)
        self.keys = torch.empty((self.max_pairs,), dtype=torch.int64, device=dev) if self.keep_keys else None
        ws = _lib.ls2_bin_sort_workspace(self.cam, self.n, self.max_pairs)
        self.workspace = torch.empty((ws,), dtype=torch.uint8, device=dev)

    # ---------------------------------------------------------------- stages
    def project(self, means, scales, quats):
        _lib.ls2_project(self.cam, means, scales, quats, self.mean2d, self.conic, self.depth, self.radius,
                         self.tiles_touched)

    def bin_sort(self, sync: bool = True):
        """Bins and sorts; with sync=True grows the pair buffers if needed and
        returns P.  With sync=False no host synchronisation happens (the
        capacity must already suffice)."""
        while True:
            try:
                P = _lib.ls2_bin_sort(self.cam, self.mean2d, self.radius, self.depth, self.max_pairs, self.keys,
                                      self.ids, self.tile_ranges, self.workspace, sync=sync)
                if sync:
                    self.num_pairs = P
                return P
            except LS2Error as e:
                if e.status != _lib.LS2_ERR_CAPACITY:
                    raise
                self._alloc_pairs(int(e.num_pairs * 1.25) + 1024)

    def project_bin_sort(self, means, scales, quats, sync: bool = True):
        """project() then bin_sort() in one call (the binning's first pass
        projects; the same outputs bit for bit, one launch fewer)."""
        while True:
            try:
                P = _lib.ls2_project_bin_sort(self.cam, means, scales, quats, self.mean2d, self.conic, self.depth,
                                              self.radius, self.max_pairs, self.keys, self.ids, self.tile_ranges,
                                              self.workspace, tiles_touched=self.tiles_touched, sync=sync)
                if sync:
                    self.num_pairs = P
                return P
            except LS2Error as e:
                if e.status != _lib.LS2_ERR_CAPACITY:
                    raise
                self._alloc_pairs(int(e.num_pairs * 1.25) + 1024)

    def splat(self, opacity, topk_idx, topk_w):
        _lib.ls2_splat_sparse(self.cam, self.levels, self.K, self.L, self.tile_ranges, self.ids, self.mean2d,
                              self.conic, opacity, topk_idx, topk_w, self.coef, self.final_T, self.last)

    def splat_decode(self, opacity, topk_idx, topk_w, dictionary, keep_coef: bool = False):
        """Splat and bf16 decode in one pass (the coefficient map is written
        only with keep_coef, in bfloat16): the bf16 feature map of
        splat() (bf16 map) + decode(), bit for bit."""
        if self.feat is None or self.feat.dtype != torch.bfloat16:
            self.feat = torch.empty((self.levels, self.H, self.W, self.D), dtype=torch.bfloat16, device=self.device)
        if getattr(self, "_sd_ws", None) is None:
            self._sd_ws = torch.empty((_lib.ls2_splat_decode_workspace(self.L, self.D),), dtype=torch.uint8,
                                      device=self.device)
        coef = None
        if keep_coef:
            if self.coef.dtype != torch.bfloat16:
                raise ValueError("splat_decode keeps a bfloat16 map (Pipeline(coef_dtype=torch.bfloat16))")
            coef = self.coef
        _lib.ls2_splat_decode(self.cam, self.levels, self.K, self.L, self.tile_ranges, self.ids, self.mean2d,
                              self.conic, opacity, topk_idx, topk_w, dictionary, self.feat, self._sd_ws, coef,
                              self.final_T, self.last)
        return self.feat

    def splat_decode_query(self, opacity, topk_idx, topk_w, dictionary, pos, neg, tau: float = 1.0,
                           keep_feat: bool = True):
        """Splat, bf16 decode and relevancy in one pass: the relevancy equals
        ls2_query on the bf16 feature map bit for bit; with keep_feat=False
        the feature map is not written at all."""
        if self.relevancy is None:
            self.relevancy = torch.empty((self.levels, self.H, self.W), dtype=torch.float32, device=self.device)
        n_neg = neg.numel() // self.D
        if getattr(self, "_sdq_key", None) != n_neg:
            self._sdq_ws = torch.empty((_lib.ls2_splat_decode_query_workspace(self.L, self.D, n_neg),),
                                       dtype=torch.uint8, device=self.device)
            self._sdq_key = n_neg
        feat = None
        if keep_feat:
            if self.feat is None or self.feat.dtype != torch.bfloat16:
                self.feat = torch.empty((self.levels, self.H, self.W, self.D), dtype=torch.bfloat16,
                                        device=self.device)
            feat = self.feat
        _lib.ls2_splat_decode_query(self.cam, self.levels, self.K, self.L, self.tile_ranges, self.ids, self.mean2d,
                                    self.conic, opacity, topk_idx, topk_w, dictionary, pos, neg, self.relevancy,
                                    self._sdq_ws, feat=feat, final_T=self.final_T, last=self.last, tau=tau)
        return self.relevancy

    def splat_dense(self, opacity, weights):
        """Dense form (all L coefficients per Gaussian) into the same buffers."""
        _lib.ls2_splat_dense(self.cam, self.levels, self.L, self.tile_ranges, self.ids, self.mean2d, self.conic,
                             opacity, weights, self.coef, self.final_T, self.last)

    def decode(self, dictionary, compute=LS2_BF16, out_dtype=torch.bfloat16):
        m = self.levels * self.H * self.W
        if self.feat is None or self.feat.dtype != out_dtype:
            self.feat = torch.empty((self.levels, self.H, self.W, self.D), dtype=out_dtype, device=self.device)
        _lib.ls2_dict_decode(self.coef.view(m, self.L), dictionary, self.feat.view(m, self.D), compute)
        return self.feat

    def query(self, pos, neg, tau: float = 1.0):
        if self.relevancy is None:
            self.relevancy = torch.empty((self.levels, self.H, self.W), dtype=torch.float32, device=self.device)
        _lib.ls2_query(self.feat, pos, neg, self.relevancy, tau)
        return self.relevancy

    def decode_query(self, dictionary, pos, neg, tau: float = 1.0, keep_feat: bool = True):
        """bf16 decode and relevancy in one pass (the relevancy is formed while
        each tile of F is on chip); with keep_feat=False the feature map is not
        written at all."""
        m = self.levels * self.H * self.W
        if self.relevancy is None:
            self.relevancy = torch.empty((self.levels, self.H, self.W), dtype=torch.float32, device=self.device)
        feat = None
        if keep_feat:
            if self.feat is None or self.feat.dtype != torch.bfloat16:
                self.feat = torch.empty((self.levels, self.H, self.W, self.D), dtype=torch.bfloat16,
                                        device=self.device)
            feat = self.feat.view(m, self.D)
        _lib.ls2_dict_decode_query(self.coef.view(m, self.L), dictionary, pos, neg, self.relevancy.view(m), feat, tau)
        return self.relevancy

    def query_coef(self, dictionary, pos, neg, tau: float = 1.0):
        """Relevancy straight from the coefficient map (Eq. 7), no feature map."""
        if self.relevancy is None:
            self.relevancy = torch.empty((self.levels, self.H, self.W), dtype=torch.float32, device=self.device)
        if self.coef.dtype != torch.float32:
            raise ValueError("query_coef needs the float32 coefficient map (Pipeline(coef_dtype=torch.float32))")
        n_neg = neg.numel() // self.D
        key = (self.L, n_neg)
        if getattr(self, "_qc_key", None) != key:
            self._qc_ws = torch.empty((_lib.ls2_query_coef_workspace(self.L, n_neg),), dtype=torch.uint8,
                                      device=self.device)
            self._qc_key = key
        m = self.levels * self.H * self.W
        _lib.ls2_query_coef(self.coef.view(m, self.L), dictionary, pos, neg, self.relevancy.view(m), self._qc_ws, tau)
        return self.relevancy

    def feature_map(self, means, scales, quats, opacity, topk_idx, topk_w, dictionary, compute=LS2_BF16,
                    out_dtype=torch.bfloat16, sync: bool = True, fused: bool = False):
        """One feature-map frame: project, bin and sort, splat, decode (with
        fused=True: bf16 compute and output, projection and binning in one
        call, splat and decode in one pass)."""
        if fused:
            if compute != LS2_BF16 or out_dtype != torch.bfloat16:
                raise ValueError("the fused frame computes and writes bfloat16")
            self.project_bin_sort(means, scales, quats, sync=sync)
            return self.splat_decode(opacity, topk_idx, topk_w, dictionary)
        self.project(means, scales, quats)
        self.bin_sort(sync=sync)
        self.splat(opacity, topk_idx, topk_w)
        return self.decode(dictionary, compute, out_dtype)


class Gradients:
    """Gradient buffers of one scene size (all float32, overwritten per step)."""

    def __init__(self, n, levels, K, L, D, H, W, device):
        f32 = torch.float32
        self.coef = torch.empty((levels, H, W, L), dtype=f32, device=device)      # dL/dcoef
        self.dictionary = torch.empty((L, D), dtype=f32, device=device)
        self.mean2d = torch.empty((n, 2), dtype=f32, device=device)
        self.conic = torch.empty((n, 3), dtype=f32, device=device)
        self.opacity = torch.empty((n,), dtype=f32, device=device)
        self.topk_w = torch.empty((n, levels, K), dtype=f32, device=device)
        self.means = torch.empty((n, 3), dtype=f32, device=device)
        self.scales = torch.empty((n, 3), dtype=f32, device=device)
        self.quats = torch.empty((n, 4), dtype=f32, device=device)


class ForwardState:
    """What the backward of one forward frame reads: the camera, the tile
    lists, the projected Gaussians and the compositing state (coefficient
    map, final T and the position of each pixel's last contributor).  Either
    views of a trainer's buffers (valid until its next frame) or a copy that
    stays valid whatever the trainer renders afterwards."""

    FIELDS = ("coef", "tile_ranges", "ids", "final_T", "last", "mean2d", "conic", "radius")

    def __init__(self, cam, **tensors):
        self.cam = type(cam).from_buffer_copy(cam)
        for k in self.FIELDS:
            setattr(self, k, tensors[k])

    def copy(self):
        return ForwardState(self.cam, **{k: getattr(self, k).clone() for k in self.FIELDS})


class Trainer(Pipeline):
    """Forward + backward of the feature-map objective (float32 throughout):
    project -> bin_sort -> splat -> decode -> feature loss, then
    decode_backward -> splat_backward -> project_backward.  With codes given
    as logits (Section 3.3), ls2_sparse_codes forms the K (index, weight)
    pairs first and ls2_sparse_codes_backward closes the chain."""

    def __init__(self, cam, n, levels=1, K=4, L=64, D=512, max_pairs=None, device="cuda"):
        super().__init__(cam, n, levels, K, L, D, max_pairs, device)
        m = levels * self.H * self.W
        dev = self.device
        self.grad = Gradients(n, levels, K, L, D, self.H, self.W, dev)
        self.d_feat = torch.empty((levels, self.H, self.W, D), dtype=torch.float32, device=dev)
        self.loss = torch.zeros((1,), dtype=torch.float64, device=dev)
        self.loss_ws = torch.empty((_lib.ls2_feature_loss_workspace(m),), dtype=torch.uint8, device=dev)
        self.dec_ws = torch.empty((max(1, _lib.ls2_dict_decode_backward_workspace(m, L, D)),), dtype=torch.uint8,
                                  device=dev)
        # decode fused with the loss where the kernel exists (L <= 64, D <= 512)
        self.fused_loss = L in (32, 64) and D % 128 == 0 and D <= 512
        if self.fused_loss:
            self.fused_ws = torch.empty((_lib.ls2_decode_feature_loss_workspace(m, D),), dtype=torch.uint8,
                                        device=dev)
            # decode + loss + decode backward in one pass (step(): dL/dF stays on chip)
            self.onepass_ws = torch.empty((_lib.ls2_decode_loss_backward_workspace(m, L, D),), dtype=torch.uint8,
                                          device=dev)
        self.topk_idx = None   # codes formed from logits (codes())
        self.topk_w = None
        self.d_logits = None

    def state(self) -> ForwardState:
        """The forward state of the last frame, as views of this trainer's
        buffers (``.copy()`` keeps it past the next frame)."""
        P = self.num_pairs if self.num_pairs is not None else self.max_pairs
        return ForwardState(self.cam, coef=self.coef, tile_ranges=self.tile_ranges, ids=self.ids[:max(P, 1)],
                            final_T=self.final_T, last=self.last, mean2d=self.mean2d, conic=self.conic,
                            radius=self.radius)

    def codes(self, logits):
        """Sparse codes of logits [n, levels, L] (softmax, top K, renormalise):
        (topk_idx, topk_w) in this trainer's buffers."""
        if self.topk_idx is None:
            shape = (self.n, self.levels, self.K)
            self.topk_idx = torch.empty(shape, dtype=torch.int32, device=self.device)
            self.topk_w = torch.empty(shape, dtype=torch.float32, device=self.device)
        _lib.ls2_sparse_codes(logits, self.K, self.topk_idx, self.topk_w)
        return self.topk_idx, self.topk_w

    def decode_loss(self, dictionary, target, keep_feat=False):
        """Float32 decode + loss + dL/dF; the feature map is kept only if asked."""
        m = self.levels * self.H * self.W
        if self.fused_loss:
            feat = None
            if keep_feat:
                if self.feat is None or self.feat.dtype != torch.float32:
                    self.feat = torch.empty((self.levels, self.H, self.W, self.D), dtype=torch.float32,
                                            device=self.device)
                feat = self.feat.view(m, self.D)
            _lib.ls2_decode_feature_loss(self.coef.view(m, self.L), dictionary, target.view(m, self.D), self.loss,
                                         self.d_feat.view(m, self.D), self.fused_ws, feat)
        else:
            self.decode(dictionary, LS2_F32, torch.float32)
            _lib.ls2_feature_loss(self.feat, target, self.loss, self.d_feat, self.loss_ws)
        return self.loss

    def forward_loss(self, scene, target, sync=True, keep_feat=False):
        """Renders the scene and evaluates the loss and dL/dF (float32).  A
        scene with "logits" [n, levels, L] instead of topk_idx / topk_w gets
        its codes from them first."""
        if "logits" in scene:
            scene["topk_idx"], scene["topk_w"] = self.codes(scene["logits"])
        self.project(scene["means"], scene["scales"], scene["quats"])
        self.bin_sort(sync=sync)
        self.splat(scene["opacity"], scene["topk_idx"], scene["topk_w"])
        return self.decode_loss(scene["dictionary"], target, keep_feat=keep_feat)

    def backward(self, scene, d_feat=None, state: ForwardState | None = None):
        """Gradients of the loss (or of any dL/dF given as d_feat) with
        respect to every differentiable input, into ``self.grad``; ``state``
        is the forward frame to differentiate (default: the last one).  A
        scene with "logits" also gets dL/dlogits (``self.d_logits``)."""
        g = self.grad
        st = self.state() if state is None else state
        m = self.levels * self.H * self.W
        G = (self.d_feat if d_feat is None else d_feat).view(m, self.D)
        _lib.ls2_dict_decode_backward(st.coef.view(m, self.L), scene["dictionary"], G, g.coef.view(m, self.L),
                                      g.dictionary, self.dec_ws)
        return self._backward_render(scene, st)

    def _backward_render(self, scene, st):
        """splat, projection (and code) backward from g.coef = dL/dcoef."""
        g = self.grad
        _lib.ls2_splat_sparse_backward(st.cam, self.levels, self.K, self.L, st.tile_ranges, st.ids,
                                       st.mean2d, st.conic, scene["opacity"], scene["topk_idx"],
                                       scene["topk_w"], st.final_T, st.last, g.coef, g.mean2d, g.conic,
                                       g.opacity, g.topk_w)
        _lib.ls2_project_backward(st.cam, scene["means"], scene["scales"], scene["quats"], st.radius, g.mean2d,
                                  g.conic, g.means, g.scales, g.quats)
        if "logits" in scene:
            if self.d_logits is None:
                self.d_logits = torch.empty((self.n, self.levels, self.L), dtype=torch.float32, device=self.device)
            _lib.ls2_sparse_codes_backward(scene["topk_idx"], scene["topk_w"], g.topk_w, self.d_logits)
        return g

    def set_camera(self, cam):
        """Switch to another view of the same image size (buffers are reused)."""
        c = _lib.make_camera(cam)
        if (c.width, c.height) != (self.W, self.H):
            raise ValueError("set_camera: image size differs from the trainer's buffers")
        self.cam = c

    def accumulate_into(self, total):
        """total.<name> += self.grad.<name> for every gradient buffer (a
        ``Gradients`` of the same shapes), e.g. over the views of a step."""
        for name in ("dictionary", "means", "scales", "quats", "opacity", "topk_w"):
            _lib.ls2_accumulate(getattr(self.grad, name), getattr(total, name))

    def step(self, scene, target, sync=True):
        """One training step: the loss and every gradient (into ``self.grad``).
        Where the one-pass kernel exists (L <= 64, D <= 512) the decode, the
        loss and the decode gradients are formed together and dL/dF is not
        materialised (``self.d_feat`` is then not updated)."""
        if not self.fused_loss:
            loss = self.forward_loss(scene, target, sync=sync)
            return loss, self.backward(scene)
        if "logits" in scene:
            scene["topk_idx"], scene["topk_w"] = self.codes(scene["logits"])
        self.project_bin_sort(scene["means"], scene["scales"], scene["quats"], sync=sync)
        self.splat(scene["opacity"], scene["topk_idx"], scene["topk_w"])
        m = self.levels * self.H * self.W
        g = self.grad
        _lib.ls2_decode_loss_backward(self.coef.view(m, self.L), scene["dictionary"], target.view(m, self.D),
                                      self.loss, g.coef.view(m, self.L), g.dictionary, self.onepass_ws)
        return self.loss, self._backward_render(scene, self.state())


def _render_forward(ctx, trainer, scene):
    feat = trainer.feature_map(scene["means"], scene["scales"], scene["quats"], scene["opacity"],
                               scene["topk_idx"], scene["topk_w"], scene["dictionary"], compute=LS2_F32,
                               out_dtype=torch.float32)
    # the backward differentiates this frame even if the trainer renders
    # other views (or other scenes) before it runs
    ctx.trainer = trainer
    ctx.state = trainer.state().copy()
    ctx.scene = scene
    return feat.clone()


class LS2Render(torch.autograd.Function):
    """Differentiable feature map F (float32, [levels, H, W, D]) of a scene,
    with the hand-written HIP backward.  ``trainer`` supplies the buffers;
    each call keeps its own copy of the forward state, so several frames
    (views) may be rendered before one backward.  topk_idx is discrete and
    carries no gradient."""

    @staticmethod
    def forward(ctx, trainer, means, scales, quats, opacity, topk_idx, topk_w, dictionary):
        scene = dict(means=means.contiguous(), scales=scales.contiguous(), quats=quats.contiguous(),
                     opacity=opacity.contiguous(), topk_idx=topk_idx.contiguous(), topk_w=topk_w.contiguous(),
                     dictionary=dictionary.contiguous())
        return _render_forward(ctx, trainer, scene)

    @staticmethod
    def backward(ctx, d_feat):
        g = ctx.trainer.backward(ctx.scene, d_feat.contiguous(), state=ctx.state)
        return (None, g.means.clone(), g.scales.clone(), g.quats.clone(), g.opacity.clone(), None,
                g.topk_w.clone(), g.dictionary.clone())


class LS2RenderLogits(torch.autograd.Function):
    """LS2Render with the codes given as logits [n, levels, L] (Section 3.3:
    softmax, top K, renormalise, learned jointly with the codebook): the
    gradient reaches the logits through ls2_sparse_codes_backward."""

    @staticmethod
    def forward(ctx, trainer, means, scales, quats, opacity, logits, dictionary):
        idx, w = trainer.codes(logits.contiguous())
        scene = dict(means=means.contiguous(), scales=scales.contiguous(), quats=quats.contiguous(),
                     opacity=opacity.contiguous(), topk_idx=idx.clone(), topk_w=w.clone(),
                     dictionary=dictionary.contiguous(), logits=logits)
        return _render_forward(ctx, trainer, scene)

    @staticmethod
    def backward(ctx, d_feat):
        tr = ctx.trainer
        g = tr.backward(ctx.scene, d_feat.contiguous(), state=ctx.state)
        return (None, g.means.clone(), g.scales.clone(), g.quats.clone(), g.opacity.clone(), tr.d_logits.clone(),
                g.dictionary.clone())


def to_device(scene, device="cuda"):
    """Scene arrays (numpy, from ``gen``) as contiguous device tensors."""
    t = lambda a, dt: torch.from_numpy(a).to(device=device, dtype=dt).contiguous()  # noqa: E731
    return dict(means=t(scene.means, torch.float32), scales=t(scene.scales, torch.float32),
                quats=t(scene.quats, torch.float32), opacity=t(scene.opacity, torch.float32),
                topk_idx=t(scene.topk_idx, torch.int32), topk_w=t(scene.topk_w, torch.float32),
                dictionary=t(scene.dictionary, torch.float32))


__all__ = ["Pipeline", "Trainer", "Gradients", "ForwardState", "LS2Render", "LS2RenderLogits", "to_device",
           "LS2_F32", "LS2_BF16"]
