"""One GES optimisation step on the HIP library: frequency mask -> render -> loss -> adjoint -> Adam.

The step follows the paper's training recipe:
  * loss L = lambda_L1 L1 + lambda_ssim L_ssim + lambda_omega L_omega with lambda_ssim = 0.2,
    lambda_omega = 0.5 and lambda_L1 = 1 - lambda_ssim - lambda_omega (Sec. 4.4, Eq. final; App. B.2);
  * the frequency mask M_omega at omega = iteration / total iterations (Sec. 4.3, linear schedule),
    40,000 iterations in all (App. B.2);
  * Adam with per-group learning rates, the position rate decaying log-linearly from 1.6e-4 to 1.6e-6
    over 30,000 steps (App. B.2).
Every stage runs in the library's kernels; this module only owns buffers and orders the calls on one stream.
By default the Adam update runs inside the backward pass (ges_render_backward_adam), so the parameter
gradients never go through memory.  Several views of one step are rendered and back-propagated through one
launch sequence (the ..._views calls; batch_views=False renders them one after another, with the same bits).
The loss schedule (omega and lambda_L1) comes from the library (ges_loss_schedule).
After the update, every shape_prune_interval iterations the splats whose opacity is below min_opacity or
whose beta is below min_beta are removed with their moments, and every shape_reset_interval iterations every
beta goes back to 2 (Sec. 4.4; Sec. 5.2; App. B.2: intervals 100 and 1,000).  When both fall on one
iteration, pruning comes first, so it sees the learned shapes.
Densification kept from Gaussian splatting (Sec. 5.2; App. B.2): until densify_until the backward pass
accumulates each visible splat's NDC mean-2D gradient norm; after densify_from, every densify_interval
iterations splats whose mean statistic reaches grad_threshold are cloned (small) or split in two (large,
relative to percent_dense * scene_extent), with normal draws from a seeded device generator, before the
pruning; every opacity_reset_interval iterations every opacity is capped at 0.01.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import ges as G

GROUP_ORDER = ("means", "sh", "opacity_logits", "beta", "quats", "log_scales")


@dataclass
class TrainConfig:
    total_iterations: int = 40000
    lam_ssim: float = 0.2
    lam_omega: float = 0.5
    lr_pos_init: float = 0.00016
    lr_pos_final: float = 0.0000016
    lr_pos_max_steps: int = 30000
    lr_pos_scale: float = 1.0              # scene extent multiplier of the position rates
    lr_feature: float = 0.0025
    lr_opacity: float = 0.05
    lr_shape: float = 0.001
    lr_rotation: float = 0.001
    lr_scaling: float = 0.005
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15
    shape_prune_interval: int = 100        # 0 switches pruning off
    shape_reset_interval: int = 1000       # 0 switches the reset off
    min_opacity: float = 0.005
    min_beta: float = 0.5                  # Sec. 5.2 (App. B.2 gives 0.005)
    beta_init: float = 2.0
    densify_from: int = 500
    densify_until: int = 15000
    densify_interval: int = 100            # 0 switches densification off
    grad_threshold: float = 0.0003
    percent_dense: float = 0.01
    scene_extent: float = 1.0
    opacity_reset_interval: int = 3000     # 0 switches the reset off
    seed: int = 0
    falloff: int = G.FALLOFF_PHI
    tile_cull: int = G.TILES_ELLIPSE
    rho: float = 0.1
    bg: tuple = (0.0, 0.0, 0.0)
    batch_views: bool = True               # the views of a step share one launch sequence


class TrainStep:
    """Owns the workspaces of training one scene against one view; ``step(it)`` updates the scene in place.

    scene: dict of contiguous float32 CUDA tensors (means, log_scales, quats, opacity_logits, sh, beta).
    """

    def __init__(self, scene: dict, cam, target, cfg: TrainConfig | None = None):
        """cam, target: one view, or equal-sized lists of views of one resolution trained together: the loss is
        the mean over the views, their gradients are summed (view order) before one update."""
        self.cfg = cfg or TrainConfig()
        self.scene = scene
        self.cams = list(cam) if isinstance(cam, (list, tuple)) else [cam]
        self.targets = [t.contiguous() for t in (target if isinstance(target, (list, tuple)) else [target])]
        if len(self.cams) != len(self.targets) or not self.cams:
            raise ValueError("one target per camera")
        if any((c.width, c.height) != (self.cams[0].width, self.cams[0].height) for c in self.cams):
            raise ValueError("the views of one step share a resolution")
        self.cam, self.target = self.cams[0], self.targets[0]
        dev = self.target.device
        self.cstructs = [G.camera_struct(c) for c in self.cams]
        self.c = self.cstructs[0]
        self.p = G.params_struct(self.cfg.falloff, self.cfg.tile_cull, self.cfg.rho, self.cfg.bg)
        H, W = self.cam.height, self.cam.width
        B = len(self.cams)
        self.batched = self.cfg.batch_views and B > 1
        self._bind_scene()
        # per view: rendered image, dL/dimage and frequency mask ([B, ...]; image / dL / mask are view 0's)
        self.images = torch.empty((B, H, W, 3), dtype=torch.float32, device=dev)
        self.dLs = torch.empty_like(self.images)
        self.masks = torch.empty((B, H, W), dtype=torch.uint8, device=dev)
        self.image, self.dL, self.mask = self.images[0], self.dLs[0], self.masks[0]
        self.view_loss = torch.empty(B, dtype=torch.float32, device=dev)
        self.loss = self.view_loss[0]
        self.mask_scratch = torch.empty(G.lib().ges_mask_scratch_bytes(W, H), dtype=torch.uint8, device=dev)
        self.loss_scratch = torch.empty(G.lib().ges_loss_scratch_bytes(), dtype=torch.uint8, device=dev)
        self.ssim_scratch = torch.empty(G.lib().ges_ssim_scratch_bytes(W, H), dtype=torch.uint8, device=dev)
        self.grads = None        # parameter gradients, allocated by the first unfused step
        self.exp_avg = {k: torch.zeros_like(v) for k, v in scene.items()}
        self.exp_avg_sq = {k: torch.zeros_like(v) for k, v in scene.items()}
        self.gen = torch.Generator(device=dev).manual_seed(self.cfg.seed)
        self._reset_stats()

    def _bind_scene(self):
        """Point the splat descriptor and the frame at the current scene tensors (after creation or pruning)."""
        self.s = G.splats_struct(*(self.scene[k] for k in G.SPLAT_PARAMS))
        self.frame = G.Frame.create(self.s.n, self.cam.width, self.cam.height, self.target.device,
                                    views=len(self.cams) if self.batched else 1)
        self.grads = None
        self.keys_known = False  # a new frame has no key workspace: its first step reads the key count back

    def _reset_stats(self):
        self.grad_accum = torch.zeros(self.n, dtype=torch.float32, device=self.target.device)
        self.grad_count = torch.zeros(self.n, dtype=torch.float32, device=self.target.device)

    def check_keys(self):
        """Raise if a step rendered with a key capacity below its slot count (the overflowing pairs were
        dropped, so that step's image and gradients are incomplete).  Waits for the stream."""
        ws = self.frame.splat_ws
        for v in range(self.frame.views):
            off = self.frame.view(v).stats - ws.data_ptr()
            if int(ws[off:off + 32].view(torch.int64)[1].cpu()) & 1:
                raise RuntimeError("key capacity too small for a step rendered without reading the key count back "
                                   "(its image and gradients miss the dropped pairs)")

    def densify(self) -> int:
        """Clone or split the splats whose mean statistic reaches the threshold; returns the new count.  The
        scene, moments, statistics and frame are replaced (read ``self.scene`` afterwards)."""
        c = self.cfg
        n = self.n
        self.check_keys()
        normals = torch.randn((n, 2, 3), generator=self.gen, device=self.target.device)
        src = [self.scene, self.exp_avg, self.exp_avg_sq]
        dst = [{k: torch.empty((2 * n,) + tuple(v.shape[1:]), dtype=v.dtype, device=v.device) for k, v in d.items()}
               for d in src]
        out = G.ges_densify(src, dst, int(self.s.sh_degree), self.grad_accum, self.grad_count, normals,
                            c.grad_threshold, c.percent_dense * c.scene_extent)
        self.scene, self.exp_avg, self.exp_avg_sq = ({k: v[:out] for k, v in d.items()} for d in dst)
        self._bind_scene()
        self._reset_stats()
        return out

    def opacity_reset(self):
        G.ges_opacity_reset(self.scene["opacity_logits"], self.exp_avg["opacity_logits"],
                            self.exp_avg_sq["opacity_logits"], 0.01)

    @property
    def n(self) -> int:
        return int(self.s.n)

    def prune(self) -> int:
        """Remove the splats below the opacity or shape bound, with their moments; returns the new count.
        The scene, moment and frame tensors are replaced (read ``self.scene`` afterwards)."""
        c = self.cfg
        src = [self.scene, self.exp_avg, self.exp_avg_sq]
        dst = [{k: torch.empty_like(v) for k, v in d.items()} for d in src]
        sh_degree = int(self.s.sh_degree)
        self.check_keys()
        kept = G.ges_prune_splats(src, dst, sh_degree, c.min_opacity, c.min_beta)
        if kept == self.n:
            return kept
        # the statistics follow the survivors: a pruning between densifications keeps them aligned
        keep_stats = [{"opacity_logits": self.scene["opacity_logits"], "beta": self.scene["beta"]},
                      {"opacity_logits": self.grad_accum, "beta": self.grad_count}]
        new_stats = [{k: torch.empty_like(v) for k, v in d.items()} for d in keep_stats]
        G.ges_prune_splats(keep_stats, new_stats, sh_degree, c.min_opacity, c.min_beta)
        self.scene, self.exp_avg, self.exp_avg_sq = ({k: v[:kept] for k, v in d.items()} for d in dst)
        self._bind_scene()
        self.grad_accum = new_stats[1]["opacity_logits"][:kept].contiguous()
        self.grad_count = new_stats[1]["beta"][:kept].contiguous()
        return kept

    def shape_reset(self):
        G.ges_shape_reset(self.scene["beta"], self.exp_avg["beta"], self.exp_avg_sq["beta"], self.cfg.beta_init)

    def omega(self, it: int) -> float:
        return G.ges_loss_schedule(it, self.cfg.total_iterations, self.cfg.lam_ssim, self.cfg.lam_omega)[0]

    def learning_rates(self, it: int) -> dict:
        c = self.cfg
        pos = c.lr_pos_scale * G.ges_expon_lr(it, c.lr_pos_init, c.lr_pos_final, c.lr_pos_max_steps)
        return {"means": pos, "sh": c.lr_feature, "opacity_logits": c.lr_opacity, "beta": c.lr_shape,
                "quats": c.lr_rotation, "log_scales": c.lr_scaling}

    def step(self, it: int, read_num_keys: bool = True, fused: bool = True):
        """Iteration ``it`` (counting from 1).  With read_num_keys=False the render takes the key count from
        the device and the frame's key capacity must already hold it (an overflow is flagged in the frame and
        raised by check_keys, which densify and prune call); the first step on a new frame (after creation,
        densification or pruning) reads the count back regardless.  fused=True applies Adam inside the
        backward pass (the gradients are not stored); fused=False stores the gradients in ``self.grads`` and
        runs the stand-alone Adam step (the same bits)."""
        c = self.cfg
        _check = G._check
        L = G.lib()
        stream = G._stream(None)
        H, W = self.cam.height, self.cam.width
        B = len(self.cams)
        lrs = self.learning_rates(it)
        stats = c.densify_interval > 0 and it < c.densify_until
        acc = self.grad_accum if stats else None
        cnt = self.grad_count if stats else None
        if (B > 1 or not fused) and self.grads is None:
            self.grads = {k: torch.empty_like(v) for k, v in self.scene.items()}
        omega, lam_l1 = G.ges_loss_schedule(it, c.total_iterations, c.lam_ssim, c.lam_omega)
        read_num_keys = read_num_keys or not self.keys_known
        self.keys_known = True
        # the step's loss is the mean over the views: each view's terms carry 1/B
        lam_l1, lam_w, lam_s = lam_l1 / B, c.lam_omega / B, c.lam_ssim / B
        if self.batched:
            self._views_step(it, read_num_keys, fused, omega, lam_l1, lam_w, lam_s, lrs, acc, cnt, stream)
        for v in range(0 if self.batched else B):
            cs, target = self.cstructs[v], self.targets[v]
            self.mask, self.image, self.dL = self.masks[v], self.images[v], self.dLs[v]
            _check(L.ges_freq_mask(G._ptr(target), W, H, float(omega), G._ptr(self.mask_scratch),
                                   G._ptr(self.mask), stream))
            if read_num_keys:
                k = G.ges_preprocess(self.s, cs, self.p, self.frame.splat_ws, True)
                self.frame.ensure_keys(k)
            else:
                G.ges_preprocess(self.s, cs, self.p, self.frame.splat_ws, False)
                k = self.frame.key_capacity
            self.frame.num_keys = k
            G.ges_render_forward(self.s, cs, self.p, self.frame.splat_ws, self.frame.key_ws, k, self.frame.pixel_ws,
                                 self.image)
            loss_v = self.view_loss[v]
            G.ges_loss(self.image, target, self.mask, lam_l1, lam_w, self.dL, loss_v, self.loss_scratch)
            G.ges_ssim_loss(self.image, target, lam_s, loss_v, self.dL, self.ssim_scratch)
            ws = (self.s, cs, self.p, self.frame.splat_ws, self.frame.key_ws, self.frame.pixel_ws, self.dL)
            last = v == B - 1
            if fused and last:   # the last view's backward updates from the sum of every view's gradients
                G.ges_render_backward_adam(*ws, self.exp_avg, self.exp_avg_sq, lrs, it, c.beta1, c.beta2, c.eps,
                                           grad_accum=acc, grad_count=cnt, grads_in=self.grads if B > 1 else None)
            elif v == 0 and acc is None:
                G.ges_render_backward(*ws, self.grads)
            else:
                if v == 0:
                    for g in self.grads.values():
                        g.zero_()
                G.ges_render_backward_accumulate(*ws, self.grads, acc, cnt)
        if not fused:
            groups = [(self.scene[k], self.grads[k], self.exp_avg[k], self.exp_avg_sq[k], lrs[k])
                      for k in GROUP_ORDER]
            G.ges_adam_step(groups, it, c.beta1, c.beta2, c.eps)
        self.mask, self.image, self.dL = self.masks[0], self.images[0], self.dLs[0]
        self.loss = self.view_loss.sum() if B > 1 else self.view_loss[0]
        if stats and it > c.densify_from and it % c.densify_interval == 0:
            self.densify()
        if c.shape_prune_interval and it % c.shape_prune_interval == 0:
            self.prune()
        if c.shape_reset_interval and it % c.shape_reset_interval == 0:
            self.shape_reset()
        if c.opacity_reset_interval and it % c.opacity_reset_interval == 0:
            self.opacity_reset()
        return self.loss

    def _views_step(self, it, read_num_keys, fused, omega, lam_l1, lam_w, lam_s, lrs, acc, cnt, stream):
        """The step's views through one launch sequence: masks and losses per view, everything else batched."""
        c = self.cfg
        L = G.lib()
        H, W = self.cam.height, self.cam.width
        f = self.frame
        for v, target in enumerate(self.targets):
            G._check(L.ges_freq_mask(G._ptr(target), W, H, float(omega), G._ptr(self.mask_scratch),
                                     G._ptr(self.masks[v]), stream))
        if read_num_keys:
            k = G.ges_preprocess_views(self.s, self.cstructs, self.p, f.splat_ws, True)
            f.ensure_keys(k)
        else:
            G.ges_preprocess_views(self.s, self.cstructs, self.p, f.splat_ws, False)
            k = f.key_capacity
        f.num_keys = k
        G.ges_render_forward_views(self.s, self.cstructs, self.p, f.splat_ws, f.key_ws, k, f.pixel_ws, self.images)
        for v, target in enumerate(self.targets):
            loss_v = self.view_loss[v]
            G.ges_loss(self.images[v], target, self.masks[v], lam_l1, lam_w, self.dLs[v], loss_v, self.loss_scratch)
            G.ges_ssim_loss(self.images[v], target, lam_s, loss_v, self.dLs[v], self.ssim_scratch)
        ws = (self.s, self.cstructs, self.p, f.splat_ws, f.key_ws, f.pixel_ws, self.dLs)
        if fused:
            G.ges_render_backward_views_adam(*ws, self.exp_avg, self.exp_avg_sq, lrs, it, c.beta1, c.beta2, c.eps,
                                             grads=self.grads, grad_accum=acc, grad_count=cnt)
        else:
            G.ges_render_backward_views(*ws, self.grads, False, acc, cnt)
