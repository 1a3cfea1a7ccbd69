"""torch.autograd.Function over the HIP rasterizer (forward and the reverse-order adjoint).

PyTorch supplies device memory and the current stream; the forward calls
ges_preprocess + ges_render_forward, the backward ges_render_backward.
"""
from __future__ import annotations

import torch

from . import ges as G


class GESRasterize(torch.autograd.Function):
    """image = GESRasterize.apply(means, log_scales, quats, opacity_logits, sh, beta, cam, settings)

    settings: dict(falloff, tile_cull, rho, bg).  Gradients are returned for the six splat tensors.
    """

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, beta, cam, settings):
        tensors = [t.contiguous() for t in (means, log_scales, quats, opacity_logits, sh, beta)]
        s = G.splats_struct(*tensors)
        c = G.camera_struct(cam)
        p = G.params_struct(settings.get("falloff", G.FALLOFF_PHI), settings.get("tile_cull", G.TILES_SQUARE),
                            settings.get("rho", 0.1), settings.get("bg", (0.0, 0.0, 0.0)))
        frame = settings.get("frame")
        if frame is None or frame.n != s.n or frame.width != c.width or frame.height != c.height:
            frame = G.Frame.create(s.n, c.width, c.height, means.device)
        k = G.ges_preprocess(s, c, p, frame.splat_ws, True)
        frame.ensure_keys(k)
        out = torch.empty((c.height, c.width, 3), dtype=torch.float32, device=means.device)
        G.ges_render_forward(s, c, p, frame.splat_ws, frame.key_ws, k, frame.pixel_ws, out)
        ctx.frame, ctx.structs, ctx.tensors = frame, (s, c, p), tensors
        ctx.save_for_backward(*tensors)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        means, log_scales, quats, opacity_logits, sh, beta = ctx.saved_tensors
        s, c, p = ctx.structs
        grads = {"means": torch.empty_like(means), "log_scales": torch.empty_like(log_scales),
                 "quats": torch.empty_like(quats), "opacity_logits": torch.empty_like(opacity_logits),
                 "sh": torch.empty_like(sh), "beta": torch.empty_like(beta)}
        G.ges_render_backward(s, c, p, ctx.frame.splat_ws, ctx.frame.key_ws, ctx.frame.pixel_ws,
                              grad_out.contiguous(), grads)
        return (grads["means"], grads["log_scales"], grads["quats"], grads["opacity_logits"], grads["sh"],
                grads["beta"], None, None)


def rasterize(scene: dict, cam, **settings):
    return GESRasterize.apply(scene["means"], scene["log_scales"], scene["quats"], scene["opacity_logits"],
                              scene["sh"], scene["beta"], cam, settings)
