"""Differentiable binary64 preprocess written with plain PyTorch CPU ops.

TEST INFRASTRUCTURE ONLY.  It restates, vectorised over splats, the per-splat
preprocess of the C++ oracle's F64 mode (GES, arXiv 2402.10128):

* scale s = exp(log-scale); opacity o = sigmoid(logit);
* unit quaternion -> rotation R; Sigma = (R S)(R S)^T with S = diag(phi * s) where
  phi = 2 / (1 + exp(-(rho beta - 2 rho))) in the PHI falloff (Sec. 4.2, Eq. approx),
  phi = 2 Gamma(3/beta) / Gamma(1/beta) in the PHI_EXACT variant (Eq. probablity, normalised to 1 at
  beta = 2; Gaussian falloff) and phi = 1 in the GEF falloff (Eq. ges);
* EWA (Sec. 4.1): Sigma' = J W Sigma W^T J^T + 0.3 I with W the camera rotation and
  J the perspective Jacobian at the camera-space mean (guard-clamped x/z, y/z);
* conic = inverse of Sigma'; mean2D = (fx x/z + cx, fy y/z + cy);
* colour = sum of real SH (degree <= 3) at the unit view direction + 0.5, clamped at 0.

Autograd through it gives the chain rule from the 2-D splat quantities to the
parameters.  Decisions (guard clamp, colour clamp, visibility) are taken from a
record passed in, so the derivative is the one of the branch the renderer took.
"""
from __future__ import annotations

import math

import numpy as np
import torch

PI = math.pi
C0 = 0.5 * math.sqrt(1.0 / PI)
C1 = 0.5 * math.sqrt(3.0 / PI)
C2A = 0.5 * math.sqrt(15.0 / PI)
C2B = 0.25 * math.sqrt(5.0 / PI)
C2C = 0.25 * math.sqrt(15.0 / PI)
C3A = 0.25 * math.sqrt(35.0 / (2.0 * PI))
C3B = 0.5 * math.sqrt(105.0 / PI)
C3C = 0.25 * math.sqrt(21.0 / (2.0 * PI))
C3D = 0.25 * math.sqrt(7.0 / PI)
C3E = 0.25 * math.sqrt(105.0 / PI)


def sh_basis(d: torch.Tensor, degree: int) -> torch.Tensor:
    """Real SH with Condon-Shortley phase at unit directions d [n,3] -> [n,(degree+1)^2]."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    Y = [torch.full_like(x, C0)]
    if degree >= 1:
        Y += [-C1 * y, C1 * z, -C1 * x]
    if degree >= 2:
        xx, yy, zz = x * x, y * y, z * z
        Y += [C2A * x * y, -C2A * y * z, C2B * (2 * zz - xx - yy), -C2A * x * z, C2C * (xx - yy)]
    if degree >= 3:
        Y += [-C3A * y * (3 * xx - yy), C3B * x * y * z, -C3C * y * (4 * zz - xx - yy),
              C3D * z * (2 * zz - 3 * xx - 3 * yy), -C3C * x * (4 * zz - xx - yy), C3E * z * (xx - yy),
              -C3A * x * (xx - 3 * yy)]
    return torch.stack(Y, dim=1)


def quat_to_rot(q: torch.Tensor) -> torch.Tensor:
    q = q / torch.linalg.norm(q, dim=1, keepdim=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], dim=1)
    return R.reshape(-1, 3, 3)


def preprocess(params: dict, sh_degree: int, cam, falloff: int = 0, rho: float = 0.1,
               clamp_bits: np.ndarray | None = None) -> dict:
    """params: float64 tensors means [n,3], log_scales [n,3], quats [n,4], opacity_logits [n], sh [n,K,3],
    beta [n].  Returns u, v, depth, conic a/b/c, qmax, opacity, rgb [n,3], beta."""
    mu = params["means"]
    Rv = torch.as_tensor(np.asarray(cam.R, np.float32).astype(np.float64)).reshape(3, 3)
    tv = torch.as_tensor(np.asarray(cam.t, np.float32).astype(np.float64))
    fx, fy = float(np.float32(cam.fx)), float(np.float32(cam.fy))
    cx, cy = float(np.float32(cam.cx)), float(np.float32(cam.cy))
    p = mu @ Rv.T + tv
    z = p[:, 2]
    s = torch.exp(params["log_scales"])
    o = torch.sigmoid(params["opacity_logits"])
    beta = params["beta"]
    rho = float(np.float32(rho))          # the renderer receives rho as binary32
    if falloff == 0:
        phi = 2.0 / (1.0 + torch.exp(-(rho * beta - 2.0 * rho)))
    elif falloff == 2:
        # exact modification 2 Gamma(3/beta) / Gamma(1/beta) (Eq. probablity, normalised to 1 at beta = 2)
        phi = 2.0 * torch.exp(torch.lgamma(3.0 / beta) - torch.lgamma(1.0 / beta))
    else:
        phi = torch.ones_like(beta)
    Rq = quat_to_rot(params["quats"])
    Mm = Rq * (phi[:, None] * s)[:, None, :]
    Sig = Mm @ Mm.transpose(1, 2)
    limx = 1.3 * (0.5 * cam.width / fx)
    limy = 1.3 * (0.5 * cam.height / fy)
    txz, tyz = p[:, 0] / z, p[:, 1] / z
    if clamp_bits is None:
        txz = torch.clamp(txz, -limx, limx)
        tyz = torch.clamp(tyz, -limy, limy)
    else:
        cb = torch.as_tensor(clamp_bits.astype(np.int64))
        cxm, cym = (cb & 8) != 0, (cb & 16) != 0
        txz = torch.where(cxm, torch.clamp(txz, -limx, limx).detach(), txz)
        tyz = torch.where(cym, torch.clamp(tyz, -limy, limy).detach(), tyz)
    xc, yc = txz * z, tyz * z
    zero = torch.zeros_like(z)
    J = torch.stack([fx / z, zero, -fx * xc / (z * z), zero, fy / z, -fy * yc / (z * z)], dim=1).reshape(-1, 2, 3)
    T = J @ Rv
    cov = T @ Sig @ T.transpose(1, 2)
    c00 = cov[:, 0, 0] + 0.3
    c01 = cov[:, 0, 1]
    c11 = cov[:, 1, 1] + 0.3
    det = c00 * c11 - c01 * c01
    a, b, c = c11 / det, -c01 / det, c00 / det
    u = fx * p[:, 0] / z + cx
    v = fy * p[:, 1] / z + cy
    L2 = 2.0 * torch.log(255.0 * o)
    qmax = L2 if falloff != 1 else torch.exp((2.0 / beta) * torch.log(L2))
    # colour
    Rnp = np.asarray(cam.R, np.float32).astype(np.float64).reshape(3, 3)
    campos = torch.as_tensor(-Rnp.T @ np.asarray(cam.t, np.float32).astype(np.float64))
    d = mu - campos
    d = d / torch.linalg.norm(d, dim=1, keepdim=True)
    Y = sh_basis(d, sh_degree)
    rgb = torch.einsum("nk,nkc->nc", Y, params["sh"]) + 0.5
    if clamp_bits is None:
        rgb = torch.clamp(rgb, min=0.0)
    else:
        cb = torch.as_tensor(clamp_bits.astype(np.int64))
        mask = torch.stack([(cb >> k) & 1 for k in range(3)], dim=1) != 0
        rgb = torch.where(mask, torch.zeros_like(rgb), rgb)
    return dict(u=u, v=v, depth=z, a=a, b=b, c=c, qmax=qmax, opacity=o, rgb=rgb, beta=beta)


def to_params(arrays: dict, requires_grad: bool = False) -> dict:
    out = {}
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "beta"):
        t = torch.as_tensor(np.asarray(arrays[k], dtype=np.float64)).clone()
        t.requires_grad_(requires_grad)
        out[k] = t
    return out


def chain_to_params(arrays: dict, sh_degree: int, cam, g2d: np.ndarray, visible: np.ndarray, clamp_bits,
                    falloff: int = 0, rho: float = 0.1) -> dict:
    """Backpropagate per-splat 2-D gradients g2d [n,10] = d/d(u,v,a,b,c,o,r,g,b,beta) to the parameters."""
    P = to_params(arrays, requires_grad=True)
    out = preprocess(P, sh_degree, cam, falloff, rho, clamp_bits)
    g = torch.as_tensor(g2d) * torch.as_tensor(visible.astype(np.float64))[:, None]
    cols = [out["u"], out["v"], out["a"], out["b"], out["c"], out["opacity"], out["rgb"][:, 0], out["rgb"][:, 1],
            out["rgb"][:, 2]]
    total = sum((g[:, k] * torch.nan_to_num(cols[k])).sum() for k in range(9))
    if falloff == 1:
        total = total + (g[:, 9] * out["beta"]).sum()
    grads = torch.autograd.grad(total, [P[k] for k in P], allow_unused=True)
    res = {}
    for k, gr in zip(P, grads):
        res[k] = np.zeros(P[k].shape) if gr is None else gr.detach().numpy()
        # culled splats get exactly zero gradient
        res[k][~visible.astype(bool)] = 0.0
    return res


def abs_chain(arrays: dict, sh_degree: int, cam, a2d: np.ndarray, visible: np.ndarray, clamp_bits,
              falloff: int = 0, rho: float = 0.1) -> dict:
    """|J|^T a per splat: the bound on how far parameter gradients can move when each 2-D gradient
    component k of a splat is uncertain by a2d[:, k] >= 0.  Splats are independent, so one backward
    pass per 2-D component (unit weight on that component of every splat) yields every splat's
    Jacobian row for that component."""
    P = to_params(arrays, requires_grad=True)
    out = preprocess(P, sh_degree, cam, falloff, rho, clamp_bits)
    cols = [out["u"], out["v"], out["a"], out["b"], out["c"], out["opacity"], out["rgb"][:, 0], out["rgb"][:, 1],
            out["rgb"][:, 2], out["beta"]]
    vis = torch.as_tensor(visible.astype(np.float64))
    res = {k: np.zeros(P[k].shape) for k in P}
    ncol = 10 if falloff == 1 else 9
    for k in range(ncol):
        total = (torch.nan_to_num(cols[k]) * vis).sum()
        grads = torch.autograd.grad(total, [P[q] for q in P], retain_graph=True, allow_unused=True)
        w = a2d[:, k]
        for name, gr in zip(P, grads):
            if gr is None:
                continue
            J = np.abs(gr.detach().numpy())
            res[name] += J * w.reshape((-1,) + (1,) * (J.ndim - 1))
    for name in res:
        res[name][~visible.astype(bool)] = 0.0
    return res


def record_from(out: dict, base_record):
    """A binary64 record (for the C++ renderer) whose continuous fields come from ``out`` and whose
    decisions (visibility, rect, clamp bits) come from ``base_record``."""
    from .oracle import Record
    n = out["u"].shape[0]
    r = Record.empty(n)
    det = lambda t: t.detach().numpy().astype(np.float64)
    r.u[:], r.v[:], r.depth[:] = det(out["u"]), det(out["v"]), det(out["depth"])
    r.conic[:] = np.stack([det(out["a"]), det(out["b"]), det(out["c"])], axis=1)
    r.qmax[:], r.opacity[:] = det(out["qmax"]), det(out["opacity"])
    r.rgb[:] = det(out["rgb"])
    r.beta[:] = det(out["beta"])
    r.radius[:] = base_record.radius
    r.rect[:] = base_record.rect
    r.tiles_touched[:] = base_record.tiles_touched
    r.clamp_bits[:] = base_record.clamp_bits
    vis = base_record.tiles_touched > 0
    for arr in (r.u, r.v, r.depth, r.qmax, r.opacity, r.beta):
        arr[~vis] = 0.0
    r.conic[~vis] = 0.0
    r.rgb[~vis] = 0.0
    return r
