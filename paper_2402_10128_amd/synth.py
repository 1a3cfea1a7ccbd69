"""Seeded synthetic GES scenes and cameras.

This module only draws random inputs and builds pinhole cameras; it holds none
of the rendering arithmetic.  Both the HIP path and the CPU oracle consume what
it produces, so every array is float32 and C-contiguous.

Scene recipes (all parameters in the form the paper states the problem in,
Sec. 4.1: position, log-scale, quaternion, opacity logit, SH colour, shape beta):

* ``uniform``  -- means U[-1,1]^3, log-scales N(-3,0.5), SH degree 0 with the DC
  colour U[0,1], beta U[1,4], opacity sigmoid(N(0,1)).
* ``clusters`` -- means from 64 isotropic clusters (sigma 0.3) with centres
  U[-5,5]^3, log-scales N(-4,0.7), opacity sigmoid(N(0,1.5)), SH degree 3 with
  DC colour U[0,1] and higher orders N(0,0.05), beta log-uniform [0.5,8].
* ``overlap``  -- 16 dense clusters (sigma 0.25) on a 4x4 grid in front of the
  camera, one log-scale axis N(-1.5,0.5) and two N(-5,0.5) (long axis in a
  random direction via the random quaternion), opacity sigmoid(N(1,1)),
  beta U[0.5,2], SH degree 3.

The DC colour c is stored as the SH coefficient (c - 0.5) / Y00 so that the
rendered colour of a degree-0 splat is exactly c before clamping.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

Y00 = 0.28209479177387814  # 1 / (2 sqrt(pi)), the l=0 real SH value


@dataclass
class Camera:
    width: int
    height: int
    R: np.ndarray          # (3,3) float32, world -> camera rotation (rows = camera axes)
    t: np.ndarray          # (3,) float32, world -> camera translation
    fx: float
    fy: float
    cx: float
    cy: float
    near: float = 0.2

    def as_dict(self):
        return dict(width=self.width, height=self.height, R=self.R, t=self.t,
                    fx=self.fx, fy=self.fy, cx=self.cx, cy=self.cy, near=self.near)


@dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    beta: np.ndarray
    sh_degree: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def arrays(self):
        return dict(means=self.means, log_scales=self.log_scales, quats=self.quats,
                    opacity_logits=self.opacity_logits, sh=self.sh, beta=self.beta)


def look_at(position, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)):
    """World->camera (R, t) for a camera at ``position`` looking at ``target``.

    Camera axes: x right, y down (image rows grow downwards), z forward.
    """
    p = np.asarray(position, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - p
    f /= np.linalg.norm(f)
    x = np.cross(f, np.asarray(up, dtype=np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f], axis=0)
    t = -R @ p
    return R.astype(np.float32), t.astype(np.float32)


def pinhole(width: int, height: int, position, target=(0.0, 0.0, 0.0), fov_x_deg: float = 60.0,
            near: float = 0.2) -> Camera:
    R, t = look_at(position, target)
    fx = width / (2.0 * math.tan(math.radians(fov_x_deg) / 2.0))
    return Camera(width=int(width), height=int(height), R=R, t=t, fx=float(np.float32(fx)),
                  fy=float(np.float32(fx)), cx=(width - 1) / 2.0, cy=(height - 1) / 2.0, near=near)


def orbit_camera(rng: np.random.Generator, width: int, height: int, radius: float = 8.0) -> Camera:
    az = rng.uniform(0.0, 2.0 * math.pi)
    el = math.radians(rng.uniform(-20.0, 20.0))
    pos = radius * np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
    return pinhole(width, height, pos)


def _normal(rng, mean, std, size):
    return (rng.standard_normal(size, dtype=np.float32) * np.float32(std) + np.float32(mean)).astype(np.float32)


def _uniform(rng, lo, hi, size):
    return (rng.random(size, dtype=np.float32) * np.float32(hi - lo) + np.float32(lo)).astype(np.float32)


def _quats(rng, n):
    q = rng.standard_normal((n, 4), dtype=np.float32)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def _sh(rng, n, degree, dc_rgb, high_std):
    k = (degree + 1) ** 2
    sh = np.empty((n, k, 3), dtype=np.float32)
    sh[:, 0, :] = (dc_rgb - np.float32(0.5)) / np.float32(Y00)
    if k > 1:
        sh[:, 1:, :] = _normal(rng, 0.0, high_std, (n, k - 1, 3))
    return sh


def scene_uniform(n: int, seed: int) -> Scene:
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(n, 3)).astype(np.float32)
    log_scales = rng.normal(-3.0, 0.5, size=(n, 3)).astype(np.float32)
    quats = _quats(rng, n)
    logits = rng.normal(0.0, 1.0, size=n).astype(np.float32)
    sh = _sh(rng, n, 0, rng.uniform(0.0, 1.0, size=(n, 3)), 0.0)
    beta = rng.uniform(1.0, 4.0, size=n).astype(np.float32)
    return Scene(means, log_scales, quats, logits, sh, beta, 0, dict(kind="uniform", seed=seed))


def scene_clusters(n: int, seed: int, degree: int = 3, n_clusters: int = 64) -> Scene:
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-5.0, 5.0, size=(n_clusters, 3)).astype(np.float32)
    which = rng.integers(0, n_clusters, size=n)
    means = (centres[which] + _normal(rng, 0.0, 0.3, (n, 3))).astype(np.float32)
    log_scales = _normal(rng, -4.0, 0.7, (n, 3))
    quats = _quats(rng, n)
    logits = _normal(rng, 0.0, 1.5, n)
    sh = _sh(rng, n, degree, _uniform(rng, 0.0, 1.0, (n, 3)), 0.05)
    beta = np.exp(_uniform(rng, math.log(0.5), math.log(8.0), n)).astype(np.float32)
    return Scene(means, log_scales, quats, logits, sh, beta, degree, dict(kind="clusters", seed=seed))


def scene_clusters_device(n: int, seed: int, device, degree: int = 3, n_clusters: int = 64) -> dict:
    """The ``clusters`` recipe drawn by torch's generator on ``device`` (a dict of float32 tensors).

    Same distributions as :func:`scene_clusters`, different random stream: used where millions of
    resident splats are needed quickly and no oracle looks at them (the serving benchmark).
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f32 = dict(dtype=torch.float32, device=device, generator=g)
    centres = torch.rand((n_clusters, 3), **f32) * 10.0 - 5.0
    which = torch.randint(0, n_clusters, (n,), device=device, generator=g)
    means = centres[which] + 0.3 * torch.randn((n, 3), **f32)
    log_scales = -4.0 + 0.7 * torch.randn((n, 3), **f32)
    quats = torch.randn((n, 4), **f32)
    quats = quats / quats.norm(dim=1, keepdim=True)
    logits = 1.5 * torch.randn((n,), **f32)
    k = (degree + 1) ** 2
    sh = torch.empty((n, k, 3), dtype=torch.float32, device=device)
    sh[:, 0, :] = (torch.rand((n, 3), **f32) - 0.5) / Y00
    if k > 1:
        sh[:, 1:, :] = 0.05 * torch.randn((n, k - 1, 3), **f32)
    beta = torch.exp(math.log(0.5) + (math.log(8.0) - math.log(0.5)) * torch.rand((n,), **f32))
    return dict(means=means.contiguous(), log_scales=log_scales.contiguous(), quats=quats.contiguous(),
                opacity_logits=logits.contiguous(), sh=sh, beta=beta.contiguous())


def scene_overlap(n: int, seed: int, cam: Camera, depth_range=(6.0, 10.0)) -> Scene:
    """Heavy-overlap scene: 16 dense clusters laid out in front of ``cam``."""
    rng = np.random.default_rng(seed)
    # cluster centres on a 4x4 grid spanning 60% of the frame, depth 6..10 along the view axis
    gx, gy = np.meshgrid(np.linspace(-0.3, 0.3, 4), np.linspace(-0.3, 0.3, 4))
    depth = rng.uniform(*depth_range, size=16)
    ndc = np.stack([gx.ravel(), gy.ravel()], axis=1)
    half_w = cam.width / (2.0 * cam.fx)
    half_h = cam.height / (2.0 * cam.fy)
    cam_pts = np.stack([ndc[:, 0] * 2 * half_w * depth, ndc[:, 1] * 2 * half_h * depth, depth], axis=1)
    R = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    centres = (cam_pts - t) @ R  # camera -> world: R^T (p - t)
    which = rng.integers(0, 16, size=n)
    means = (centres[which].astype(np.float32) + _normal(rng, 0.0, 0.25, (n, 3))).astype(np.float32)
    log_scales = _normal(rng, -5.0, 0.5, (n, 3))
    log_scales[:, 0] = _normal(rng, -1.5, 0.5, n)
    quats = _quats(rng, n)
    logits = _normal(rng, 1.0, 1.0, n)
    sh = _sh(rng, n, 3, _uniform(rng, 0.0, 1.0, (n, 3)), 0.05)
    beta = _uniform(rng, 0.5, 2.0, n)
    return Scene(means, log_scales, quats, logits, sh, beta, 3, dict(kind="overlap", seed=seed))


def random_target(rng: np.random.Generator, width: int, height: int) -> np.ndarray:
    return rng.uniform(0.0, 1.0, size=(height, width, 3)).astype(np.float32)


# ---- the five workloads -------------------------------------------------------------------

SERVING_SIZES = (200_000, 500_000, 1_000_000, 1_000_000, 2_000_000, 2_000_000, 3_000_000, 4_000_000)
SERVING_RESOLUTIONS = ((256, 256), (512, 512), (1280, 720), (1920, 1080))

CONFIG_NAMES = {
    0: "fwd+bwd 1k splats 64x64 (uniform cube, SH0)",
    1: "fwd+bwd 1M splats 1600x1040 (64 clusters, SH3)",
    2: "train step 3M splats 1920x1080 (64 clusters, SH3, L1 + freq-masked L1)",
    3: "fwd+bwd 5M splats 1920x1080 (16 dense anisotropic clusters)",
    4: "serving: 8 resident scenes 0.2M..4M splats, mixed resolutions",
}


def make_config(k: int, n_override: int | None = None, seed: int | None = None):
    """Inputs for workload ``k``: dict(scene=..., camera=..., target=..., extra...).

    ``n_override`` shrinks the splat count (same recipe) for parity tests.
    """
    seed = 1000 + k if seed is None else seed
    if k == 0:
        n = 1000 if n_override is None else n_override
        sc = scene_uniform(n, seed)
        cam = pinhole(64, 64, (0.0, 0.0, -4.0))
        tgt = random_target(np.random.default_rng(seed + 7), 64, 64)
        return dict(scene=sc, camera=cam, target=tgt, loss="l1")
    if k in (1, 2):
        n = (1_000_000 if k == 1 else 3_000_000) if n_override is None else n_override
        sc = scene_clusters(n, seed)
        w, h = (1600, 1040) if k == 1 else (1920, 1080)
        cam = orbit_camera(np.random.default_rng(seed + 1), w, h)
        tgt = random_target(np.random.default_rng(seed + 7), w, h)
        return dict(scene=sc, camera=cam, target=tgt, loss="l1" if k == 1 else "l1+freq", omega=0.75)
    if k == 3:
        n = 5_000_000 if n_override is None else n_override
        cam = pinhole(1920, 1080, (0.0, 0.0, -8.0))
        sc = scene_overlap(n, seed, cam)
        tgt = random_target(np.random.default_rng(seed + 7), 1920, 1080)
        return dict(scene=sc, camera=cam, target=tgt, loss="l1")
    if k == 4:
        sizes = list(SERVING_SIZES)
        if n_override is not None:
            sizes = [max(1, int(s * n_override / 4_000_000)) for s in sizes]
        scenes = [scene_clusters(s, seed + 10 * i) for i, s in enumerate(sizes)]
        return dict(scenes=scenes, resolutions=list(SERVING_RESOLUTIONS))
    raise ValueError(f"unknown workload {k}")


def serving_requests(n_req: int, n_scenes: int, resolutions, seed: int = 2000):
    """Request list: (scene index, camera) with a uniformly drawn resolution and orbit camera."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_req):
        s = int(rng.integers(0, n_scenes))
        w, h = resolutions[int(rng.integers(0, len(resolutions)))]
        out.append((s, orbit_camera(np.random.default_rng(seed + 1 + i), w, h)))
    return out


# ---- the 1-D mixture simulation (Sec. 3.2; App. A.3) ------------------------------------------------
MIX_SIGNALS = ("square", "triangle", "parabolic", "half_sinusoid", "gaussian", "exponential")
MIX_MODEL_IDS = {"gmm": 0, "dog": 1, "log": 2, "gef": 3}
MIX_NS = (2, 5, 8, 10, 15, 20, 50, 100)


def mixture_signals(x: np.ndarray, width: float) -> np.ndarray:
    """The six ground-truth signals of App. A.3 on the grid x, [6, len(x)] binary32: square, triangle and
    parabola of support (-width/2, width/2), a half period of a sine over that support, a Gaussian of standard
    deviation `width` and exp(-|x|) over the support."""
    x = np.asarray(x, np.float64)
    half = width / 2.0
    inside = (x > -half) & (x < half)
    rows = [inside.astype(np.float64),
            np.where(inside, half - np.abs(x), 0.0),
            np.where(inside, half * half - x * x, 0.0),
            np.where(inside, np.sin((x + half) * math.pi / width), 0.0),
            np.exp(-(x * x) / (2.0 * width * width)),
            np.where(inside, np.exp(-np.abs(x)), 0.0)]
    return np.stack(rows).astype(np.float32)


def mixture_workload(seed: int = 0, models=("gmm", "dog", "log", "gef"), ns=MIX_NS, runs: int = 20,
                     weights=("positive", "free"), m: int = 1000, x_range=(-5.0, 5.0), width: float = 2.0):
    """Problems of the 1-D simulation: every model x signal x N x run x weight mode.

    Returns dict(problems [P, 4] int32 (model, n, positive, target), targets [6, m], params [P, 128, 4]
    binary32 initial values, x0, dx, and the recipe).  Initial values per component: w_raw ~ N(0, 0.5),
    mu ~ U(-2, 2), s ~ U(0.2, 1.0), beta = 2 (every GEF starts Gaussian); one seeded draw per run."""
    rng = np.random.default_rng(seed)
    x0, x1 = x_range
    dx = (x1 - x0) / (m - 1) if m > 1 else 0.0
    x = x0 + dx * np.arange(m, dtype=np.float64)
    targets = mixture_signals(x, width)
    probs, params = [], []
    for model in models:
        for sig in range(len(MIX_SIGNALS)):
            for n in ns:
                for run in range(runs):
                    for mode in weights:
                        th = np.zeros((128, 4), np.float32)
                        th[:n, 0] = rng.normal(0.0, 0.5, n)
                        th[:n, 1] = rng.uniform(-2.0, 2.0, n)
                        th[:n, 2] = rng.uniform(0.2, 1.0, n)
                        th[:n, 3] = 2.0
                        probs.append((MIX_MODEL_IDS[model], n, 1 if mode == "positive" else 0, sig))
                        params.append(th)
    return dict(problems=np.array(probs, np.int32).reshape(-1, 4), targets=targets,
                params=np.array(params, np.float32).reshape(-1, 128, 4), x0=float(x0), dx=float(dx), m=m,
                x=x, width=width)
