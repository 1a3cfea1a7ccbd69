"""Densification (clone/split), its statistic and the opacity reset on the GPU against the oracle.

Copies and the kept/clone/split decision (binary64 comparisons on both sides) are bit-exact; split children's
log-scales are one binary64 subtraction rounded to binary32 on both sides (bit-exact); their means are
mu + R(s z) evaluated in binary64 with the device's exp and rounded to binary32, so they are compared to
2.5e-7 relative (one binary32 rounding).  The statistic is a binary64 norm added in binary32 and compared to
the oracle's statistic of its own backward within the gradient tolerance (1e-3 of the largest)."""
import numpy as np
import pytest
import torch

from oracle import densify as OD
from oracle import oracle as O
from paper_2402_10128_amd import ges as G
from paper_2402_10128_amd import synth
from paper_2402_10128_amd.train import TrainConfig, TrainStep

from .parity_helpers import GRAD_RTOL, oracle_full, to_device

pytestmark = pytest.mark.gpu
NAMES = G.SPLAT_PARAMS


def _inputs(rng, n, deg, nsets):
    K = (deg + 1) ** 2
    shapes = {"means": (n, 3), "log_scales": (n, 3), "quats": (n, 4), "opacity_logits": (n,), "sh": (n, K, 3),
              "beta": (n,)}
    sets = [{k: rng.normal(size=s).astype(np.float32) for k, s in shapes.items()} for _ in range(nsets)]
    sets[0]["log_scales"] = rng.uniform(-6, -1, (n, 3)).astype(np.float32)
    accum = (rng.uniform(0, 0.001, n) * rng.integers(0, 5, n)).astype(np.float32)
    count = rng.integers(0, 5, n).astype(np.float32)
    normals = rng.standard_normal((n, 2, 3)).astype(np.float32)
    return sets, accum, count, normals


def _gpu_densify(sets, accum, count, normals, deg, thr=0.0003, sthr=0.05):
    dev = torch.device("cuda:0")
    n = len(accum)
    src = [{k: torch.from_numpy(v).to(dev) for k, v in s.items()} for s in sets]
    cap = 2 * n + 1
    dst = [{k: torch.full((cap,) + tuple(v.shape[1:]), float("nan"), device=dev) for k, v in s.items()} for s in src]
    out = G.ges_densify(src, dst, deg, torch.from_numpy(accum).to(dev), torch.from_numpy(count).to(dev),
                        torch.from_numpy(normals).to(dev), thr, sthr)
    torch.cuda.synchronize()
    return out, [{k: v[:out].cpu().numpy() for k, v in d.items()} for d in dst]


def _same(got, want, means):
    if means:
        return np.allclose(got, want, rtol=2.5e-7, atol=1e-7)
    return np.array_equal(got.view(np.uint32), want.astype(np.float32).view(np.uint32))


@pytest.mark.parametrize("n,deg,nsets", [(5000, 3, 3), (1, 0, 1), (0, 1, 2), (777, 1, 3), (3000, 2, 2)],
                         ids=["sh3", "one", "empty", "sh1", "sh2"])
def test_densify_matches_oracle(n, deg, nsets):
    sets, accum, count, normals = _inputs(np.random.default_rng(n), n, deg, nsets)
    n_out, got = _gpu_densify(sets, accum, count, normals, deg)
    out, outm, kind = OD.densify(sets[0], sets[1:], accum, count, normals, 0.0003, 0.05)
    assert n_out == len(out["beta"])
    for j, want in enumerate([out] + outm):
        for k in NAMES:
            assert _same(got[j][k], want[k], j == 0 and k == "means"), (j, k)


def test_densify_full_scene_sampled():
    """The 3M-splat scene with synthetic statistics: the oracle classifies every splat; 3,000 sampled splats
    are densified by the oracle one at a time and their output rows (kept row, clone, children) compared."""
    cfg = synth.make_config(2)
    arr = {k: np.ascontiguousarray(v, np.float32) for k, v in cfg["scene"].arrays().items()}
    n = arr["beta"].shape[0]
    rng = np.random.default_rng(11)
    accum = (rng.uniform(0, 0.0012, n) * rng.integers(0, 4, n)).astype(np.float32)
    count = rng.integers(0, 4, n).astype(np.float32)
    normals = rng.standard_normal((n, 2, 3)).astype(np.float32)
    mom = {k: rng.normal(size=v.shape).astype(np.float32) for k, v in arr.items()}
    ext = float(np.exp(np.median(arr["log_scales"].max(axis=1)))) * 1.0
    n_out, got = _gpu_densify([arr, mom], accum, count, normals, 3, 0.0003, ext)
    kind = OD.classify(accum, count, arr["log_scales"], 0.0003, ext)
    U, Cn, S = int((kind != 2).sum()), int((kind == 1).sum()), int((kind == 2).sum())
    assert n_out == U + Cn + 2 * S and Cn > 0 and S > 0
    upos = np.cumsum(kind != 2) - 1
    cpos = U + np.cumsum(kind == 1) - 1
    spos = U + Cn + 2 * (np.cumsum(kind == 2) - 1)
    for i in rng.choice(n, 3000, replace=False):
        one, (onem,), _ = OD.densify({k: v[[i]] for k, v in arr.items()}, [{k: v[[i]] for k, v in mom.items()}],
                                     accum[[i]], count[[i]], normals[[i]], 0.0003, ext)
        rows = [upos[i]] if kind[i] == 0 else [upos[i], cpos[i]] if kind[i] == 1 else [spos[i], spos[i] + 1]
        for r_i, r in enumerate(rows):
            for k in NAMES:
                assert _same(got[0][k][r], one[k][r_i], k == "means"), (i, kind[i], k)
                assert _same(got[1][k][r], onem[k][r_i], False), (i, kind[i], k)


def test_densify_statistic_and_opacity_reset():
    """One fused backward on the 1,000-splat workload accumulates, for every visible splat, the NDC norm of the
    oracle's mean-2D gradient and one visit; the opacity reset caps opacities at 0.01 on the logit."""
    cfg_w = synth.make_config(0)
    sc, cam = cfg_w["scene"], cfg_w["camera"]
    arrays = sc.arrays()
    g = np.random.default_rng(4).standard_normal((cam.height, cam.width, 3)).astype(np.float32)
    ref = oracle_full(arrays, sc.sh_degree, cam, 0, 1, dL=g.astype(np.float64))
    vis = ref["rec"].tiles_touched > 0
    want, wcount = OD.accumulate(np.zeros(len(vis)), np.zeros(len(vis)), ref["g2d"][:, 0], ref["g2d"][:, 1], vis,
                                 cam.width, cam.height)
    t = to_device(arrays)
    s = G.splats_struct(*(t[k] for k in NAMES))
    c, p = G.camera_struct(cam), G.params_struct(0, 1, 0.1, (0.0, 0.0, 0.0))
    frame = G.Frame.create(s.n, cam.width, cam.height, "cuda")
    k = G.ges_preprocess(s, c, p, frame.splat_ws, True)
    frame.ensure_keys(k)
    out = torch.empty((cam.height, cam.width, 3), device="cuda")
    G.ges_render_forward(s, c, p, frame.splat_ws, frame.key_ws, k, frame.pixel_ws, out)
    acc = torch.zeros(s.n, device="cuda")
    cnt = torch.zeros(s.n, device="cuda")
    zeros = {k: torch.zeros_like(v) for k, v in t.items()}
    G.ges_render_backward_adam(s, c, p, frame.splat_ws, frame.key_ws, frame.pixel_ws, torch.from_numpy(g).cuda(),
                               zeros, {k: torch.zeros_like(v) for k, v in t.items()},
                               {k: 0.0 for k in NAMES}, 1, grad_accum=acc, grad_count=cnt)
    torch.cuda.synchronize()
    assert np.array_equal(cnt.cpu().numpy(), wcount.astype(np.float32))
    assert np.abs(acc.cpu().numpy() - want).max() <= GRAD_RTOL * want.max()
    logits = torch.tensor([-6.0, -4.59511985013459, -4.5, 0.0, 3.0], device="cuda")
    m, v = torch.ones_like(logits), torch.ones_like(logits)
    G.ges_opacity_reset(logits, m, v, 0.01)
    want_l, _, _ = OD.opacity_reset(np.array([-6.0, -4.59511985013459, -4.5, 0.0, 3.0], np.float32), np.ones(5),
                                    np.ones(5))
    assert np.array_equal(logits.cpu().numpy(), want_l.astype(np.float32)) and not m.any() and not v.any()


def test_training_densify_hook():
    """The step's statistics and densification on the 1,000-splat workload: after one step every visible
    splat has one visit; densify() then keeps the unsplit splats first, in order and unchanged, grows the set
    by one per clone and per split, and training goes on with finite losses."""
    import math
    cfg_w = synth.make_config(0)
    sc, cam = cfg_w["scene"], cfg_w["camera"]
    cfg = TrainConfig(shape_prune_interval=0, densify_from=10 ** 6, grad_threshold=1e-7,
                      scene_extent=float(np.exp(np.median(sc.arrays()["log_scales"].max(axis=1)))) / 0.01)
    ts = TrainStep(to_device(sc.arrays()), cam, torch.as_tensor(np.asarray(cfg_w["target"], np.float32)).cuda(), cfg)
    ts.step(1)
    torch.cuda.synchronize()
    acc, cnt = ts.grad_accum.cpu().numpy(), ts.grad_count.cpu().numpy()
    before = {k: v.cpu().numpy().copy() for k, v in ts.scene.items()}
    assert set(np.unique(cnt)) <= {0.0, 1.0} and cnt.sum() > 0
    mean = np.where(cnt > 0, acc.astype(np.float64) / np.maximum(cnt, 1), 0.0)
    sel = mean >= cfg.grad_threshold
    small = before["log_scales"].astype(np.float64).max(axis=1) <= math.log(cfg.percent_dense * cfg.scene_extent)
    clones, splits = int((sel & small).sum()), int((sel & ~small).sum())
    assert clones > 0 and splits > 0
    n0 = ts.n
    out = ts.densify()
    assert out == ts.n == n0 + clones + splits
    unsplit = ~(sel & ~small)
    for k in NAMES:
        assert np.array_equal(ts.scene[k][: int(unsplit.sum())].cpu().numpy(), before[k][unsplit]), k
    assert float(ts.grad_count.sum().cpu()) == 0.0
    losses = [float(ts.step(it).cpu()) for it in (2, 3)]
    assert all(np.isfinite(losses))
