"""The composed training step (mask -> render -> L1 + SSIM + frequency loss -> adjoint -> Adam) against the
oracle's step on the 1,000-splat 64x64 workload, and a short optimisation that must lower the loss.
Parameter gradients are held per element to the parity bound (1e-3 of max(|r|, 1e-2 rms)) beyond the render's
allowance plus what the GPU's binary32 loss gradient moves them by.

Each stage has its own parity test; here the stages are chained as the step chains them.  The oracle
renders in binary64, so its loss gradient and the GPU's agree only where the L1 sign is settled: the seed is
chosen so that no pixel lies within the image tolerance of its target.  Adam's first step moves each
parameter by lr g / (|g| + eps), i.e. by lr times the sign of its gradient: where the gradient exceeds
2e-3 of its group's largest (twice the gradient tolerance) the sign is settled and the moves agree to
1e-6 lr; elsewhere the GPU's move is at most lr."""
import numpy as np
import pytest
import torch

from oracle import loss as OL
from oracle import optim as OP
from oracle import preprocess_f64 as PF
from oracle import ssim as OS
from paper_2402_10128_amd import ges as G
from paper_2402_10128_amd import synth
from paper_2402_10128_amd.train import GROUP_ORDER, TrainConfig, TrainStep

from .parity_helpers import GRAD_RTOL, IMG_ATOL, allowance2d, assert_grad_ok, grad3d_check, oracle_full, to_device

pytestmark = pytest.mark.gpu
B1, B2, EPS = (float(np.float32(x)) for x in (OP.BETA1, OP.BETA2, OP.EPS))


def _oracle_step(arrays, deg, cam, target, it, cfg):
    ref = oracle_full(arrays, deg, cam, cfg.falloff, cfg.tile_cull)
    assert not ref["out"]["flags"].any(), "a pixel has a floating-point-ambiguous decision at this seed"
    img = ref["out"]["img"]
    omega = it / cfg.total_iterations
    mask = OL.freq_mask(target.astype(np.float64), omega)
    lam_l1 = 1.0 - cfg.lam_ssim - cfg.lam_omega
    l1, g1 = OL.loss_and_grad(img, target.astype(np.float64), mask, lam_l1, cfg.lam_omega)
    ls, gs = OS.ssim_loss_and_grad(img, target.astype(np.float64))
    dL = g1 + cfg.lam_ssim * gs
    ref = oracle_full(arrays, deg, cam, cfg.falloff, cfg.tile_cull, dL=dL)
    return dict(img=img, mask=mask, loss=l1 + cfg.lam_ssim * ls, grads=ref["grads"], dL=dL, full=ref)


def _step_allowance(arrays, deg, cam, cfg, full, dL_ref, dL_gpu):
    """Parameter-gradient allowance of the composed step: the render's own (ambiguous decisions, binary32
    evaluation and summation) plus what the GPU's binary32 loss gradient changes -- the gradient is linear in
    dL/dI, so sum |per-pixel term of (dL_gpu - dL_ref)| (the oracle's mass of that difference) bounds it."""
    _, _, mass_d, _, _ = full["orc"].backward2d(full["rec"], dL_gpu.astype(np.float64) - dL_ref, full["values"],
                                                full["ranges"], with_delta=True)
    rec = full["rec"]
    a2 = allowance2d(full["delta"], full["ebound"], full["mass"]) + mass_d
    return PF.abs_chain(arrays, deg, cam, a2, rec.tiles_touched > 0, rec.clamp_bits, cfg.falloff, cfg.rho)


@pytest.mark.parametrize("fused", [True, False], ids=["fused", "two_calls"])
def test_train_step_matches_oracle_step(fused):
    cfg_w = synth.make_config(0)
    sc, cam, target = cfg_w["scene"], cfg_w["camera"], np.asarray(cfg_w["target"], np.float32)
    arrays = sc.arrays()
    cfg = TrainConfig()
    ref = _oracle_step(arrays, sc.sh_degree, cam, target, 1, cfg)
    assert not np.any(np.abs(ref["img"] - target) <= IMG_ATOL), "an L1 sign is unsettled at this seed"
    scene = to_device(arrays)
    p0 = {k: v.clone() for k, v in scene.items()}
    ts = TrainStep(scene, cam, torch.as_tensor(target).cuda(), cfg)
    loss = float(ts.step(1, fused=False).cpu()) if not fused else None
    if fused:
        # the fused step stores no gradients: take them from an unfused backward of the same frame first
        ts_g = TrainStep({k: v.clone() for k, v in scene.items()}, cam, torch.as_tensor(target).cuda(), cfg)
        ts_g.step(1, fused=False)
        grads_gpu = ts_g.grads
        dL_gpu = ts_g.dL.cpu().numpy()
        loss = float(ts.step(1, fused=True).cpu())
    else:
        grads_gpu = ts.grads
        dL_gpu = ts.dL.cpu().numpy()
    torch.cuda.synchronize()
    allow = _step_allowance(arrays, sc.sh_degree, cam, cfg, ref["full"], ref["dL"], dL_gpu)
    print(f"  dL/dI: GPU against oracle, largest difference {np.abs(dL_gpu - ref['dL']).max():.2e} "
          f"(largest |dL/dI| {np.abs(ref['dL']).max():.2e})")
    assert np.array_equal(ts.mask.cpu().numpy(), ref["mask"])
    assert np.abs(ts.image.cpu().numpy() - ref["img"]).max() <= IMG_ATOL
    assert abs(loss - ref["loss"]) <= 1e-4, (loss, ref["loss"])
    lrs = {"means": OP.position_lr(1), "sh": OP.LR["sh"], "opacity_logits": OP.LR["opacity_logits"],
           "beta": OP.LR["beta"], "quats": OP.LR["quats"], "log_scales": OP.LR["log_scales"]}
    for k in GROUP_ORDER:
        g_ref = np.asarray(ref["grads"][k], np.float64).ravel()
        g_gpu = grads_gpu[k].cpu().numpy().astype(np.float64).ravel()
        gmax = np.abs(g_ref).max()
        assert_grad_ok(k, grad3d_check(g_gpu, g_ref, allow[k]))
        pr, _, _ = OP.adam_step(p0[k].cpu().numpy().ravel(), g_ref, 0.0, 0.0, 1, lrs[k], B1, B2, EPS)
        move = scene[k].cpu().numpy().astype(np.float64).ravel() - p0[k].cpu().numpy().astype(np.float64).ravel()
        move_ref = pr - p0[k].cpu().numpy().astype(np.float64).ravel()
        settled = np.abs(g_ref) > 2 * GRAD_RTOL * gmax
        tol = 1e-6 * lrs[k] + 2.5e-7 * np.abs(p0[k].cpu().numpy().ravel())
        assert np.all(np.abs(move - move_ref)[settled] <= tol[settled]), k
        assert np.all(np.abs(move)[~settled] <= lrs[k] * (1 + 1e-6) + tol[~settled]), k


def test_training_lowers_the_loss():
    """30 steps toward the oracle's image of the same scene with its colours and opacities disturbed."""
    cfg_w = synth.make_config(0)
    sc, cam = cfg_w["scene"], cfg_w["camera"]
    arrays = sc.arrays()
    target = oracle_full(arrays, sc.sh_degree, cam, 0, 1)["out"]["img"].astype(np.float32)
    rng = np.random.default_rng(12)
    start = {k: np.array(v, np.float32) for k, v in arrays.items()}
    start["sh"] = start["sh"] + rng.normal(0, 0.2, start["sh"].shape).astype(np.float32)
    start["opacity_logits"] = start["opacity_logits"] + rng.normal(0, 0.5, start["opacity_logits"].shape).astype(
        np.float32)
    scene = to_device(start)
    ts = TrainStep(scene, cam, torch.as_tensor(target).cuda(), TrainConfig())
    losses = [float(ts.step(it).cpu()) for it in range(1, 31)]
    print("losses", [round(x, 5) for x in losses])
    assert all(np.isfinite(losses))
    assert min(losses[-5:]) < 0.8 * losses[0], losses


@pytest.mark.parametrize("workload,n", [(0, None), (1, 200_000)], ids=["1k_64x64", "200k_1600x1040"])
def test_fused_backward_adam_equals_two_calls(workload, n):
    """Three steps of the training step with Adam fused into the backward pass and with the stand-alone
    Adam kernel after a stored-gradient backward: parameters and both moments identical bit for bit."""
    cfg_w = synth.make_config(workload, n_override=n)
    sc, cam = cfg_w["scene"], cfg_w["camera"]
    target = torch.as_tensor(np.asarray(cfg_w["target"], np.float32)).cuda()
    runs = []
    for fused in (True, False):
        scene = to_device(sc.arrays())
        ts = TrainStep(scene, cam, target, TrainConfig())
        for it in range(1, 4):
            ts.step(it, fused=fused)
        torch.cuda.synchronize()
        runs.append((scene, ts.exp_avg, ts.exp_avg_sq))
    for k in GROUP_ORDER:
        for a, b in zip(runs[0], runs[1]):
            assert torch.equal(a[k], b[k]), k


def test_prune_and_shape_reset_hooks():
    """The step's hooks on the 1,000-splat workload with betas spread over [0.2, 3]: pruning at iteration 2
    keeps exactly the splats at or above both bounds (checked on the state just before it), in order and with
    their moments; the shape reset at iteration 3 sets every beta to 2 and clears its moments; training then
    goes on with finite losses."""
    import math
    cfg_w = synth.make_config(0)
    sc, cam = cfg_w["scene"], cfg_w["camera"]
    arrays = {k: np.array(v, np.float32) for k, v in sc.arrays().items()}
    arrays["beta"] = np.random.default_rng(3).uniform(0.2, 3.0, arrays["beta"].shape).astype(np.float32)
    cfg = TrainConfig(shape_prune_interval=0, shape_reset_interval=0, min_beta=0.5)
    ts = TrainStep(to_device(arrays), cam, torch.as_tensor(np.asarray(cfg_w["target"], np.float32)).cuda(), cfg)
    ts.step(1)
    ts.step(2)
    before = {k: v.cpu().numpy().copy() for k, v in ts.scene.items()}
    m_before = {k: v.cpu().numpy().copy() for k, v in ts.exp_avg.items()}
    kept = ts.prune()
    bound = math.log(cfg.min_opacity / (1 - cfg.min_opacity))
    keep = ~(before["opacity_logits"].astype(np.float64) < bound) & ~(before["beta"].astype(np.float64) < 0.5)
    assert kept == int(keep.sum()) == ts.n and 0 < kept < len(keep)
    for k in G.SPLAT_PARAMS:
        assert np.array_equal(ts.scene[k].cpu().numpy(), before[k][keep]), k
        assert np.array_equal(ts.exp_avg[k].cpu().numpy(), m_before[k][keep]), k
    ts.cfg.shape_reset_interval = 3
    loss = float(ts.step(3).cpu())
    torch.cuda.synchronize()
    assert torch.all(ts.scene["beta"] == 2.0) and not ts.exp_avg["beta"].any() and not ts.exp_avg_sq["beta"].any()
    losses = [loss] + [float(ts.step(it).cpu()) for it in (4, 5)]
    assert all(np.isfinite(losses))


def test_accumulating_backward_matches_the_oracle_sum_over_views():
    """Two views of the 1,000-splat workload: the first view's backward, then the second's added with
    ges_render_backward_accumulate, against the sum of the oracle's gradients of both views (within the
    parity bound beyond the summed allowances for floating-point-ambiguous decisions)."""
    cfg_w = synth.make_config(0)
    sc, cam0 = cfg_w["scene"], cfg_w["camera"]
    cam1 = synth.pinhole(cam0.width, cam0.height, (0.6, -0.4, -3.8))
    arrays = sc.arrays()
    rng = np.random.default_rng(17)
    dLs = [rng.standard_normal((cam0.height, cam0.width, 3)).astype(np.float32) for _ in range(2)]
    refs = [oracle_full(arrays, sc.sh_degree, cam, 0, 1, dL=d.astype(np.float64)) for cam, d in zip((cam0, cam1), dLs)]
    t = to_device(arrays)
    s = G.splats_struct(*(t[k] for k in G.SPLAT_PARAMS))
    p = G.params_struct(0, 1, 0.1, (0.0, 0.0, 0.0))
    frame = G.Frame.create(s.n, cam0.width, cam0.height, "cuda")
    grads = {k: torch.empty_like(v) for k, v in t.items()}
    out = torch.empty((cam0.height, cam0.width, 3), device="cuda")
    for v, cam in enumerate((cam0, cam1)):
        c = G.camera_struct(cam)
        k = G.ges_preprocess(s, c, p, frame.splat_ws, True)
        frame.ensure_keys(k)
        G.ges_render_forward(s, c, p, frame.splat_ws, frame.key_ws, k, frame.pixel_ws, out)
        ws = (s, c, p, frame.splat_ws, frame.key_ws, frame.pixel_ws, torch.from_numpy(dLs[v]).cuda())
        if v == 0:
            G.ges_render_backward(*ws, grads)
        else:
            G.ges_render_backward_accumulate(*ws, grads)
    torch.cuda.synchronize()
    for k in G.SPLAT_PARAMS:
        want = np.asarray(refs[0]["grads"][k]) + np.asarray(refs[1]["grads"][k])
        allow = np.asarray(refs[0]["allow"][k]) + np.asarray(refs[1]["allow"][k])
        assert_grad_ok(k, grad3d_check(grads[k].cpu().numpy(), want, allow))


def test_multi_view_step_fused_equals_two_calls():
    """A two-view training step: the fused update from the summed gradients (grads_in) and the stand-alone
    Adam after both views' accumulated backward give the same bits over three steps."""
    cfg_w = synth.make_config(0)
    sc, cam0 = cfg_w["scene"], cfg_w["camera"]
    cam1 = synth.pinhole(cam0.width, cam0.height, (0.6, -0.4, -3.8))
    tg = torch.as_tensor(np.asarray(cfg_w["target"], np.float32)).cuda()
    tg1 = torch.flip(tg, dims=[1]).contiguous()
    runs = []
    for fused in (True, False):
        scene = to_device(sc.arrays())
        ts = TrainStep(scene, [cam0, cam1], [tg, tg1], TrainConfig())
        losses = [float(ts.step(it, fused=fused).cpu()) for it in range(1, 4)]
        torch.cuda.synchronize()
        runs.append((scene, ts.exp_avg, ts.exp_avg_sq, ts.grad_accum, ts.grad_count, losses))
    for k in GROUP_ORDER:
        for a, b in zip(runs[0][:3], runs[1][:3]):
            assert torch.equal(a[k], b[k]), k
    assert torch.equal(runs[0][3], runs[1][3]) and torch.equal(runs[0][4], runs[1][4])
    assert runs[0][5] == runs[1][5] and all(np.isfinite(runs[0][5]))
    assert 0 < float(runs[0][4].max().cpu()) <= 3 * 2          # at most one visit per view and step
