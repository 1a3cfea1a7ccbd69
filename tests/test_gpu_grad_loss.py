"""GPU gradients against central finite differences of the binary64 oracle, the autograd Function,
and the frequency-masked loss kernels against the oracle's loss."""
import numpy as np
import pytest
import torch

from oracle import loss as OL
from oracle import oracle as O
from paper_2402_10128_amd import synth

from .fd_helpers import central_fd, random_picks
from .parity_helpers import GRAD_RTOL, ambiguous_splats, gpu_render, oracle_full, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("falloff", [O.FALLOFF_PHI, O.FALLOFF_GEF], ids=["phi", "gef"])
def test_gpu_grads_vs_central_fd_1000_params(falloff):
    """1,000 random scalar parameters of the 1,000-splat 64x64 workload (PHI and GEF falloff)."""
    cfg = synth.make_config(0)
    sc, cam = cfg["scene"], cfg["camera"]
    g = np.random.default_rng(21).standard_normal((cam.height, cam.width, 3)).astype(np.float32)
    gpu = gpu_render(sc.arrays(), 0, cam, falloff, dL=g)
    ref = oracle_full(sc.arrays(), 0, cam, falloff, dL=g.astype(np.float64))
    amb = ambiguous_splats(ref["g2d"][:, :10], ref["delta"][:, :10])   # FD is undefined across a flipped decision
    picks = random_picks(sc.arrays(), (ref["rec"].tiles_touched > 0) & ~amb, 1000, seed=5 + falloff)
    fd, _ = central_fd(sc.arrays(), 0, cam, falloff, g.astype(np.float64), picks)
    got, want = [], []
    for (name, idx), f in zip(picks, fd):
        if f is None:
            continue
        got.append(gpu["grads"][name][idx])
        want.append(f)
    got, want = np.array(got, np.float64), np.array(want)
    floor = 1e-2 * np.sqrt(np.mean(want ** 2))
    rel = np.abs(got - want) / np.maximum(np.abs(want), floor)
    print(f"[fd] falloff={falloff} checked {len(want)} excluded {len(picks) - len(want)} "
          f"max {rel.max():.2e} p99 {np.percentile(rel, 99):.2e}")
    assert len(want) >= 900
    assert rel.max() <= GRAD_RTOL, rel.max()


def test_autograd_function_matches_abi():
    from paper_2402_10128_amd.autograd import rasterize
    cfg = synth.make_config(0, n_override=500)
    sc, cam = cfg["scene"], cfg["camera"]
    t = to_device(sc.arrays())
    for v in t.values():
        v.requires_grad_(True)
    img = rasterize(t, cam)
    g = torch.randn_like(img)
    (img * g).sum().backward()
    ref = gpu_render(sc.arrays(), 0, cam, dL=g.detach().cpu().numpy())
    np.testing.assert_array_equal(img.detach().cpu().numpy(), ref["img"])
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "beta"):
        np.testing.assert_allclose(t[k].grad.cpu().numpy(), ref["grads"][k], rtol=1e-5, atol=1e-7)


def test_freq_mask_and_loss_vs_oracle():
    from paper_2402_10128_amd import ges as G
    rng = np.random.default_rng(8)
    H, W = 108, 192
    # a target with structure: smooth blobs plus noise
    yy, xx = np.mgrid[0:H, 0:W]
    tgt = (0.5 + 0.4 * np.sin(xx / 9.0)[..., None] * np.cos(yy / 13.0)[..., None]
           + 0.05 * rng.standard_normal((H, W, 3))).astype(np.float32)
    img = rng.uniform(size=(H, W, 3)).astype(np.float32)
    for omega in (0.75, 0.3, 0.5, 1.0, 0.0, 1 / 40000):
        m_gpu = G.ges_freq_mask(torch.as_tensor(tgt).cuda(), omega).cpu().numpy()
        m_ref = OL.freq_mask(tgt.astype(np.float64), omega)
        # pixels whose normalised response lies within 1e-4 of the threshold may go either way
        resp = OL.dog_response(tgt.astype(np.float64), omega if omega > 0.5 else omega + 0.5)
        near = np.abs(resp - 0.5) < 1e-4
        near_full = near[np.arange(H)[:, None] // 5, np.arange(W)[None, :] // 5]
        assert np.array_equal(m_gpu[~near_full], m_ref[~near_full]), int((m_gpu != m_ref).sum())
    mask = m_ref
    L, dL = G.ges_loss(torch.as_tensor(img).cuda(), torch.as_tensor(tgt).cuda(), torch.as_tensor(mask).cuda(), 0.5, 0.5)
    L_ref, g_ref = OL.loss_and_grad(img.astype(np.float64), tgt.astype(np.float64), mask, 0.5, 0.5)
    assert abs(float(L.cpu()) - L_ref) <= 1e-5 * max(1.0, abs(L_ref))
    np.testing.assert_allclose(dL.cpu().numpy(), g_ref, rtol=1e-6, atol=1e-12)
