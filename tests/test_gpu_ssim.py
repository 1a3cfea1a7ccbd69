"""SSIM term of the training loss on the GPU against the binary64 oracle: ragged sizes (one tile, partial
tiles, single rows and columns, a single pixel), the accumulate-into contract, identical images, run-to-run
determinism, and the full 1920x1080 image.

Tolerance (binary32 kernel): the local statistics carry rounding of order 1e-7; the variance terms divide
by s_x + s_y + C2 >= C2 ~ 1e-3, so each SSIM value and each partial-derivative map can be off by ~1e-4 of
its scale.  The loss is a mean over h w 3 values whose errors do not share a sign: |dL| <= 2e-6 +
1e-6 |L|.  The gradient is compared to its largest magnitude: |d grad| <= 1e-4 max|grad|."""
import numpy as np
import pytest
import torch

from oracle import ssim as OS
from paper_2402_10128_amd import ges as G
from paper_2402_10128_amd import synth

pytestmark = pytest.mark.gpu
LAM = 0.2


def _pair(H, W, seed, noise=0.1):
    rng = np.random.default_rng(seed)
    tgt = rng.random((H, W, 3)).astype(np.float32)
    img = np.clip(tgt + noise * rng.standard_normal((H, W, 3)), 0, 1).astype(np.float32)
    return img, tgt, rng


def _gpu(img, tgt, loss0, dl0):
    dev = torch.device("cuda:0")
    ti, tt = torch.from_numpy(img).to(dev), torch.from_numpy(tgt).to(dev)
    loss = torch.tensor(loss0, dtype=torch.float32, device=dev)
    dl = torch.from_numpy(dl0).to(dev)
    G.ges_ssim_loss(ti, tt, LAM, loss, dl)
    torch.cuda.synchronize()
    return float(loss.cpu()), dl.cpu().numpy().astype(np.float64)


def _check(img, tgt, loss0, dl0, loss, dl):
    lref, gref = OS.ssim_loss_and_grad(img, tgt)
    want = loss0 + LAM * lref
    assert abs(loss - want) <= 2e-6 + 1e-6 * abs(want), (loss, want)
    scale = max(np.abs(LAM * gref).max(), 1e-30)
    err = np.abs(dl - (dl0 + LAM * gref)).max() / scale
    assert err <= 1e-4, err


@pytest.mark.parametrize("H,W", [(32, 32), (45, 70), (1, 1), (1, 33), (33, 1), (100, 37)])
def test_ssim_ragged_sizes_accumulate(H, W):
    img, tgt, rng = _pair(H, W, H * 1000 + W)
    dl0 = (rng.standard_normal((H, W, 3)) * 1e-3).astype(np.float32)
    loss, dl = _gpu(img, tgt, 0.25, dl0)
    _check(img, tgt, 0.25, dl0, loss, dl)


def test_ssim_identical_images_add_nothing():
    img, _, _ = _pair(70, 90, 3)
    dl0 = np.zeros_like(img)
    loss, dl = _gpu(img, img, 0.0, dl0)
    assert abs(loss) <= 2e-6
    assert np.abs(dl).max() <= 1e-4 / img.size


def test_ssim_deterministic():
    img, tgt, _ = _pair(200, 300, 4)
    z = np.zeros_like(img)
    a = _gpu(img, tgt, 0.0, z)
    b = _gpu(img, tgt, 0.0, z)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_ssim_full_size_1080p():
    """The 1920x1080 training target against a perturbed copy (the rendered image's role), every element."""
    cfg = synth.make_config(2, n_override=1000)
    tgt = np.asarray(cfg["target"], np.float32)
    rng = np.random.default_rng(9)
    img = np.clip(tgt + 0.05 * rng.standard_normal(tgt.shape), 0, 1).astype(np.float32)
    z = np.zeros_like(img)
    loss, dl = _gpu(img, tgt, 0.0, z)
    _check(img, tgt, 0.0, z, loss, dl)
