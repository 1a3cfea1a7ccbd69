"""Fused Adam kernel (App. B.2 training step) against the binary64 oracle: several steps over the six
splat parameter groups at a small size (ragged blocks, an empty group, a group that is not 16-byte aligned),
and one step at the 3,000,000-splat size on sampled elements.

Tolerance (binary32 kernel, binary64 oracle; eps32 = 2^-24): each step rounds m, v and p a few times, so
after k steps |dm| <= 4e-7 k max|g| (m may cancel, so the bound scales with the largest gradient), |dv| <=
1e-6 k |v|, and p drifts by at most 2.5e-7 k |p| from its own rounding plus lr times the error of
m_hat / (sqrt(v_hat) + eps), which stays below 2e-5 when that ratio is of order one (the seeded states
keep it so).  Gradients are exact zeros or have magnitudes in [1e-8, 1e2], away from binary32 underflow
of g^2.  The oracle takes the binary32 values of b1 and b2 that the kernel receives."""
import numpy as np
import pytest
import torch

from oracle import optim as OP
from paper_2402_10128_amd import ges as G

pytestmark = pytest.mark.gpu

B1, B2, EPS = float(np.float32(OP.BETA1)), float(np.float32(OP.BETA2)), float(np.float32(OP.EPS))
# per-splat float counts of the six groups and their App. B.2 learning rates
GROUPS = [("means", 3, OP.LR["means"]), ("sh", 48, OP.LR["sh"]), ("opacity_logits", 1, OP.LR["opacity_logits"]),
          ("beta", 1, OP.LR["beta"]), ("quats", 4, OP.LR["quats"]), ("log_scales", 3, OP.LR["log_scales"])]


def _grads(rng, count):
    mag = 10.0 ** rng.uniform(-8, 2, count)
    g = (rng.choice([-1.0, 1.0], count) * mag).astype(np.float32)
    g[rng.random(count) < 0.1] = 0.0
    return g


def _run(n, steps, misalign=False, empty=False, seed=0):
    rng = np.random.default_rng(seed)
    dev = torch.device("cuda:0")
    host, devs, grads_all = [], [], []
    for gi, (name, per, lr) in enumerate(GROUPS):
        count = 0 if (empty and gi == 2) else n * per
        p0 = rng.standard_normal(count).astype(np.float32)
        host.append([p0.astype(np.float64), np.zeros(count), np.zeros(count), float(np.float32(lr))])
        off = 1 if (misalign and gi == 1) else 0    # a view one float into its buffer is only 4-byte aligned
        bufs = [torch.zeros(count + off, dtype=torch.float32, device=dev)[off:] for _ in range(4)]
        bufs[0].copy_(torch.from_numpy(p0))
        devs.append(bufs)
    gmax = [np.zeros(len(h[0])) for h in host]
    for t in range(1, steps + 1):
        groups = []
        for gi, (h, d) in enumerate(zip(host, devs)):
            g = _grads(rng, len(h[0]))
            gmax[gi] = np.maximum(gmax[gi], np.abs(g))
            d[1].copy_(torch.from_numpy(g))
            h[0], h[1], h[2] = OP.adam_step(h[0], g, h[1], h[2], t, h[3], B1, B2, EPS)
            groups.append((d[0], d[1], d[2], d[3], h[3]))
        G.ges_adam_step(groups, t, B1, B2, EPS)
    torch.cuda.synchronize()
    for gi, (h, d) in enumerate(zip(host, devs)):
        p, m, v = (x.cpu().numpy().astype(np.float64) for x in (d[0], d[2], d[3]))
        k = steps
        assert np.all(np.abs(m - h[1]) <= 4e-7 * k * gmax[gi]), GROUPS[gi][0]
        assert np.all(np.abs(v - h[2]) <= 1e-6 * k * h[2] + 1e-45), GROUPS[gi][0]
        err = np.abs(p - h[0])
        bound = 2.5e-7 * k * np.abs(h[0]) + 2e-5 * h[3] * k
        assert np.all(err <= bound), (GROUPS[gi][0], float((err / bound).max()))


@pytest.mark.parametrize("n", [1237, 4096], ids=["ragged", "aligned"])
def test_adam_multi_step_parity(n):
    _run(n, steps=5, seed=n)


def test_adam_unaligned_and_empty_groups():
    _run(333, steps=3, misalign=True, empty=True, seed=7)


def test_adam_zero_gradient_keeps_zero_state_and_params():
    dev = torch.device("cuda:0")
    p = torch.randn(1000, device=dev)
    p0 = p.clone()
    z = [torch.zeros(1000, device=dev) for _ in range(3)]
    G.ges_adam_step([(p, z[0], z[1], z[2], 0.01)], 1)
    torch.cuda.synchronize()
    assert torch.equal(p, p0) and not z[1].any() and not z[2].any()


def test_adam_full_size_one_step_sampled():
    """One step (t = 1000) over all six groups of 3,000,000 splats from seeded moment states, checked on
    200,000 sampled elements per group (the update is elementwise, so the oracle takes the samples alone)."""
    n = 3_000_000
    rng = np.random.default_rng(2024)
    gen = torch.Generator(device="cuda:0").manual_seed(5)
    dev = torch.device("cuda:0")
    groups, checks = [], []
    t = 1000
    for name, per, lr in GROUPS:
        count = n * per
        p = torch.randn(count, device=dev, generator=gen)
        g = torch.randn(count, device=dev, generator=gen) * 0.1
        m = torch.randn(count, device=dev, generator=gen) * 0.05
        v = (m.abs() + 0.1) ** 2 * (0.5 + 1.5 * torch.rand(count, device=dev, generator=gen))
        idx = np.sort(rng.choice(count, 200_000, replace=False))
        ti = torch.from_numpy(idx).to(dev)
        before = [x[ti].cpu().numpy().astype(np.float64) for x in (p, g, m, v)]
        lr32 = float(np.float32(lr))
        groups.append((p, g, m, v, lr32))
        checks.append((name, ti, before, lr32))
    G.ges_adam_step(groups, t, B1, B2, EPS)
    torch.cuda.synchronize()
    for (name, ti, (p0, g0, m0, v0), lr), (p, _, m, v, _) in zip(checks, groups):
        pr, mr, vr = OP.adam_step(p0, g0, m0, v0, t, lr, B1, B2, EPS)
        pg, mg, vg = (x[ti].cpu().numpy().astype(np.float64) for x in (p, m, v))
        assert np.all(np.abs(mg - mr) <= 4e-7 * np.maximum(np.abs(m0), np.abs(g0))), name
        assert np.all(np.abs(vg - vr) <= 1e-6 * vr), name
        assert np.all(np.abs(pg - pr) <= 2.5e-7 * np.abs(pr) + 4e-6 * lr), name
