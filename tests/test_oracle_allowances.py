"""Pins of the oracle's binary32 compositing branch and of the allowances its backward returns
(Sec. 4.2, Eq. transimttance: front-to-back compositing and its derivative).

A GPU gradient is accepted when its error lies within
    delta         the other branch of a termination / clamp decision that binary32 may take either way,
    ebound        a first-order bound on the binary32 evaluation error of every per-pixel term,
    gamma * mass  the rounding of binary32 sums of those terms,
so each is pinned here against something other than the oracle itself:
  * closed forms of the compositing derivative written front to back (the oracle recurs back to front
    through the colour composited behind each splat);
  * an independent binary32 compositor (numpy float32 arithmetic, round to nearest) whose exp2, log2 and
    reciprocal results are the exact values rounded in a chosen direction (within one ulp), so that their
    errors add up coherently, as the bound assumes they may.
Splat geometry is put on a 1/64 grid so that q is exact in every precision and only the compositing
arithmetic rounds.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2402_10128_amd import synth

U32 = 2.0 ** -24
F = np.float32


def _camera(W, H):
    return synth.Camera(W, H, np.eye(3, dtype=np.float32), np.zeros(3, np.float32), 50.0, 50.0, 0.0, 0.0, 0.2)


def _record(splats, W, H):
    """A hand-built record: splats are dicts with u, v, a, b, c, qmax, o, rgb, beta (depth = list order)."""
    n = len(splats)
    rec = O.Record.empty(n)
    TX, TY = (W + 15) // 16, (H + 15) // 16
    for i, s in enumerate(splats):
        rec.u[i], rec.v[i] = s["u"], s["v"]
        rec.depth[i] = 1.0 + 0.01 * i
        rec.conic[i] = (s["a"], s["b"], s["c"])
        rec.qmax[i] = s["qmax"]
        rec.opacity[i] = s["o"]
        rec.rgb[i] = s["rgb"]
        rec.beta[i] = s.get("beta", 2.0)
        rec.radius[i] = 1000
        rec.rect[i] = (0, 0, TX - 1, TY - 1)
        rec.tiles_touched[i] = TX * TY
    return rec


def _oracle(n, W, H, falloff=O.FALLOFF_PHI, bg=(0.0, 0.0, 0.0)):
    arr = dict(means=np.zeros((n, 3), np.float32), log_scales=np.zeros((n, 3), np.float32),
               quats=np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)), opacity_logits=np.zeros(n, np.float32),
               sh=np.zeros((n, 1, 3), np.float32), beta=np.full(n, 2.0, np.float32))
    return O.Oracle(arr, 0, _camera(W, H), falloff=falloff, tile_cull=O.TILES_SQUARE, bg=bg)


def _run(splats, W, H, g, falloff=O.FALLOFF_PHI, bg=(0.0, 0.0, 0.0)):
    orc = _oracle(len(splats), W, H, falloff, bg)
    rec = _record(splats, W, H)
    _, vals, ranges = orc.build_keys(rec)
    out = orc.render(rec, vals, ranges)
    g2d, delta, mass, ebound, _ = orc.backward2d(rec, g, vals, ranges, with_delta=True)
    return out, g2d, delta, mass, ebound


def _grid(rng, lo, hi):
    return float(np.round(rng.uniform(lo, hi) * 64.0) / 64.0)


# ---- closed form, front to back --------------------------------------------------------------------------
def closed_form_pixel(splats, px, py, g, bg=(0.0, 0.0, 0.0), flip_term_at=None, flip_clamp_at=None):
    """Colour and per-splat terms of one pixel by the front-to-back sums
        C = sum_j c_j alpha_j T_j + T_fin bg,  T_j = prod_{k<j} (1 - alpha_k),
        dC/dc_j = alpha_j T_j,
        dC/dalpha_j = c_j T_j - (sum_{m>j} c_m alpha_m T_m + T_fin bg) / (1 - alpha_j),
    PHI falloff G = exp(-q/2).  Returns (C, T_fin, {index: 10 terms})."""
    g = np.asarray(g, np.float64)
    bg = np.asarray(bg, np.float64)
    T = 1.0
    used = []
    for j, s in enumerate(splats):
        dx, dy = s["u"] - px, s["v"] - py
        q = s["a"] * dx * dx + 2 * s["b"] * dx * dy + s["c"] * dy * dy
        if not q <= s["qmax"]:
            continue
        G = math.exp(-0.5 * max(q, 0.0))
        clamped = s["o"] * G > 0.99
        if j == flip_clamp_at:
            clamped = not clamped
        alpha = 0.99 if clamped else s["o"] * G
        stop = T * (1 - alpha) < 1e-4
        if j == flip_term_at:
            stop = not stop
        if stop:
            break
        used.append((j, alpha, T, G, q, dx, dy, clamped))
        T *= 1 - alpha
    Tfin = T
    C = sum(np.asarray(splats[j]["rgb"]) * a * t for j, a, t, *_ in used) + Tfin * bg
    terms = {}
    for k, (j, alpha, Tj, G, q, dx, dy, clamped) in enumerate(used):
        s = splats[j]
        behind = sum((np.asarray(splats[m]["rgb"]) * am * tm for m, am, tm, *_ in used[k + 1:]), np.zeros(3))
        dalpha = float(g @ (np.asarray(s["rgb"]) * Tj - (behind + Tfin * bg) / (1 - alpha)))
        v = np.zeros(10)
        v[6:9] = alpha * Tj * g
        if not clamped:
            v[5] = G * dalpha
            dq = -0.5 * G * s["o"] * dalpha
            v[0] = dq * 2 * (s["a"] * dx + s["b"] * dy)
            v[1] = dq * 2 * (s["b"] * dx + s["c"] * dy)
            v[2] = dq * dx * dx
            v[3] = dq * 2 * dx * dy
            v[4] = dq * dy * dy
        terms[j] = v
    return C, Tfin, terms


def _stack_for_termination(margin):
    """Three splats over pixel (0, 0) whose third brings T (1 - alpha) to 1e-4 (1 + margin)."""
    base = [dict(u=0.25, v=-0.125, a=0.5, b=0.0625, c=0.25, qmax=9.0, rgb=(0.9, 0.2, 0.4)),
            dict(u=-0.375, v=0.125, a=0.25, b=-0.03125, c=0.375, qmax=9.0, rgb=(0.1, 0.8, 0.3)),
            dict(u=0.125, v=0.25, a=0.375, b=0.0, c=0.5, qmax=9.0, rgb=(0.5, 0.5, 0.95))]
    G = [math.exp(-0.5 * (s["a"] * s["u"] ** 2 + 2 * s["b"] * s["u"] * s["v"] + s["c"] * s["v"] ** 2)) for s in base]
    alphas = [0.97, 0.96]
    for s, a, gg in zip(base, alphas, G):
        s["o"] = a / gg
    T2 = (1 - alphas[0]) * (1 - alphas[1])
    a3 = 1 - 1e-4 * (1 + margin) / T2
    base[2]["o"] = a3 / G[2]
    return base


def test_delta_is_the_other_termination_branch():
    sp = _stack_for_termination(4e-4)          # within the 1e-3 flag margin
    g = np.array([[[0.7, -1.3, 0.4]]])
    out, g2d, delta, mass, _ = _run(sp, 1, 1, g)
    assert out["flags"][0, 0] == 1
    C, _, prim = closed_form_pixel(sp, 0, 0, g[0, 0])
    _, _, alt = closed_form_pixel(sp, 0, 0, g[0, 0], flip_term_at=2)
    assert 2 in prim and 2 not in alt
    np.testing.assert_allclose(out["img"][0, 0], C, rtol=1e-9, atol=1e-12)
    for j in range(3):
        np.testing.assert_allclose(g2d[j], prim[j], rtol=1e-7, atol=1e-12)
        want = np.abs(alt.get(j, np.zeros(10)) - prim[j])
        np.testing.assert_allclose(delta[j], want, rtol=1e-7, atol=1e-12)
    assert delta[2, 6] > 0 and delta[0, 5] > 0
    # outside the margin: no flag, no allowance
    sp = _stack_for_termination(2e-3)
    out, _, delta, _, _ = _run(sp, 1, 1, g)
    assert out["flags"][0, 0] == 0 and not delta.any()


def test_delta_is_the_other_clamp_branch():
    sp = _stack_for_termination(0.5)            # termination far from its threshold
    for s in sp:
        s["o"] *= 0.3
    gq = math.exp(-0.5 * (sp[0]["a"] * sp[0]["u"] ** 2 + 2 * sp[0]["b"] * sp[0]["u"] * sp[0]["v"]
                          + sp[0]["c"] * sp[0]["v"] ** 2))
    sp[0]["o"] = (0.99 + 4e-6) / gq              # o G within 1e-5 of the clamp
    g = np.array([[[0.7, -1.3, 0.4]]])
    _, g2d, delta, _, _ = _run(sp, 1, 1, g)
    _, _, prim = closed_form_pixel(sp, 0, 0, g[0, 0])
    _, _, alt = closed_form_pixel(sp, 0, 0, g[0, 0], flip_clamp_at=0)
    assert not prim[0][:6].any() and alt[0][5] != 0     # clamped: no opacity or geometry gradient
    for j in range(3):
        np.testing.assert_allclose(g2d[j], prim[j], rtol=1e-7, atol=1e-12)
        np.testing.assert_allclose(delta[j], np.abs(alt[j] - prim[j]), rtol=1e-7, atol=1e-12)


def test_delta_vanishes_without_ambiguous_pixels(oracle_mod):
    cfg = synth.make_config(0)
    sc, cam = cfg["scene"], cfg["camera"]
    arr = {k: v.copy() for k, v in sc.arrays().items()}
    arr["opacity_logits"] = np.full_like(arr["opacity_logits"], -2.5)   # o = 0.076: T stays far above 1e-4
    orc = O.Oracle(arr, sc.sh_degree, cam)
    rec = orc.preprocess()
    _, vals, ranges = orc.build_keys(rec)
    out = orc.render(rec, vals, ranges)
    g = np.random.default_rng(5).standard_normal((cam.height, cam.width, 3))
    _, delta, mass, ebound, _ = orc.backward2d(rec, g, vals, ranges, with_delta=True)
    assert not out["flags"].any() and not delta.any()
    assert mass.any() and ebound.any()


def test_mass_is_the_sum_of_absolute_terms():
    rng = np.random.default_rng(11)
    sp = []
    for _ in range(3):
        sp.append(dict(u=_grid(rng, 2, 14), v=_grid(rng, 2, 14), a=_grid(rng, 0.05, 0.2), b=_grid(rng, -0.03, 0.03),
                       c=_grid(rng, 0.05, 0.2), qmax=_grid(rng, 6, 9), o=float(rng.uniform(0.2, 0.5)),
                       rgb=tuple(rng.uniform(0, 1, 3))))
    g = rng.standard_normal((16, 16, 3))
    _, g2d, delta, mass, _ = _run(sp, 16, 16, g)
    want_g = np.zeros((3, 10))
    want_m = np.zeros((3, 10))
    for py in range(16):
        for px in range(16):
            for j, s in enumerate(sp):    # no pixel may sit on an alpha-floor decision
                dx, dy = s["u"] - px, s["v"] - py
                q = s["a"] * dx * dx + 2 * s["b"] * dx * dy + s["c"] * dy * dy
                assert abs(q - s["qmax"]) > 1e-6
            _, _, terms = closed_form_pixel(sp, px, py, g[py, px])
            for j, v in terms.items():
                want_g[j] += v
                want_m[j] += np.abs(v)
    assert not delta.any()
    np.testing.assert_allclose(g2d[:, :9], want_g[:, :9], rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(mass[:, :9], want_m[:, :9], rtol=1e-9, atol=1e-15)
    assert (want_m[:, :9] > np.abs(want_g[:, :9]) * 1.01).any()   # some components cancel across pixels


# ---- the binary32 compositing branch -------------------------------------------------------------------
def _fma32(a, b, c):
    """binary32 fused multiply-add: the exact a*b + c, rounded once (Fraction arithmetic)."""
    from fractions import Fraction
    exact = Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c))
    f = F(float(exact))                      # nearest double, then nearest float ...
    lo, hi = (f, np.nextafter(f, F(np.inf))) if Fraction(float(f)) <= exact else (np.nextafter(f, F(-np.inf)), f)
    dlo, dhi = exact - Fraction(float(lo)), Fraction(float(hi)) - exact
    if dlo != dhi:                           # ... corrected to the nearest float of the exact value
        return lo if dlo < dhi else hi
    return lo if int(lo.view(np.uint32)) % 2 == 0 else hi


def test_f32_branch_decides_on_the_binary32_q():
    """A splat whose quadratic form rounds in binary32 to exactly its q_max: the binary32 branch composites
    it (q <= q_max), the binary64 branch skips it (the exact q exceeds q_max).  The pixel value is worked
    by hand from the binary32 q with G = exp(-q/2) in binary64."""
    rng = np.random.default_rng(1)
    for _ in range(10000):
        u, v = F(rng.uniform(0.1, 3.0)), F(rng.uniform(0.1, 3.0))
        a, b, c = F(rng.uniform(0.2, 1.0)), F(rng.uniform(-0.1, 0.1)), F(rng.uniform(0.2, 1.0))
        dx, dy = u - F(0.0), v - F(0.0)
        t = _fma32(a, dx, (b + b) * dy)
        q32 = _fma32(t, dx, (c * dy) * dy)
        q64 = float(a) * float(dx) ** 2 + 2.0 * float(b) * float(dx) * float(dy) + float(c) * float(dy) ** 2
        if q64 > float(q32) * (1 + 1e-12) and q32 > 0:
            break
    else:
        pytest.fail("no binary32 rounding-down case found")
    sp = [dict(u=float(u), v=float(v), a=float(a), b=float(b), c=float(c), qmax=float(q32), o=0.5,
               rgb=(0.75, 0.5, 0.25))]
    orc = _oracle(1, 1, 1)
    rec = _record(sp, 1, 1)
    _, vals, ranges = orc.build_keys(rec)
    img32 = orc.render(rec, vals, ranges, mode=O.MODE_F32)["img"][0, 0]
    img64 = orc.render(rec, vals, ranges, mode=O.MODE_F64)["img"][0, 0]
    alpha = 0.5 * math.exp(-0.5 * float(q32))
    np.testing.assert_allclose(img32, np.array([0.75, 0.5, 0.25]) * alpha, rtol=1e-15)
    assert not img64.any()


@pytest.mark.parametrize("falloff", [O.FALLOFF_PHI, O.FALLOFF_GEF], ids=["phi", "gef"])
def test_f32_branch_matches_f64_branch_on_the_same_records(oracle_mod, falloff):
    """Workload 0: the binary32 compositing branch against the binary64 one on the same (binary32) records.
    Only q differs (binary32 vs binary64 evaluation), so pixels agree to rounding unless an alpha-floor or
    termination decision falls the other way."""
    cfg = synth.make_config(0)
    sc, cam = cfg["scene"], cfg["camera"]
    orc = O.Oracle(sc.arrays(), sc.sh_degree, cam, falloff=falloff)
    rec = orc.preprocess(O.MODE_F32)
    _, vals, ranges = orc.build_keys(rec)
    a = orc.render(rec, vals, ranges, mode=O.MODE_F32)
    b = orc.render(rec, vals, ranges, mode=O.MODE_F64)
    same = (a["n_contrib"] == b["n_contrib"]) & ~a["flags"].astype(bool) & ~b["flags"].astype(bool)
    err = np.abs(a["img"] - b["img"]).max(axis=2)
    print(f"pixels compared {int(same.sum())} of {same.size}, max err {err[same].max():.2e}")
    assert same.mean() > 0.995
    assert err[same].max() < 2e-6
    assert np.abs(a["final_T"] - b["final_T"])[same].max() < 2e-6


# ---- the binary32 evaluation bound ---------------------------------------------------------------------
K_PHI = F(-0.5 * math.log2(math.e))


def _tr(x, mode):
    """A transcendental result: the exact value rounded to binary32 to nearest (mode 0), up (1) or down (-1)."""
    f = F(x)
    if mode > 0 and float(f) < x:
        f = np.nextafter(f, F(np.inf))
    elif mode < 0 and float(f) > x:
        f = np.nextafter(f, F(-np.inf))
    return f


def emulate_pixel(splats, px, py, g, bg, falloff, mode):
    """Independent binary32 compositor: forward front to back, backward back to front recovering T by
    T / (1 - alpha) (reciprocal then product).  Returns (n_composited, {index: 10 binary32 terms})."""
    g = [F(x) for x in g]
    bgv = [F(x) for x in bg]
    T = F(1.0)
    used = []
    for j, s in enumerate(splats):
        u, v, a, b, c, qmax, o, beta = (F(s[k]) for k in ("u", "v", "a", "b", "c", "qmax", "o", "beta"))
        dx, dy = u - F(px), v - F(py)
        q = F(float(a) * float(dx) ** 2 + 2.0 * float(b) * float(dx) * float(dy) + float(c) * float(dy) ** 2)
        if not q <= qmax:
            continue
        qc = max(q, F(0.0))
        l = qb = F(0.0)
        if falloff == O.FALLOFF_PHI:
            G = _tr(2.0 ** float(K_PHI * qc), mode)
        elif qc > 0:
            l = _tr(math.log2(float(qc)), mode)
            qb = _tr(2.0 ** float(F(0.5) * beta * l), mode)
            G = _tr(2.0 ** float(K_PHI * qb), mode)
        else:
            G = F(1.0)
        oG = o * G
        clamped = oG > F(0.99)
        alpha = F(0.99) if clamped else oG
        t = T * (F(1.0) - alpha)
        if t < F(1e-4):
            break
        used.append((j, alpha, G, q, qc, l, qb, dx, dy, clamped))
        T = t
    Tfin = T
    bgg = bgv[0] * g[0] + bgv[1] * g[1] + bgv[2] * g[2]
    S = [F(0.0)] * 3
    terms = {}
    for (j, alpha, G, q, qc, l, qb, dx, dy, clamped) in reversed(used):
        s = splats[j]
        a, b, c, o, beta = (F(s[k]) for k in ("a", "b", "c", "o", "beta"))
        col = [F(x) for x in s["rgb"]]
        inv = _tr(1.0 / float(F(1.0) - alpha), mode)
        T = T * inv
        out = np.zeros(10)
        w = alpha * T
        for ch in range(3):
            out[6 + ch] = w * g[ch]
        d = [col[ch] - S[ch] for ch in range(3)]
        dalpha = (d[0] * g[0] + d[1] * g[1] + d[2] * g[2]) * T - Tfin * bgg * inv
        for ch in range(3):
            S[ch] = S[ch] + alpha * d[ch]
        if not clamped:
            gd = G * dalpha
            out[5] = gd
            if q < 0:
                dq = F(0.0)
            elif falloff == O.FALLOFF_PHI:
                dq = F(-0.5) * o * gd
            else:
                qf = max(qc, F(1e-12))
                qpow = _tr(2.0 ** float((F(0.5) * beta - F(1.0)) * _tr(math.log2(float(qf)), mode)), mode)
                dq = (F(-0.25) * beta * o) * qpow * gd
                if qc > 0:
                    out[9] = (F(-0.25 * math.log(2.0)) * o) * (qb * l) * gd
            out[0] = F(2.0) * dq * (a * dx + b * dy)
            out[1] = F(2.0) * dq * (b * dx + c * dy)
            out[2] = dq * (dx * dx)
            out[3] = F(2.0) * dq * (dx * dy)
            out[4] = dq * (dy * dy)
        terms[j] = out
    return len(used), terms


def _random_stack(rng, n, falloff, similar=False):
    """n splats over pixel (0, 0); similar=True gives every splat nearly the same colour, so that the colour
    behind each splat cancels its own in dL/dalpha."""
    base = rng.uniform(0, 1, 3)
    sp = []
    for _ in range(n):
        hi = rng.random() < 0.5
        rgb = base + rng.uniform(-0.01, 0.01, 3) if similar else rng.uniform(0, 1, 3)
        sp.append(dict(u=_grid(rng, -1.5, 1.5), v=_grid(rng, -1.5, 1.5), a=_grid(rng, 0.1, 1.0),
                       b=_grid(rng, -0.1, 0.1), c=_grid(rng, 0.1, 1.0), qmax=_grid(rng, 4.0, 11.0),
                       o=float(F(rng.uniform(0.85, 1.0) if hi else rng.uniform(0.05, 0.85))),
                       rgb=tuple(float(F(x)) for x in rgb),
                       beta=float(F(rng.uniform(0.5, 4.0))) if falloff == O.FALLOFF_GEF else 2.0))
    return sp


@pytest.mark.parametrize("falloff", [O.FALLOFF_PHI, O.FALLOFF_GEF], ids=["phi", "gef"])
def test_ebound_bounds_a_binary32_compositor(falloff):
    """One pixel, stacks of 2-14 splats with opacities up to 1 (deep transmittance, clamps), backgrounds on and
    off, transcendentals rounded to nearest / up / down: every binary32 term lies within the oracle's bound
    of the binary64 term, and the bound is reached to within a factor 30 somewhere (it is not vacuous)."""
    rng = np.random.default_rng(2024 + falloff)
    worst = 0.0
    checked = 0
    for trial in range(600):
        sp = _random_stack(rng, int(rng.integers(2, 15)), falloff, similar=trial % 3 == 2)
        g = rng.standard_normal(3)
        bg = (0.0, 0.0, 0.0) if trial % 2 == 0 else tuple(float(F(x)) for x in rng.uniform(0, 1, 3))
        out, g2d, delta, mass, ebound = _run(sp, 1, 1, g.reshape(1, 1, 3), falloff, bg)
        if out["flags"].any() or delta.any():
            continue       # ambiguous decisions are delta's business
        for mode in (0, 1, -1):
            nc, terms = emulate_pixel(sp, 0, 0, g, bg, falloff, mode)
            if nc != len([j for j in range(len(sp)) if g2d[j].any() or mass[j].any()]):
                continue
            for j, v in terms.items():
                err = np.abs(v - g2d[j])
                assert np.all(err <= ebound[j] * (1 + 1e-9) + 1e-300), (trial, mode, j, err, ebound[j])
                nz = ebound[j] > 0
                if nz.any():
                    worst = max(worst, float((err[nz] / ebound[j][nz]).max()))
                checked += 1
    print(f"terms checked {checked}, largest error / bound {worst:.3f}")
    assert checked > 1000
    assert worst > 1.0 / 30.0


def test_ebound_and_mass_bound_a_binary32_tile_sum():
    """A 16x16 tile, 40 splats: binary32 terms summed per splat in binary32 pixel by pixel (serial order)
    stay within ebound + gamma_255 * mass of the oracle's binary64 gradient."""
    rng = np.random.default_rng(77)
    sp = []
    for _ in range(40):
        sp.append(dict(u=_grid(rng, -2, 18), v=_grid(rng, -2, 18), a=_grid(rng, 0.02, 0.3), b=_grid(rng, -0.02, 0.02),
                       c=_grid(rng, 0.02, 0.3), qmax=_grid(rng, 5.0, 11.0), o=float(F(rng.uniform(0.1, 0.99))),
                       rgb=tuple(float(F(x)) for x in rng.uniform(0, 1, 3)), beta=2.0))
    g = rng.standard_normal((16, 16, 3)).astype(np.float32)
    out, g2d, delta, mass, ebound = _run(sp, 16, 16, g.astype(np.float64))
    sums = np.zeros((40, 10), np.float32)
    for py in range(16):
        for px in range(16):
            _, terms = emulate_pixel(sp, px, py, g[py, px], (0.0, 0.0, 0.0), O.FALLOFF_PHI, 1)
            for j, v in terms.items():
                sums[j] = sums[j] + v.astype(np.float32)
    gamma = 255 * U32 / (1 - 255 * U32)
    allow = delta + ebound + gamma * mass
    err = np.abs(sums.astype(np.float64) - g2d)
    assert np.all(err <= allow * (1 + 1e-9) + 1e-300)
    assert mass.sum() > 0 and (err > 0).any()


@pytest.mark.parametrize("falloff", [O.FALLOFF_PHI, O.FALLOFF_GEF], ids=["phi", "gef"])
def test_ebound_single_splat_far_from_the_centre(falloff):
    """One splat near its alpha floor (q close to q_max, the largest exponent argument): the rounding of the
    argument of exp2 dominates there.  Every term within the bound; the colour term reaches it closely."""
    rng = np.random.default_rng(99 + falloff)
    worst = 0.0
    for trial in range(3000):
        a, c = _grid(rng, 0.2, 1.0), _grid(rng, 0.2, 1.0)
        u, v = _grid(rng, 1.0, 3.0), _grid(rng, 1.0, 3.0)
        q = a * u * u + c * v * v
        sp = [dict(u=u, v=v, a=a, b=0.0, c=c, qmax=q + 1.0 / 64, o=float(F(rng.uniform(0.3, 0.98))),
                   rgb=tuple(float(F(x)) for x in rng.uniform(0.2, 1, 3)),
                   beta=float(F(rng.uniform(0.5, 4.0))) if falloff == O.FALLOFF_GEF else 2.0)]
        g = rng.standard_normal(3)
        out, g2d, delta, mass, ebound = _run(sp, 1, 1, g.reshape(1, 1, 3), falloff)
        for mode in (1, -1):
            _, terms = emulate_pixel(sp, 0, 0, g, (0.0, 0.0, 0.0), falloff, mode)
            err = np.abs(terms[0] - g2d[0])
            assert np.all(err <= ebound[0] * (1 + 1e-9) + 1e-300), (trial, mode, err, ebound[0])
            worst = max(worst, float((err[6:9] / ebound[0][6:9]).max()))
    print(f"largest colour-term error / bound {worst:.3f}")
    assert worst > 0.4
