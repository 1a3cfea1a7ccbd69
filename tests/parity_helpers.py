"""Helpers for the GPU-vs-oracle parity tests: run both sides on the same seeded inputs and compare.

Tolerances (stated per result):
  * per-splat records, keys, sort order, tile ranges: bit-exact (mismatch count must be 0);
  * image: <= 1e-5 absolute per FP32 channel on pixels whose termination decision is not within
    1e-3 (relative) of the 1e-4 threshold; flagged pixels must match one of the two branches;
  * gradients: |g - r| / max(|r|, 1e-2 * rms(r)) <= 1e-3 per tensor, beyond a derived allowance for what
    a binary32 implementation may legitimately differ by (allowance2d); entries whose allowance is
    negligible are held to the plain bound, and the entries that pass only through the allowance are
    counted and reported.
"""
from __future__ import annotations

import numpy as np
import torch

from oracle import oracle as O
from oracle import preprocess_f64 as PF
from paper_2402_10128_amd import ges as G

IMG_ATOL = 1e-5
GRAD_RTOL = 1e-3
GRAD_FLOOR = 1e-2
# Rounding of the GPU's sums of per-pixel terms.  A term reaches its (tile, splat) sum through at most 12
# binary32 roundings: 4 pixels accumulated per lane, 16 lanes per row reduced in 4 levels, 4 rows in 2,
# the splat's scale factor (o times the constant of dG/dq, or 2), and spares; the per-tile sums are
# then added in binary64 (at most 8,160 tiles).  Hence |error| <= gamma_12 * sum|terms| (Higham, Sec. 4.2),
# with sum|terms| the oracle's `mass`.
U32 = 2.0 ** -24
TILE_SUM_ROUNDINGS = 12
GAMMA_SUM = TILE_SUM_ROUNDINGS * U32 / (1.0 - TILE_SUM_ROUNDINGS * U32) + 8160 * 2.0 ** -53


def to_device(arrays: dict, device="cuda"):
    return {k: torch.as_tensor(np.ascontiguousarray(v, np.float32)).to(device) for k, v in arrays.items()}


def gpu_render(arrays, sh_degree, cam, falloff=0, tile_cull=0, rho=0.1, bg=(0.0, 0.0, 0.0), dL=None):
    """Forward (+ optional backward) on the GPU; returns numpy results and the frame arrays."""
    sc = to_device(arrays)
    s = G.splats_struct(sc["means"], sc["log_scales"], sc["quats"], sc["opacity_logits"], sc["sh"], sc["beta"])
    c = G.camera_struct(cam)
    p = G.params_struct(falloff, tile_cull, rho, bg, flags=G.RASTER_KEEP_GRAD2D)
    frame = G.Frame.create(s.n, c.width, c.height)
    k = G.ges_preprocess(s, c, p, frame.splat_ws, True)
    frame.ensure_keys(k)
    out = torch.empty((c.height, c.width, 3), dtype=torch.float32, device="cuda")
    G.ges_render_forward(s, c, p, frame.splat_ws, frame.key_ws, k, frame.pixel_ws, out)
    res = dict(img=out.cpu().numpy(), num_keys=k)
    if dL is not None:
        grads = {kk: torch.empty_like(sc[kk]) for kk in ("means", "log_scales", "quats", "opacity_logits", "sh", "beta")}
        G.ges_render_backward(s, c, p, frame.splat_ws, frame.key_ws, frame.pixel_ws,
                              torch.as_tensor(np.ascontiguousarray(dL, np.float32)).cuda(), grads)
        res["grads"] = {kk: v.cpu().numpy() for kk, v in grads.items()}
    torch.cuda.synchronize()
    res.update(G.frame_arrays(frame, s.n))
    return res


RECORD_FIELDS = [("u", 0), ("v", 1), ("a", 2), ("b", 3), ("c", 4), ("qmax", 5), ("opacity", 6), ("beta", 7),
                 ("r", 8), ("g", 9), ("b_", 10), ("depth", 11)]


def record_mismatches(gpu_rec: np.ndarray, orc: O.Record) -> dict:
    """Mismatch counts per record field, binary32 bits vs the oracle's F32 record (visible splats)."""
    vis = orc.tiles_touched > 0
    gvis = gpu_rec[:, 15].view(np.uint32) > 0
    out = {"visible": int((vis != gvis).sum())}
    ref = {"u": orc.u, "v": orc.v, "a": orc.conic[:, 0], "b": orc.conic[:, 1], "c": orc.conic[:, 2],
           "qmax": orc.qmax, "opacity": orc.opacity, "beta": orc.beta, "r": orc.rgb[:, 0], "g": orc.rgb[:, 1],
           "b_": orc.rgb[:, 2], "depth": orc.depth}
    both = vis & gvis
    for name, col in RECORD_FIELDS:
        g = gpu_rec[both, col].view(np.uint32)
        r = ref[name][both].astype(np.float32).view(np.uint32)
        out[name] = int((g != r).sum())
    words = gpu_rec.view(np.uint32)
    radius = (words[:, 12] & 0xFFFFFF).astype(np.int64)
    flags = (words[:, 12] >> 24).astype(np.int64)
    out["radius"] = int((radius[both] != orc.radius[both]).sum())
    out["flags"] = int((flags[both] != orc.clamp_bits[both]).sum())
    rect = np.stack([words[:, 13] & 0xFFFF, words[:, 13] >> 16, words[:, 14] & 0xFFFF, words[:, 14] >> 16], 1)
    out["rect"] = int((rect[both] != orc.rect[both]).any(axis=1).sum())
    out["tiles_touched"] = int((words[both, 15].astype(np.int64) != orc.tiles_touched[both]).sum())
    return out


def image_compare(gpu_img, orc_out, pixels_mask=None):
    """Max error on unflagged pixels, and whether every flagged pixel matches one branch."""
    ref, alt, fl = orc_out["img"], orc_out["alt"], orc_out["flags"].astype(bool)
    if pixels_mask is None:
        pixels_mask = np.ones(fl.shape, bool)
    err = np.abs(gpu_img.astype(np.float64) - ref).max(axis=2)
    unf = pixels_mask & ~fl
    flagged = pixels_mask & fl
    err_alt = np.abs(gpu_img.astype(np.float64) - alt).max(axis=2)
    flag_ok = np.minimum(err, err_alt)[flagged]
    return dict(max_err=float(err[unf].max()) if unf.any() else 0.0,
                p99_err=float(np.percentile(err[unf], 99)) if unf.any() else 0.0,
                flagged=int(flagged.sum()),
                flagged_max_err=float(flag_ok.max()) if flagged.any() else 0.0)


def grad_rel_err(g, r):
    g = np.asarray(g, np.float64).ravel()
    r = np.asarray(r, np.float64).ravel()
    rms = np.sqrt(np.mean(r * r)) if r.size else 0.0
    floor = max(GRAD_FLOOR * rms, 1e-30)
    rel = np.abs(g - r) / np.maximum(np.abs(r), floor)
    nrm = np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-30)
    return dict(max=float(rel.max()) if rel.size else 0.0, p99=float(np.percentile(rel, 99)) if rel.size else 0.0,
                norm=float(nrm))


def allowance2d(delta, ebound, mass):
    """Per 2-D component: the other branch of ambiguous decisions (delta), the first-order binary32 error
    bound of the per-pixel terms (ebound) and the rounding of their binary32 sums (GAMMA_SUM * mass)."""
    return delta + ebound + GAMMA_SUM * mass


def _excess(g, r, allow, floor):
    """Error beyond the allowance relative to max(|r|, floor); counts of entries that pass only through the
    allowance, and the largest plain relative error over entries whose allowance is negligible
    (below 1e-4 of max(|r|, floor)): those must meet the plain bound."""
    scale = np.maximum(np.abs(r), floor)
    err = np.abs(g - r)
    excess = np.maximum(err - allow, 0.0) / scale
    plain = err / scale
    negligible = allow <= 1e-4 * scale
    return dict(max=float(excess.max()) if excess.size else 0.0,
                only_by_allowance=int(((plain > GRAD_RTOL) & (excess <= GRAD_RTOL)).sum()),
                entries=int(excess.size),
                plain_max_negligible_allowance=float(plain[negligible].max()) if negligible.any() else 0.0,
                allowance_over_tol_median=float(np.median(allow / scale / GRAD_RTOL)) if excess.size else 0.0)


def grad2d_check(g, r, delta, mass, ebound):
    """2-D accumulators against the oracle (see _excess); ambiguous entries are those with delta > 0."""
    g = np.asarray(g, np.float64)
    r = np.asarray(r, np.float64)
    floor = np.maximum(GRAD_FLOOR * np.sqrt(np.mean(r * r, axis=0, keepdims=True)), 1e-30)
    out = _excess(g, r, allowance2d(delta, ebound, mass), floor)
    out["ambiguous_entries"] = int((delta > 0).sum())
    return out


def grad3d_check(g, r, allow):
    """Parameter gradients: error beyond the propagated allowance |J|^T a (see _excess)."""
    g = np.asarray(g, np.float64).ravel()
    r = np.asarray(r, np.float64).ravel()
    a = np.asarray(allow, np.float64).ravel()
    floor = max(GRAD_FLOOR * np.sqrt(np.mean(r * r)), 1e-30) if r.size else 1.0
    return _excess(g, r, a, floor)


def assert_grad_ok(name, res):
    """The parity bound: nothing beyond the allowance, and the plain bound where the allowance is negligible."""
    print(f"  {name}: beyond allowance {res['max']:.2e}, passing only by the allowance {res['only_by_allowance']} "
          f"of {res['entries']}, plain max where the allowance is negligible "
          f"{res['plain_max_negligible_allowance']:.2e}, median allowance / tolerance "
          f"{res['allowance_over_tol_median']:.2e}", flush=True)
    assert res["max"] <= GRAD_RTOL, (name, res)
    assert res["plain_max_negligible_allowance"] <= GRAD_RTOL, (name, res)


def ambiguous_splats(r2d, delta):
    """Splats whose 2-D gradient may legitimately move by at least a tenth of the tolerance because of a
    floating-point-ambiguous decision in one of their pixels (see grad2d_check).  Their parameter
    gradients are reported but not held to the strict bound, since the allowance passes through the
    preprocess chain rule unbounded by a simple per-component factor."""
    floor = np.maximum(GRAD_FLOOR * np.sqrt(np.mean(r2d * r2d, axis=0, keepdims=True)), 1e-30)
    return (delta > 0.1 * GRAD_RTOL * np.maximum(np.abs(r2d), floor)).any(axis=1)


def oracle_full(arrays, sh_degree, cam, falloff=0, tile_cull=0, rho=0.1, bg=(0.0, 0.0, 0.0), dL=None):
    orc = O.Oracle(arrays, sh_degree, cam, falloff=falloff, tile_cull=tile_cull, rho=rho, bg=bg)
    rec = orc.preprocess(O.MODE_F32)
    keys, vals, ranges = orc.build_keys(rec)
    out = orc.render(rec, vals, ranges)
    res = dict(orc=orc, rec=rec, keys=keys, values=vals, ranges=ranges, out=out)
    if dL is not None:
        g2d, delta, mass, ebound, _ = orc.backward2d(rec, dL, vals, ranges, with_delta=True)
        res["g2d"] = g2d
        res["delta"] = delta
        res["mass"] = mass
        res["ebound"] = ebound
        vis = rec.tiles_touched > 0
        res["grads"] = PF.chain_to_params(arrays, sh_degree, cam, g2d, vis, rec.clamp_bits, falloff, rho)
        res["allow"] = PF.abs_chain(arrays, sh_degree, cam, allowance2d(delta, ebound, mass), vis, rec.clamp_bits,
                                    falloff, rho)
    return res
