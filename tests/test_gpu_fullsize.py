"""Parity at full workload sizes, in the launch configuration the benchmark times.

The oracle cannot render a 3M-splat 1080p frame in seconds, so these tests compare
  * every per-splat record (bit-exact), every tile range and the key count (bit-exact, from the
    oracle's per-tile counts over the whole frame);
  * the sorted list, the image and n_contrib of ~60 sampled tiles: random ones, a 4x4 block and the
    tile with the longest list;
  * gradients of a loss whose image gradient is non-zero only on the sampled tiles, so that the
    oracle's backward over those tiles is the exact full gradient: 2-D accumulators of every splat,
    and parameter gradients of every splat those tiles reach (all others must be exactly zero).
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import preprocess_f64 as PF
from paper_2402_10128_amd import synth

from .parity_helpers import (GRAD_RTOL, IMG_ATOL, allowance2d, ambiguous_splats, assert_grad_ok, gpu_render,
                             grad2d_check, grad3d_check, image_compare, record_mismatches)

pytestmark = pytest.mark.gpu

FULL = [
    # (name, workload, falloff)
    ("w1_1M_1600x1040_phi", 1, O.FALLOFF_PHI),
    ("w1_1M_1600x1040_gef", 1, O.FALLOFF_GEF),
    ("w2_3M_1080p_phi", 2, O.FALLOFF_PHI),
    ("w3_5M_1080p_overlap_phi", 3, O.FALLOFF_PHI),
]


def _sample_tiles(counts, TX, TY, seed):
    rng = np.random.default_rng(seed)
    T = TX * TY
    pick = set(rng.choice(T, size=min(40, T), replace=False).tolist())
    cx, cy = TX // 2 - 2, TY // 2 - 2
    pick.update((cy + dy) * TX + cx + dx for dy in range(4) for dx in range(4))
    pick.add(int(np.argmax(counts)))
    return np.array(sorted(pick), np.int32)


@pytest.mark.parametrize("case", FULL, ids=[c[0] for c in FULL])
def test_full_size_sampled_parity(case):
    name, wl, falloff = case
    cull = O.TILES_ELLIPSE
    cfg = synth.make_config(wl)
    sc, cam = cfg["scene"], cfg["camera"]
    arr = sc.arrays()
    print(f"[fullsize] {name}: {sc.n} splats {cam.width}x{cam.height}", flush=True)
    orc = O.Oracle(arr, sc.sh_degree, cam, falloff=falloff, tile_cull=cull)
    rec = orc.preprocess(O.MODE_F32)
    counts = orc.tile_counts(rec)
    TX, TY = orc.TX, orc.TY
    tiles = _sample_tiles(counts, TX, TY, seed=wl)
    # image gradient: random on the sampled tiles, zero elsewhere
    rng = np.random.default_rng(100 + wl)
    dL = np.zeros((cam.height, cam.width, 3), np.float32)
    pix_mask = np.zeros((cam.height, cam.width), bool)
    for t in tiles:
        x0, y0 = (t % TX) * 16, (t // TX) * 16
        blk = dL[y0:y0 + 16, x0:x0 + 16]
        blk[...] = rng.standard_normal(blk.shape).astype(np.float32)
        pix_mask[y0:y0 + 16, x0:x0 + 16] = True
    gpu = gpu_render(arr, sc.sh_degree, cam, falloff, cull, dL=dL)

    mm = record_mismatches(gpu["records"], rec)
    print("  record mismatches", mm, flush=True)
    assert all(v == 0 for v in mm.values()), mm
    K = int(counts.sum())
    assert gpu["keys"] == K and gpu["num_keys"] >= K, (gpu["keys"], gpu["num_keys"], K)
    assert np.array_equal(gpu["sorted_tiles"], np.repeat(np.arange(TX * TY), counts)), "sorted tile ids differ"
    ends = np.cumsum(counts)
    ref_ranges = np.stack([ends - counts, ends], 1)
    ref_ranges[counts == 0] = 0
    assert np.array_equal(gpu["ranges"].astype(np.int64), ref_ranges), "tile ranges differ"

    # per sampled tile: the sorted list, then the oracle's render/backward over those tiles
    vals, ranges, pos = [], np.zeros((TX * TY, 2), np.int64), 0
    for t in tiles:
        lst = orc.tile_list(rec, int(t))
        g0, g1 = gpu["ranges"][t]
        assert np.array_equal(gpu["sorted_ids"][int(g0):int(g1)], lst), f"sorted list of tile {t} differs"
        ranges[t] = (pos, pos + len(lst))
        pos += len(lst)
        vals.append(lst)
    values = np.concatenate(vals).astype(np.uint32)
    print(f"  {len(tiles)} tiles sampled, longest list {int(counts.max())}, K={K}", flush=True)
    out = orc.render(rec, values, ranges, tiles=tiles)
    cmp = image_compare(gpu["img"], out, pixels_mask=pix_mask)
    print("  image", cmp, flush=True)
    assert cmp["max_err"] <= IMG_ATOL and cmp["flagged_max_err"] <= IMG_ATOL, cmp
    unf = pix_mask & ~out["flags"].astype(bool)
    assert np.array_equal(gpu["n_contrib"][unf], out["n_contrib"][unf].astype(np.uint32))

    g2d, delta, mass, ebound, _ = orc.backward2d(rec, dL.astype(np.float64), values, ranges, tiles=tiles, with_delta=True)
    ncomp = 10 if falloff == O.FALLOFF_GEF else 9
    chk = grad2d_check(gpu["grad2d"][:, :ncomp], g2d[:, :ncomp], delta[:, :ncomp], mass[:, :ncomp],
                       ebound[:, :ncomp])
    assert_grad_ok("grad2d", chk)

    reach = np.abs(g2d).sum(axis=1) > 0
    idx = np.nonzero(reach)[0]
    sub = {k: v[idx] for k, v in arr.items()}
    vis = rec.tiles_touched[idx] > 0
    clamp = rec.clamp_bits[idx]
    ref = PF.chain_to_params(sub, sc.sh_degree, cam, g2d[idx], vis, clamp, falloff, 0.1)
    allow = PF.abs_chain(sub, sc.sh_degree, cam, allowance2d(delta[idx], ebound[idx], mass[idx]), vis, clamp,
                         falloff, 0.1)
    amb = ambiguous_splats(g2d[idx, :ncomp], delta[idx, :ncomp])
    print(f"  {len(idx)} splats reached, {int(amb.sum())} with an ambiguous decision", flush=True)
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "beta"):
        g = gpu["grads"][k]
        rest = np.ones(g.shape[0], bool)
        rest[idx] = False
        assert not np.any(g[rest]), f"{k}: gradient of a splat outside the sampled tiles"
        assert_grad_ok(k, grad3d_check(g[idx], ref[k], allow[k]))
