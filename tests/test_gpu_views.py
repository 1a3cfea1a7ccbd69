"""Several views of one scene per launch sequence (the ..._views calls) on the GPU.

Each view of a batched step must be exactly what the single-view calls give for it: records, tile ranges,
every tile's sorted list, image, final transmittance, n_contrib and the 2-D gradients are compared bit for
bit, and the summed parameter gradients against the single-view backward of view 0 followed by the
accumulating backward of the others (Sec. 4.2, Eq. transimttance; Sec. 4.4).  The summed gradients are also
held to the oracle's per-view sum, and the batched optimisation step to the one-view-at-a-time step.
"""
import numpy as np
import pytest
import torch

from paper_2402_10128_amd import ges as G
from paper_2402_10128_amd import synth
from paper_2402_10128_amd.train import GROUP_ORDER, TrainConfig, TrainStep

from .parity_helpers import assert_grad_ok, grad3d_check, oracle_full, to_device

pytestmark = pytest.mark.gpu

CASES = [
    # (name, splats, width, height, views, falloff, tile_cull)
    ("20k_256x192_3views_phi_ellipse", 20_000, 256, 192, 3, G.FALLOFF_PHI, G.TILES_ELLIPSE),
    ("20k_200x136_4views_gef_square", 20_000, 200, 136, 4, G.FALLOFF_GEF, G.TILES_SQUARE),
    ("5k_75x61_3views_gef_ellipse", 5_000, 75, 61, 3, G.FALLOFF_GEF, G.TILES_ELLIPSE),   # ragged tiles
]


def _cams(w, h, views, seed):
    rng = np.random.default_rng(seed)
    return [synth.orbit_camera(rng, w, h) for _ in range(views)]


def _sequential(t, s, cams, p, dLs, n, w, h):
    """Every view through the single-view calls: per-view arrays and the accumulated gradients."""
    frame = G.Frame.create(n, w, h, "cuda")
    grads = {k: torch.empty_like(x) for k, x in t.items()}
    per_view, view_grads = [], []
    for v, cam in enumerate(cams):
        c = G.camera_struct(cam)
        k = G.ges_preprocess(s, c, p, frame.splat_ws, True)
        frame.ensure_keys(k)
        img = torch.empty((h, w, 3), device="cuda")
        G.ges_render_forward(s, c, p, frame.splat_ws, frame.key_ws, k, frame.pixel_ws, img)
        ws = (s, c, p, frame.splat_ws, frame.key_ws, frame.pixel_ws, dLs[v])
        if v == 0:
            G.ges_render_backward(*ws, grads)
        else:
            G.ges_render_backward_accumulate(*ws, grads)
        a = G.frame_arrays(frame, n)
        a["img"] = img.cpu().numpy()
        per_view.append(a)
        gv = {k: torch.empty_like(x) for k, x in t.items()}   # this view's gradients alone
        G.ges_render_backward(*ws, gv)
        view_grads.append(gv)
    return per_view, grads, view_grads


def _struct(t):
    return G.splats_struct(*(t[k] for k in G.SPLAT_PARAMS))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_views_equal_single_view_calls(case):
    name, n, w, h, views, falloff, cull = case
    print(f"[views] {name}", flush=True)
    sc = synth.scene_clusters(n, 900)
    t = to_device(sc.arrays())
    s = _struct(t)
    cams = _cams(w, h, views, 901)
    p = G.params_struct(falloff, cull, 0.1, (0.0, 0.0, 0.0), flags=G.RASTER_KEEP_GRAD2D)
    rng = np.random.default_rng(902)
    dL = torch.as_tensor(rng.standard_normal((views, h, w, 3)).astype(np.float32)).cuda()
    seq, seq_grads, view_grads = _sequential(t, s, cams, p, [dL[v] for v in range(views)], n, w, h)

    frame = G.Frame.create(n, w, h, "cuda", views=views)
    cs = [G.camera_struct(c) for c in cams]
    k = G.ges_preprocess_views(s, cs, p, frame.splat_ws, True)
    keys = sum(int(a["stats"][0]) for a in seq)
    assert k == keys if cull == G.TILES_SQUARE else k >= keys, (k, keys)
    frame.ensure_keys(k)
    imgs = torch.empty((views, h, w, 3), device="cuda")
    G.ges_render_forward_views(s, cs, p, frame.splat_ws, frame.key_ws, k, frame.pixel_ws, imgs)
    grads = {g: torch.empty_like(x) for g, x in t.items()}
    G.ges_render_backward_views(s, cs, p, frame.splat_ws, frame.key_ws, frame.pixel_ws, dL, grads)
    torch.cuda.synchronize()
    tiles = seq[0]["ranges"].shape[0]
    base = 0
    for v in range(views):
        a = G.frame_arrays(frame, n, view=v)
        r = seq[v]
        assert np.array_equal(a["records"].view(np.uint32), r["records"].view(np.uint32)), (v, "records")
        assert int(a["stats"][0]) == int(r["stats"][0]) and int(a["stats"][1]) == 0, (v, "key count / error word")
        # batch ranges are offsets into the batch's sorted pairs: the same lists, shifted
        lens_a = a["ranges"][:, 1].astype(np.int64) - a["ranges"][:, 0]
        lens_r = r["ranges"][:, 1].astype(np.int64) - r["ranges"][:, 0]
        assert np.array_equal(lens_a, lens_r), (v, "tile list lengths")
        for tile in np.nonzero(lens_r)[0]:
            g0, g1 = a["ranges"][tile]
            q0, q1 = r["ranges"][tile]
            assert np.array_equal(a["sorted_ids"][g0:g1], r["sorted_ids"][q0:q1]), (v, tile)
            assert np.all(a["sorted_tiles"][g0:g1] == v * tiles + tile), (v, tile)
        base += int(lens_r.sum())
        assert np.array_equal(imgs[v].cpu().numpy().view(np.uint32), r["img"].view(np.uint32)), (v, "image")
        assert np.array_equal(a["final_T"].view(np.uint32), r["final_T"].view(np.uint32)), (v, "final_T")
        assert np.array_equal(a["n_contrib"], r["n_contrib"]), (v, "n_contrib")
        assert np.array_equal(a["grad2d"][:, :10].view(np.uint64), r["grad2d"][:, :10].view(np.uint64)), (v, "grad2d")
    assert base == sum(int(a["stats"][0]) for a in seq)
    for g in G.SPLAT_PARAMS:
        assert torch.equal(grads[g], seq_grads[g]), g
    # accumulate = 1 adds every view's gradients once more, in view order
    twice = {g: x.clone() for g, x in grads.items()}
    G.ges_render_backward_views(s, cs, p, frame.splat_ws, frame.key_ws, frame.pixel_ws, dL, twice, accumulate=True)
    for g in G.SPLAT_PARAMS:
        want = grads[g].clone()
        for gv in view_grads:
            want = want + gv[g]
        assert torch.equal(twice[g], want), g


def test_views_gradients_match_the_oracle_sum():
    """Three views of the 1,000-splat 64x64 workload, batched: the summed parameter gradients against the sum
    of the oracle's per-view gradients, per element, beyond the summed allowances."""
    cfg_w = synth.make_config(0)
    sc, cam0 = cfg_w["scene"], cfg_w["camera"]
    cams = [cam0, synth.pinhole(cam0.width, cam0.height, (0.6, -0.4, -3.8)),
            synth.pinhole(cam0.width, cam0.height, (-0.9, 0.3, -3.5))]
    arrays = sc.arrays()
    rng = np.random.default_rng(23)
    dLs = rng.standard_normal((3, cam0.height, cam0.width, 3)).astype(np.float32)
    refs = [oracle_full(arrays, sc.sh_degree, c, 0, 1, dL=d.astype(np.float64)) for c, d in zip(cams, dLs)]
    t = to_device(arrays)
    s = _struct(t)
    p = G.params_struct(0, 1, 0.1, (0.0, 0.0, 0.0))
    frame = G.Frame.create(s.n, cam0.width, cam0.height, "cuda", views=3)
    cs = [G.camera_struct(c) for c in cams]
    k = G.ges_preprocess_views(s, cs, p, frame.splat_ws, True)
    frame.ensure_keys(k)
    imgs = torch.empty((3, cam0.height, cam0.width, 3), device="cuda")
    G.ges_render_forward_views(s, cs, p, frame.splat_ws, frame.key_ws, k, frame.pixel_ws, imgs)
    grads = {g: torch.empty_like(x) for g, x in t.items()}
    G.ges_render_backward_views(s, cs, p, frame.splat_ws, frame.key_ws, frame.pixel_ws,
                                torch.from_numpy(dLs).cuda(), grads)
    torch.cuda.synchronize()
    for g in G.SPLAT_PARAMS:
        want = sum(np.asarray(r["grads"][g]) for r in refs)
        allow = sum(np.asarray(r["allow"][g]) for r in refs)
        assert_grad_ok(g, grad3d_check(grads[g].cpu().numpy(), want, allow))


@pytest.mark.parametrize("fused", [True, False], ids=["fused", "two_calls"])
def test_batched_training_step_equals_view_by_view(fused):
    """Three views trained together for four steps (densification statistics on): the batched step and the
    view-by-view step leave identical parameters, moments, statistics and losses."""
    cfg_w = synth.make_config(0)
    sc, cam0 = cfg_w["scene"], cfg_w["camera"]
    cams = [cam0, synth.pinhole(cam0.width, cam0.height, (0.6, -0.4, -3.8)),
            synth.pinhole(cam0.width, cam0.height, (-0.9, 0.3, -3.5))]
    tg = torch.as_tensor(np.asarray(cfg_w["target"], np.float32)).cuda()
    targets = [tg, torch.flip(tg, dims=[1]).contiguous(), torch.flip(tg, dims=[0]).contiguous()]
    runs = []
    for batched in (True, False):
        scene = to_device(sc.arrays())
        ts = TrainStep(scene, cams, targets, TrainConfig(batch_views=batched))
        assert ts.batched == batched
        losses = [float(ts.step(it, fused=fused).cpu()) for it in range(1, 5)]
        torch.cuda.synchronize()
        runs.append((scene, ts.exp_avg, ts.exp_avg_sq, ts.grad_accum, ts.grad_count, losses))
    for k in GROUP_ORDER:
        for a, b in zip(runs[0][:3], runs[1][:3]):
            assert torch.equal(a[k], b[k]), k
    assert torch.equal(runs[0][3], runs[1][3]) and torch.equal(runs[0][4], runs[1][4])
    assert runs[0][5] == runs[1][5] and all(np.isfinite(runs[0][5]))
    assert 0 < float(runs[0][4].max().cpu()) <= 3 * 4
