"""Serving on the GPU: a request's image is bit-identical alone, in a mixed batch and through the plain
render path; batched serving beats one-request-at-a-time serving in throughput and p99 latency."""
import numpy as np
import pytest
import torch

from paper_2402_10128_amd import ges as G
from paper_2402_10128_amd import synth
from paper_2402_10128_amd.serve import Server, run_stream

from .parity_helpers import to_device

pytestmark = pytest.mark.gpu

RES = [(256, 256), (512, 512), (320, 180), (640, 360)]


def _scenes(sizes, seed=500):
    return [to_device(synth.scene_clusters(n, seed + i).arrays()) for i, n in enumerate(sizes)]


def _requests(n_req, n_scenes, seed=2000):
    return synth.serving_requests(n_req, n_scenes, RES, seed=seed)


def test_alone_equals_mixed_equals_plain_render():
    scenes = _scenes([20_000, 50_000, 80_000])
    reqs = _requests(12, len(scenes))
    outs_mixed = [torch.zeros((c.height, c.width, 3), device="cuda") for _, c in reqs]
    outs_alone = [torch.zeros_like(o) for o in outs_mixed]
    with Server(4 << 30, max_slots=8) as s:
        ids = [s.add_scene(sc) for sc in scenes]
        # mixed: everything at once (batched)
        rids = [s.submit(ids[k], cam, out) for (k, cam), out in zip(reqs, outs_mixed)]
        s.drain()
        sizes = [s.poll(r)["batch_size"] for r in rids]
        assert all(s.poll(r)["state"] == "DONE" for r in rids)
        # alone: one at a time
        for (k, cam), out in zip(reqs, outs_alone):
            r = s.submit(ids[k], cam, out)
            s.drain()
            assert s.poll(r)["batch_size"] == 1
    print("batch sizes in the mix:", sizes)
    assert max(sizes) > 1
    for a, b in zip(outs_alone, outs_mixed):
        assert torch.equal(a, b)
    # and equal to the plain render path (same kernels, single view)
    for (k, cam), out in zip(reqs[:4], outs_alone[:4]):
        img, _ = G.render(scenes[k], cam, tile_cull=G.TILES_ELLIPSE)
        assert torch.equal(img, out)


def test_batched_beats_sequential_throughput_and_p99():
    scenes = _scenes([200_000, 500_000, 1_000_000])
    reqs = _requests(48, len(scenes), seed=2100)
    outs = [torch.zeros((c.height, c.width, 3), device="cuda") for _, c in reqs]
    results = {}
    for mode in ("sequential", "batched"):
        with Server(16 << 30, max_slots=16, sequential=(mode == "sequential")) as s:
            ids = [s.add_scene(sc) for sc in scenes]
            rq = [(ids[k], cam) for k, cam in reqs]
            run_stream(s, rq[:8], outs[:8], None)          # warm-up
            results[mode] = run_stream(s, rq, outs, None)
    seq, bat = results["sequential"], results["batched"]
    print(f"sequential: {seq['mpix_s']:.1f} Mpix/s p50 {seq['p50_ms']:.2f} p99 {seq['p99_ms']:.2f}")
    print(f"batched:    {bat['mpix_s']:.1f} Mpix/s p50 {bat['p50_ms']:.2f} p99 {bat['p99_ms']:.2f} "
          f"mean batch {bat['mean_batch']:.1f}")
    assert seq["all_done"] and bat["all_done"]
    assert bat["mpix_s"] > seq["mpix_s"]
    assert bat["p99_ms"] < seq["p99_ms"]
