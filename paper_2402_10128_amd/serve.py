"""Python front end of the continuous-batching render server (ges_serve_* in libges.so).

The server thread, admission by the pool budget, batching and the device work all live in the
library; this module marshals arguments and runs the latency/throughput experiment.
"""
from __future__ import annotations

import ctypes as C
import threading
import time

import numpy as np

from . import ges as G

REQ_STATES = {0: "QUEUED", 1: "RUNNING", 2: "DONE", 3: "FAILED", 4: "REJECTED", 5: "CANCELLED"}


class Server:
    """A render server over resident scenes.

    simulated: None for the GPU server, else dict(keys_per_view, batch_ns, per_view_ns, fail_scene) for the
    host-only scheduler test harness (no device memory is touched).
    """

    def __init__(self, pool_bytes: int, max_slots: int = 16, queue_capacity: int = 4096, falloff: int = 0,
                 tile_cull: int = 1, rho: float = 0.1, bg=(0.0, 0.0, 0.0), sequential: bool = False,
                 simulated: dict | None = None, device="cuda"):
        cfg = G.ges_serve_config()
        cfg.max_slots, cfg.queue_capacity = int(max_slots), int(queue_capacity)
        cfg.falloff, cfg.tile_cull, cfg.rho = int(falloff), int(tile_cull), float(rho)
        cfg.bg[:] = [float(b) for b in bg]
        cfg.sequential = 1 if sequential else 0
        self._h = C.c_void_p()
        self._keep = []
        self.pool = None
        if simulated is None:
            import torch
            self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=device)
            G._check(G.lib().ges_serve_create(C.byref(cfg), C.c_void_p(self.pool.data_ptr()), int(pool_bytes),
                                              C.byref(self._h)))
        else:
            G._check(G.lib().ges_serve_create_simulated(C.byref(cfg), int(pool_bytes),
                                                        int(simulated.get("keys_per_view", 1000)),
                                                        int(simulated.get("batch_ns", 1_000_000)),
                                                        int(simulated.get("per_view_ns", 100_000)),
                                                        int(simulated.get("fail_scene", -1)), C.byref(self._h)))

    def add_scene(self, scene) -> int:
        """scene: dict of CUDA float32 tensors, or (simulated server) dict(n=..., sh_degree=...)."""
        if "means" in scene:
            s = G.splats_struct(scene["means"], scene["log_scales"], scene["quats"], scene["opacity_logits"],
                                scene["sh"], scene["beta"])
            self._keep.append(scene)
        else:
            s = G.ges_splats()
            s.n, s.sh_degree = int(scene["n"]), int(scene.get("sh_degree", 3))
            for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "beta"):
                setattr(s, k, 1 << 20)   # never dereferenced by the simulated executor
        sid = C.c_int32(0)
        G._check(G.lib().ges_serve_add_scene(self._h, C.byref(s), C.byref(sid)))
        return sid.value

    def submit(self, scene_id: int, cam, out_ptr, inspect=None) -> int:
        """out_ptr: a CUDA float32 tensor [h,w,3] or (simulated) any non-zero integer.  inspect: optional
        256-byte-aligned CUDA uint8 tensor receiving the request's frame arrays (see inspect_arrays)."""
        ptr = out_ptr.data_ptr() if hasattr(out_ptr, "data_ptr") else int(out_ptr)
        rid = C.c_uint64(0)
        if inspect is None:
            G._check(G.lib().ges_serve_submit(self._h, int(scene_id), C.byref(G.camera_struct(cam)), C.c_void_p(ptr),
                                              C.byref(rid)))
        else:
            G._check(G.lib().ges_serve_submit_inspect(self._h, int(scene_id), C.byref(G.camera_struct(cam)),
                                                      C.c_void_p(ptr), C.c_void_p(inspect.data_ptr()),
                                                      inspect.numel(), C.byref(rid)))
        return rid.value

    def poll(self, rid: int) -> dict:
        info = G.ges_request_info()
        G._check(G.lib().ges_serve_poll(self._h, int(rid), C.byref(info)))
        return dict(state=REQ_STATES[info.state], status=info.status, t_submit_ns=info.t_submit_ns,
                    t_start_ns=info.t_start_ns, t_done_ns=info.t_done_ns, num_keys=info.num_keys,
                    batch_size=info.batch_size)

    def drain(self):
        G._check(G.lib().ges_serve_drain(self._h))

    def close(self):
        if self._h:
            G._check(G.lib().ges_serve_destroy(self._h))
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def run_stream(server: Server, requests, outs, rate_hz: float | None, seed: int = 0):
    """Submit (scene_id, camera) requests with Poisson arrivals at rate_hz (None: all at once), wait
    for all, and return per-request latency (ms) and the throughput (Mpix/s) over the whole run."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, len(requests)) if rate_hz else np.zeros(len(requests))
    ids = []
    t0 = time.perf_counter()
    t_next = t0
    for (sid, cam), out, gap in zip(requests, outs, gaps):
        t_next += gap
        while True:
            d = t_next - time.perf_counter()
            if d <= 0:
                break
            time.sleep(min(d, 0.002))
        while True:
            try:
                ids.append(server.submit(sid, cam, out))
                break
            except G.GESError as e:   # queue full: back off briefly
                if e.status != 5:
                    raise
                time.sleep(0.0005)
    server.drain()
    infos = [server.poll(i) for i in ids]
    lat = np.array([(x["t_done_ns"] - x["t_submit_ns"]) / 1e6 for x in infos])
    t_first = min(x["t_submit_ns"] for x in infos)
    t_last = max(x["t_done_ns"] for x in infos)
    px = sum(cam.width * cam.height for _, cam in requests)
    ok = all(x["state"] == "DONE" for x in infos)
    return dict(p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()), mpix_s=px / ((t_last - t_first) / 1e9) / 1e6, all_done=ok,
                mean_batch=float(np.mean([x["batch_size"] for x in infos])), infos=infos)


def _align256(x: int) -> int:
    return (x + 255) // 256 * 256


def inspect_arrays(buf, n: int, width: int, height: int, batch_keys: int) -> dict:
    """numpy copies of a served request's inspection buffer, laid out as ges_serve_submit_inspect documents."""
    tiles = ((width + 15) // 16) * ((height + 15) // 16)
    px = width * height
    off_ranges = _align256(64 * n)
    off_nc = off_ranges + _align256(8 * tiles)
    off_hdr = off_nc + _align256(4 * px)
    off_ids = off_hdr + 256
    b = buf.cpu().numpy()
    out = dict(records=b[:64 * n].view(np.float32).reshape(n, 16),
               ranges=b[off_ranges:off_ranges + 8 * tiles].view(np.uint32).reshape(tiles, 2),
               n_contrib=b[off_nc:off_nc + 4 * px].view(np.uint32).reshape(height, width),
               header=b[off_hdr:off_hdr + 32].view(np.uint64))
    if b.size >= off_ids + 8 * batch_keys:
        out["ids"] = b[off_ids:off_ids + 8 * batch_keys].view(np.uint32).reshape(batch_keys, 2)[:, 0]
    return out
