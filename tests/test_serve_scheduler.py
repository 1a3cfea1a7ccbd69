"""Host-only tests of the serving scheduler (admission, budget, batching, failures) through the
simulated executor of libges: no GPU needed, no device memory touched."""
import os
import time

import numpy as np
import pytest

from paper_2402_10128_amd import ges as G
from paper_2402_10128_amd import synth

pytestmark = pytest.mark.skipif(not os.path.exists(G.LIB_PATH), reason="libges.so not built")

from paper_2402_10128_amd.serve import Server  # noqa: E402

CAM = synth.pinhole(256, 256, (0.0, 0.0, -4.0))


def req_bytes(n, w, h):
    sb, _ = G.ges_workspace_query(n, w, h)
    return sb


def wait_all(server, ids, timeout=10.0):
    t0 = time.time()
    while time.time() - t0 < timeout:
        infos = [server.poll(i) for i in ids]
        if all(x["state"] in ("DONE", "FAILED", "REJECTED", "CANCELLED") for x in infos):
            return infos
        time.sleep(0.002)
    raise TimeoutError


def test_all_requests_complete_in_fifo_order_with_batches():
    with Server(1 << 30, max_slots=4, simulated=dict(batch_ns=2_000_000, per_view_ns=100_000)) as s:
        sid = s.add_scene(dict(n=10_000))
        ids = [s.submit(sid, CAM, 1) for _ in range(20)]
        s.drain()
        infos = [s.poll(i) for i in ids]
    assert all(x["state"] == "DONE" and x["status"] == 0 for x in infos)
    starts = [x["t_start_ns"] for x in infos]
    assert starts == sorted(starts)                      # admitted in arrival order
    assert max(x["batch_size"] for x in infos) > 1       # requests that waited were batched together
    assert max(x["batch_size"] for x in infos) <= 4


def test_sequential_mode_renders_one_request_per_batch():
    with Server(1 << 30, max_slots=8, sequential=True, simulated=dict(batch_ns=200_000)) as s:
        sid = s.add_scene(dict(n=1000))
        ids = [s.submit(sid, CAM, 1) for _ in range(10)]
        s.drain()
        assert all(s.poll(i)["batch_size"] == 1 for i in ids)


def test_budget_limits_concurrency_but_everything_finishes():
    n = 200_000
    one = req_bytes(n, 256, 256)
    # room for the view tables and about two requests' workspaces plus their keys
    pool = 2 * one + 3 * (1 << 20) + 2 * 100_000 * 20
    with Server(pool, max_slots=8, simulated=dict(keys_per_view=100_000, batch_ns=1_000_000)) as s:
        sid = s.add_scene(dict(n=n))
        ids = [s.submit(sid, CAM, 1) for _ in range(12)]
        s.drain()
        infos = [s.poll(i) for i in ids]
    assert all(x["state"] == "DONE" for x in infos), infos
    assert max(x["batch_size"] for x in infos) <= 2


def test_request_larger_than_pool_is_rejected():
    with Server(1 << 20, simulated={}) as s:
        sid = s.add_scene(dict(n=5_000_000))
        rid = s.submit(sid, CAM, 1)
        info = s.poll(rid)
    assert info["state"] == "REJECTED" and info["status"] == 3   # GES_ERR_OUT_OF_MEMORY


def test_queue_full_returns_busy():
    with Server(1 << 30, max_slots=1, queue_capacity=3, simulated=dict(batch_ns=50_000_000)) as s:
        sid = s.add_scene(dict(n=1000))
        accepted, busy = 0, 0
        for _ in range(10):
            try:
                s.submit(sid, CAM, 1)
                accepted += 1
            except G.GESError as e:
                assert e.status == 5
                busy += 1
        assert busy > 0 and accepted >= 3


def test_bad_arguments():
    with Server(1 << 30, simulated={}) as s:
        sid = s.add_scene(dict(n=1000))
        with pytest.raises(G.GESError) as e:
            s.submit(sid + 7, CAM, 1)
        assert e.value.status == 6   # NOT_FOUND
        bad = synth.Camera(64, 64, np.eye(3, dtype=np.float32) * 2, np.zeros(3, np.float32), 50, 50, 32, 32, 0.2)
        with pytest.raises(G.GESError) as e:
            s.submit(sid, bad, 1)
        assert e.value.status == 1   # INVALID_ARGUMENT
        with pytest.raises(G.GESError) as e:
            s.submit(sid, CAM, 0)
        assert e.value.status == 1


def test_executor_failure_fails_batch_and_server_keeps_serving():
    with Server(1 << 30, max_slots=1, simulated=dict(fail_scene=1, batch_ns=100_000)) as s:
        good = s.add_scene(dict(n=1000))
        bad = s.add_scene(dict(n=1000))
        ids = [s.submit(good, CAM, 1), s.submit(bad, CAM, 1), s.submit(good, CAM, 1)]
        s.drain()
        states = [s.poll(i) for i in ids]
    assert [x["state"] for x in states] == ["DONE", "FAILED", "DONE"]
    assert states[1]["status"] == 4   # GES_ERR_DEVICE


def test_destroy_cancels_queued_requests():
    s = Server(1 << 30, max_slots=1, simulated=dict(batch_ns=30_000_000))
    sid = s.add_scene(dict(n=1000))
    ids = [s.submit(sid, CAM, 1) for _ in range(6)]
    time.sleep(0.005)
    h = s._h
    s.close()   # returns after the running batches finished; queued ones are cancelled
    assert h is not None


def test_continuous_batching_admits_arrivals_while_busy():
    """Requests arriving during a batch are taken together by the next one (not one at a time)."""
    with Server(1 << 30, max_slots=16, simulated=dict(batch_ns=5_000_000, per_view_ns=50_000)) as s:
        sid = s.add_scene(dict(n=1000))
        first = s.submit(sid, CAM, 1)
        t0 = time.monotonic()   # the first batch has taken the first request (it runs for 5 ms)
        while s.poll(first)["state"] == "QUEUED" and time.monotonic() - t0 < 5.0:
            time.sleep(0.0001)
        rest = [s.submit(sid, CAM, 1) for _ in range(8)]
        s.drain()
        b0 = s.poll(first)["batch_size"]
        later = [s.poll(i)["batch_size"] for i in rest]
    assert b0 == 1
    assert max(later) >= 4


def test_inspection_submit_validates_its_buffer():
    """ges_serve_submit_inspect: the layout size of ges_serve_inspect_bytes (records, ranges, n_contrib,
    header, batch ids, each 256-byte aligned), a misaligned buffer and one too small for the view refused
    before the request is queued."""
    n, w, h = 10_000, 256, 256
    a = lambda x: (x + 255) // 256 * 256
    want = a(64 * n) + a(8 * 256) + a(4 * w * h) + 256 + a(8 * 1000)
    assert G.lib().ges_serve_inspect_bytes(n, w, h, 1000) == want
    assert G.lib().ges_serve_inspect_bytes(n, 0, h, 0) == 0

    class Buf:   # a stand-in device buffer: never dereferenced by the simulated executor
        def __init__(self, ptr, size):
            self.ptr, self.size = ptr, size

        def data_ptr(self):
            return self.ptr

        def numel(self):
            return self.size

    with Server(1 << 30, max_slots=4, simulated=dict(batch_ns=100_000)) as s:
        sid = s.add_scene(dict(n=n))
        with pytest.raises(G.GESError) as e:
            s.submit(sid, CAM, 1, inspect=Buf((1 << 30) + 8, want))
        assert e.value.status == 1
        with pytest.raises(G.GESError) as e:
            s.submit(sid, CAM, 1, inspect=Buf(1 << 30, G.lib().ges_serve_inspect_bytes(n, w, h, 0) - 1))
        assert e.value.status == 2
        rid = s.submit(sid, CAM, 1)
        s.drain()
        assert s.poll(rid)["state"] == "DONE"
