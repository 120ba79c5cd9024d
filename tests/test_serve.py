"""The server's scheduler on the CPU with a fake executor of simulated durations: memory and
slot admission, first-come-first-served order, rejection, cancellation, failures that release
their slot and memory, overload, and continuous admission while other work runs."""
import threading
import time

import numpy as np
import pytest

from paper_2505_18764_amd.serve import FWD, FWD_BWD, Request, Server


class FakeExec:
    def __init__(self, dur=0.01, fail_launch=(), fail_done=()):
        self.dur, self.fail_launch, self.fail_done = dur, set(fail_launch), set(fail_done)
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.launched = []

    def need_bytes(self, req):
        return 1000 * (req.scene + 1) * (2 if req.mode == FWD_BWD else 1)

    def launch(self, slot, req):
        if req.rid in self.fail_launch:
            raise RuntimeError("launch failed")
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
            self.launched.append(req.rid)
        d = self.dur(req) if callable(self.dur) else self.dur
        return {"t": time.perf_counter() + d, "req": req, "closed": False}

    def done(self, h):
        if time.perf_counter() < h["t"]:
            return False
        if not h["closed"]:
            h["closed"] = True
            with self.lock:
                self.active -= 1
        if h["req"].rid in self.fail_done:
            raise RuntimeError("kernel failed")
        return True

    def result(self, h):
        return {"rid": h["req"].rid}


def _req(i, scene=0, mode=FWD):
    return Request(rid=i, scene=scene, width=64, height=48, mode=mode)


def test_slots_pool_and_fifo():
    ex = FakeExec(dur=0.02)
    srv = Server(ex, pool_bytes=5000, slots=3).start()
    rs = [srv.submit(_req(i, scene=i % 2)) for i in range(12)]
    for r in rs:
        assert r.wait(10)
    srv.stop()
    assert all(r.status == "done" for r in rs)
    assert srv.peak_running <= 3 and ex.max_active <= 3
    assert srv.peak_in_use <= 5000
    assert ex.launched == sorted(ex.launched)            # admitted in arrival order
    assert srv.in_use == 0 and sorted(srv.free_slots) == [0, 1, 2]


def test_reject_cancel_and_failures_release_resources():
    ex = FakeExec(dur=0.03, fail_launch={3}, fail_done={4})
    srv = Server(ex, pool_bytes=4000, slots=1)
    big = srv.submit(_req(0, scene=10))                  # 11000 B > pool
    assert big.status == "rejected" and big.wait(0)
    rs = [srv.submit(_req(i)) for i in range(1, 7)]
    assert srv.cancel(rs[1])                             # rid 2, still waiting
    srv.start()
    for r in rs:
        assert r.wait(10)
    srv.stop()
    st = {r.rid: r.status for r in rs}
    assert st == {1: "done", 2: "cancelled", 3: "failed", 4: "failed", 5: "done", 6: "done"}
    assert 2 not in ex.launched and srv.in_use == 0 and srv.free_slots == [0]
    s = srv.summary()
    assert s["rejected"] == 1 and s["failed"] == 2 and s["cancelled"] == 1 and s["served"] == 3


def test_continuous_admission_while_running():
    """A request that arrives while others run starts when the first slot frees, long before
    the earlier requests have all finished."""
    ex = FakeExec(dur=lambda r: 0.3 if r.rid < 2 else 0.01)
    srv = Server(ex, pool_bytes=10_000, slots=2).start()
    a, b = srv.submit(_req(0)), srv.submit(_req(1))
    time.sleep(0.05)
    c = srv.submit(_req(2))
    d = srv.submit(_req(3))
    for r in (a, b, c, d):
        assert r.wait(10)
    srv.stop()
    assert c.t_admit >= min(a.t_done, b.t_done) - 1e-3   # waited for a free slot ...
    assert c.t_admit < max(a.t_done, b.t_done) + 0.05    # ... not for the whole batch


def test_memory_admission_blocks_head_of_line():
    ex = FakeExec(dur=0.05)
    srv = Server(ex, pool_bytes=3000, slots=4).start()
    r0 = srv.submit(_req(0, scene=1))                    # 2000 B
    r1 = srv.submit(_req(1, scene=1))                    # 2000 B: must wait for r0's memory
    r2 = srv.submit(_req(2, scene=0))                    # 1000 B: fits, but may not overtake
    for r in (r0, r1, r2):
        assert r.wait(10)
    srv.stop()
    assert r1.t_admit >= r0.t_done - 1e-3
    assert r2.t_admit >= r1.t_admit
    assert srv.peak_in_use <= 3000


def test_overload_queues_then_drains():
    ex = FakeExec(dur=0.004)
    srv = Server(ex, pool_bytes=1 << 30, slots=2).start()
    rs = []
    for i in range(120):                                 # offered 1000/s vs capacity ~500/s
        rs.append(srv.submit(_req(i)))
        time.sleep(0.001)
    for r in rs:
        assert r.wait(20)
    srv.stop()
    s = srv.summary()
    assert s["served"] == 120
    lat = np.array([r.latency for r in rs])
    assert lat[-10:].mean() > 3 * lat[:10].mean()        # the queue grew under overload
