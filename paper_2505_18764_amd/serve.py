"""Continuous-batching render server with memory admission.

Requests (scene, resolution, mode FWD or FWD_BWD) arrive at any time. A scheduler thread admits
the oldest waiting request as soon as a slot (a HIP stream) is free and the request's memory fits
the pool; every buffer the path uses has a size that is a closed form of (N, W, H, format), so the
need is known before launch. Admitted requests run concurrently on their slots' streams and so
overlap on the device; completion is detected with events, which releases the slot and the memory
and records the arrival-to-completion latency. A request larger than the whole pool is rejected;
a waiting request can be cancelled; an executor failure releases its slot and memory.

The executor is pluggable: GpuExecutor runs the HIP path; tests drive the scheduler on the CPU
with a fake executor of simulated durations.

Run as a module for the serving workload (16 scenes of 50k-3M Gaussians, 640x480-1920x1080,
Poisson arrivals, 70 % forward / 30 % forward+backward, FP16 framebuffers):
    python -m paper_2505_18764_amd.serve [--requests 2000] [--rate 200]
"""
from __future__ import annotations

import argparse
import collections
import dataclasses
import json
import threading
import time

import numpy as np

FWD, FWD_BWD = "fwd", "fwd_bwd"


@dataclasses.dataclass
class Request:
    rid: int
    scene: int
    width: int
    height: int
    mode: str = FWD
    arrival: float = 0.0
    status: str = "pending"     # pending | running | done | rejected | cancelled | failed
    need: int = 0
    t_admit: float = 0.0
    t_done: float = 0.0
    error: str = ""
    result: object = None
    keep_result: bool = False
    event: threading.Event = dataclasses.field(default_factory=threading.Event)

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival

    def wait(self, timeout=None) -> bool:
        return self.event.wait(timeout)


class Server:
    def __init__(self, executor, pool_bytes: int, slots: int = 4, poll_s: float = 1e-4):
        self.ex = executor
        self.pool = int(pool_bytes)
        self.nslots = int(slots)
        self.poll_s = poll_s
        self.lock = threading.Lock()
        self.waiting = collections.deque()
        self.free_slots = list(range(self.nslots))
        self.running = {}                  # slot -> (request, handle)
        self.in_use = 0
        self.peak_in_use = 0
        self.peak_running = 0
        self.done = []
        self._stop = threading.Event()
        self._thread = None

    # ---- client side ----
    def submit(self, req: Request) -> Request:
        req.arrival = req.arrival or time.perf_counter()
        req.need = int(self.ex.need_bytes(req))
        with self.lock:
            if req.need > self.pool:
                req.status, req.error = "rejected", f"needs {req.need} B > pool {self.pool} B"
                req.t_done = time.perf_counter()
                req.event.set()
                self.done.append(req)
                return req
            self.waiting.append(req)
        return req

    def cancel(self, req: Request) -> bool:
        with self.lock:
            if req.status == "pending" and req in self.waiting:
                self.waiting.remove(req)
                req.status = "cancelled"
                req.t_done = time.perf_counter()
                req.event.set()
                self.done.append(req)
                return True
        return False

    # ---- scheduler ----
    def start(self):
        self._stop.clear()
        self._thread = threading.Thread(target=self._loop, name="gsr-server", daemon=True)
        self._thread.start()
        return self

    def stop(self, drain: bool = True, timeout: float = 600.0):
        if drain:
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < timeout:
                with self.lock:
                    if not self.waiting and not self.running:
                        break
                time.sleep(1e-3)
        self._stop.set()
        if self._thread:
            self._thread.join()

    def step(self) -> bool:
        """One scheduling round: retire finished work, then admit. Returns True if anything
        changed (used by the loop and by tests that drive the scheduler by hand)."""
        changed = False
        for slot, (req, h) in list(self.running.items()):
            try:
                fin = self.ex.done(h)
            except Exception as e:          # the executor failed: release and report
                fin, req.status, req.error = True, "failed", repr(e)
            if fin:
                if req.status != "failed":
                    try:
                        res = self.ex.result(h)
                        req.result = res if req.keep_result else None
                        req.status = "done"
                    except Exception as e:
                        req.status, req.error = "failed", repr(e)
                req.t_done = time.perf_counter()
                with self.lock:
                    del self.running[slot]
                    self.free_slots.append(slot)
                    self.in_use -= req.need
                    self.done.append(req)
                req.event.set()
                changed = True
        while True:
            with self.lock:
                if not self.waiting or not self.free_slots:
                    break
                req = self.waiting[0]
                if self.in_use + req.need > self.pool:
                    break                       # first come, first served: no overtaking
                self.waiting.popleft()
                slot = self.free_slots.pop()
                self.in_use += req.need
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                req.status, req.t_admit = "running", time.perf_counter()
            try:
                h = self.ex.launch(slot, req)
            except Exception as e:
                req.status, req.error = "failed", repr(e)
                req.t_done = time.perf_counter()
                with self.lock:
                    self.free_slots.append(slot)
                    self.in_use -= req.need
                    self.done.append(req)
                req.event.set()
                changed = True
                continue
            with self.lock:
                self.running[slot] = (req, h)
                self.peak_running = max(self.peak_running, len(self.running))
            changed = True
        return changed

    def _loop(self):
        while not self._stop.is_set():
            if not self.step():
                time.sleep(self.poll_s)

    def summary(self, skip: int = 0) -> dict:
        served = [r for r in self.done if r.status == "done"]
        served.sort(key=lambda r: r.rid)
        served = [r for r in served if r.rid >= skip]
        lat = np.array([r.latency for r in served]) * 1e3
        span = (max(r.t_done for r in served) - min(r.arrival for r in served)) if served else 0.0
        return {"served": len(served),
                "rejected": sum(r.status == "rejected" for r in self.done),
                "failed": sum(r.status == "failed" for r in self.done),
                "cancelled": sum(r.status == "cancelled" for r in self.done),
                "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
                "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
                "mean_ms": float(lat.mean()) if len(lat) else None,
                "views_per_s": len(served) / span if span > 0 else None,
                "peak_pool_bytes": self.peak_in_use, "peak_concurrent": self.peak_running,
                "pool_bytes": self.pool, "slots": self.nslots}


# ---- the HIP executor ------------------------------------------------------------------------

class GpuExecutor:
    """Runs requests on the HIP path, one stream per slot. Scenes stay resident in HBM."""

    def __init__(self, scenes: dict, cameras: dict, cfg=None, device="cuda:0", grad_seed=551):
        import torch
        from . import _lib as L
        from .render import RasterConfig
        self.torch, self.L = torch, L
        self.dev = torch.device(device)
        self.scenes = scenes                      # id -> (means3d, scales, quats, opac, sh)
        self.cameras = cameras                    # (W, H) -> camera object
        self.cfg = cfg or RasterConfig(fb_format="f16", reduce_mode="tile")
        self.streams = {}
        self.grads = {}
        g = np.random.default_rng(grad_seed)
        for (W, H) in cameras:
            self.grads[(W, H)] = torch.from_numpy(
                g.uniform(-1, 1, size=(3, H, W)).astype(np.float32)).to(self.dev)

    def need_bytes(self, req: Request) -> int:
        n = int(self.scenes[req.scene][0].shape[0])
        W, H = req.width, req.height
        L, c = self.L, self.cfg.c()
        b = L.gs_workspace_size("all", n, W, H, c) + L.gs_framebuffer_size(W, H, self.cfg.fb_format)
        b += W * H * 4 * 4                      # image + T
        b += n * (2 + 3 + 3 + 1) * 4 + n * 8 + 64   # projected splats, keys, ids
        if req.mode == FWD_BWD:
            k = self.scenes[req.scene][4].shape[1]
            b += n * 9 * 4 + n * (3 + 3 + 4 + 1 + 3 * k) * 4
        return int(b) + 4096

    def _stream(self, slot):
        if slot not in self.streams:
            self.streams[slot] = self.torch.cuda.Stream(device=self.dev)   # default priority
        return self.streams[slot]

    def launch(self, slot: int, req: Request):
        from . import render as R
        torch = self.torch
        s = self._stream(slot)
        cam = self.cameras[(req.width, req.height)]
        sc = self.scenes[req.scene]
        with torch.cuda.stream(s):
            ws = R.Workspace(self.dev)
            p = R.project(*sc, cam, self.cfg, ws)
            R.raster_setup(p, self.cfg, ws)           # shared by the forward and the backward
            f = R.raster_forward(p, self.cfg, ws, reuse_setup=True)
            out = {"image": f["image"]}
            if req.mode == FWD_BWD:
                g2 = R.raster_backward(p, f["fb"], self.grads[(req.width, req.height)], self.cfg,
                                       ws, reuse_setup=True)
                out["grads2d"] = {k: v for k, v in g2.items() if v is not None}
                out["grads"] = R.project_backward(*sc, cam, self.cfg, g2)
            ev = torch.cuda.Event()
            ev.record(s)
        return {"event": ev, "out": out, "keep": (ws, p, f)}

    def done(self, h) -> bool:
        return h["event"].query()

    def result(self, h):
        return h["out"]


def serving_cameras(resolutions, fx_ref=900.0, ref_w=1024):
    import synth
    return {(W, H): synth.camera_front(W, H, fx_ref * W / ref_w) for (W, H) in resolutions}


def load_scenes(device, count=16, scale=1.0):
    """The 16 serving scenes (seeds 500-515, 50k-3M Gaussians log-spaced), resident on device."""
    import torch
    import synth
    scenes = {}
    for j, (seed, n) in enumerate(synth.serving_scenes(count)):
        sc = synth.scene3d(max(1000, int(n * scale)), seed=seed)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        scenes[j] = (t(sc.means3d), t(sc.scales), t(sc.quats), t(sc.opacities), t(sc.sh))
    return scenes


def run_load(server: Server, reqs, warmup: int):
    """Submit requests at their arrival offsets (a feeder thread); wait for all to finish."""
    t0 = time.perf_counter()
    out = []
    for i, (t_arr, scene, (W, H), fwd_only) in enumerate(reqs):
        now = time.perf_counter() - t0
        if t_arr > now:
            time.sleep(t_arr - now)
        r = Request(rid=i, scene=scene, width=W, height=H, mode=FWD if fwd_only else FWD_BWD,
                    arrival=time.perf_counter())
        out.append(server.submit(r))
    for r in out:
        r.wait()
    return server.summary(skip=warmup)


def main():
    import torch
    import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--pool-gb", type=float, default=64.0)
    ap.add_argument("--scene-scale", type=float, default=1.0)
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    scenes = load_scenes(dev, scale=args.scene_scale)
    cams = serving_cameras(synth.CFG5_RESOLUTIONS)
    ex = GpuExecutor(scenes, cams)
    srv = Server(ex, int(args.pool_gb * (1 << 30)), slots=args.slots).start()
    reqs = synth.serving_requests(args.requests + args.warmup, args.rate)
    summ = run_load(srv, reqs, args.warmup)
    srv.stop()
    summ.update(offered_rate=args.rate, requests=args.requests, warmup=args.warmup)
    print(json.dumps(summ))


if __name__ == "__main__":
    main()
