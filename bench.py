"""Benchmark: forward + backward ms per view for 1M clustered Gaussians at 1600x1064.

One step = one view through the whole path: projection (gs_preprocess), depth sort (gs_sort),
forward raster (gs_raster_fwd), backward raster (gs_raster_bwd) and projection backward
(gs_preprocess_bwd), with dL/dC ~ U[-1, 1] (the paper's backward protocol, Sec. 4). Inputs are
resident in HBM before the timed region. The headline is the FP16-framebuffer path; the FP32
path is timed the same way and reported beside it.

Prints one JSON line (rank 0). Single GPU only.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FLOPs per fragment of the method's own arithmetic:
FLOP_FWD_PER_COVERED = 24   # alpha of one fragment + the blend of Eq. 2
FLOP_BWD_PER_LIVE = 69      # alpha, Eqs. 3/5/6/7, the chain rule to 9 parameters, their reduction
# FP32 vector peaks of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA) x 2.4 GHz = 78.6 TFLOP/s
# for one FP32 operation per lane and cycle; the published 157.3 counts the packed two-wide FP32
# instructions, which this library's build disables, so 78.6 is the ceiling its kernels can reach.
PEAK_FP32_TFLOPS = 78.6
PEAK_FP32_PACKED_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# Framebuffer bytes of the method per fragment (the algorithmic bytes of the survey's roofline,
# what a render target holding the state in memory would move): S = state bytes per pixel.
STATE_BYTES = {"f32": 16, "f16": 8, "unorm16": 8, "bf16": 8, "unorm8": 4}


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None, help="override the Gaussian count")
    ap.add_argument("--formats", default="f16,f32,unorm16")
    ap.add_argument("--reduce", default="tile")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-blocks", type=int, default=96)
    ap.add_argument("--no-variants", action="store_true",
                    help="skip Table 1's reduction modes, the X sweep and the forward T-cull")
    ap.add_argument("--no-micro", action="store_true",
                    help="skip the HBM-copy and FP32-atomic microbenchmarks")
    ap.add_argument("--no-fit", action="store_true", help="skip the 300-step fitting run")
    ap.add_argument("--cpu-full", action="store_true",
                    help="only time the CPU oracle on whole frames (cfg1, cfg2) and a cfg3 sample, "
                         "at all host threads and at one; prints a JSON line")
    ap.add_argument("--no-tile", action="store_true", help="skip the tile-based baseline")
    ap.add_argument("--no-views", action="store_true",
                    help="skip the several-views-per-call measurement (fitting workload)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="measured requests of each serving run (0: skip); 200 more are warmup")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 512 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--no-format-errors", action="store_true",
                    help="skip the low-precision gradient error table")
    ap.add_argument("--summarize-pmc", metavar="DIR",
                    help="write profiles/traffic.json from DIR/{fetch,write,cfetch,cwrite} "
                         "rocprofv3 databases and the kernel table from DIR/kt (no GPU work)")
    return ap.parse_args()


def _profile(name, kernels, field):
    """Sum over the given kernels of `field` in the committed profile summary profiles/<name>, if
    every entry was taken with the current kernel sources; else None."""
    from paper_2505_18764_amd import pmc
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    h = pmc.source_hash()
    tot = 0.0
    for k in kernels:
        e = d.get(k)
        if not e or e.get("source_hash") != h or e.get(field) is None:
            return None
        tot += e[field]
    return tot


def _traffic(kernels):
    """HBM bytes per launch of the given kernels (summed) from the committed PMC summary."""
    return _profile("traffic.json", kernels, "bytes_per_launch")


def format_error_table(g, g_ref):
    """The paper's mixed-precision error measure (Sec. 4.6, Table 4): RMSE of all gradient
    elements against the FP32 path, and the mean relative error |g - g_ref| / |g_ref| over the
    elements whose reference magnitude lies in [10, inf), [0.1, 10) and [1e-3, 0.1)."""
    g = np.asarray(g, np.float64).reshape(-1)
    r = np.asarray(g_ref, np.float64).reshape(-1)
    out = {"rmse": float(np.sqrt(np.mean((g - r) ** 2))) if r.size else 0.0}
    a = np.abs(r)
    for name, lo, hi in (("mre_10_inf", 10.0, np.inf), ("mre_0.1_10", 0.1, 10.0),
                         ("mre_1e-3_0.1", 1e-3, 0.1)):
        m = (a >= lo) & (a < hi)
        out[name] = float(np.mean(np.abs(g[m] - r[m]) / a[m])) if m.any() else None
        out["n_" + name[4:]] = int(m.sum())
    return out


# consecutive lanes whose FP32 atomic adds reach the L2 as one request (a 64-byte line)
LANES_PER_ATOMIC_REQUEST = 16

# the launches of the timed raster stages (paper mode, FP16 at rest, no counters)
FWD_KERNELS = ("k_raster_fwd<-1, false, false, false>",)
BWD_KERNELS = ("k_raster_bwd<-1, false, false, true>",)


def main():
    args = _parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the path has no multi-GPU "
              "component; views are independent and would shard one view per GPU.", file=sys.stderr)
        sys.exit(2)
    if args.summarize_pmc:
        from paper_2505_18764_amd import pmc
        d = args.summarize_pmc
        A = ("python -u bench.py --steps 3 --warmup 1 --no-cpu --no-tile --serve-requests 0 "
             "--no-format-errors --no-views --no-variants --no-fit --formats f16")
        B = A + " --no-micro"
        KT = B.replace("--steps 3", "--steps 5")
        cmd = "\n".join([
            "cd /tmp && export TMPDIR=/tmp && R=<repository root>",
            f"rocprofv3 --pmc FETCH_SIZE --kernel-trace -d $OUT/fetch -o run -- {B.replace('bench.py', '$R/bench.py')}",
            f"rocprofv3 --pmc WRITE_SIZE --kernel-trace -d $OUT/write -o run -- {B.replace('bench.py', '$R/bench.py')}",
            "rocprofv3 --pmc FETCH_SIZE --kernel-trace -d $OUT/cfetch -o run -- python -u $R/bench.py --copy-probe",
            "rocprofv3 --pmc WRITE_SIZE --kernel-trace -d $OUT/cwrite -o run -- python -u $R/bench.py --copy-probe",
            "python bench.py --summarize-pmc $OUT"])
        res = pmc.summarize(os.path.join(d, "fetch"), os.path.join(d, "write"),
                            os.path.join(d, "cfetch"), os.path.join(d, "cwrite"), 512 << 20,
                            os.path.join(ROOT, "profiles"), cmd,
                            "1M clustered Gaussians, 1600x1064, FP16 framebuffer")
        print(json.dumps({k: v for k, v in res.items() if k.startswith("_")}))
        if os.path.isdir(os.path.join(d, "sq")):
            scmd = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU "
                    "SQ_INSTS_LDS SQ_WAVES SQ_INSTS_VALU_TRANS_F32 SQ_BUSY_CYCLES --kernel-trace "
                    f"-d $OUT/sq -o run -- {B.replace('bench.py', '$R/bench.py')}")
            pmc.issue_summary(os.path.join(d, "sq"),
                              os.path.join(ROOT, "profiles", "issue_1M_1600x1064_f16.md"), scmd,
                              "1M clustered Gaussians, 1600x1064, FP16 framebuffer")
        if os.path.isdir(os.path.join(d, "atom")):
            acmd = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc " + " ".join(pmc.ATOMIC_COUNTERS)
                    + f" --kernel-trace -d $OUT/atom -o run -- {A.replace('bench.py', '$R/bench.py')}")
            pmc.atomic_summary(os.path.join(d, "atom"),
                               os.path.join(ROOT, "profiles", "atomics_1M_1600x1064_f16.md"), acmd,
                               "1M clustered Gaussians, 1600x1064, FP16 framebuffer; the FP32 "
                               "atomic microbenchmark")
        if os.path.isdir(os.path.join(d, "stall1")) and os.path.isdir(os.path.join(d, "stall2")):
            cmds = [f"cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc {' '.join(c)} --kernel-trace "
                    f"-d $OUT/stall{i + 1} -o run -- {B.replace('bench.py', '$R/bench.py')}"
                    for i, c in enumerate(pmc.STALL_COUNTERS)]
            pmc.stall_summary([os.path.join(d, "stall1"), os.path.join(d, "stall2")],
                              os.path.join(ROOT, "profiles", "stalls_1M_1600x1064_f16.md"), cmds,
                              "1M clustered Gaussians, 1600x1064, FP16 framebuffer")
        if os.path.isdir(os.path.join(d, "kt")):
            kcmd = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats -d $OUT/kt "
                    f"-o run -- {KT.replace('bench.py', '$R/bench.py')}")
            pmc.trace_summary(os.path.join(d, "kt"),
                              os.path.join(ROOT, "profiles", "kernels_1M_1600x1064_f16.md"), kcmd,
                              "1M clustered Gaussians, 1600x1064, FP16 framebuffer",
                              note="Six views: one warm-up, one instrumented (the INSTR = true "
                                   "instances count fragments: a forward with the saturation "
                                   "exit, a forward of every covered fragment and a backward), "
                                   "five timed (the timed loop's views and the stage timings).")
        return
    if args.cpu_full:
        cpu_full(args)
        return
    import torch
    import synth
    from paper_2505_18764_amd import render as R

    if args.copy_probe:
        a = torch.empty(512 << 20, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel(), "copies": 3}))
        return

    dev = torch.device("cuda:0")
    c3 = dict(synth.CFG3)
    if args.n:
        c3["n"] = args.n
    W, H = c3["width"], c3["height"]
    sc = synth.scene3d(c3["n"], seed=c3["seed"])
    cam = synth.camera_front(W, H, c3["fx"])
    G = synth.image_grad(W, H, c3["grad_seed"])
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    inp = [t(sc.means3d), t(sc.scales), t(sc.quats), t(sc.opacities), t(sc.sh)]
    Gd = t(G)
    torch.cuda.synchronize()

    def run_format(fmt, reduce_mode, t_min_fwd=0.0, steps=args.steps, warmup=args.warmup,
                   composite_all=False):
        cfg = R.RasterConfig(fb_format=fmt, reduce_mode=reduce_mode, t_min_fwd=t_min_fwd,
                             composite_all=composite_all)
        ws = R.Workspace(dev)
        # preallocated outputs: the timed steps allocate nothing
        p = R.project(*inp, cam, cfg, ws)
        f = R.raster_forward(p, cfg, ws)
        g2 = R.raster_backward(p, f["fb"], Gd, cfg, ws)
        g3 = R.project_backward(*inp, cam, cfg, g2)
        torch.cuda.synchronize()
        # fragment counts of this workload (instrumented runs, outside the timed region): the
        # fragments the timed forward composites (with its saturation exit) and the backward
        # visits, and every covered fragment (paper mode's full walk, the algorithmic count)
        st = R.new_stats(dev)
        R.raster_forward(p, cfg, ws, fb=f["fb"], image=f["image"], T=f["T"], stats=st)
        R.raster_backward(p, f["fb"], Gd, cfg, ws, stats=st, out=g2)
        st_all = R.new_stats(dev)
        cfg_all = dataclasses.replace(cfg, composite_all=True)
        R.raster_forward(p, cfg_all, ws, fb=f["fb"], image=f["image"], T=f["T"], stats=st_all)
        torch.cuda.synchronize()
        stats = R.read_stats(st)
        stats["fwd_covered_full_walk"] = R.read_stats(st_all)["fwd_covered"]
        nvis = int(p.n_visible.item())

        # every call below runs on torch's current stream, which the events are recorded on; the
        # raster_fwd / raster_bwd stages are then the k_raster_fwd launch alone and the
        # k_raster_bwd launch between a gradient-buffer fill and the scatter to splat ids
        def step(ev=None):
            rec = (lambda i: ev[i].record()) if ev else (lambda i: None)
            rec(0)
            q = R.project(*inp, cam, cfg, ws, sort=False)
            rec(1)
            R.sort_(q, ws)
            rec(2)
            R.raster_setup(q, cfg, ws)
            rec(3)
            R.raster_forward(q, cfg, ws, fb=f["fb"], image=f["image"], T=f["T"], reuse_setup=True)
            rec(4)
            R.raster_backward(q, f["fb"], Gd, cfg, ws, out=g2, reuse_setup=True)
            rec(5)
            R.project_backward(*inp, cam, cfg, g2, out=g3)
            rec(6)

        names = ["preprocess", "sort", "raster_setup", "raster_fwd", "raster_bwd", "preprocess_bwd"]
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
               for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(evs[i])
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / steps
        per = {k: float(np.mean([e[j].elapsed_time(e[j + 1]) for e in evs]))
               for j, k in enumerate(names)}
        total = float(np.mean([e[0].elapsed_time(e[len(names)]) for e in evs]))
        return dict(fmt=fmt, ms_per_view=total, wall_ms_per_view=wall, stages_ms=per,
                    stats=stats, n_visible=nvis, ws_bytes=ws.nbytes)

    def run_tile(steps=max(3, args.steps // 2), warmup=1):
        """The tile-based comparison rasterizer on the same view: projection, per-splat tile
        counts, host readback of the pair count, pair duplication + 64-bit sort + ranges +
        forward, backward, projection backward. Buffers are sized in the warmup, so the timed
        steps allocate nothing (the paper's tile-based timings also exclude allocation)."""
        cfg = R.RasterConfig(fb_format="f32")
        ws = R.Workspace(dev)
        q = R.project(*inp, cam, cfg, ws, sort=False)
        f = R.tile_forward(q, cfg, ws)
        g2 = R.tile_backward(q, f, Gd, cfg, ws)
        g3 = R.project_backward(*inp, cam, cfg, g2)
        torch.cuda.synchronize()
        times = []
        for i in range(warmup + steps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
            ev[0].record()
            q = R.project(*inp, cam, cfg, ws, sort=False)
            ev[1].record()
            ff = R.tile_forward(q, cfg, ws, out=f)      # includes the pair-count readback
            ev[2].record()
            R.tile_backward(q, ff, Gd, cfg, ws, out=g2)
            ev[3].record()
            R.project_backward(*inp, cam, cfg, g2, out=g3)
            ev[4].record()
            torch.cuda.synchronize()
            if i >= warmup:
                times.append([ev[j].elapsed_time(ev[j + 1]) for j in range(4)])
        med = np.median(np.array(times), axis=0)
        names = ["preprocess", "tile_fwd_incl_readback", "tile_bwd", "preprocess_bwd"]
        return {"ms_per_view": float(med.sum()),
                "stages_ms": {k: round(float(v), 4) for k, v in zip(names, med)},
                "n_pairs": int(ff["n_pairs"]),
                "pair_buffer_bytes": int(ff["capacity"]) * 12 * 2, "ws_bytes": ws.nbytes}

    results = {}
    for fmt in args.formats.split(","):
        results[fmt] = run_format(fmt, args.reduce)
    tile = run_tile() if not args.no_tile else None
    head_fmt = "f16" if "f16" in results else list(results)[0]
    head = results[head_fmt]
    st = head["stats"]
    # F: fragments the forward composites (its saturation exit stops where no later fragment can
    # change the stored colour); F_all: every covered fragment (the method's own count)
    F, F_all, Lv = st["fwd_covered"], st["fwd_covered_full_walk"], st["bwd_live"]
    A = st["bwd_atomic_sets"]
    fwd_ms, bwd_ms = head["stages_ms"]["raster_fwd"], head["stages_ms"]["raster_bwd"]
    S = STATE_BYTES[head_fmt]
    micro = None if args.no_micro else micro_run(dev)
    # the method's framebuffer bytes (Proc. 1's state loads and stores, the blend's read-modify-
    # write, 4 bytes a channel for FP32, 2 for the 16-bit formats): forward F 2S; backward
    # (F - L) s_T + L (2S + 12) + A 36 (culled fragments read T only; a live one reads and
    # writes the state and reads dL/dC; 36 bytes per atomic set of nine gradients)
    s_T = S // 4
    alg_bytes = {"raster_fwd": F * 2 * S,
                 "raster_bwd": (F_all - Lv) * s_T + Lv * (2 * S + 12) + A * 36}
    roof = {}
    for name, ms, flops, keys in (("raster_fwd", fwd_ms, F * FLOP_FWD_PER_COVERED, FWD_KERNELS),
                                  ("raster_bwd", bwd_ms, Lv * FLOP_BWD_PER_LIVE, BWD_KERNELS)):
        ach = flops / (ms * 1e-3) / 1e12
        tr = _traffic(keys) if head_fmt == "f16" else None
        issue = _profile("issue.json", keys[:1], "share") if head_fmt == "f16" else None
        alg_gbs = alg_bytes[name] / (ms * 1e-3) / 1e9
        r = {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS,
             "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4),
             "traffic": None if tr is None else round(tr),
             "peak_published_packed": PEAK_FP32_PACKED_TFLOPS,
             "frac_of_published": round(ach / PEAK_FP32_PACKED_TFLOPS, 4),
             "valu_issue_share": None if issue is None else round(issue, 3),
             "flops_per_launch": flops, "ms": round(ms, 4), "kernels": list(keys),
             "algorithmic_bytes": alg_bytes[name], "algorithmic_gbs": round(alg_gbs, 1),
             "algorithmic_over_hbm_peak": round(alg_gbs / PEAK_HBM_GBS, 3),
             "measured_hbm_gbs": None if tr is None else round(tr / (ms * 1e-3) / 1e9, 1),
             "measured_hbm_frac": None if tr is None else round(tr / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
        if micro:
            r["hbm_copy_gbs_measured"] = micro["copy_gbs"]
        roof[name] = r
    if micro:
        # the backward's atomics against the measured FP32-atomic throughput. By adds: each set
        # adds nine values, first with a returning add, then (when its rounding error is not
        # zero) a second add of that error. By requests: 16 consecutive lanes' adds travel as one
        # 64-byte request (the microbenchmark's counters: 67.1M adds, 4.19M L2 requests), and the
        # kernel's own request counts come from the committed counter profile.
        n_at = 9 * A
        rate = micro["atomic_per_s"]
        t_ret = n_at / rate["spread_return"]
        t_plain = n_at / rate["spread"]
        at = {"sets": A, "returning_adds": n_at, "error_adds_at_most": n_at,
              "bound_ms_by_adds": round((t_ret + t_plain) * 1e3, 4),
              "rate_per_s_measured": rate, "lanes_per_request": LANES_PER_ATOMIC_REQUEST}
        req_ret = _profile("atomics.json", BWD_KERNELS, "TCP_TCC_ATOMIC_WITH_RET_REQ_sum")
        req_plain = _profile("atomics.json", BWD_KERNELS, "TCP_TCC_ATOMIC_WITHOUT_RET_REQ_sum")
        if req_ret is not None and req_plain is not None:
            t_req = (req_ret / (rate["spread_return"] / LANES_PER_ATOMIC_REQUEST) +
                     req_plain / (rate["spread"] / LANES_PER_ATOMIC_REQUEST))
            at.update(requests_with_return=round(req_ret), requests_without_return=round(req_plain),
                      bound_ms_by_requests=round(t_req * 1e3, 4),
                      frac_of_kernel_time=round(t_req * 1e3 / bwd_ms, 4))
        else:
            at["frac_of_kernel_time"] = round((t_ret + t_plain) * 1e3 / bwd_ms, 4)
        roof["raster_bwd"]["atomics"] = at
    dom = "raster_fwd" if fwd_ms >= bwd_ms else "raster_bwd"

    extra = {}
    if not args.no_variants:
        extra["variants"] = variants_run(run_format, inp, cam, Gd, R, head_fmt, args)

    format_errors = None
    if not args.no_format_errors:
        format_errors = format_error_run(inp, cam, Gd, R, dev)

    views = None if args.no_views else views_run(dev)
    fitting = None if args.no_fit else fitting_run(dev)

    serving = None
    if args.serve_requests > 0:
        serving = serving_run(args.serve_requests, dev)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(sc, cam, G, args.cpu_blocks)

    line = {
        "metric": "fwd+bwd ms/view @1M splats 1600x1064 (FP16 vs FP32 FB); p50/p99 latency",
        "value": round(head["ms_per_view"], 4),
        "unit": "ms/view",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_view"], 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{c3['n']} clustered 3D Gaussians (SH deg 3), {W}x{H}, "
                               f"fx={c3['fx']}, dL/dC~U[-1,1]; framebuffer {head_fmt}, "
                               f"reduction {args.reduce}, paper mode (no forward T-cull)",
                   "framebuffer": head_fmt, "arithmetic": "f32", "n": c3["n"], "width": W,
                   "height": H},
        "views_per_s": round(1e3 / head["ms_per_view"], 2),
        "formats": {k: {"ms_per_view": round(v["ms_per_view"], 4),
                        "stages_ms": {s: round(x, 4) for s, x in v["stages_ms"].items()},
                        "wall_ms_per_view": round(v["wall_ms_per_view"], 4)}
                    for k, v in results.items()},
        "fragments": {"covered": F_all, "composited": F, "live": Lv,
                      "n_visible": head["n_visible"],
                      "covered_per_s": round(F_all / (fwd_ms * 1e-3), 1),
                      "composited_per_s": round(F / (fwd_ms * 1e-3), 1),
                      "live_per_s": round(Lv / (bwd_ms * 1e-3), 1),
                      "atomic_rate": round(A / max(1, Lv), 5),
                      "cohesion": round(st["bwd_cohesive"] / max(1, st["bwd_wave_reductions"] +
                                                                   st["bwd_quad_reductions"]), 4),
                      "stats": st},
        "roofline": dict(roof[dom], kernel=dom),
        "roofline_kernels": roof,
        "microbench": micro,
        "workspace_bytes": head["ws_bytes"],
        "tile_baseline": tile,
        "format_errors": format_errors,
        "views_per_call": views,
        "fitting": fitting,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


def format_error_run(inp, cam, Gd, R, dev):
    """Gradients of the 3D parameters (means, scales, quaternions, opacities, SH) with each
    low-precision framebuffer against the FP32 framebuffer on the benchmark view, in the two
    rounding modes (state rounded at rest; rounded after every fragment as a render target)."""
    import torch

    def grads(fmt, rnd):
        cfg = R.RasterConfig(fb_format=fmt, fb_round=rnd, reduce_mode="tile")
        ws = R.Workspace(dev)
        p = R.project(*inp, cam, cfg, ws)
        f = R.raster_forward(p, cfg, ws)
        g2 = R.raster_backward(p, f["fb"], Gd, cfg, ws)
        g3 = R.project_backward(*inp, cam, cfg, g2)
        torch.cuda.synchronize()
        return np.concatenate([g3[k].detach().cpu().numpy().reshape(-1)
                               for k in ("means3d", "scales", "quats", "opacities", "sh")])

    ref = grads("f32", "at_rest")
    out = {"reference": "FP32 framebuffer", "parameters": "means, scales, quats, opacities, SH"}
    for rnd in ("at_rest", "per_fragment"):
        for fmt in ("f16", "unorm16", "bf16", "unorm8"):
            out[f"{fmt}/{rnd}"] = {k: (round(v, 5) if isinstance(v, float) else v)
                                   for k, v in format_error_table(grads(fmt, rnd), ref).items()}
    return out


def views_run(dev, steps=10, warmup=2):
    """The fitting workload's step over all its cameras (500k Gaussians, 8 ring cameras,
    1280x720, FP16 framebuffer, dL/dC ~ U[-1, 1] per view): projection, sort, raster setup,
    forward, backward and projection backward with the 3D gradients summed over the views, run as
    8 one-view calls (the sums added by torch) and as calls of 2, 4 and 8 views (the library sums).
    Returns ms per view of each."""
    import torch
    import synth
    from paper_2505_18764_amd import render as R
    c = synth.CFG4
    W, H = c["width"], c["height"]
    sc = synth.scene3d(c["n_train"], seed=c["seed_train"])
    cams = [synth.camera_ring(k, c["cameras"], width=W, height=H, fx=c["fx"])
            for k in range(c["cameras"])]
    V = len(cams)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    inp = [t(sc.means3d), t(sc.scales), t(sc.quats), t(sc.opacities), t(sc.sh)]
    Gd = t(np.stack([synth.image_grad(W, H, 300 + v) for v in range(V)]))
    cfg = R.RasterConfig(fb_format="f16", reduce_mode="tile")
    keys3 = ("means3d", "scales", "quats", "opacities", "sh")

    def make(vb):
        ws = R.Workspace(dev)
        cs = cams[:vb] if vb > 1 else cams[0]
        q = R.project(*inp, cs, cfg, ws)
        R.raster_setup(q, cfg, ws)
        f = R.raster_forward(q, cfg, ws, reuse_setup=True)
        g2 = R.raster_backward(q, f["fb"], Gd[:vb] if vb > 1 else Gd[0], cfg, ws, reuse_setup=True)
        g3 = R.project_backward(*inp, cs, cfg, g2)
        return ws, f, g2, g3

    def run(vb):
        ws, f, g2, g3 = make(vb)
        acc = {k: torch.zeros_like(x) for k, x in zip(keys3, inp)}

        def step():
            for a in acc.values():
                a.zero_()
            for v0 in range(0, V, vb):
                cs = cams[v0:v0 + vb] if vb > 1 else cams[v0]
                Gv = Gd[v0:v0 + vb] if vb > 1 else Gd[v0]
                q = R.project(*inp, cs, cfg, ws)
                R.raster_setup(q, cfg, ws)
                R.raster_forward(q, cfg, ws, fb=f["fb"], image=f["image"], T=f["T"],
                                 reuse_setup=True)
                R.raster_backward(q, f["fb"], Gv, cfg, ws, out=g2, reuse_setup=True)
                R.project_backward(*inp, cs, cfg, g2, out=g3)
                for k in keys3:
                    acc[k].add_(g3[k])

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps / V

    out = {"workload": f"{c['n_train']} clustered 3D Gaussians, {V} ring cameras, {W}x{H}, "
                       "FP16 framebuffer, tile reduction; 3D gradients summed over the views",
           "ms_per_view": {}}
    for vb in (1, 2, 4, 8):
        out["ms_per_view"][f"{vb}_views_per_call"] = round(run(vb), 4)
    return out


def micro_run(dev, reps=5):
    """The measured ceilings: a 1 GiB copy with the library's own copy kernel (best of `reps`,
    bytes read + written per second), and FP32 global atomic adds per second in three patterns
    over a 64 MB slot buffer (the size of the gradient slots of 800k splats)."""
    import torch
    from paper_2505_18764_amd import _lib as L
    st = torch.cuda.current_stream().cuda_stream
    nb = 1 << 30
    a = torch.ones(nb // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    best = 1e9
    for _ in range(reps):
        ev[0].record()
        L.gs_micro_copy(a, b, nb, st)
        ev[1].record()
        torch.cuda.synchronize()
        best = min(best, ev[0].elapsed_time(ev[1]))
    del a, b
    out = {"copy_bytes": nb, "copy_gbs": round(2 * nb / (best * 1e-3) / 1e9, 1)}
    nslots = 1 << 24
    slots = torch.zeros(nslots, dtype=torch.float32, device=dev)
    per = 64
    rates = {}
    for mode in ("spread", "spread_return", "wave_same"):
        L.gs_micro_atomic_f32(slots, nslots, 4, mode, st)          # warm
        ev[0].record()
        L.gs_micro_atomic_f32(slots, nslots, per, mode, st)
        ev[1].record()
        torch.cuda.synchronize()
        rates[mode] = round(per * L.MICRO_THREADS / (ev[0].elapsed_time(ev[1]) * 1e-3), 0)
    out["atomic_per_s"] = rates
    out["atomic_slots_bytes"] = nslots * 4
    return out


def variants_run(run_format, inp, cam, Gd, R, fmt, args):
    """Table 1's comparison on the benchmark view: the backward raster with each gradient
    reduction (naive, quad, wave and hybrid with X = 0 (no threshold), 4 and 8, the lane pre-sum
    and the tile reduction): ms of the gs_raster_bwd stage and atomic sets per live fragment;
    then the whole view with the forward T-culled (NEXT-1), and with the forward compositing
    every covered fragment (no saturation exit)."""
    import torch
    dev = inp[0].device
    cfg0 = R.RasterConfig(fb_format=fmt, reduce_mode="tile")
    ws = R.Workspace(dev)
    p = R.project(*inp, cam, cfg0, ws)
    R.raster_setup(p, cfg0, ws)
    f = R.raster_forward(p, cfg0, ws, reuse_setup=True)
    out = {}
    cases = [("naive", 8), ("quad", 8), ("wave", 0), ("wave", 4), ("wave", 8), ("hybrid", 0),
             ("hybrid", 4), ("hybrid", 8), ("hybrid_lane", 8), ("tile", 8)]
    for mode, X in cases:
        cfg = R.RasterConfig(fb_format=fmt, reduce_mode=mode, reduce_threshold=X)
        g2 = R.raster_backward(p, f["fb"], Gd, cfg, ws, reuse_setup=True)
        stt = R.new_stats(dev)
        R.raster_backward(p, f["fb"], Gd, cfg, ws, reuse_setup=True, stats=stt, out=g2)
        torch.cuda.synchronize()
        s = R.read_stats(stt)
        reps = 2 if mode == "naive" else 5
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            R.raster_backward(p, f["fb"], Gd, cfg, ws, reuse_setup=True, out=g2)
        ev[1].record()
        torch.cuda.synchronize()
        key = mode if mode in ("naive", "quad", "hybrid_lane", "tile") else f"{mode}_X{X}"
        out[key] = {"raster_bwd_ms": round(ev[0].elapsed_time(ev[1]) / reps, 4),
                    "atomic_rate": round(s["bwd_atomic_sets"] / max(1, s["bwd_live"]), 5)}
    r = run_format(fmt, args.reduce, t_min_fwd=float(np.float32(1e-4)),
                   steps=max(3, args.steps // 2), warmup=1)
    out["fwd_tcull"] = {"ms_per_view": round(r["ms_per_view"], 4),
                        "stages_ms": {k: round(v, 4) for k, v in r["stages_ms"].items()}}
    # every covered fragment composited (no saturation exit; depth split): the same image
    r = run_format(fmt, args.reduce, steps=max(3, args.steps // 2), warmup=1, composite_all=True)
    out["composite_all"] = {"ms_per_view": round(r["ms_per_view"], 4),
                            "stages_ms": {k: round(v, 4) for k, v in r["stages_ms"].items()}}
    return out


def fitting_run(dev, steps=300):
    """The fitting workload (500k Gaussians fitted to a hidden 500k scene over 8 ring cameras at
    1280x720, Adam lr 1e-3, one view per step through the autograd Function): ms per step over
    all 300 steps (device events), and the loss at the first and last step."""
    import torch
    import synth
    from paper_2505_18764_amd import render as R
    from paper_2505_18764_amd import train as TR
    c = synth.CFG4
    W, H = c["width"], c["height"]
    cams = [synth.camera_ring(k, c["cameras"], width=W, height=H, fx=c["fx"])
            for k in range(c["cameras"])]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    hidden = synth.scene3d(c["n_hidden"], seed=c["seed_hidden"])
    cfg = R.RasterConfig(reduce_mode="tile")
    ws = R.Workspace(dev)
    with torch.no_grad():
        targets = [R.rasterize_gaussians(t(hidden.means3d), t(hidden.scales), t(hidden.quats),
                                         t(hidden.opacities), t(hidden.sh), cm, cfg, ws)[0].clone()
                   for cm in cams]
    sc = synth.scene3d(c["n_train"], seed=c["seed_train"])
    params = TR.GaussianParams(t(sc.means3d), t(sc.scales), t(sc.quats), t(sc.opacities), t(sc.sh))
    TR.fit(params, cams, targets, 5, cfg=cfg)                      # warm up the kernels
    params = TR.GaussianParams(t(sc.means3d), t(sc.scales), t(sc.quats), t(sc.opacities), t(sc.sh))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    hist = TR.fit(params, cams, targets, steps, cfg=cfg, log_every=steps)
    e1.record()
    torch.cuda.synchronize()
    return {"workload": f"{c['n_train']} Gaussians fitted to a hidden {c['n_hidden']} over "
                        f"{c['cameras']} ring cameras, {W}x{H}, Adam lr 1e-3, one view per step, "
                        "FP32 framebuffer, tile reduction",
            "steps": steps, "ms_per_step": round(e0.elapsed_time(e1) / steps, 4),
            "loss_first": round(hist[0][1], 6), "loss_last": round(hist[-1][1], 6)}


def serving_run(n_requests, dev, warmup=200, rate=200.0, saturating_rate=3000.0):
    """Continuous-batching server on 16 resident scenes (50k-3M Gaussians), resolutions
    640x480-1920x1080, 70 % FWD / 30 % FWD_BWD, FP16 framebuffer, 64 GB pool, 4 streams: the
    specified Poisson stream at `rate`/s (warmup + n_requests), then an offered rate well above
    what the server sustains, which measures its capacity and the latency under overload."""
    import synth
    from paper_2505_18764_amd import serve as S
    scenes = S.load_scenes(dev)
    ex = S.GpuExecutor(scenes, S.serving_cameras(synth.CFG5_RESOLUTIONS))
    out = {}
    for name, r in (("spec", rate), ("saturating", saturating_rate)):
        srv = S.Server(ex, 64 << 30, slots=4).start()
        summ = S.run_load(srv, synth.serving_requests(n_requests + warmup, r), warmup)
        srv.stop()
        summ.update(offered_rate_per_s=r, requests=n_requests, warmup=warmup)
        out[name] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in summ.items()}
    out["capacity_views_per_s"] = out["saturating"]["views_per_s"]
    return out


def _cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_threads():
    """The host share of one GPU: OMP_NUM_THREADS where the launcher sets it, else the cores
    this process may run on."""
    nth = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    return max(1, min(nth, len(os.sched_getaffinity(0))))


def _oracle_view_sample(sc, cam, G, blocks, nth, seed=77):
    """FP64 oracle seconds for one view, from a sample: the projection of all Gaussians, the raster
    forward + backward on `blocks` random 32x32 blocks scaled to the frame, the projection
    backward on 2 % of the Gaussians scaled to all."""
    import oracle
    import synth
    cfg = oracle.OracleConfig(nthreads=nth)
    t0 = time.perf_counter()
    pre = oracle.preprocess(sc, cam, cfg)
    t_pre = time.perf_counter() - t0
    order = oracle.visible_order(pre["keys"])
    m2, cn, rgb = (pre["means2d"].astype(np.float32), pre["conic"].astype(np.float32),
                   pre["rgb"].astype(np.float32))
    g = np.random.default_rng(seed)
    W, H = cam.width, cam.height
    t_r, px = 0.0, 0
    for _ in range(blocks):
        x0, y0 = int(g.integers(0, W - 32)), int(g.integers(0, H - 32))
        t0 = time.perf_counter()
        oracle.raster(m2, cn, sc.opacities, rgb, order, W, H, crop=(x0, y0, 32, 32), dL_dimg=G,
                      cfg=cfg)
        t_r += time.perf_counter() - t0
        px += 32 * 32
    sub = g.choice(sc.n, size=max(1, sc.n // 50), replace=False)
    s2 = synth.Scene(means3d=sc.means3d[sub], scales=sc.scales[sub], quats=sc.quats[sub],
                     opacities=sc.opacities[sub], sh=sc.sh[sub], sh_degree=sc.sh_degree)
    gg = g.normal(size=(len(sub), 9))
    t0 = time.perf_counter()
    oracle.preprocess_vjp(s2, cam, gg[:, 0:2], gg[:, 2:5], gg[:, 6:9], gg[:, 5], cfg)
    t_vjp = (time.perf_counter() - t0) * sc.n / len(sub)
    total = t_pre + t_r * (W * H / px) + t_vjp
    return total, dict(t_pre=t_pre, t_raster=t_r, px=px, scale=W * H / px, t_vjp=t_vjp,
                       n_sub=len(sub))


def _oracle_full_2d(s, W, H, G, nth):
    import oracle
    t0 = time.perf_counter()
    oracle.raster(s.means2d, s.conics, s.opacities, s.rgb, oracle.depth_order(s.depth), W, H,
                  dL_dimg=G, cfg=oracle.OracleConfig(nthreads=nth))
    return time.perf_counter() - t0


def cpu_baseline(sc, cam, G, blocks):
    """The FP64 oracle on this host: the benchmark view from a bounded sample (`blocks` 32x32
    blocks at all host threads, a quarter of them at one thread), and the whole 1000-splat 128x128
    2D view (cfg1) at both thread counts. Times are scaled to ms per view."""
    import synth
    nth = _host_threads()
    tot_n, d_n = _oracle_view_sample(sc, cam, G, blocks, nth)
    b1 = max(4, blocks // 4)
    tot_1, d_1 = _oracle_view_sample(sc, cam, G, b1, 1, seed=78)
    c1 = synth.CFG1
    s1 = synth.splats2d(n=c1["n"], width=c1["width"], height=c1["height"], seed=c1["seed"])
    G1 = synth.image_grad(c1["width"], c1["height"], 31)
    cfg1_n = _oracle_full_2d(s1, c1["width"], c1["height"], G1, nth)
    cfg1_1 = _oracle_full_2d(s1, c1["width"], c1["height"], G1, 1)
    return {"value": round(tot_n * 1e3, 1), "unit": "ms/view", "cores": nth, "kind": "oracle",
            "cpu_model": _cpu_model(),
            "sample": f"FP64 oracle, benchmark view: projection of all {sc.n} Gaussians "
                      f"({d_n['t_pre']:.2f} s); raster fwd+bwd on {blocks} random 32x32 blocks "
                      f"({d_n['px']} px, {d_n['t_raster']:.2f} s) scaled by {d_n['scale']:.0f}x; "
                      f"projection backward on {d_n['n_sub']} Gaussians scaled by "
                      f"{sc.n / d_n['n_sub']:.0f}x",
            "stages_s": {"projection": round(d_n["t_pre"], 3),
                         "raster_fwd_bwd": round(d_n["t_raster"] * d_n["scale"], 2),
                         "projection_bwd": round(d_n["t_vjp"], 2),
                         "note": "the projection and its complex-step backward are numpy (one "
                                 "thread whatever `cores` says); the raster is the C oracle on "
                                 "`cores` OpenMP threads"},
            "one_thread": {"value": round(tot_1 * 1e3, 1), "unit": "ms/view", "cores": 1,
                           "sample": f"as above with {b1} blocks",
                           "stages_s": {"projection": round(d_1["t_pre"], 3),
                                        "raster_fwd_bwd": round(d_1["t_raster"] * d_1["scale"], 2),
                                        "projection_bwd": round(d_1["t_vjp"], 2)}},
            "cfg1_full_frame_ms": {"cores_all": round(cfg1_n * 1e3, 2),
                                   "cores_1": round(cfg1_1 * 1e3, 2)}}


def cpu_full(args):
    """The oracle on whole frames: cfg1 (1000 splats, 128x128) and cfg2 (200k Gaussians,
    1024x768: projection, raster forward + backward of the whole image, projection backward), at
    all host threads and at one; and the benchmark view from a 96-block sample at both. Host
    work only (no GPU)."""
    import oracle
    import synth
    nth = _host_threads()
    out = {"cpu_model": _cpu_model(), "threads_all": nth}
    c1 = synth.CFG1
    s1 = synth.splats2d(n=c1["n"], width=c1["width"], height=c1["height"], seed=c1["seed"])
    G1 = synth.image_grad(c1["width"], c1["height"], 31)
    _oracle_full_2d(s1, c1["width"], c1["height"], G1, nth)     # starts the OpenMP threads
    out["cfg1_full_s"] = {str(k): round(_oracle_full_2d(s1, c1["width"], c1["height"], G1, k), 4)
                          for k in (nth, 1)}
    print(json.dumps({"cfg1_full_s": out["cfg1_full_s"]}), flush=True)
    c2 = synth.CFG2
    sc2 = synth.scene3d(c2["n"], seed=c2["seed"])
    cam2 = synth.camera_front(c2["width"], c2["height"], c2["fx"])
    G2 = synth.image_grad(c2["width"], c2["height"], c2["grad_seed"])
    out["cfg2_full_s"] = {}
    for k in (nth, 1):
        cfg = oracle.OracleConfig(nthreads=k)
        t0 = time.perf_counter()
        r = oracle.render_scene(sc2, cam2, dL_dimg=G2, cfg=cfg)
        t_fwd = time.perf_counter() - t0
        print(json.dumps({"cfg2_threads": k, "render_s": round(t_fwd, 2)}), flush=True)
        t0 = time.perf_counter()
        og = r["grad"]
        oracle.preprocess_vjp(sc2, cam2, og[:, 0:2], og[:, 2:5], og[:, 6:9], og[:, 5], cfg)
        out["cfg2_full_s"][str(k)] = round(t_fwd + time.perf_counter() - t0, 2)
        print(json.dumps({"cfg2_threads": k, "s": out["cfg2_full_s"][str(k)]}), flush=True)
    c3 = synth.CFG3
    sc3 = synth.scene3d(c3["n"], seed=c3["seed"])
    cam3 = synth.camera_front(c3["width"], c3["height"], c3["fx"])
    G3 = synth.image_grad(c3["width"], c3["height"], c3["grad_seed"])
    out["cfg3_sampled_ms_per_view"] = {}
    for k, blocks in ((nth, 96), (1, 24)):
        tot, d = _oracle_view_sample(sc3, cam3, G3, blocks, k)
        out["cfg3_sampled_ms_per_view"][str(k)] = {"ms": round(tot * 1e3, 1), "blocks": blocks}
        print(json.dumps({"cfg3_threads": k, **out["cfg3_sampled_ms_per_view"][str(k)]}), flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
