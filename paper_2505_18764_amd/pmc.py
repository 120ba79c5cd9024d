"""HBM traffic per kernel launch from rocprofv3 PMC databases.

Two counter passes over the same program, one with ``--pmc FETCH_SIZE`` and one with
``--pmc WRITE_SIZE`` (each with ``--kernel-trace``), give per-dispatch kilobytes read from and
written to device memory. The counters' scale is calibrated against a plain device-to-device
copy of known size (``bench.py --copy-probe``, 512 MiB copied three times), profiled the same
two ways: the calibration factor of each counter is bytes copied / (counter KiB x 1024).

``summarize`` writes ``traffic.json`` (per kernel: scaled bytes read, written, and their sum per
launch, the mean launch duration, and the hash of the kernel sources the counters were taken
with; a consumer ignores entries whose hash differs from the current sources) and a short
markdown table. ``trace_summary`` turns a ``--kernel-trace --stats`` database into a markdown
table of kernel durations; ``issue_summary`` turns an SQ instruction-counter pass into the VALU
issue share of each kernel.
"""
from __future__ import annotations

import collections
import hashlib
import json
import os
import re
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))


def source_hash() -> str:
    """Hash of the HIP sources and the build flags (the counters describe the kernels these
    build)."""
    h = hashlib.sha256()
    d = os.path.join(HERE, "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    from .build import FLAGS, SOURCE_FLAGS
    flags = [f for i, f in enumerate(FLAGS) if f != "-I" and (i == 0 or FLAGS[i - 1] != "-I")]
    h.update(" ".join(flags).encode())              # no paths: the hash is the same on any host
    for src in sorted(SOURCE_FLAGS):
        h.update((src + " " + " ".join(SOURCE_FLAGS[src])).encode())
    return h.hexdigest()[:16]


def short_name(n: str) -> str:
    n = re.sub(r"\(.*$", "", n)
    return n.replace("void ", "").replace("gsr::", "").strip()


def _db(path: str) -> str:
    if os.path.isdir(path):
        for root, _, files in os.walk(path):
            for f in files:
                if f.endswith("_results.db"):
                    return os.path.join(root, f)
        raise FileNotFoundError(f"no *_results.db under {path}")
    return path


def counter_means(path: str) -> dict:
    """{kernel: {counter: mean value per dispatch, '_calls': n, '_dur_ns': mean duration}}."""
    cur = sqlite3.connect(_db(path)).cursor()
    vals = collections.defaultdict(lambda: collections.defaultdict(dict))
    dur = collections.defaultdict(dict)
    for k, c, v, d, du in cur.execute(
            "select kernel_name, counter_name, value, dispatch_id, duration from counters_collection"):
        k = short_name(k)
        vals[k][c][d] = vals[k][c].get(d, 0.0) + float(v)
        dur[k][d] = float(du)
    out = {}
    for k, cs in vals.items():
        out[k] = {c: sum(dv.values()) / len(dv) for c, dv in cs.items()}
        out[k]["_calls"] = len(dur[k])
        out[k]["_dur_ns"] = sum(dur[k].values()) / max(1, len(dur[k]))
    return out


def _copy_kernel(m: dict) -> str:
    cands = [k for k in m if "copy" in k.lower()]
    if not cands:
        raise ValueError("no copy kernel in the calibration database")
    return max(cands, key=lambda k: m[k]["_dur_ns"])


def summarize(fetch_db, write_db, copy_fetch_db, copy_write_db, copy_bytes: int, out_dir: str,
              command: str, workload: str) -> dict:
    f, w = counter_means(fetch_db), counter_means(write_db)
    cf, cw = counter_means(copy_fetch_db), counter_means(copy_write_db)
    kf, kw = _copy_kernel(cf), _copy_kernel(cw)
    fac_f = copy_bytes / (cf[kf]["FETCH_SIZE"] * 1024.0)
    fac_w = copy_bytes / (cw[kw]["WRITE_SIZE"] * 1024.0)
    h = source_hash()
    res = {"_calibration": {"copy_bytes": copy_bytes, "fetch_factor": fac_f, "write_factor": fac_w,
                            "copy_kernel": kf},
           "_command": command, "_workload": workload}
    for k in sorted(set(f) & set(w)):
        if "FETCH_SIZE" not in f[k] or "WRITE_SIZE" not in w[k]:
            continue
        rd = f[k]["FETCH_SIZE"] * 1024.0 * fac_f
        wr = w[k]["WRITE_SIZE"] * 1024.0 * fac_w
        res[k] = {"read_bytes": rd, "write_bytes": wr, "bytes_per_launch": rd + wr,
                  "mean_ns": f[k]["_dur_ns"], "calls": f[k]["_calls"], "source_hash": h}
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, "traffic.json"), "w") as fh:
        json.dump(res, fh, indent=1)
    lines = [f"# HBM traffic per launch: {workload}", "",
             "Commands (run from the repository root on one MI355X; `$OUT` is any scratch "
             "directory):", "", "```", command, "```", "",
             f"Calibration: a {copy_bytes / 2**20:.0f} MiB device copy reads FETCH_SIZE x "
             f"{fac_f:.3f} and WRITE_SIZE x {fac_w:.3f} (bytes per counter byte).", "",
             "| kernel | calls | mean us | read MB | written MB | GB/s |", "|---|---:|---:|---:|---:|---:|"]
    for k, v in sorted(((k, v) for k, v in res.items() if not k.startswith("_")),
                       key=lambda kv: -kv[1]["mean_ns"] * kv[1]["calls"]):
        if v["mean_ns"] * v["calls"] < 20_000:
            continue
        gbs = v["bytes_per_launch"] / v["mean_ns"]
        lines.append(f"| `{k}` | {v['calls']} | {v['mean_ns'] / 1e3:.1f} | {v['read_bytes'] / 1e6:.1f} | "
                     f"{v['write_bytes'] / 1e6:.1f} | {gbs:.0f} |")
    lines += ["", f"Source hash of the kernels measured: `{h}`."]
    with open(os.path.join(out_dir, "traffic_1M_1600x1064_f16.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return res


def trace_summary(path: str, out_md: str, command: str, workload: str, note: str = "") -> list:
    """Markdown table of kernel durations (calls, total, mean, share) from a rocprofv3
    ``--kernel-trace`` database; returns the rows."""
    cur = sqlite3.connect(_db(path)).cursor()
    rows = list(cur.execute(
        "select name, total_calls, total_duration, average, percentage from top_kernels"))
    lines = [f"# Kernel durations: {workload}", "",
             "Command (on one MI355X; `$R` is the repository root, `$OUT` any scratch directory):",
             "", "```", command, "```", "",
             "| kernel | calls | total us | avg us | % |", "|---|---:|---:|---:|---:|"]
    out = []
    for n, c, tot, avg, pct in rows:
        if pct < 0.05:
            continue
        k = short_name(n)
        out.append((k, int(c), tot, avg, pct))       # the view reports microseconds
        lines.append(f"| `{k}` | {int(c)} | {tot:.1f} | {avg:.1f} | {pct:.1f} |")
    lines += ["", f"Source hash of the kernels measured: `{source_hash()}`."]
    if note:
        lines += ["", note]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return out


CLOCK_HZ = 2.4e9          # MI355X peak engine clock
SIMDS = 256 * 4           # 256 CUs x 4 SIMDs
VALU_CYCLES = 4           # a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles


def issue_summary(path: str, out_md: str, command: str, workload: str, top: int = 8) -> dict:
    """Per kernel: wave instructions issued per launch (SQ_INSTS_VALU, _SALU, _LDS,
    _VALU_TRANS_F32) and the VALU issue share = 4 x VALU instructions / (launch duration x
    clock x 1024 SIMDs), i.e. the fraction of the chip's SIMD cycles the kernel's VALU work
    fills at the peak clock; also the same share without the transcendental instructions, which
    gfx950 issues to a pipeline of their own (a share above 1 with them counted shows it)."""
    m = counter_means(path)
    res = {}
    lines = [f"# Instruction issue per launch: {workload}", "",
             "Command (on one MI355X; `$R` is the repository root, `$OUT` any scratch directory):",
             "", "```", command, "```", "",
             "VALU share = 4 cycles x SQ_INSTS_VALU / (mean launch duration x 2.4 GHz x 1024 SIMDs);",
             "a value near 1 means the SIMDs issue a VALU instruction almost every cycle. The",
             "transcendentals (SQ_INSTS_VALU_TRANS_F32, counted in SQ_INSTS_VALU) issue to a",
             "pipeline of their own on gfx950, so a share above 1 is possible; the last column",
             "leaves them out.", "",
             "| kernel | mean us | VALU (M) | trans (M) | SALU (M) | LDS (M) | VALU share "
             "| share without trans |",
             "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for k in sorted(m, key=lambda k: -m[k]["_dur_ns"] * m[k]["_calls"])[:top]:
        v = m[k]
        if "SQ_INSTS_VALU" not in v:
            continue
        dur = v["_dur_ns"] * 1e-9
        share = VALU_CYCLES * v["SQ_INSTS_VALU"] / (dur * CLOCK_HZ * SIMDS)
        trans = v.get("SQ_INSTS_VALU_TRANS_F32", 0)
        share_nt = VALU_CYCLES * (v["SQ_INSTS_VALU"] - trans) / (dur * CLOCK_HZ * SIMDS)
        res[k] = dict(valu=v["SQ_INSTS_VALU"], share=share, share_no_trans=share_nt,
                      mean_ns=v["_dur_ns"])
        lines.append(f"| `{k}` | {v['_dur_ns'] / 1e3:.1f} | {v['SQ_INSTS_VALU'] / 1e6:.1f} | "
                     f"{v.get('SQ_INSTS_VALU_TRANS_F32', 0) / 1e6:.1f} | "
                     f"{v.get('SQ_INSTS_SALU', 0) / 1e6:.1f} | {v.get('SQ_INSTS_LDS', 0) / 1e6:.1f} | "
                     f"{share:.2f} | {share_nt:.2f} |")
    h = source_hash()
    lines += ["", f"Source hash of the kernels measured: `{h}`."]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    js = {k: dict(v, source_hash=h) for k, v in res.items()}
    js["_command"] = command
    with open(os.path.join(os.path.dirname(out_md), "issue.json"), "w") as fh:
        json.dump(js, fh, indent=1)
    return res


# L2-side and L1-side atomic request counters (summed over the L2 channels / L1 instances): the
# requests the L2 executes, those it forwards to memory, and the vector-L1 requests with and
# without a returned value.
ATOMIC_COUNTERS = ("TCC_ATOMIC_sum", "TCC_EA0_ATOMIC_sum", "TCP_TCC_ATOMIC_WITH_RET_REQ_sum",
                   "TCP_TCC_ATOMIC_WITHOUT_RET_REQ_sum")


def _longest_dispatches(path: str, prefix: str) -> dict:
    """{kernel: {counter: value, '_calls': 1, '_dur_ns': duration}} for the longest dispatch of
    each kernel whose name starts with `prefix` (a microbenchmark's measured launch, not its
    warm-up)."""
    cur = sqlite3.connect(_db(path)).cursor()
    per = collections.defaultdict(lambda: collections.defaultdict(dict))
    for k, c, v, d, du in cur.execute(
            "select kernel_name, counter_name, value, dispatch_id, duration from counters_collection"):
        k = short_name(k)
        if k.startswith(prefix):
            per[k][d][c] = per[k][d].get(c, 0.0) + float(v)
            per[k][d]["_dur_ns"] = float(du)
    out = {}
    for k, ds in per.items():
        best = max(ds.values(), key=lambda e: e["_dur_ns"])
        out[k] = dict(best, _calls=1)
    return out


def atomic_summary(path: str, out_md: str, command: str, workload: str, top: int = 10) -> dict:
    """Per kernel that issues atomics: the counters of ATOMIC_COUNTERS per launch and the L2
    atomic rate (TCC_ATOMIC per second of launch time); for the atomic microbenchmark, its
    measured launch (the longest) rather than the mean with its warm-up."""
    m = counter_means(path)
    m.update(_longest_dispatches(path, "k_micro_atomic"))
    res = {}
    lines = [f"# Atomic requests per launch: {workload}", "",
             "Command (on one MI355X; `$R` is the repository root, `$OUT` any scratch directory):",
             "", "```", command, "```", "",
             "| kernel | calls | mean us | L2 atomics (M) | to memory (M) | L1 req. with return (M) "
             "| L1 req. without return (M) | L2 atomics / s (G) |",
             "|---|---:|---:|---:|---:|---:|---:|---:|"]
    rows = [k for k in m if m[k].get("TCC_ATOMIC_sum", 0) > 0]
    for k in sorted(rows, key=lambda k: -m[k]["_dur_ns"] * m[k]["_calls"])[:top]:
        v = m[k]
        rate = v["TCC_ATOMIC_sum"] / (v["_dur_ns"] * 1e-9)
        res[k] = {c: v.get(c) for c in ATOMIC_COUNTERS}
        res[k].update(mean_ns=v["_dur_ns"], calls=v["_calls"], l2_atomics_per_s=rate)
        cells = [f"{v.get(c, 0) / 1e6:.2f}" for c in ATOMIC_COUNTERS]
        lines.append(f"| `{k}` | {v['_calls']} | {v['_dur_ns'] / 1e3:.1f} | " + " | ".join(cells)
                     + f" | {rate / 1e9:.1f} |")
    h = source_hash()
    lines += ["", f"Source hash of the kernels measured: `{h}`."]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    js = {k: dict(v, source_hash=h) for k, v in res.items()}
    js["_command"] = command
    with open(os.path.join(os.path.dirname(out_md), "atomics.json"), "w") as fh:
        json.dump(js, fh, indent=1)
    return res


STALL_COUNTERS = (("SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
                   "SQ_WAIT_INST_LDS", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS",
                   "SQ_LDS_BANK_CONFLICT"),
                  ("SQ_THREAD_CYCLES_VALU", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_VALU",
                   "SQ_ACTIVE_INST_SCA", "SQ_ACTIVE_INST_MISC", "SQ_INSTS_BRANCH", "SQ_WAVES",
                   "SQ_INSTS_SMEM"))


def stall_summary(paths, out_md: str, commands, workload: str, top: int = 6) -> dict:
    """Where the waves of each kernel spend their time, from two counter passes: the shares of
    resident wave-cycles (SQ_WAVE_CYCLES) spent waiting on a dependency (SQ_WAIT_ANY), ready but
    not issued (SQ_WAIT_INST_ANY), and issuing VALU, scalar, LDS and other instructions; and the
    active lanes per VALU instruction (SQ_THREAD_CYCLES_VALU / SQ_ACTIVE_INST_VALU)."""
    m1, m2 = counter_means(paths[0]), counter_means(paths[1])
    res = {}
    lines = [f"# Wave time by state: {workload}", "",
             "Commands (on one MI355X; `$R` is the repository root, `$OUT` any scratch directory):",
             "", "```", *commands, "```", "",
             "Shares of the resident wave-cycles (SQ_WAVE_CYCLES) of each kernel: waiting on a",
             "dependency such as a memory result or a barrier (SQ_WAIT_ANY), ready but not issued",
             "because another wave had the issue slot (SQ_WAIT_INST_ANY), and issuing VALU, scalar",
             "(SALU and SMEM), LDS and miscellaneous instructions (SQ_ACTIVE_INST_*, from the second",
             "pass, scaled by that pass's SQ_ACTIVE_INST_VALU to the first's). Lanes per VALU",
             "instruction = SQ_THREAD_CYCLES_VALU / SQ_ACTIVE_INST_VALU (64 = no idle lanes).", "",
             "| kernel | mean us | wait (dependency) | wait (issue) | VALU | scalar | LDS | misc "
             "| lanes per VALU |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for k in sorted(set(m1) & set(m2), key=lambda k: -m1[k]["_dur_ns"] * m1[k]["_calls"])[:top]:
        a, b = m1[k], m2[k]
        wc = a.get("SQ_WAVE_CYCLES", 0.0)
        if not wc or not b.get("SQ_ACTIVE_INST_VALU"):
            continue
        sc = a["SQ_ACTIVE_INST_VALU"] / b["SQ_ACTIVE_INST_VALU"]
        r = {"wait_dependency": a["SQ_WAIT_ANY"] / wc, "wait_issue": a["SQ_WAIT_INST_ANY"] / wc,
             "valu": a["SQ_ACTIVE_INST_VALU"] / wc,
             "scalar": b.get("SQ_ACTIVE_INST_SCA", 0.0) * sc / wc,
             "lds": a.get("SQ_ACTIVE_INST_LDS", 0.0) / wc,
             "misc": b.get("SQ_ACTIVE_INST_MISC", 0.0) * sc / wc,
             "lanes_per_valu": b.get("SQ_THREAD_CYCLES_VALU", 0.0) / b["SQ_ACTIVE_INST_VALU"],
             "mean_ns": a["_dur_ns"]}
        res[k] = r
        lines.append(f"| `{k}` | {a['_dur_ns'] / 1e3:.1f} | {r['wait_dependency']:.2f} | "
                     f"{r['wait_issue']:.2f} | {r['valu']:.2f} | {r['scalar']:.2f} | "
                     f"{r['lds']:.2f} | {r['misc']:.2f} | {r['lanes_per_valu']:.1f} |")
    h = source_hash()
    lines += ["", f"Source hash of the kernels measured: `{h}`."]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return res
