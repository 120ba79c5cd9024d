"""The benchmark's format error measure (the paper's RMSE and binned mean relative error) on
inputs whose answer is known by hand."""
import numpy as np
import pytest

import bench


def test_format_error_table_known_values():
    ref = np.array([20.0, -40.0, 1.0, -5.0, 0.01, 0.05, 1e-4, 0.0])
    g = ref.copy()
    g[0] += 2.0          # 10 % in [10, inf)
    g[1] -= 2.0          #  5 % in [10, inf)
    g[2] += 0.5          # 50 % in [0.1, 10)
    g[4] += 0.01         # 100 % in [1e-3, 0.1)
    g[6] += 1.0          # below the bins: counts only in the RMSE
    t = bench.format_error_table(g, ref)
    assert t["mre_10_inf"] == pytest.approx((0.10 + 0.05) / 2)
    assert t["mre_0.1_10"] == pytest.approx((0.5 + 0.0) / 2)
    assert t["mre_1e-3_0.1"] == pytest.approx((1.0 + 0.0) / 2)
    assert (t["n_10_inf"], t["n_0.1_10"], t["n_1e-3_0.1"]) == (2, 2, 2)
    assert t["rmse"] == pytest.approx(np.sqrt((4 + 4 + 0.25 + 1e-4 + 1.0) / 8))


def test_format_error_table_empty_bins():
    t = bench.format_error_table(np.zeros(3), np.zeros(3))
    assert t["rmse"] == 0.0 and t["mre_10_inf"] is None


def test_roofline_kernels_are_in_the_traffic_summary():
    """The launches bench.py prices its roofline on are named as the committed counters name
    them (the kernel templates' instances), so the traffic figure can be found."""
    import json
    import os
    d = json.load(open(os.path.join(os.path.dirname(bench.__file__), "profiles", "traffic.json")))
    for k in bench.FWD_KERNELS + bench.BWD_KERNELS:
        assert k in d, k


def _counter_db(path, rows):
    """A rocprofv3-shaped counter database: rows of (kernel, counter, value, dispatch, ns)."""
    import sqlite3
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, "
                "value real, dispatch_id integer, duration real)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?, ?)", rows)
    con.commit()
    con.close()


def test_counter_summaries_from_a_synthetic_database(tmp_path):
    """The counter summaries bench.py commits: per-dispatch values summed over counter instances
    and averaged over dispatches; the wave-state shares; the atomic rate; the micro kernel's
    measured (longest) launch instead of the mean with its warm-up."""
    from paper_2505_18764_amd import pmc
    k = "void gsr::k_raster_bwd<-1, false, false, true>(int, float*)"
    s1 = [(k, "SQ_WAVE_CYCLES", 500.0, d, 1000.0) for d in (1, 2)] + \
         [(k, "SQ_WAVE_CYCLES", 500.0, d, 1000.0) for d in (1, 2)] + \
         [(k, c, v, d, 1000.0) for d in (1, 2) for c, v in
          (("SQ_WAIT_ANY", 400.0), ("SQ_WAIT_INST_ANY", 200.0), ("SQ_ACTIVE_INST_VALU", 250.0),
           ("SQ_ACTIVE_INST_LDS", 10.0), ("SQ_BUSY_CYCLES", 1.0), ("SQ_WAIT_INST_LDS", 1.0),
           ("SQ_LDS_BANK_CONFLICT", 0.0))]
    s2 = [(k, c, v, d, 1000.0) for d in (1, 2) for c, v in
          (("SQ_THREAD_CYCLES_VALU", 60.0 * 125.0), ("SQ_ACTIVE_INST_VALU", 125.0),
           ("SQ_ACTIVE_INST_SCA", 50.0), ("SQ_ACTIVE_INST_MISC", 10.0), ("SQ_INSTS_VALU", 1.0),
           ("SQ_INSTS_BRANCH", 1.0), ("SQ_WAVES", 1.0), ("SQ_INSTS_SMEM", 1.0))]
    _counter_db(str(tmp_path / "s1.db"), s1)
    _counter_db(str(tmp_path / "s2.db"), s2)
    m = pmc.counter_means(str(tmp_path / "s1.db"))
    kk = "k_raster_bwd<-1, false, false, true>"
    assert m[kk]["SQ_WAVE_CYCLES"] == 1000.0 and m[kk]["_calls"] == 2   # two instances summed
    r = pmc.stall_summary([str(tmp_path / "s1.db"), str(tmp_path / "s2.db")],
                          str(tmp_path / "st.md"), ["cmd"], "w")[kk]
    assert r["wait_dependency"] == pytest.approx(0.4) and r["wait_issue"] == pytest.approx(0.2)
    assert r["valu"] == pytest.approx(0.25) and r["lanes_per_valu"] == pytest.approx(60.0)
    assert r["scalar"] == pytest.approx(50.0 * 2.0 / 1000.0)     # scaled by the VALU ratio
    mk = "void gsr::k_micro_atomic<0>(float*, unsigned int, int, float*)"
    at = [(mk, "TCC_ATOMIC_sum", 10.0, 1, 100.0), (mk, "TCC_ATOMIC_sum", 160.0, 2, 1600.0)] + \
         [(k, "TCC_ATOMIC_sum", 50.0, d, 1000.0) for d in (3, 4)]
    _counter_db(str(tmp_path / "at.db"), at)
    a = pmc.atomic_summary(str(tmp_path / "at.db"), str(tmp_path / "at.md"), "cmd", "w")
    assert a["k_micro_atomic<0>"]["TCC_ATOMIC_sum"] == 160.0          # the measured launch
    assert a[kk]["l2_atomics_per_s"] == pytest.approx(50.0 / 1e-6)
