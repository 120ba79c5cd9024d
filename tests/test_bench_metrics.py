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
