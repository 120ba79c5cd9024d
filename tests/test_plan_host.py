"""The raster's tile schedulers run on the CPU (no GPU): plan.hpp's bucket_order, the code every
schedule of the GPU path uses (the forward's tile order, the depth split's work-item order, the
backward's tile order), is compiled for the host with a sequential emulation of one workgroup
whose threads run each phase in a seeded random order. Each result must be a permutation of the
work items, heaviest bucket first, padded with -1; the depth split's segment counts must fit the
workspace's fixed item capacity. Adversarial weights: all equal, all zero, ties at bucket edges,
the largest uint32, one tile holding everything, heavy tails, tile counts 1 to 2^18."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "plan_host.hip")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def plan(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("plan") / "libplan_host.so")
    subprocess.run([HIPCC, "--offload-host-only", "-O2", "-std=c++17", "-fPIC", "-shared",
                    "-o", out, SRC], check=True, capture_output=True)
    L = ctypes.CDLL(out)
    P = ctypes.c_void_p
    L.plan_bucket_order.argtypes = [P, ctypes.c_int, ctypes.c_uint32, P, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_uint64]
    L.plan_weight_bucket.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    L.plan_segment_cap.restype = ctypes.c_uint32
    L.plan_segment_cap.argtypes = [ctypes.c_ulonglong, ctypes.c_int]
    L.plan_segment_count.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    L.plan_cut_target.restype = ctypes.c_uint32
    L.plan_cut_target.argtypes = [ctypes.c_uint32, ctypes.c_int, ctypes.c_int]
    return L


def _order(L, w, pad=None, wmax=None, nthreads=1024, seed=0):
    w = np.ascontiguousarray(w, np.uint32)
    count = w.size
    pad = count if pad is None else pad
    wmax = int(w.max()) if (wmax is None and count) else int(wmax or 0)
    out = np.full(max(pad, 1), 0x7777, np.int32)
    L.plan_bucket_order(w.ctypes.data_as(ctypes.c_void_p), count, wmax,
                        out.ctypes.data_as(ctypes.c_void_p), pad, nthreads, seed)
    return out[:pad]


def _check_order(L, w, out, wmax):
    count = len(w)
    np.testing.assert_array_equal(np.sort(out[:count]), np.arange(count))   # a permutation
    assert (out[count:] == -1).all()
    b = np.array([L.plan_weight_bucket(int(w[i]), wmax) for i in out[:count]])
    assert (np.diff(b) >= 0).all()                                          # heaviest first


def _cases():
    g = np.random.default_rng(5)
    yield "all equal 1", np.full(1, 7)
    yield "all equal 4096", np.full(4096, 123)
    yield "all zero 8192", np.zeros(8192)
    yield "all max 1000", np.full(1000, 2**32 - 1)
    edges = (np.arange(1024) * 4097 // 1024).astype(np.int64)            # wmax 4096: bucket edges
    yield "bucket edges", np.clip(np.concatenate([edges - 1, edges, edges + 1, [4096]]), 0, 4096)
    yield "one heavy tile", np.concatenate([[2**28], np.zeros(4095)])
    yield "uint32 extremes", np.array([0, 1, 2**31, 2**32 - 2, 2**32 - 1, 5] * 100)
    yield "lognormal 8192", np.minimum(g.lognormal(8, 3, 8192), 2**32 - 1)
    yield "ragged 1025", g.integers(0, 50, 1025)
    yield "large image 2^18", g.integers(0, 10**6, 2**18)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bucket_order_is_a_heaviest_first_permutation(plan, seed):
    for name, w in _cases():
        w = np.asarray(w, np.uint64).astype(np.uint32)
        wmax = int(w.max())
        out = _order(plan, w, seed=seed)
        _check_order(plan, w, out, wmax)


def test_bucket_order_pads_and_tolerates_a_small_wmax(plan):
    g = np.random.default_rng(8)
    w = g.integers(0, 1000, 3000).astype(np.uint32)
    out = _order(plan, w, pad=4 * 3000)                  # the item order's padded capacity
    _check_order(plan, w, out, int(w.max()))
    # a bound below some weights still gives a permutation (those weights share bucket 0)
    out = _order(plan, w, wmax=10)
    np.testing.assert_array_equal(np.sort(out), np.arange(3000))
    # weights whose scaled value leaves the int range (a zero bound, weights near 2^32)
    w2 = np.array([2**32 - 1, 2**31, 5, 0, 2**32 - 1], np.uint32)
    for wmax in (0, 1, 2**20):
        out = _order(plan, w2, wmax=wmax)
        np.testing.assert_array_equal(np.sort(out), np.arange(5))
    out = _order(plan, np.zeros(0, np.uint32), pad=16)   # no items at all
    assert (out == -1).all()


@pytest.mark.parametrize("nthreads", [1, 64, 1000, 1024])
def test_bucket_order_any_workgroup_size(plan, nthreads):
    w = np.random.default_rng(nthreads).integers(0, 2**20, 5000).astype(np.uint32)
    _check_order(plan, w, _order(plan, w, nthreads=nthreads, seed=nthreads), int(w.max()))


def test_weight_bucket_is_monotone(plan):
    for wmax in (0, 1, 1023, 1024, 4096, 10**6, 2**24 + 1, 2**32 - 1):
        xs = sorted(set(np.linspace(0, wmax, 3000).astype(np.uint64).tolist() + [wmax]))
        b = [plan.plan_weight_bucket(int(x), wmax) for x in xs]
        assert all(0 <= v < 1024 for v in b)
        assert all(b1 >= b2 for b1, b2 in zip(b, b[1:])), wmax   # heavier: same or earlier
        assert b[0] == 1023                                        # weight 0: the last bucket
        if wmax >= 1023:
            assert b[-1] == 0                                      # the maximum: the first


@pytest.mark.parametrize("ntiles", [1, 2, 17, 4096])
def test_depth_split_fits_its_item_capacity(plan, ntiles):
    ipt, mseg = plan.plan_items_per_tile(), plan.plan_max_segments()
    g = np.random.default_rng(ntiles)
    for w in (np.full(ntiles, 5000), np.zeros(ntiles), g.integers(0, 2**16, ntiles),
              np.minimum(g.lognormal(6, 3, ntiles), 2**28),
              np.concatenate([[2**28], np.zeros(ntiles - 1)])):
        w = w.astype(np.uint64)
        cap = plan.plan_segment_cap(int(w.sum()), ntiles)
        assert cap >= 1
        k = np.array([plan.plan_segment_count(int(x), cap) for x in w])
        assert ((k >= 1) & (k <= mseg)).all()
        assert k.sum() <= ipt * ntiles                    # the items array never overflows
        for wt, kt in zip(w[:64], k[:64]):
            tg = [plan.plan_cut_target(int(wt), j, int(kt)) for j in range(int(kt) + 1)]
            assert tg[0] == 0 and tg[-1] == wt           # cuts run from the front to the end
            assert all(a <= b for a, b in zip(tg, tg[1:]))
