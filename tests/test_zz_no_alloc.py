"""gs_sort_noalloc (the depth sort with the library's fixed per-device scratch, for callers that
cannot allocate) against gs_sort with a caller workspace, through the C ABI: bit-exact keys and
ids on two calls in a row, the second smaller than the first (the scratch keeps the first call's
contents), a visible prefix shorter than n, and the size limit rejected before any launch."""
import numpy as np
import pytest

import synth
from tests.helpers import t

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2505_18764_amd import _lib as L  # noqa: E402


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _with_workspace(keys, n_visible):
    n = keys.size
    k = t(keys.view(np.int32))
    ids = t(np.arange(n, dtype=np.int32))
    nv = t(np.array([n_visible], np.int32))
    need = L.gs_workspace_size("sort", n, 1, 1, L.GsConfig())
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
    L.gs_sort(n, k, ids, nv, ws, ws.numel(), _stream())
    return k, ids


def _noalloc(keys, n_visible):
    n = keys.size
    k = t(keys.view(np.int32))
    ids = t(np.arange(n, dtype=np.int32))
    nv = t(np.array([n_visible], np.int32))
    L.gs_sort_noalloc(n, k, ids, nv, _stream())
    return k, ids


def test_noalloc_sort_equals_workspace_sort_on_two_calls():
    cases = [(1_000_000, 1_000_000, 40_000, 61),     # the benchmark's splat count, many ties
             (123_457, 100_000, 300, 62)]            # then a smaller call with a ragged prefix
    for n, nv, ties, seed in cases:
        keys = synth.sorted_key_case(n, seed=seed, tie_levels=ties)
        print(f"[noalloc] n {n} n_visible {nv} tie levels {ties}", flush=True)
        kw, iw = _with_workspace(keys, nv)
        kn, inn = _noalloc(keys, nv)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(inn.cpu().numpy(), iw.cpu().numpy())
        np.testing.assert_array_equal(kn.cpu().numpy(), kw.cpu().numpy())
        assert (inn.cpu().numpy()[nv:] == np.arange(nv, n)).all()   # the rest left in place


def test_noalloc_sort_limits():
    assert L.NOALLOC_SORT_MAX_N == 1 << 22
    nv = t(np.array([0], np.int32))
    with pytest.raises(L.GsrError) as ei:          # rejected on the host, nothing launched
        L.gs_sort_noalloc(L.NOALLOC_SORT_MAX_N + 1, 0x1000, 0x1000, nv, _stream())
    assert ei.value.status == 2 and "at most" in str(ei.value)
    L.gs_sort_noalloc(0, None, None, nv, _stream())  # n = 0: nothing to do
