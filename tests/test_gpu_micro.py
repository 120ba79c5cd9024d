"""The microbenchmarks that measure the raster's ceilings do the work they are timed for: the
copy copies, and every atomic add lands (the values added are exact in FP32, so each slot's sum
is exact)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2505_18764_amd import _lib as L  # noqa: E402


def test_micro_copy_copies():
    st = torch.cuda.current_stream().cuda_stream
    a = torch.arange(1 << 20, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    L.gs_micro_copy(a, b, a.numel() * 4, st)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("mode", ["spread", "spread_return", "wave_same"])
def test_micro_atomics_all_land(mode):
    st = torch.cuda.current_stream().cuda_stream
    nslots = 1 << 16
    s = torch.zeros(nslots, dtype=torch.float32, device="cuda")
    per = 4
    L.gs_micro_atomic_f32(s, nslots, per, mode, st)
    torch.cuda.synchronize()
    # 4 x 2^20 adds of 1/64 spread evenly over 2^16 slots: each slot ends at exactly 1
    np.testing.assert_array_equal(s.cpu().numpy(), np.ones(nslots, np.float32))
