"""Serving on the GPU: requests of different scenes, sizes and modes admitted concurrently on
several streams give the same images, bit for bit, as each request run alone, and the same
gradients to the rounding of atomic accumulation order."""
import numpy as np
import pytest

import synth
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2505_18764_amd import render as R  # noqa: E402
from paper_2505_18764_amd import serve as S  # noqa: E402


def _scenes(dev):
    out = {}
    for j, n in enumerate([20_000, 60_000, 150_000, 5_000]):
        sc = synth.scene3d(n, seed=600 + j)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        out[j] = (t(sc.means3d), t(sc.scales), t(sc.quats), t(sc.opacities), t(sc.sh))
    return out


def test_results_alone_equal_results_in_the_mix():
    dev = torch.device("cuda:0")
    res = [(320, 240), (640, 480), (400, 300)]
    ex = S.GpuExecutor(_scenes(dev), S.serving_cameras(res))
    g = np.random.default_rng(3)
    specs = [(int(g.integers(0, 4)), res[int(g.integers(0, 3))],
              S.FWD if g.uniform() < 0.6 else S.FWD_BWD) for _ in range(24)]
    srv = S.Server(ex, pool_bytes=8 << 30, slots=4).start()
    mix = [srv.submit(S.Request(rid=i, scene=sc, width=W, height=H, mode=m, keep_result=True))
           for i, (sc, (W, H), m) in enumerate(specs)]
    for r in mix:
        assert r.wait(120)
    srv.stop()
    assert all(r.status == "done" for r in mix)
    assert srv.peak_running > 1                          # work really overlapped on the device

    def alone(i, sc, W, H, m):
        srv1 = S.Server(ex, pool_bytes=8 << 30, slots=1).start()
        r = srv1.submit(S.Request(rid=i, scene=sc, width=W, height=H, mode=m, keep_result=True))
        assert r.wait(120)
        srv1.stop()
        return r.result

    worst3d = 0.0
    for i, (sc, (W, H), m) in enumerate(specs):
        a, b = mix[i].result, alone(i, sc, W, H, m)
        np.testing.assert_array_equal(a["image"].cpu().numpy(), b["image"].cpu().numpy())
        if m == S.FWD_BWD:
            # the raster gradients are summed with FP32 atomics whose order varies from run to
            # run (also for a request run alone): equal to the rounding of that order
            for k in a["grads2d"]:
                assert rel_l2(a["grads2d"][k].cpu().numpy(), b["grads2d"][k].cpu().numpy()) <= 1e-5, k
            # the projection backward is per-splat and deterministic: the 3D gradients served in
            # the mix are exactly those of the mix's own raster gradients (its chain rule can
            # amplify the rounding above: near-plane splats have conic gradients ~1e7)
            g3 = R.project_backward(*ex.scenes[sc], ex.cameras[(W, H)], ex.cfg, a["grads2d"])
            torch.cuda.synchronize()
            for k in a["grads"]:
                np.testing.assert_array_equal(a["grads"][k].cpu().numpy(), g3[k].cpu().numpy())
                worst3d = max(worst3d, rel_l2(a["grads"][k].cpu().numpy(),
                                              b["grads"][k].cpu().numpy()))
    print("3D gradients, mix vs alone, worst rel-L2", worst3d)
    # the served 3D gradients of a request are the same alone and in the mix within the FP16
    # gradient limit (the requests' framebuffers are FP16)
    assert worst3d <= 1e-2, worst3d
