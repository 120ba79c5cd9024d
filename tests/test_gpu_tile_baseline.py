"""GPU parity of the tile-based comparison rasterizer (gs_tile_prepare / gs_tile_raster_fwd /
gs_tile_raster_bwd): it computes the oracle's function with forward and backward T-culling at
the same threshold, so it must match the oracle run with t_min_fwd = t_min_bwd, and the main
rasterizer run with forward T-culling."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import check_schedule, group_errors, grads9, rel_l2, t

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2505_18764_amd import render as R  # noqa: E402

TMIN = float(np.float32(1e-4))


def _tile(p, G, cfg):
    ws = R.Workspace()
    f = R.tile_forward(p, cfg, ws)
    b = R.tile_backward(p, f, t(G), cfg, ws)
    torch.cuda.synchronize()
    return f, b


@pytest.mark.parametrize("W,H,n,seed", [(128, 128, 1000, 1), (100, 70, 3000, 2), (17, 33, 200, 3)])
def test_tile_baseline_2d(W, H, n, seed):
    s = synth.splats2d(n=n, width=W, height=H, seed=seed, log_s_mean=np.log(4.0))
    s.opacities[:] = np.clip(s.opacities * 1.5, 0, 0.97).astype(np.float32)
    G = synth.image_grad(W, H, seed + 7)
    cfg = R.RasterConfig()
    p = R.prepare_2d(t(s.means2d), t(s.conics), t(s.opacities), t(s.rgb), t(s.depth), W, H, cfg,
                     R.Workspace())
    f, b = _tile(p, G, cfg)
    ref = oracle.raster(s.means2d, s.conics, s.opacities, s.rgb, oracle.depth_order(s.depth), W, H,
                        dL_dimg=G, cfg=oracle.OracleConfig(t_min_fwd=TMIN, beta=1e-6, beta_abs=4e-6,
                                                           tau=1e-4))
    ok = ref["amb"] == 0
    img = f["image"].cpu().numpy()
    assert np.abs(img - ref["img"])[:, ok].max() <= 1e-5
    assert np.abs(f["T"].cpu().numpy() - ref["T"])[ok].max() <= 1e-5
    e = group_errors(grads9(b), ref["grad"])
    print(W, H, n, "pairs", f["n_pairs"], e)
    assert max(e.values()) <= 1e-4, e
    # the same function as the main path with forward T-culling: its schedules are permutations
    # of the tiles, no kernel met an out-of-range entry, and its per-pixel coverage and live
    # counts are the oracle's at every pixel with no borderline decision
    cfgt = R.RasterConfig(t_min_fwd=TMIN)
    ws = R.Workspace()
    mf = R.raster_forward(p, cfgt, ws, coverage=True)
    mb = R.raster_backward(p, mf["fb"], t(G), cfgt, ws, live=True)
    assert R.raster_status(p, cfgt, ws) == 0
    check_schedule(R, p, cfgt, ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(mf["coverage"].cpu().numpy()[ok], ref["cov"][ok])
    np.testing.assert_array_equal(mb["live"].cpu().numpy()[ok], ref["live"][ok])
    assert np.abs(mf["image"].cpu().numpy() - img)[:, ok].max() <= 2e-5
    gm, gb = grads9(mb), grads9(b)
    e_mb = rel_l2(gm, gb)
    if e_mb > 2e-4:     # name the splats that differ, against the oracle too
        d = np.abs(gm - gb).max(axis=1)
        for i in np.argsort(-d)[:5]:
            print("splat", i, "main", gm[i], "tile", gb[i], "oracle", ref["grad"][i])
        print("main vs oracle", group_errors(gm, ref["grad"]), "tile vs oracle",
              group_errors(gb, ref["grad"]))
    assert e_mb <= 2e-4


def test_tile_baseline_on_projected_scene():
    """Dense clustered scene; both sides read the oracle's projection (rounded to FP32)."""
    sc = synth.scene3d(40_000, seed=8)
    cam = synth.camera_front(256, 192, 900 * 256 / 1024)
    W, H = cam.width, cam.height
    G = synth.image_grad(W, H, 18)
    pre = oracle.preprocess(sc, cam)
    order = oracle.visible_order(pre["keys"])
    cul = np.setdiff1d(np.arange(sc.n), order)
    ids = np.concatenate([order, cul]).astype(np.int32)
    keys = pre["keys"][ids].view(np.int32)
    arr = dict(means2d=pre["means2d"].astype(np.float32), conics=pre["conic"].astype(np.float32),
               rgb=pre["rgb"].astype(np.float32), opacities=sc.opacities.astype(np.float32))
    p = R.Projected(means2d=t(arr["means2d"]), conics=t(arr["conics"]), rgb=t(arr["rgb"]),
                    opacities=t(arr["opacities"]), depth=t(np.zeros(sc.n, np.float32)),
                    keys=t(keys), ids=t(ids), n_visible=t(np.array([len(order)], np.int32)),
                    width=W, height=H)
    cfg = R.RasterConfig()
    f, b = _tile(p, G, cfg)
    ref = oracle.raster(arr["means2d"], arr["conics"], arr["opacities"], arr["rgb"], order, W, H,
                        dL_dimg=G, cfg=oracle.OracleConfig(t_min_fwd=TMIN, beta=1e-6,
                                                           beta_abs=4e-6, tau=1e-4))
    ok = ref["amb"] == 0
    assert ok.mean() > 0.9
    assert np.abs(f["image"].cpu().numpy() - ref["img"])[:, ok].max() <= 1e-5
    e = group_errors(grads9(b), ref["grad"])
    print("pairs", f["n_pairs"], e)
    assert max(e.values()) <= 1e-4, e
    assert f["n_pairs"] > len(order)
