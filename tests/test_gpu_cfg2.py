"""Parity on the whole 1024x768 image of the 200k-Gaussian clustered scene, element by element:
the ordered path (shared setup, depth-split forward, tile-mode backward, as the benchmark runs it)
in FP32 and FP16, the instrumented forward's per-pixel coverage, and the tile-based comparison
rasterizer. Both sides read the oracle's FP64 projection rounded to FP32."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import group_errors, grads9, t

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")

from paper_2505_18764_amd import render as R  # noqa: E402

TMIN = float(np.float32(1e-4))
BAND = dict(beta=1e-6, beta_abs=4e-6, tau=1e-4)


@pytest.fixture(scope="module")
def scene():
    c = synth.CFG2
    sc = synth.scene3d(c["n"], seed=c["seed"])
    cam = synth.camera_front(c["width"], c["height"], c["fx"])
    W, H = cam.width, cam.height
    pre = oracle.preprocess(sc, cam)
    order = oracle.visible_order(pre["keys"])
    cul = np.setdiff1d(np.arange(sc.n), order)
    ids = np.concatenate([order, cul]).astype(np.int32)
    arr = dict(means2d=pre["means2d"].astype(np.float32), conics=pre["conic"].astype(np.float32),
               rgb=pre["rgb"].astype(np.float32), opacities=sc.opacities.astype(np.float32))
    p = R.Projected(means2d=t(arr["means2d"]), conics=t(arr["conics"]), rgb=t(arr["rgb"]),
                    opacities=t(arr["opacities"]), depth=t(np.zeros(sc.n, np.float32)),
                    keys=t(pre["keys"][ids].view(np.int32)), ids=t(ids),
                    n_visible=t(np.array([len(order)], np.int32)), width=W, height=H)
    ocfg = oracle.OracleConfig(**BAND)
    # dL/dC ~ U[-1, 1], zeroed where the oracle flags a decision the FP32 path could take the
    # other way (including the backward's T tests, hence the pass with dL/dC = 1)
    ones = np.ones((3, H, W), np.float32)
    flags = oracle.raster(arr["means2d"], arr["conics"], arr["opacities"], arr["rgb"], order, W, H,
                          dL_dimg=ones, cfg=ocfg, want_grad=False)["amb"]
    G = synth.image_grad(W, H, c["grad_seed"])
    G[:, flags > 0] = 0.0
    ref = oracle.raster(arr["means2d"], arr["conics"], arr["opacities"], arr["rgb"], order, W, H,
                        dL_dimg=G, cfg=ocfg)
    return dict(arr=arr, order=order, p=p, W=W, H=H, G=G, ref=ref)


@pytest.mark.parametrize("fmt", ["f32", "f16"])
def test_cfg2_whole_image(scene, fmt):
    p, G, ref = scene["p"], scene["G"], scene["ref"]
    cfg = R.RasterConfig(fb_format=fmt, reduce_mode="tile")
    ws = R.Workspace()
    R.raster_setup(p, cfg, ws)
    f = R.raster_forward(p, cfg, ws, reuse_setup=True)
    b = R.raster_backward(p, f["fb"], t(G), cfg, ws, live=True, reuse_setup=True)
    fc = R.raster_forward(p, cfg, ws, coverage=True, reuse_setup=True)
    torch.cuda.synchronize()
    ok = ref["amb"] == 0
    assert ok.mean() > 0.95
    img, T = f["image"].cpu().numpy(), f["T"].cpu().numpy()
    d_img = np.abs(img - ref["img"])[:, ok].max()
    d_T = np.abs(T - ref["T"])[ok].max()
    e = group_errors(grads9(b), ref["grad"])
    print(fmt, "covered/px", ref["cov"].mean(), "image max-abs", d_img, "T", d_T, "grad", e)
    np.testing.assert_array_equal(fc["coverage"].cpu().numpy()[ok], ref["cov"][ok])
    np.testing.assert_array_equal(b["live"].cpu().numpy()[ok], ref["live"][ok])
    if fmt == "f32":
        assert d_img <= 1e-5 and d_T <= 1e-5
        assert e["all"] <= 1e-4, e
    else:
        assert d_img <= 2e-3
        assert e["all"] <= 1e-2, e


def test_cfg2_tile_baseline(scene):
    """The tile-based comparison rasterizer (Sec. 2.1.3-2.1.4) on the same view. It T-culls in
    the forward, so the oracle runs with the same forward threshold."""
    arr, order, p, W, H = scene["arr"], scene["order"], scene["p"], scene["W"], scene["H"]
    ocfg = oracle.OracleConfig(t_min_fwd=TMIN, **BAND)
    ones = np.ones((3, H, W), np.float32)
    flags = oracle.raster(arr["means2d"], arr["conics"], arr["opacities"], arr["rgb"], order, W, H,
                          dL_dimg=ones, cfg=ocfg, want_grad=False)["amb"]
    G = synth.image_grad(W, H, synth.CFG2["grad_seed"])
    G[:, flags > 0] = 0.0
    cfg = R.RasterConfig()
    ws = R.Workspace()
    f = R.tile_forward(p, cfg, ws)
    b = R.tile_backward(p, f, t(G), cfg, ws)
    torch.cuda.synchronize()
    ref = oracle.raster(arr["means2d"], arr["conics"], arr["opacities"], arr["rgb"], order, W, H,
                        dL_dimg=G, cfg=ocfg)
    ok = ref["amb"] == 0
    assert ok.mean() > 0.9
    d = np.abs(f["image"].cpu().numpy() - ref["img"])[:, ok].max()
    e = group_errors(grads9(b), ref["grad"])
    print("tile baseline: pairs", f["n_pairs"], "image max-abs", d, "grad", e)
    assert d <= 1e-5
    assert e["all"] <= 1e-4, e
