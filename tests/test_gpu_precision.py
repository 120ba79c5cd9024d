"""The precision sweep at the benchmark view (1M clustered Gaussians, 1600x1064): each framebuffer
format (FP32, FP16, unorm16, BF16) against the FP64 oracle on four 256x256 crops, the centre crop
(672, 404) and three 8-aligned crops drawn with seed 33 (Sec. 3.3, mixed-precision rendering;
Table 4 measures the same formats). Both sides read the oracle's FP64 projection rounded to FP32,
so the error is the raster's: the loss is supported on the crop (dL/dC ~ U[-1, 1] there, zero
elsewhere and at pixels with a borderline oracle decision, R19), and the gradients of all splats
w.r.t. (mean2d, conic, opacity, rgb) are compared per parameter group and over all.

The GPU runs the benchmark's configuration: shared setup, depth-split forward, tile reduction.
Bars: FP32 image 1e-5 max-abs and gradients 1e-4 per group; unorm16 (state rounded at rest) the
mixed-precision limits, image 2e-3 and gradients 1e-2 over all parameters. FP16 at rest meets the
image limit but not the gradient limit on every crop: the backward starts from the stored C
(Procedure 1), whose half-precision rounding (up to 2.4e-4 near 1) is large against c T - C' for
the fragments far behind, and the gradients of the crops measure 1.0e-2 to 1.5e-2 over all
parameters. That is asserted only as a regression guard (3e-2), and stated as a miss. BF16 at
rest is held only to its own storage rounding (half a step, 2^-8 relative: 2e-3 near 1)."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import group_errors, grads9, t

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")

from paper_2505_18764_amd import render as R  # noqa: E402

CROP = 256


def _crops(W, H):
    g = np.random.default_rng(33)
    out = [(672, 404)]
    while len(out) < 4:
        x0 = int(g.integers(0, (W - CROP) // 8 + 1)) * 8
        y0 = int(g.integers(0, (H - CROP) // 8 + 1)) * 8
        if (x0, y0) not in out:
            out.append((x0, y0))
    return out


@pytest.fixture(scope="module")
def view():
    c = synth.CFG3
    sc = synth.scene3d(c["n"], seed=c["seed"])
    cam = synth.camera_front(c["width"], c["height"], c["fx"])
    pre = oracle.preprocess(sc, cam)
    order = oracle.visible_order(pre["keys"])
    cul = np.setdiff1d(np.arange(sc.n), order)
    ids = np.concatenate([order, cul]).astype(np.int32)
    arr = dict(means2d=pre["means2d"].astype(np.float32), conics=pre["conic"].astype(np.float32),
               rgb=pre["rgb"].astype(np.float32), opacities=sc.opacities.astype(np.float32))
    W, H = cam.width, cam.height
    p = R.Projected(means2d=t(arr["means2d"]), conics=t(arr["conics"]), rgb=t(arr["rgb"]),
                    opacities=t(arr["opacities"]), depth=t(np.zeros(sc.n, np.float32)),
                    keys=t(pre["keys"][ids].view(np.int32)), ids=t(ids),
                    n_visible=t(np.array([len(order)], np.int32)), width=W, height=H)
    return dict(arr=arr, order=order, p=p, W=W, H=H)


FORMATS = [(f, r) for r in ("at_rest", "per_fragment") for f in ("f32", "f16", "unorm16", "bf16")]
LIMITS = {"f32": (1e-5, 1e-4), "unorm16": (2e-3, 1e-2)}


@pytest.mark.parametrize("k", range(4))
def test_formats_against_fp64_oracle_on_crops(view, k):
    arr, order, p, W, H = view["arr"], view["order"], view["p"], view["W"], view["H"]
    x0, y0 = _crops(W, H)[k]
    crop = (x0, y0, CROP, CROP)
    ocfg = oracle.OracleConfig(beta=1e-6, beta_abs=4e-6, tau=1e-4)
    ones = np.ones((3, H, W), np.float32)             # runs the backward loop for its T flags
    amb = oracle.raster(arr["means2d"], arr["conics"], arr["opacities"], arr["rgb"], order, W, H,
                        crop=crop, dL_dimg=ones, cfg=ocfg, want_grad=False)["amb"]
    ok = amb == 0
    Gc = synth.image_grad(CROP, CROP, 330 + k)
    Gc[:, ~ok] = 0.0
    G = np.zeros((3, H, W), np.float32)
    G[:, y0:y0 + CROP, x0:x0 + CROP] = Gc
    ref = oracle.raster(arr["means2d"], arr["conics"], arr["opacities"], arr["rgb"], order, W, H,
                        crop=crop, dL_dimg=G, cfg=ocfg)
    print(f"[precision] crop {k} at ({x0}, {y0}): covered/px {ref['cov'].mean():.0f}, "
          f"live/px {ref['live'].mean():.1f}, flagged px {1 - ok.mean():.4f}", flush=True)
    Gd = t(G)
    for fmt, rnd in FORMATS:
        cfg = R.RasterConfig(fb_format=fmt, fb_round=rnd, reduce_mode="tile")
        ws = R.Workspace()
        R.raster_setup(p, cfg, ws)
        f = R.raster_forward(p, cfg, ws, reuse_setup=True)
        b = R.raster_backward(p, f["fb"], Gd, cfg, ws, reuse_setup=True)
        assert R.raster_status(p, cfg, ws) == 0
        torch.cuda.synchronize()
        img = f["image"].cpu().numpy()[:, y0:y0 + CROP, x0:x0 + CROP]
        Tg = f["T"].cpu().numpy()[y0:y0 + CROP, x0:x0 + CROP]
        d_img = float(np.abs(img - ref["img"])[:, ok].max())
        d_T = float(np.abs(Tg - ref["T"])[ok].max())
        e = group_errors(grads9(b), ref["grad"])
        print(f"[precision] crop {k} {fmt}/{rnd}: image max-abs {d_img:.3e}, T max-abs {d_T:.3e}, "
              "grad " + ", ".join(f"{g} {v:.3e}" for g, v in e.items()), flush=True)
        if rnd != "at_rest":
            continue          # reported: per-fragment FP16 and BF16 fail the limits (R20)
        if fmt == "f32":
            assert d_img <= 1e-5 and d_T <= 1e-5 and max(e.values()) <= 1e-4, (d_img, d_T, e)
        elif fmt in LIMITS:
            li, lg = LIMITS[fmt]
            assert d_img <= li and d_T <= li and e["all"] <= lg, (fmt, d_img, d_T, e)
        elif fmt == "f16":      # image limit met; gradient limit missed (see above): guard only
            assert d_img <= 2e-3 and d_T <= 2e-3 and e["all"] <= 3e-2, (d_img, d_T, e)
        else:   # BF16: the error is its storage rounding, at most half a step (2^-8 relative)
            tol = 2.0 ** -8 * np.abs(ref["img"]) + 1e-5
            assert (np.abs(img - ref["img"]) <= tol)[:, ok].all(), d_img
            assert (np.abs(Tg - ref["T"]) <= 2.0 ** -8 * ref["T"] + 1e-5)[ok].all(), d_T
