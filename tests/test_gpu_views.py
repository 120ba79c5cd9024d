"""Several views of one scene per launch (the library's view batching, grid y = view): every stage
run over V cameras at once against the same stages run one view at a time (bit-exact where no
atomic is involved), the summed 3D gradients against the FP64 oracle's chain summed over the views,
the batched autograd Function, and the edge cases (no splats, a view that sees nothing, the
largest batch)."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import certain_grad, rel_l2, t

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2505_18764_amd import _lib as L  # noqa: E402
from paper_2505_18764_amd import render as R  # noqa: E402

W, H = 192, 144
FX = 900.0 * W / 1024


def _ring(count, w=W, h=H):
    return [synth.camera_ring(k, count, width=w, height=h, fx=900.0 * w / 1024)
            for k in range(count)]


def _args(sc):
    return [t(sc.means3d), t(sc.scales), t(sc.quats), t(sc.opacities), t(sc.sh)]


G2D = ("means2d", "conics", "opacities", "rgb")
G3D = ("means3d", "scales", "quats", "opacities", "sh")


@pytest.mark.parametrize("fmt,bg", [("f32", (0.0, 0.0, 0.0)), ("f16", (0.25, 0.5, 0.1))])
def test_batched_stages_match_one_view_calls(fmt, bg):
    sc = synth.scene3d(20_000, seed=21)
    cams = _ring(3)
    V = len(cams)
    args = _args(sc)
    cfg = R.RasterConfig(fb_format=fmt, reduce_mode="tile", background=bg)
    G = np.stack([synth.image_grad(W, H, 40 + v) for v in range(V)])
    # batched: shared setup, forward, backward, summed projection backward
    ws = R.Workspace()
    pb = R.project(*args, cams, cfg, ws)
    R.raster_setup(pb, cfg, ws)
    fb = R.raster_forward(pb, cfg, ws, reuse_setup=True)
    bb = R.raster_backward(pb, fb["fb"], t(G), cfg, ws, live=True, reuse_setup=True)
    g3b = R.project_backward(*args, cams, cfg, bb)
    torch.cuda.synchronize()
    print(f"[views] {fmt} n_visible per view", pb.n_visible.tolist(), flush=True)
    assert pb.means2d.shape == (V, sc.n, 2) and fb["image"].shape == (V, 3, H, W)
    bg_sum = np.zeros(3)
    g3s = {k: 0.0 for k in G3D}
    for v in range(V):
        w1 = R.Workspace()
        p = R.project(*args, cams[v], cfg, w1)
        f = R.raster_forward(p, cfg, w1)
        b = R.raster_backward(p, f["fb"], t(G[v]), cfg, w1, live=True)
        torch.cuda.synchronize()
        for k in ("means2d", "conics", "rgb", "depth", "keys", "ids"):
            assert torch.equal(getattr(pb, k)[v], getattr(p, k)), (v, k)
        assert int(pb.n_visible[v]) == int(p.n_visible[0])
        # the forward has no atomics: the same bits
        assert torch.equal(fb["fb"][v], f["fb"]), v
        assert torch.equal(fb["image"][v], f["image"]) and torch.equal(fb["T"][v], f["T"]), v
        assert torch.equal(bb["live"][v], b["live"]), v
        # the backward's FP32 atomics add in a run-dependent order
        for k in G2D:
            e = rel_l2(bb[k][v].cpu().numpy(), b[k].cpu().numpy())
            assert e <= 1e-6, (v, k, e)
        bg_sum += b["background"].cpu().numpy()
        # per-view projection backward from the batched call's own 2D gradients
        g3 = R.project_backward(*args, cams[v], cfg, {k: bb[k][v] for k in G2D})
        for k in G3D:
            g3s[k] = g3s[k] + g3[k].double().cpu().numpy()
    np.testing.assert_allclose(bb["background"].cpu().numpy(), bg_sum, rtol=1e-5, atol=1e-6)
    for k in G3D:
        e = rel_l2(g3b[k].cpu().numpy(), g3s[k])
        print("[views] summed 3D gradient", k, e)
        assert e <= 1e-6, (k, e)


@pytest.mark.parametrize("mode", ["hybrid", "tile"])
def test_batched_chain_against_oracle(mode):
    """GPU projection -> sort -> raster -> projection backward over three views in one call each,
    against the oracle's FP64 chain per view with its complex-step projection backward, summed
    over the views."""
    sc = synth.scene3d(20_000, seed=9)
    cams = _ring(3)
    V = len(cams)
    ocfg = oracle.OracleConfig(beta=1e-5, beta_abs=2e-3, tau=1e-3)
    # dL/dC zero at the pixels with a borderline decision (R19; up to 1.7 % of them here): there
    # the FP32 rounding of the projected means alone flips decisions and moves the mean2d
    # gradients of view 2 by 1.2e-4 (the same with the FP64 projection rounded to FP32)
    G = np.stack([certain_grad(synth.image_grad(W, H, 60 + v),
                               oracle.render_scene(sc, cams[v], cfg=ocfg)["amb"]) for v in range(V)])
    cfg = R.RasterConfig(reduce_mode=mode)
    ws = R.Workspace()
    args = _args(sc)
    p = R.project(*args, cams, cfg, ws)
    f = R.raster_forward(p, cfg, ws)
    b = R.raster_backward(p, f["fb"], t(G), cfg, ws)
    g3 = R.project_backward(*args, cams, cfg, b)
    torch.cuda.synchronize()
    ov = None
    for v in range(V):
        ref = oracle.render_scene(sc, cams[v], dL_dimg=G[v], cfg=ocfg)
        ok = ref["amb"] == 0
        d = np.abs(f["image"][v].cpu().numpy() - ref["img"])[:, ok].max()
        print(f"[views] {mode} view {v} image max-abs (unflagged)", d, "flagged px", (~ok).mean())
        assert d <= 1e-5
        og = ref["grad"]
        r = oracle.preprocess_vjp(sc, cams[v], og[:, 0:2], og[:, 2:5], og[:, 6:9], og[:, 5])
        # this view's share: the projection backward of the batched call's 2D gradients
        gv = R.project_backward(*args, cams[v], cfg, {k: b[k][v] for k in G2D})
        e2 = {k: rel_l2(b[k][v].cpu().numpy(), og[:, s]) for k, s in
              (("means2d", slice(0, 2)), ("conics", slice(2, 5)), ("opacities", 5),
               ("rgb", slice(6, 9)))}
        e3 = {k: rel_l2(gv[k].cpu().numpy(), r[k]) for k in r}
        print(f"[views] {mode} view {v} 2D", e2, "3D", e3)
        ov = r if ov is None else {k: ov[k] + r[k] for k in r}
    errs = {k: rel_l2(g3[k].cpu().numpy(), ov[k]) for k in ov}
    allg = rel_l2(np.concatenate([g3[k].cpu().numpy().reshape(-1) for k in ov]),
                  np.concatenate([ov[k].reshape(-1) for k in ov]))
    print(f"[views] {mode} summed 3D gradient rel-L2", errs, "all", allg)
    assert max(max(errs.values()), allg) <= 1e-4, (errs, allg)


def test_batched_autograd_sums_the_views():
    sc = synth.scene3d(8_000, seed=23)
    cams = _ring(4)
    cfg = R.RasterConfig(fb_format="f16", reduce_mode="tile")
    G = t(np.stack([synth.image_grad(W, H, 70 + v) for v in range(len(cams))]))
    leaves = [x.clone().requires_grad_(True) for x in _args(sc)]
    img, T = R.rasterize_gaussians(*leaves, cams, cfg)
    assert img.shape == (len(cams), 3, H, W) and T.shape == (len(cams), H, W)
    (img * G).sum().backward()
    got = [x.grad.clone() for x in leaves]
    ref = [torch.zeros_like(x) for x in leaves]
    for v, cam in enumerate(cams):
        ls = [x.detach().clone().requires_grad_(True) for x in leaves]
        i1, _ = R.rasterize_gaussians(*ls, cam, cfg)
        assert torch.equal(i1, img[v].detach())
        (i1 * G[v]).sum().backward()
        for r, x in zip(ref, ls):
            r += x.grad
    torch.cuda.synchronize()
    for k, a, b in zip(G3D, got, ref):
        e = rel_l2(a.cpu().numpy(), b.cpu().numpy())
        print("[views] autograd", k, e)
        assert e <= 1e-5, (k, e)


def test_batched_edge_cases():
    cfg = R.RasterConfig(reduce_mode="tile", background=(0.5, 0.25, 1.0))
    # no splats: every view is the background with T = 1 and zero gradients
    sc0 = synth.scene3d(0, seed=1)
    cams = _ring(2)
    ws = R.Workspace()
    args0 = _args(sc0)
    p0 = R.project(*args0, cams, cfg, ws)
    f0 = R.raster_forward(p0, cfg, ws)
    b0 = R.raster_backward(p0, f0["fb"], t(np.ones((2, 3, H, W), np.float32)), cfg, ws)
    torch.cuda.synchronize()
    assert p0.n_visible.tolist() == [0, 0]
    assert (f0["T"] == 1).all()
    for c, val in enumerate((0.5, 0.25, 1.0)):
        assert (f0["image"][:, c] == val).all()
    np.testing.assert_allclose(b0["background"].cpu().numpy(), [2.0 * W * H] * 3, rtol=1e-6)
    # a view that sees nothing between two that do, and the largest batch (16 views)
    sc = synth.scene3d(3_000, seed=5)
    args = _args(sc)
    # outside the scene's shell (radius 5), looking away from it
    away = synth.Camera(viewmat=synth._lookat(np.array([0.0, 0.0, -20.0]),
                                              np.array([0.0, 0.0, -30.0]),
                                              np.array([0.0, 1.0, 0.0])),
                        fx=FX, fy=FX, cx=W / 2.0, cy=H / 2.0, width=W, height=H, znear=0.2)
    ring = _ring(L.MAX_VIEWS)
    batches = {"blind view": [ring[0], away, ring[3]], "16 views": ring}
    for name, cs in batches.items():
        ws = R.Workspace()
        p = R.project(*args, cs, cfg, ws)
        f = R.raster_forward(p, cfg, ws)
        torch.cuda.synchronize()
        print(f"[views] {name}: n_visible", p.n_visible.tolist(), flush=True)
        for v in (0, 1, len(cs) - 1):
            w1 = R.Workspace()
            q = R.project(*args, cs[v], cfg, w1)
            g = R.raster_forward(q, cfg, w1)
            torch.cuda.synchronize()
            assert int(p.n_visible[v]) == int(q.n_visible[0])
            assert torch.equal(f["image"][v], g["image"]) and torch.equal(f["T"][v], g["T"])
        if name == "blind view":
            assert int(p.n_visible[1]) == 0 and (f["T"][1] == 1).all()
    with pytest.raises(ValueError):
        R.project(*args, _ring(L.MAX_VIEWS + 1), cfg, R.Workspace())
