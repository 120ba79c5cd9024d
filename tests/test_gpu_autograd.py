"""The autograd Function against the oracle: its gradients (through the torch activations) agree
with the oracle's chain, with central finite differences of the FP64 oracle on 64 randomly
sampled raw parameters, and a short fit lowers the photometric loss."""
import copy

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import rel_l2, t

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2505_18764_amd import render as R  # noqa: E402
from paper_2505_18764_amd import train as TR  # noqa: E402

TMIN = float(np.float32(1e-4))


def _small(n=2000, seed=41, W=96, H=72):
    sc = synth.scene3d(n, seed=seed, log_scale_mean=-2.5, log_scale_sd=0.5)
    cam = synth.camera_ring(1, 8, width=W, height=H, fx=1125.0 * W / 1280)
    return sc, cam


def _raw(sc):
    o = np.clip(sc.opacities.astype(np.float64), 1e-4, 1 - 1e-4)
    return dict(means3d=sc.means3d.astype(np.float64), log_scales=np.log(sc.scales.astype(np.float64)),
                quats=sc.quats.astype(np.float64), logits=np.log(o / (1 - o)),
                sh=sc.sh.astype(np.float64))


def _scene_from_raw(raw, deg):
    return synth.Scene(means3d=raw["means3d"], scales=np.exp(raw["log_scales"]), quats=raw["quats"],
                       opacities=1 / (1 + np.exp(-raw["logits"])), sh=raw["sh"], sh_degree=deg)


def test_autograd_gradients_match_oracle_chain():
    sc, cam = _small()
    G = synth.image_grad(cam.width, cam.height, 5)
    p = TR.GaussianParams(t(sc.means3d), t(sc.scales), t(sc.quats), t(sc.opacities), t(sc.sh))
    img, T = TR.render(p, cam, R.RasterConfig(), R.Workspace())
    (img * t(G)).sum().backward()
    torch.cuda.synchronize()
    ref = oracle.render_scene(sc, cam, dL_dimg=G,
                              cfg=oracle.OracleConfig(beta=1e-5, beta_abs=2e-3, tau=1e-3))
    og = ref["grad"]
    v = oracle.preprocess_vjp(sc, cam, og[:, 0:2], og[:, 2:5], og[:, 6:9], og[:, 5])
    # chain through the torch activations: d/dlog_s = s * d/ds, d/dlogit = o (1 - o) d/do
    s64, o64 = sc.scales.astype(np.float64), sc.opacities.astype(np.float64)
    exp_ = dict(means=v["means3d"], log_scales=v["scales"] * s64, quats=v["quats"],
                logits=v["opacities"] * o64 * (1 - o64), sh=v["sh"])
    got = dict(means=p.means.grad, log_scales=p.log_scales.grad, quats=p.quats.grad,
               logits=p.logits.grad, sh=p.sh.grad)
    errs = {k: rel_l2(got[k].cpu().numpy(), exp_[k]) for k in exp_}
    print(errs)
    assert max(errs.values()) <= 1e-4, errs           # the FP32 gradient contract, per group
    assert T.requires_grad          # a loss on T reaches the splats through dL/dT_final


def test_finite_differences_on_64_parameters():
    """Central differences of the FP64 oracle (loss = mean squared error against a target
    rendered from a hidden scene) on 64 seeded raw parameters, forward and backward T-culling at
    the same threshold so that the analytic gradient is the exact derivative."""
    sc, cam = _small(seed=41)
    hidden, _ = _small(seed=40)
    W, H = cam.width, cam.height
    ocfg = oracle.OracleConfig(t_min_fwd=TMIN)
    target = oracle.render_scene(hidden, cam, cfg=ocfg)["img"]
    raw = _raw(sc)
    deg = sc.sh_degree

    def oracle_loss(r):
        out = oracle.render_scene(_scene_from_raw(r, deg), cam, cfg=ocfg)
        return float(np.mean((out["img"] - target) ** 2)), out

    # GPU analytic gradient through the autograd Function
    cfg = R.RasterConfig(t_min_fwd=TMIN)
    p = TR.GaussianParams(t(sc.means3d), t(sc.scales), t(sc.quats), t(sc.opacities), t(sc.sh))
    img, _ = TR.render(p, cam, cfg, R.Workspace())
    loss = torch.mean((img - t(target.astype(np.float32))) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    grads = dict(means3d=p.means.grad.cpu().numpy(), log_scales=p.log_scales.grad.cpu().numpy(),
                 quats=p.quats.grad.cpu().numpy(), logits=p.logits.grad.cpu().numpy(),
                 sh=p.sh.grad.cpu().numpy())
    base_l, base = oracle_loss(raw)
    vis = np.flatnonzero(base["pre"]["visible"])
    g = np.random.default_rng(synth.CFG4["fd_seed"])
    names = ["means3d", "log_scales", "quats", "logits", "sh"]
    fd, an = [], []
    tries = 0
    while len(fd) < 64 and tries < 400:
        tries += 1
        nm = names[g.integers(0, len(names))]
        i = int(vis[g.integers(0, len(vis))])
        comp = tuple(int(g.integers(0, d)) for d in raw[nm].shape[1:])
        idx = (i,) + comp
        th = raw[nm][idx]
        h = 1e-6 * max(1.0, abs(th))
        vals, outs = [], []
        for sgn in (1, -1):
            r2 = copy.deepcopy(raw)
            r2[nm][idx] = th + sgn * h
            l, o = oracle_loss(r2)
            vals.append(l)
            outs.append(o)
        if any((o["cov"] != base["cov"]).any() or (o["pre"]["visible"] != base["pre"]["visible"]).any()
               for o in outs):
            continue                                   # a discrete decision flipped: resample
        d = (vals[0] - vals[1]) / (2 * h)
        if abs(d) < 1e-12 and abs(grads[nm][idx]) < 1e-12:
            continue                                   # parameter without influence
        fd.append(d)
        an.append(float(grads[nm][idx]))
    fd, an = np.array(fd), np.array(an)
    err = rel_l2(an, fd)
    print("FD samples", len(fd), "rel-L2", err)
    assert len(fd) == 64
    assert err <= 1e-4, err                           # GPU vs FD on the FP64 oracle (R21)


@pytest.mark.parametrize("views_per_step", [1, 4])
def test_short_fit_lowers_loss(views_per_step):
    c = synth.CFG4
    W, H = 160, 90
    cams = [synth.camera_ring(k, 8, width=W, height=H, fx=c["fx"] * W / c["width"]) for k in range(8)]
    hidden = synth.scene3d(20_000, seed=c["seed_hidden"])
    init = synth.scene3d(20_000, seed=c["seed_train"])
    cfg = R.RasterConfig(fb_format="f16", reduce_mode="hybrid_lane")
    ws = R.Workspace()
    with torch.no_grad():
        targets = [R.rasterize_gaussians(t(hidden.means3d), t(hidden.scales), t(hidden.quats),
                                         t(hidden.opacities), t(hidden.sh), cam, cfg, ws)[0].clone()
                   for cam in cams]
    p = TR.GaussianParams(t(init.means3d), t(init.scales), t(init.quats), t(init.opacities),
                          t(init.sh))
    hist = TR.fit(p, cams, targets, steps=80 if views_per_step == 1 else 40, lr=1e-2, cfg=cfg,
                  log_every=8 if views_per_step == 1 else 4, views_per_step=views_per_step)
    first = np.mean([l for _, l in hist[:2]])
    last = np.mean([l for _, l in hist[-2:]])
    print(hist)
    assert last < 0.7 * first
