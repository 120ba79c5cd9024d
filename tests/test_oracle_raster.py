"""Pins for the oracle's compositing and gradient procedure (CPU only).

Each test checks the oracle against something other than its own code: closed forms of special
configurations, a mass integral, central finite differences of its forward, the paper's sum form
of dL/dalpha (Eq. 4) against its recurrence form (Eq. 7), library rounding routines, and brute
force against the prefiltered mode. A plausible slip in the oracle (a dropped term, a sign, a
swapped index or operand) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def _cfg(**kw):
    return oracle.OracleConfig(**kw)


def test_constants_match_paper():
    g = json.load(open(GOLD))
    c = oracle.OracleConfig()
    assert c.alpha_min == pytest.approx(g["alpha_min"]["value"], rel=1e-7)
    assert c.t_min_bwd == pytest.approx(g["t_min_bwd"]["value"], rel=1e-7)
    assert c.t_min_fwd == 0.0   # hardware blending in the paper's forward cannot T-cull (Sec. 2.1.4)


# ---- closed forms -------------------------------------------------------------------------

def _slabs(opac, rgb, n_extra=0):
    """Splats with a zero conic: q = 0, so alpha = o at every pixel (a uniform slab)."""
    k = len(opac)
    return dict(means2d=np.zeros((k, 2)), conics=np.zeros((k, 3)),
                opacities=np.asarray(opac, float), rgb=np.asarray(rgb, float))


@pytest.mark.parametrize("K,o", [(1, 0.3), (5, 0.3), (17, 0.45), (40, 0.2)])
def test_identical_slabs_geometric_series(K, o):
    c = np.array([0.2, 0.5, 0.9])
    s = _slabs([o] * K, [c] * K)
    out = oracle.raster(**s, order=np.arange(K), width=4, height=3,
                        cfg=_cfg(prefilter=False, t_min_bwd=0.0))
    Tk = (1.0 - o) ** K
    np.testing.assert_allclose(out["img"][:, 0, 0], c * (1.0 - Tk), rtol=1e-13)
    np.testing.assert_allclose(out["T"], Tk, rtol=1e-13)
    assert (out["cov"] == K).all()


@pytest.mark.parametrize("o", [0.3, 0.5, 0.77])
def test_tcull_live_count_is_exact(o):
    """Fragment i (1-based) is live iff (1-o)^(i-1) >= 1e-4 (Procedure 1 T-Culling)."""
    K = 80
    t = float(np.float32(1e-4))
    expect = sum(1 for i in range(1, K + 1) if (1.0 - o) ** (i - 1) >= t)
    # keep away from the threshold so no decision is borderline
    assert min(abs((1.0 - o) ** (i - 1) / t - 1.0) for i in range(1, K + 1)) > 1e-3
    s = _slabs([o] * K, [[0.5, 0.5, 0.5]] * K)
    G = np.ones((3, 2, 2))
    out = oracle.raster(**s, order=np.arange(K), width=2, height=2, dL_dimg=G,
                        cfg=_cfg(prefilter=False))
    assert (out["live"] == expect).all()
    assert (out["cov"] == K).all()                      # paper mode: no forward T-culling
    out2 = oracle.raster(**s, order=np.arange(K), width=2, height=2, dL_dimg=G,
                         cfg=_cfg(prefilter=False, t_min_fwd=t))
    assert (out2["cov"] == expect).all()


def test_two_slab_derivatives():
    """C = o1 c1 + (1 - o1) o2 c2, so dC/do1 = c1 - o2 c2, dC/do2 = (1 - o1) c2,
    dC/dc1 = o1, dC/dc2 = (1 - o1) o2 (derived by hand from Eq. 2 for two splats)."""
    o1, o2 = 0.35, 0.6
    c1, c2 = np.array([0.9, 0.1, 0.4]), np.array([0.2, 0.8, 0.6])
    G = np.array([0.7, -1.3, 0.25])
    s = _slabs([o1, o2], [c1, c2])
    Gimg = np.broadcast_to(G[:, None, None], (3, 1, 1)).copy()
    out = oracle.raster(**s, order=np.arange(2), width=1, height=1, dL_dimg=Gimg,
                        cfg=_cfg(prefilter=False, t_min_bwd=0.0))
    g = out["grad"]
    np.testing.assert_allclose(g[0, 5], G @ (c1 - o2 * c2), rtol=1e-13)
    np.testing.assert_allclose(g[1, 5], G @ ((1 - o1) * c2), rtol=1e-13)
    np.testing.assert_allclose(g[0, 6:9], G * o1, rtol=1e-13)
    np.testing.assert_allclose(g[1, 6:9], G * (1 - o1) * o2, rtol=1e-13)
    # the order matters: swapping the splats swaps the roles
    out2 = oracle.raster(**s, order=np.array([1, 0]), width=1, height=1, dL_dimg=Gimg,
                         cfg=_cfg(prefilter=False, t_min_bwd=0.0))
    np.testing.assert_allclose(out2["grad"][1, 5], G @ (c2 - o1 * c1), rtol=1e-13)


def test_slab_conic_gradient_closed_form():
    """One slab seen at pixel offset d: dalpha/da = -alpha dx^2 / 2 at a = b = c = 0."""
    o, c = 0.4, np.array([0.3, 0.6, 0.9])
    s = dict(means2d=np.array([[1.25, 2.0]]), conics=np.zeros((1, 3)),
             opacities=np.array([o]), rgb=c[None])
    G = np.zeros((3, 4, 4))
    G[:, 3, 2] = [1.0, 2.0, -0.5]          # one pixel: centre (2.5, 3.5)
    out = oracle.raster(**s, order=np.array([0]), width=4, height=4, dL_dimg=G,
                        cfg=_cfg(prefilter=False, t_min_bwd=0.0))
    dx, dy = 2.5 - 1.25, 3.5 - 2.0
    dC_dalpha = c                          # C = alpha c
    dL_dalpha = G[:, 3, 2] @ dC_dalpha
    g = out["grad"][0]
    np.testing.assert_allclose(g[2], dL_dalpha * (-0.5 * o * dx * dx), rtol=1e-13)
    np.testing.assert_allclose(g[3], dL_dalpha * (-0.5 * o * 2 * dx * dy), rtol=1e-13)
    np.testing.assert_allclose(g[4], dL_dalpha * (-0.5 * o * dy * dy), rtol=1e-13)
    np.testing.assert_allclose(g[0:2], 0.0, atol=1e-15)   # q does not depend on mu at Q = 0


def test_mass_integral_and_coverage_area():
    """For one splat with o <= alpha_max: sum over pixels of alpha -> 2 pi sqrt(det S)(o - a_min)
    and the number of covered pixels -> 2 pi ln(o / a_min) sqrt(det S) (integral of o exp(-q/2)
    over the ellipse q <= 2 ln(o / a_min); lattice error only)."""
    W = H = 400
    th = 0.6
    s1, s2 = 41.0, 23.0
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    S = R @ np.diag([s1 * s1, s2 * s2]) @ R.T
    Q = np.linalg.inv(S)
    o = 0.8
    amin = oracle.OracleConfig().alpha_min
    s = dict(means2d=np.array([[200.3, 199.6]]), conics=np.array([[Q[0, 0], Q[0, 1], Q[1, 1]]]),
             opacities=np.array([o]), rgb=np.array([[1.0, 0.0, 0.0]]))
    out = oracle.raster(**s, order=np.array([0]), width=W, height=H)
    sq = math.sqrt(np.linalg.det(S))
    mass = out["img"][0].sum()
    np.testing.assert_allclose(mass, 2 * math.pi * sq * (o - amin), rtol=2e-4)
    area = out["cov"].sum()
    np.testing.assert_allclose(area, 2 * math.pi * math.log(o / amin) * sq, rtol=5e-3)
    np.testing.assert_allclose(1.0 - out["T"], out["img"][0], rtol=1e-12)


# ---- the paper's two forms of dL/dalpha and the T recurrence --------------------------------

def test_dLdalpha_sum_form_equals_recurrence():
    """Eq. 4 (sum over later fragments) equals Eq. 7 (C' recurrence, Eq. 6) at every fragment,
    and T_i equals the product of (1 - alpha_k) over earlier fragments (Eq. 2)."""
    s = synth.splats2d(n=300, width=32, height=32, seed=9)
    order = oracle.depth_order(s.depth)
    G = np.array([0.3, -0.8, 1.1])
    for (px, py) in [(16.5, 16.5), (3.5, 28.5), (30.5, 1.5)]:
        tr, C = oracle.pixel_trace(s.means2d, s.conics, s.opacities, s.rgb, order, px, py, G,
                                   cfg=_cfg(t_min_bwd=0.0))
        assert len(tr) > 5
        alpha = tr[:, 1]
        T = np.concatenate([[1.0], np.cumprod(1.0 - alpha)[:-1]])
        np.testing.assert_allclose(tr[:, 2], T, rtol=1e-12)
        col = s.rgb[order[tr[:, 0].astype(int)]].astype(np.float64)
        contrib = (T * alpha)[:, None] * col
        np.testing.assert_allclose(contrib.sum(0), C, rtol=1e-12)
        for i in range(len(tr)):
            later = contrib[i + 1:].sum(0)
            eq4 = G @ (col[i] * T[i] - later / (1.0 - alpha[i]))
            np.testing.assert_allclose(tr[i, 6], eq4, rtol=1e-9, atol=1e-12)


# ---- central finite differences of the forward ----------------------------------------------

def _loss(s, order, W, H, G, cfg):
    out = oracle.raster(**s, order=order, width=W, height=H, cfg=cfg)
    return float(np.sum(G * out["img"])), out


def _fd_check(s, order, W, H, G, cfg, n_params=None, seed=0):
    base = oracle.raster(**s, order=order, width=W, height=H, dL_dimg=G, cfg=cfg)
    g = base["grad"]
    keys = [("means2d", 0), ("means2d", 1), ("conics", 0), ("conics", 1), ("conics", 2),
            ("opacities", None), ("rgb", 0), ("rgb", 1), ("rgb", 2)]
    n = s["opacities"].shape[0]
    checked = 0
    errs = []
    rng = np.random.default_rng(seed)
    idx = rng.permutation(n) if n_params is None else rng.choice(n, n_params, replace=False)
    for i in idx:
        for j, (name, comp) in enumerate(keys):
            th = s[name][i] if comp is None else s[name][i, comp]
            h = 1e-6 * max(1.0, abs(th))
            vals, outs = [], []
            for sign in (+1, -1):
                s2 = {k: v.copy() for k, v in s.items()}
                if comp is None:
                    s2[name][i] = th + sign * h
                else:
                    s2[name][i, comp] = th + sign * h
                L, o = _loss(s2, order, W, H, G, cfg)
                bwd = oracle.raster(**s2, order=order, width=W, height=H, dL_dimg=G, cfg=cfg,
                                    want_grad=False)
                vals.append(L)
                outs.append(bwd)
            # skip parameters whose perturbation flips a discrete decision
            if any((o["cov"] != base["cov"]).any() or (o["live"] != base["live"]).any()
                   for o in outs):
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            errs.append((fd, g[i, j]))
            checked += 1
    fd = np.array([e[0] for e in errs])
    an = np.array([e[1] for e in errs])
    return checked, fd, an


@pytest.mark.parametrize("tcull", [False, True])
def test_fd_matches_backward(tcull):
    """With t_min_fwd == t_min_bwd the backward procedure is the exact gradient of the forward;
    central differences in FP64 must agree to ~1e-7 relative."""
    g = np.random.default_rng(5)
    n = 14 if not tcull else 40
    W = H = 20
    means = g.uniform(4, 16, size=(n, 2))
    th = g.uniform(0, np.pi, n)
    sc = g.uniform(2.5, 5.0, size=(n, 2))
    conics = []
    for k in range(n):
        R = np.array([[np.cos(th[k]), -np.sin(th[k])], [np.sin(th[k]), np.cos(th[k])]])
        Q = np.linalg.inv(R @ np.diag(sc[k] ** 2) @ R.T)
        conics.append([Q[0, 0], Q[0, 1], Q[1, 1]])
    opac = g.uniform(0.5, 0.9, n) if tcull else g.uniform(0.2, 0.9, n)
    s = dict(means2d=means, conics=np.array(conics), opacities=opac, rgb=g.uniform(0, 1, (n, 3)))
    order = np.argsort(g.uniform(size=n)).astype(np.int32)
    G = g.uniform(-1, 1, size=(3, H, W))
    t = float(np.float32(1e-4)) if tcull else 0.0
    cfg = _cfg(t_min_fwd=t, t_min_bwd=t)
    if tcull:
        base = oracle.raster(**s, order=order, width=W, height=H, dL_dimg=G, cfg=cfg)
        assert (base["live"] < base["cov"]).any() or (base["T"] < 1e-3).any()
    checked, fd, an = _fd_check(s, order, W, H, G, cfg, n_params=None if not tcull else 10)
    assert checked >= 60
    scale = np.linalg.norm(an)
    assert np.abs(fd - an).max() <= 1e-6 * scale, (np.abs(fd - an).max(), scale)


def test_tcull_makes_backward_differ_from_forward_gradient():
    """Paper mode: the forward does not T-cull but Procedure 1 does, so the backward drops the
    gradients of fragments behind T < 1e-4 (Sec. 3.1.3); without the backward T-cull it is exact."""
    K = 30
    s = _slabs([0.5] * K, [[0.5, 0.4, 0.3]] * K)
    G = np.ones((3, 1, 1))
    g_cull = oracle.raster(**s, order=np.arange(K), width=1, height=1, dL_dimg=G,
                           cfg=_cfg(prefilter=False))["grad"]
    g_full = oracle.raster(**s, order=np.arange(K), width=1, height=1, dL_dimg=G,
                           cfg=_cfg(prefilter=False, t_min_bwd=0.0))["grad"]
    live = sum(1 for i in range(1, K + 1) if 0.5 ** (i - 1) >= float(np.float32(1e-4)))
    assert (g_cull[live:] == 0).all() and (g_full[live:, 5:] != 0).all()
    np.testing.assert_allclose(g_cull[:live, 6:], g_full[:live, 6:], rtol=1e-13)


# ---- prefilter vs brute force ----------------------------------------------------------------

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_prefilter_equals_brute_force(seed):
    s = synth.splats2d(n=400, width=48, height=40, seed=seed)
    order = oracle.depth_order(s.depth)
    G = synth.image_grad(48, 40, seed + 10)
    kw = dict(means2d=s.means2d, conics=s.conics, opacities=s.opacities, rgb=s.rgb, order=order,
              width=48, height=40, dL_dimg=G)
    a = oracle.raster(**kw, cfg=_cfg(prefilter=True))
    b = oracle.raster(**kw, cfg=_cfg(prefilter=False))
    for k in ("img", "T", "cov", "live", "amb"):
        np.testing.assert_array_equal(a[k], b[k])
    np.testing.assert_allclose(a["grad"], b["grad"], rtol=1e-11, atol=1e-13)
    # a crop equals the same window of the full frame, and its gradient only sees the crop
    c = oracle.raster(**kw, crop=(8, 5, 20, 17), cfg=_cfg(prefilter=True))
    np.testing.assert_array_equal(c["img"], a["img"][:, 5:22, 8:28])
    Gc = np.zeros_like(G)
    Gc[:, 5:22, 8:28] = G[:, 5:22, 8:28]
    d = oracle.raster(**{**kw, "dL_dimg": Gc}, cfg=_cfg(prefilter=True))
    np.testing.assert_allclose(c["grad"], d["grad"], rtol=1e-11, atol=1e-13)


# ---- format rounding -------------------------------------------------------------------------

def _values(seed=0, n=200000):
    g = np.random.default_rng(seed)
    v = np.concatenate([
        g.uniform(-1, 1, n), g.uniform(0, 2, n) * 10.0 ** g.integers(-9, 5, n),
        g.normal(size=n) * 1e-5, np.array([0.0, -0.0, 1.0, 65504.0, 65519.99, 65520.0, 7e4,
                                           2 ** -24, 2 ** -25, 3 * 2 ** -26, 2 ** -14])])
    return v


def test_round_f16_matches_numpy():
    v = _values()
    # exact ties between fp16 neighbours, both in the normal and the subnormal range
    ties = (np.arange(1, 2000) + 0.5) * 2.0 ** -10
    sub = (np.arange(1, 500) + 0.5) * 2.0 ** -24
    v = np.concatenate([v, ties, -ties, sub])
    np.testing.assert_array_equal(oracle.round_fmt(v, "f16"), v.astype(np.float16).astype(np.float64))


def test_round_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    v = _values(1).astype(np.float32)          # fp32-exact inputs: torch rounds fp32 -> bf16
    ties = ((np.arange(1, 3000) + 0.5) * 2.0 ** -7).astype(np.float32)
    v = np.concatenate([v, ties, -ties])
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.round_fmt(v.astype(np.float64), "bf16"), ref)


def test_round_unorm_and_f32():
    v = _values(2)
    for fmt, lv in (("unorm16", 65535.0), ("unorm8", 255.0)):
        ref = np.rint(np.clip(v, 0.0, 1.0) * lv) / lv      # numpy rint: ties to even
        np.testing.assert_array_equal(oracle.round_fmt(v, fmt), ref)
    np.testing.assert_array_equal(oracle.round_fmt(v, "f32"), v.astype(np.float32).astype(np.float64))


def test_emulation_rounds_stored_state():
    s = synth.splats2d(n=300, width=32, height=32, seed=4)
    order = oracle.depth_order(s.depth)
    kw = dict(means2d=s.means2d, conics=s.conics, opacities=s.opacities, rgb=s.rgb, order=order,
              width=32, height=32)
    ref = oracle.raster(**kw)
    rest = oracle.raster(**kw, cfg=_cfg(fb_format="f16", emulate=True, fb_round="at_rest"))
    np.testing.assert_array_equal(rest["img"], oracle.round_fmt(ref["img"], "f16"))
    f32 = oracle.raster(**kw, cfg=_cfg(fb_format="f32", emulate=True, fb_round="per_fragment"))
    assert np.abs(f32["img"] - ref["img"]).max() < 1e-6
    pf = oracle.raster(**kw, cfg=_cfg(fb_format="f16", emulate=True, fb_round="per_fragment"))
    d = np.abs(pf["img"] - ref["img"]).max()
    assert 1e-4 < d < 5e-2
    np.testing.assert_array_equal(pf["img"], oracle.round_fmt(pf["img"], "f16"))


def test_unorm_saturates_colour():
    s = _slabs([0.5], [[1.7, 0.5, -0.0]])
    G = np.ones((3, 1, 1))
    a = oracle.raster(**s, order=np.arange(1), width=1, height=1, dL_dimg=G,
                      cfg=_cfg(prefilter=False, fb_format="unorm16"))
    np.testing.assert_allclose(a["img"][:, 0, 0], [0.5, 0.25, 0.0], atol=1e-15)
    assert a["grad"][0, 6] == 0.0 and a["grad"][0, 7] == pytest.approx(0.5)


# ---- background colour and the gradient of the final transmittance --------------------------

def test_background_one_and_two_slabs_closed_form():
    """With a background bg behind the splats, Eq. 2 becomes C = sum_i T_i alpha_i c_i + T bg with
    T = prod_i (1 - alpha_i). For one slab: C = o c + (1 - o) bg, dC/do = c - bg, dT/do = -1,
    dC/dbg = 1 - o. For two: dC/do1 = c1 - o2 c2 - (1 - o2) bg, dC/do2 = (1 - o1) (c2 - bg),
    dT/do1 = -(1 - o2), dT/do2 = -(1 - o1). L = G.C + gT T (derived by hand)."""
    bg = np.array([0.15, 0.55, 0.8])
    G, gT = np.array([0.7, -1.3, 0.25]), -0.45
    Gimg = np.broadcast_to(G[:, None, None], (3, 1, 1)).copy()
    GT = np.full((1, 1), gT)
    cfg = _cfg(prefilter=False, t_min_bwd=0.0, background=tuple(bg))
    o, c = 0.35, np.array([0.9, 0.1, 0.4])
    out = oracle.raster(**_slabs([o], [c]), order=np.arange(1), width=1, height=1, dL_dimg=Gimg,
                        dL_dT=GT, cfg=cfg)
    np.testing.assert_allclose(out["img"][:, 0, 0], o * c + (1 - o) * bg, rtol=1e-14)
    np.testing.assert_allclose(out["T"][0, 0], 1 - o, rtol=1e-14)
    np.testing.assert_allclose(out["grad"][0, 5], G @ (c - bg) - gT, rtol=1e-13)
    np.testing.assert_allclose(out["grad_bg"], G * (1 - o), rtol=1e-14)
    o1, o2 = 0.35, 0.6
    c1, c2 = np.array([0.9, 0.1, 0.4]), np.array([0.2, 0.8, 0.6])
    out = oracle.raster(**_slabs([o1, o2], [c1, c2]), order=np.arange(2), width=1, height=1,
                        dL_dimg=Gimg, dL_dT=GT, cfg=cfg)
    np.testing.assert_allclose(out["grad"][0, 5], G @ (c1 - o2 * c2 - (1 - o2) * bg) - gT * (1 - o2),
                               rtol=1e-13)
    np.testing.assert_allclose(out["grad"][1, 5], G @ ((1 - o1) * (c2 - bg)) - gT * (1 - o1),
                               rtol=1e-13)
    np.testing.assert_allclose(out["grad"][1, 6:9], G * (1 - o1) * o2, rtol=1e-13)
    np.testing.assert_allclose(out["grad_bg"], G * (1 - o1) * (1 - o2), rtol=1e-14)


def test_background_and_dLdT_finite_differences():
    """L = sum_p G_p . C_p + gT_p T_p with a background: central differences of the FP64 forward
    against the backward for every parameter of a few splats and for the background."""
    g = np.random.default_rng(9)
    n, W, H = 10, 16, 14
    means = g.uniform(3, 13, size=(n, 2))
    conics = []
    for k in range(n):
        t = g.uniform(0, np.pi)
        R = np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
        Q = np.linalg.inv(R @ np.diag(g.uniform(2.0, 4.0, 2) ** 2) @ R.T)
        conics.append([Q[0, 0], Q[0, 1], Q[1, 1]])
    s = dict(means2d=means, conics=np.array(conics), opacities=g.uniform(0.2, 0.8, n),
             rgb=g.uniform(0, 1, (n, 3)))
    order = np.argsort(g.uniform(size=n)).astype(np.int32)
    G = g.uniform(-1, 1, size=(3, H, W))
    GT = g.uniform(-1, 1, size=(H, W))
    bg = np.array([0.3, 0.6, 0.2])

    def loss(s_, bg_):
        o = oracle.raster(**s_, order=order, width=W, height=H,
                          cfg=_cfg(t_min_bwd=0.0, background=tuple(bg_)))
        return float((G * o["img"]).sum() + (GT * o["T"]).sum()), o

    base = oracle.raster(**s, order=order, width=W, height=H, dL_dimg=G, dL_dT=GT,
                         cfg=_cfg(t_min_bwd=0.0, background=tuple(bg)))
    _, b0 = loss(s, bg)
    h = 1e-6
    fd, an = [], []
    # (input array, column, gradient column: mean x, y, conic a, b, c, opacity, rgb r, g, b)
    for key, col, gcol in (("opacities", None, 5), ("means2d", 0, 0), ("means2d", 1, 1),
                           ("conics", 0, 2), ("conics", 1, 3), ("conics", 2, 4), ("rgb", 0, 6)):
        for i in range(n):
            vals = []
            for sgn in (1, -1):
                s2 = {k: v.copy() for k, v in s.items()}
                if s2[key].ndim == 1:
                    s2[key][i] += sgn * h
                else:
                    s2[key][i, col] += sgn * h
                l, o = loss(s2, bg)
                if (o["cov"] != b0["cov"]).any():
                    break
                vals.append(l)
            if len(vals) == 2:
                fd.append((vals[0] - vals[1]) / (2 * h))
                an.append(base["grad"][i, gcol])
    for ch in range(3):
        bp, bm = bg.copy(), bg.copy()
        bp[ch] += h
        bm[ch] -= h
        fd.append((loss(s, bp)[0] - loss(s, bm)[0]) / (2 * h))
        an.append(base["grad_bg"][ch])
    fd, an = np.array(fd), np.array(an)
    assert len(fd) >= 50
    assert np.abs(fd - an).max() <= 1e-6 * np.linalg.norm(an), (np.abs(fd - an).max(), np.linalg.norm(an))


# ---- per-fragment format emulation, by hand -------------------------------------------------
# A render target that blends in its own format rounds the stored state after every fragment
# (Sec. 3.3). For uniform slabs (zero conic, alpha = o at every pixel) the whole computation of
# one pixel is written out below in numpy, store by store, in the order of Eq. 2 / Eq. 5 for the
# forward and Procedure 1 (Eqs. 3, 7, then the Eqs. 6 and 5 stores) for the backward, with the
# format's rounding taken from numpy (float16) or the unorm definition. Rounding placed before
# the C' update, or applied to C' but not to T, or skipped at the backward's stores, gives other
# numbers; the test checks that each such variant differs from the oracle.

def _round_np(x, fmt):
    if fmt == "f16":
        return float(np.float16(x))                      # numpy rounds double -> half (RNE)
    if fmt == "unorm16":
        return float(np.rint(min(max(x, 0.0), 1.0) * 65535.0) / 65535.0)
    raise ValueError(fmt)


def _slab_pixel_by_hand(ops, cols, G, fmt, t_min_bwd=0.0, variant=None):
    """Image, T, dL/dalpha and dL/dc of one pixel over uniform slabs, per-fragment rounding."""
    rnd = lambda x: _round_np(x, fmt)
    C, T = [0.0, 0.0, 0.0], 1.0
    for o, c in zip(ops, cols):
        C = [rnd(C[ch] + T * o * c[ch]) for ch in range(3)]          # C += T alpha c, stored
        T = rnd(T * (1.0 - o))                                        # T (1 - alpha), stored
    C = [rnd(x) for x in C]                                           # written back at rest
    ga, gc = [], []
    Cp, Tb = list(C), 1.0                                             # (C'_1, T_1) = (C, 1)
    for o, c in zip(ops, cols):
        if Tb < t_min_bwd:                                            # T-culled: state frozen
            ga.append(0.0)
            gc.append([0.0, 0.0, 0.0])
            continue
        gc.append([G[ch] * o * Tb for ch in range(3)])                # Eq. 3
        s = 0.0
        if variant == "round_before_update":
            Cp = [rnd(x) for x in Cp]
        for ch in range(3):
            s += G[ch] * (c[ch] * Tb - Cp[ch])                        # Eq. 7 numerator
        ga.append(s / (1.0 - o))
        if variant == "no_backward_rounding":
            Cp = [Cp[ch] - Tb * o * c[ch] for ch in range(3)]
            Tb = Tb * (1.0 - o)
        elif variant == "no_T_rounding":
            Cp = [rnd(Cp[ch] - Tb * o * c[ch]) for ch in range(3)]
            Tb = Tb * (1.0 - o)
        elif variant == "round_before_update":
            Cp = [Cp[ch] - Tb * o * c[ch] for ch in range(3)]
            Tb = Tb * (1.0 - o)
        else:
            Cp = [rnd(Cp[ch] - Tb * o * c[ch]) for ch in range(3)]   # Eq. 6, stored
            Tb = rnd(Tb * (1.0 - o))                                  # Eq. 5, stored
    return np.array(C), T, np.array(ga), np.array(gc)


_SLAB_CASES = {
    "one": ([0.37], [[0.8173, 0.2291, 0.5519]]),
    "two": ([0.37, 0.61], [[0.8173, 0.2291, 0.5519], [0.1367, 0.9042, 0.4433]]),
    "five": ([0.37, 0.61, 0.23, 0.52, 0.44],
             [[0.8173, 0.2291, 0.5519], [0.1367, 0.9042, 0.4433], [0.6711, 0.3105, 0.0917],
              [0.2468, 0.7531, 0.9876], [0.5050, 0.4049, 0.3048]]),
}


@pytest.mark.parametrize("fmt", ["f16", "unorm16"])
@pytest.mark.parametrize("case", list(_SLAB_CASES))
def test_per_fragment_emulation_by_hand(fmt, case):
    ops, cols = _SLAB_CASES[case]
    K = len(ops)
    G = np.array([0.7, -1.3, 0.25])
    Gimg = np.broadcast_to(G[:, None, None], (3, 1, 1)).copy()
    cfg = _cfg(prefilter=False, t_min_bwd=0.0, fb_format=fmt, emulate=True,
               fb_round="per_fragment")
    out = oracle.raster(**_slabs(ops, cols), order=np.arange(K), width=1, height=1,
                        dL_dimg=Gimg, cfg=cfg)
    C, T, ga, gc = _slab_pixel_by_hand(ops, cols, G, fmt)
    np.testing.assert_array_equal(out["img"][:, 0, 0], C)
    assert out["T"][0, 0] == T
    # opacity gradient = dL/dalpha (exp(-q/2) = 1 on a slab); colour gradient = Eq. 3
    np.testing.assert_allclose(out["grad"][:, 5], ga, rtol=1e-15, atol=0)
    np.testing.assert_allclose(out["grad"][:, 6:9], gc, rtol=1e-15, atol=0)
    # the rounding is really there: the plain FP64 result differs by about a format step
    plain = oracle.raster(**_slabs(ops, cols), order=np.arange(K), width=1, height=1,
                          dL_dimg=Gimg, cfg=_cfg(prefilter=False, t_min_bwd=0.0))
    assert np.abs(plain["img"][:, 0, 0] - C).max() > 0
    # every misplaced rounding gives other numbers, so the comparison above would catch it
    for v in ("round_before_update", "no_T_rounding", "no_backward_rounding"):
        _, _, ga_v, _ = _slab_pixel_by_hand(ops, cols, G, fmt, variant=v)
        if K > 1:
            assert np.abs(ga_v - out["grad"][:, 5]).max() > 1e-9, v


@pytest.mark.parametrize("fmt", ["f16", "unorm16"])
def test_per_fragment_emulation_with_tcull(fmt):
    """Twenty slabs of opacity 0.45: the rounded T crosses 1e-4 at a fragment the hand model
    finds, the later fragments are culled (Procedure 1), and every live fragment's dL/dalpha is
    the hand value."""
    K, o = 20, 0.45
    cols = [[0.2 + 0.03 * k, 0.9 - 0.04 * k, 0.5] for k in range(K)]
    G = np.array([0.4, 0.9, -0.6])
    Gimg = np.broadcast_to(G[:, None, None], (3, 1, 1)).copy()
    tb = float(np.float32(1e-4))
    cfg = _cfg(prefilter=False, t_min_bwd=tb, fb_format=fmt, emulate=True,
               fb_round="per_fragment")
    out = oracle.raster(**_slabs([o] * K, cols), order=np.arange(K), width=1, height=1,
                        dL_dimg=Gimg, cfg=cfg)
    C, T, ga, gc = _slab_pixel_by_hand([o] * K, cols, G, fmt, t_min_bwd=tb)
    live = int((ga != 0.0).sum())
    assert 5 < live < K and out["live"][0, 0] == live
    np.testing.assert_array_equal(out["img"][:, 0, 0], C)
    assert out["T"][0, 0] == T
    np.testing.assert_allclose(out["grad"][:, 5], ga, rtol=1e-15, atol=0)
    np.testing.assert_allclose(out["grad"][:, 6:9], gc, rtol=1e-15, atol=0)
