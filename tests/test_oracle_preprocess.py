"""Pins for the oracle's projection (EWA splatting, SH colour, culling, depth key) and its
complex-step vector-Jacobian product (CPU only).

Checks against: SH orthonormality by quadrature and the addition theorem; the Hamilton product
for the quaternion rotation; a Monte-Carlo projection of samples through the exact pinhole
model; finite differences of the pinhole map for the EWA Jacobian; an on-axis closed form;
central finite differences for the complex-step derivative; a brute-force stable sort.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import projection as P
import synth


def _gauss_sphere(nt=24, nphi=48):
    x, w = np.polynomial.legendre.leggauss(nt)          # exact for degree <= 2 nt - 1 in cos
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi   # exact for trig degree < nphi
    ct = np.repeat(x, nphi)
    st = np.sqrt(1 - ct * ct)
    ph = np.tile(phi, nt)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], 1)
    wt = np.repeat(w, nphi) * (2 * math.pi / nphi)
    return d, wt


def test_sh_orthonormal():
    d, wt = _gauss_sphere()
    Y = P.sh_basis(d, 3)
    gram = (Y * wt[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


def test_sh_addition_theorem():
    g = np.random.default_rng(0)
    d = g.normal(size=(500, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = P.sh_basis(d, 3)
    for l in range(4):
        s = (Y[:, l * l:(l + 1) ** 2] ** 2).sum(1)
        np.testing.assert_allclose(s, (2 * l + 1) / (4 * math.pi), rtol=1e-12)


def _qmul(a, b):
    w1, v1 = a[0], a[1:]
    w2, v2 = b[0], b[1:]
    return np.concatenate([[w1 * w2 - v1 @ v2], w1 * v2 + w2 * v1 + np.cross(v1, v2)])


def test_quaternion_rotation_is_hamilton_conjugation():
    g = np.random.default_rng(1)
    q = g.normal(size=(50, 4)) * g.uniform(0.3, 3.0, size=(50, 1))   # not unit: normalised inside
    R = P.quat_to_rot(q)
    for k in range(50):
        qn = q[k] / np.linalg.norm(q[k])
        v = g.normal(size=3)
        rot = _qmul(_qmul(qn, np.concatenate([[0.0], v])), qn * np.array([1, -1, -1, -1]))
        np.testing.assert_allclose(R[k] @ v, rot[1:], atol=1e-13)
        np.testing.assert_allclose(R[k] @ R[k].T, np.eye(3), atol=1e-13)
        assert np.linalg.det(R[k]) == pytest.approx(1.0)


def _cam(W=640, H=480, fx=500.0, fy=520.0, viewmat=None):
    vm = np.concatenate([np.eye(3), np.zeros((3, 1))], 1) if viewmat is None else viewmat
    return synth.Camera(viewmat=np.asarray(vm, np.float32), fx=fx, fy=fy, cx=W / 2, cy=H / 2,
                        width=W, height=H)


def _one(mean, scale, quat, opac=0.7, degree=0):
    K = (degree + 1) ** 2
    sh = np.zeros((1, K, 3))
    sh[0, 0] = [0.3, 0.5, 0.7]
    return synth.Scene(means3d=np.array([mean], np.float64), scales=np.array([scale], np.float64),
                       quats=np.array([quat], np.float64), opacities=np.array([opac]),
                       sh=sh, sh_degree=degree)


def test_on_axis_isotropic_closed_form():
    cam = _cam()
    eps = oracle.OracleConfig().eps2d
    s, z = 0.05, 3.0
    sc = _one([0.0, 0.0, z], [s, s, s], [0.3, -0.5, 0.2, 0.7])
    out = oracle.preprocess(sc, cam)
    np.testing.assert_allclose(out["means2d"][0], [cam.cx, cam.cy], atol=1e-12)
    np.testing.assert_allclose(out["cov2d"][0], [(cam.fx * s / z) ** 2 + eps, 0.0,
                                                 (cam.fy * s / z) ** 2 + eps], rtol=1e-12, atol=1e-12)
    assert out["visible"][0]


def test_ewa_matches_monte_carlo_projection():
    """Project samples of the 3D Gaussian through the exact pinhole map; their mean and
    covariance must match mu_2D and Sigma_2D - eps I (the EWA linearisation is exact to
    O((s/z)^2) for a small Gaussian)."""
    ang = 0.4
    Rv = np.array([[math.cos(ang), 0, math.sin(ang)], [0, 1, 0], [-math.sin(ang), 0, math.cos(ang)]])
    vm = np.concatenate([Rv, np.array([[0.1], [-0.2], [3.5]])], 1)
    cam = _cam(viewmat=vm)
    Rv32 = cam.viewmat[:, :3].astype(np.float64)
    t32 = cam.viewmat[:, 3].astype(np.float64)
    eps = oracle.OracleConfig().eps2d
    mean = np.array([0.3, -0.25, 0.4])
    scale = np.array([0.006, 0.003, 0.0045])
    quat = np.array([0.8, 0.3, -0.4, 0.2])
    out = oracle.preprocess(_one(mean, scale, quat), cam)
    R = P.quat_to_rot(quat[None])[0]
    S3 = R @ np.diag(scale ** 2) @ R.T
    g = np.random.default_rng(7)
    pts = g.multivariate_normal(mean, S3, size=400_000)
    t = pts @ Rv32.T + t32
    u = np.stack([cam.fx * t[:, 0] / t[:, 2] + cam.cx, cam.fy * t[:, 1] / t[:, 2] + cam.cy], 1)
    np.testing.assert_allclose(u.mean(0), out["means2d"][0], atol=1e-2)
    C = np.cov(u.T)
    cv = out["cov2d"][0]
    ref = np.array([C[0, 0] + eps, C[0, 1], C[1, 1] + eps])
    lam = max(C[0, 0], C[1, 1])
    assert np.abs(ref - cv).max() <= 1.5e-2 * lam


def test_ewa_jacobian_by_finite_differences():
    """Sigma_2D - eps I = J W Sigma_3D W^T J^T with J the derivative of the pinhole map at t,
    here taken by central differences instead of the closed form."""
    vm = np.array([[0.36, 0.48, -0.8, 0.2], [-0.8, 0.6, 0.0, -0.1], [0.48, 0.64, 0.6, 4.0]])
    cam = _cam(viewmat=vm)
    Rv = cam.viewmat[:, :3].astype(np.float64)
    tv = cam.viewmat[:, 3].astype(np.float64)
    eps = oracle.OracleConfig().eps2d
    g = np.random.default_rng(3)
    for _ in range(10):
        mean = g.uniform(-0.8, 0.8, 3)
        scale = g.uniform(0.01, 0.08, 3)
        quat = g.normal(size=4)
        out = oracle.preprocess(_one(mean, scale, quat), cam)
        t = Rv @ mean + tv
        proj = lambda tt: np.array([cam.fx * tt[0] / tt[2] + cam.cx, cam.fy * tt[1] / tt[2] + cam.cy])
        J = np.zeros((2, 3))
        for j in range(3):
            h = 1e-6 * max(1.0, abs(t[j]))
            e = np.zeros(3)
            e[j] = h
            J[:, j] = (proj(t + e) - proj(t - e)) / (2 * h)
        R = P.quat_to_rot(quat[None])[0]
        S2 = J @ Rv @ (R @ np.diag(scale ** 2) @ R.T) @ Rv.T @ J.T
        np.testing.assert_allclose(out["cov2d"][0], [S2[0, 0] + eps, S2[0, 1], S2[1, 1] + eps],
                                   rtol=1e-7)
        np.testing.assert_allclose(out["means2d"][0], proj(t), rtol=1e-12)
        cv = out["cov2d"][0]
        Q = np.linalg.inv(np.array([[cv[0], cv[1]], [cv[1], cv[2]]]))
        np.testing.assert_allclose(out["conic"][0], [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-10)


def test_colour_uses_view_direction():
    """Degree-1 SH: colour = Y00 k0 + sqrt(3/4pi)(y k1 + z k2 + x k3) + 0.5 at the unit
    direction from the camera centre to the mean."""
    cam = _cam()
    sc = _one([0.4, -0.3, 2.0], [0.02] * 3, [1, 0, 0, 0], degree=1)
    sc.sh[0, 1:] = np.array([[0.1, -0.2, 0.05], [0.3, 0.0, -0.1], [-0.2, 0.15, 0.2]])
    out = oracle.preprocess(sc, cam)
    d = np.array([0.4, -0.3, 2.0]) / np.linalg.norm([0.4, -0.3, 2.0])
    c1 = math.sqrt(3 / (4 * math.pi))
    ref = 0.5 / math.sqrt(math.pi) * sc.sh[0, 0] + c1 * (d[1] * sc.sh[0, 1] + d[2] * sc.sh[0, 2]
                                                        + d[0] * sc.sh[0, 3]) + 0.5
    np.testing.assert_allclose(out["rgb"][0], np.maximum(ref, 0), rtol=1e-12)


def test_culling_and_depth_key():
    cam = _cam()
    means = [[0, 0, 3.0], [0, 0, 0.1], [0, 0, -2.0], [50.0, 0, 3.0], [0.2, 0.1, 5.0], [0, 0, 2.0]]
    n = len(means)
    sc = synth.Scene(means3d=np.array(means, np.float32), scales=np.full((n, 3), 0.02, np.float32),
                     quats=np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)),
                     opacities=np.array([0.5, 0.5, 0.5, 0.5, 0.003, 0.9], np.float32),
                     sh=np.zeros((n, 1, 3), np.float32), sh_degree=0)
    out = oracle.preprocess(sc, cam)
    assert list(out["visible"]) == [True, False, False, False, False, True]
    k = out["keys"]
    assert k[0] == np.float32(3.0).view(np.uint32) and k[5] == np.float32(2.0).view(np.uint32)
    assert all(k[i] == 0xFFFFFFFF for i in (1, 2, 3, 4))
    assert list(oracle.visible_order(k)) == [5, 0]


def test_complex_step_matches_finite_differences():
    sc = synth.scene3d(60, seed=12, sh_degree=3)
    sc.means3d *= 0.3
    sc.scales *= 3.0
    cam = synth.camera_front(200, 150, 160.0)
    ref = oracle.preprocess(sc, cam)
    vis = ref["visible"]
    assert vis.sum() > 30
    g = np.random.default_rng(2)
    gm, gc, gr = g.normal(size=(60, 2)), g.normal(size=(60, 3)), g.normal(size=(60, 3))
    go = g.normal(size=60)
    vj = oracle.preprocess_vjp(sc, cam, gm, gc, gr, go)

    def loss(s2):
        o = P.project(np.asarray(s2.means3d, np.float64), np.asarray(s2.scales, np.float64),
                      np.asarray(s2.quats, np.float64), np.asarray(s2.opacities, np.float64),
                      np.asarray(s2.sh, np.float64), s2.sh_degree, cam,
                      oracle.OracleConfig().alpha_min, oracle.OracleConfig().eps2d, visible=vis)
        m = vis
        return (np.sum(gm[m] * o["means2d"][m]) + np.sum(gc[m] * o["conic"][m]) +
                np.sum(gr[m] * o["rgb"][m]) + np.sum(go[m] * s2.opacities[m]))

    import copy
    base = copy.deepcopy(sc)
    for name in ("means3d", "scales", "quats", "sh", "opacities"):
        arr = getattr(base, name).astype(np.float64)
        an = vj[name]
        idx = list(np.ndindex(*arr.shape))
        sel = [idx[i] for i in g.choice(len(idx), size=min(40, len(idx)), replace=False)]
        for ix in sel:
            h = 1e-6 * max(1.0, abs(arr[ix]))
            vals = []
            for sgn in (1, -1):
                s2 = copy.deepcopy(base)
                a2 = arr.copy()
                a2[ix] += sgn * h
                setattr(s2, name, a2)
                vals.append(loss(s2))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - an[ix]) <= 1e-6 * max(1.0, abs(an[ix])) + 1e-7, (name, ix, fd, an[ix])


def test_stable_sort_brute_force():
    k = synth.sorted_key_case(3000, seed=5, tie_levels=37)
    ref = [i for _, i in sorted((int(k[i]), i) for i in range(len(k)))]
    assert list(oracle.depth_order(k)) == ref
