"""FP64 reference for the projection step (EWA splatting, SH colour, culling, depth key) and
its vector-Jacobian product.

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU-baseline leg use it.

The forward follows Sec. 2.1.1-2.1.2: Sigma_3D = R S S^T R^T from a quaternion and a scale
vector; t = W mu + tau; mu_2D = proj(t); Sigma_2D = J W Sigma_3D W^T J^T (+ eps2d I, a low-pass
dilation the paper does not state; common practice); conic = Sigma_2D^{-1}; colour from real
spherical harmonics of degree <= 3 evaluated at the view direction. The paper gives neither
the SH basis nor its offset; the readings used here (orthonormal real SH, +0.5 offset, clamp
at 0) are listed in the design notes. The tests pin the basis by orthonormality and the
addition theorem, which fix every function up to its sign: the sign convention of the m != 0
functions (no Condon-Shortley phase, Y_1,-1 ~ y, Y_1,0 ~ z, Y_1,1 ~ x) is parity unpinned.
Frustum culling (Sec. 4.1) drops splats that cannot put a fragment with alpha >= alpha_min on a
pixel centre.

Every arithmetic step is written so that it also runs on complex128 inputs. The backward is
then the exact derivative of this forward by the complex-step method,
df/dx = Im f(x + i h) / h with h = 1e-30, one input component at a time for all splats at once
(splats are independent, so there is no cross-talk). Branches (culling, the colour clamp) are
decided on the real part. This gives the vector-Jacobian product to rounding without any
hand-derived chain rule.
"""
from __future__ import annotations

import math

import numpy as np

# ---- real spherical harmonics, degree <= 3 ------------------------------------------------
# Y_{l,m} as polynomials in the unit direction (x, y, z); coefficient index k = l^2 + l + m.
_S = math.sqrt
SH_C = {
    (0, 0): 0.5 * _S(1.0 / math.pi),
    (1, -1): _S(3.0 / (4.0 * math.pi)),
    (1, 0): _S(3.0 / (4.0 * math.pi)),
    (1, 1): _S(3.0 / (4.0 * math.pi)),
    (2, -2): 0.5 * _S(15.0 / math.pi),
    (2, -1): 0.5 * _S(15.0 / math.pi),
    (2, 0): 0.25 * _S(5.0 / math.pi),
    (2, 1): 0.5 * _S(15.0 / math.pi),
    (2, 2): 0.25 * _S(15.0 / math.pi),
    (3, -3): 0.25 * _S(35.0 / (2.0 * math.pi)),
    (3, -2): 0.5 * _S(105.0 / math.pi),
    (3, -1): 0.25 * _S(21.0 / (2.0 * math.pi)),
    (3, 0): 0.25 * _S(7.0 / math.pi),
    (3, 1): 0.25 * _S(21.0 / (2.0 * math.pi)),
    (3, 2): 0.25 * _S(105.0 / math.pi),
    (3, 3): 0.25 * _S(35.0 / (2.0 * math.pi)),
}


def sh_basis(d: np.ndarray, degree: int) -> np.ndarray:
    """Real SH basis values at unit directions d [N, 3] -> [N, (degree+1)^2]."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    cols = [SH_C[(0, 0)] * np.ones_like(x)]
    if degree >= 1:
        cols += [SH_C[(1, -1)] * y, SH_C[(1, 0)] * z, SH_C[(1, 1)] * x]
    if degree >= 2:
        cols += [SH_C[(2, -2)] * x * y, SH_C[(2, -1)] * y * z,
                 SH_C[(2, 0)] * (2.0 * z * z - x * x - y * y),
                 SH_C[(2, 1)] * x * z, SH_C[(2, 2)] * (x * x - y * y)]
    if degree >= 3:
        cols += [SH_C[(3, -3)] * y * (3.0 * x * x - y * y),
                 SH_C[(3, -2)] * x * y * z,
                 SH_C[(3, -1)] * y * (4.0 * z * z - x * x - y * y),
                 SH_C[(3, 0)] * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y),
                 SH_C[(3, 1)] * x * (4.0 * z * z - x * x - y * y),
                 SH_C[(3, 2)] * z * (x * x - y * y),
                 SH_C[(3, 3)] * x * (x * x - 3.0 * y * y)]
    return np.stack(cols, axis=1)


def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrix of the normalised quaternion (w, x, y, z): R v = q v q^*."""
    n = np.sqrt(np.sum(q * q, axis=1))
    w, x, y, z = (q[:, j] / n for j in range(4))
    R = np.empty((q.shape[0], 3, 3), dtype=np.result_type(q, np.float64))
    R[:, 0, 0] = 1.0 - 2.0 * (y * y + z * z)
    R[:, 0, 1] = 2.0 * (x * y - w * z)
    R[:, 0, 2] = 2.0 * (x * z + w * y)
    R[:, 1, 0] = 2.0 * (x * y + w * z)
    R[:, 1, 1] = 1.0 - 2.0 * (x * x + z * z)
    R[:, 1, 2] = 2.0 * (y * z - w * x)
    R[:, 2, 0] = 2.0 * (x * z - w * y)
    R[:, 2, 1] = 2.0 * (y * z + w * x)
    R[:, 2, 2] = 1.0 - 2.0 * (x * x + y * y)
    return R


def _cam_arrays(cam):
    vm = np.asarray(cam.viewmat, dtype=np.float32).astype(np.float64)
    return vm[:, :3], vm[:, 3]


def project(means3d, scales, quats, opacities, sh, sh_degree, cam, alpha_min, eps2d,
            visible=None):
    """The projection forward on float64 or complex128 arrays.

    Returns a dict with t (camera coords), means2d, cov2d (xx, xy, yy), conic (a, b, c), rgb,
    the half extents of the alpha >= alpha_min ellipse's bounding box, and (when ``visible`` is
    None) the visibility decision made on the real parts.
    """
    Rv, tv = _cam_arrays(cam)
    mx, my, mz = means3d[:, 0], means3d[:, 1], means3d[:, 2]
    # Camera coordinates, summed left to right (the depth key is fp32 of this FP64 tz).
    tx = ((Rv[0, 0] * mx + Rv[0, 1] * my) + Rv[0, 2] * mz) + tv[0]
    ty = ((Rv[1, 0] * mx + Rv[1, 1] * my) + Rv[1, 2] * mz) + tv[1]
    tz = ((Rv[2, 0] * mx + Rv[2, 1] * my) + Rv[2, 2] * mz) + tv[2]
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    front = np.real(tz) >= float(np.float32(cam.znear))
    tzs = np.where(front, tz, 1.0)          # keep culled rows finite
    # Local affine approximation of the perspective projection (Jacobian of proj at t).
    J = np.zeros((means3d.shape[0], 2, 3), dtype=np.result_type(means3d, np.float64))
    J[:, 0, 0] = fx / tzs
    J[:, 0, 2] = -fx * tx / (tzs * tzs)
    J[:, 1, 1] = fy / tzs
    J[:, 1, 2] = -fy * ty / (tzs * tzs)
    R = quat_to_rot(quats)
    M = R * scales[:, None, :]              # R S
    S3 = M @ np.swapaxes(M, 1, 2)           # R S S^T R^T
    Tm = J @ Rv[None, :, :]                 # J W
    S2 = Tm @ S3 @ np.swapaxes(Tm, 1, 2)
    sxx = S2[:, 0, 0] + eps2d
    sxy = S2[:, 0, 1]
    syy = S2[:, 1, 1] + eps2d
    det = sxx * syy - sxy * sxy
    dets = np.where(np.real(det) > 0, det, 1.0)
    conic = np.stack([syy / dets, -sxy / dets, sxx / dets], axis=1)
    mean2d = np.stack([fx * tx / tzs + cx, fy * ty / tzs + cy], axis=1)
    campos = -Rv.T @ tv
    v = means3d - campos[None, :]
    dirs = v / np.sqrt(np.sum(v * v, axis=1))[:, None]
    Y = sh_basis(dirs, sh_degree)
    K = (sh_degree + 1) ** 2
    val = np.einsum("nk,nkc->nc", Y, sh[:, :K, :]) + 0.5
    rgb = np.where(np.real(val) > 0, val, 0.0)
    o = np.real(opacities)
    r2 = 2.0 * np.log(np.maximum(o, 1e-300) / alpha_min)
    hx = np.sqrt(np.maximum(r2 * np.real(sxx), 0.0))
    hy = np.sqrt(np.maximum(r2 * np.real(syy), 0.0))
    out = dict(tx=tx, ty=ty, tz=tz, means2d=mean2d, cov2d=np.stack([sxx, sxy, syy], 1),
               conic=conic, rgb=rgb, hx=hx, hy=hy, det=det, front=front)
    if visible is None:
        mxr, myr = np.real(mean2d[:, 0]), np.real(mean2d[:, 1])
        W, H = cam.width, cam.height
        on_img = ((mxr + hx >= 0.5) & (mxr - hx <= W - 0.5) &
                  (myr + hy >= 0.5) & (myr - hy <= H - 0.5))
        out["visible"] = front & (o >= alpha_min) & (np.real(det) > 0) & on_img
        # decisions the FP32 GPU path could take the other way (kept for parity tests)
        mx_band = 1e-4 * (np.abs(mxr) + hx + 1.0)
        my_band = 1e-4 * (np.abs(myr) + hy + 1.0)
        near = (np.abs(mxr + hx - 0.5) <= mx_band) | (np.abs(mxr - hx - (W - 0.5)) <= mx_band) | \
               (np.abs(myr + hy - 0.5) <= my_band) | (np.abs(myr - hy - (H - 0.5)) <= my_band)
        out["ambiguous"] = front & (o >= alpha_min) & near
    else:
        out["visible"] = visible
    return out


def depth_keys(tz: np.ndarray, visible: np.ndarray) -> np.ndarray:
    """uint32 sort key: the bits of fp32(tz) (positive, so monotone); 0xFFFFFFFF when culled."""
    k = np.real(tz).astype(np.float32).view(np.uint32).copy()
    k[~visible] = np.uint32(0xFFFFFFFF)
    return k


def preprocess(scene, cam, alpha_min, eps2d):
    """FP64 projection of a scene; float64 outputs plus the fp32 depth key and visibility."""
    f64 = lambda a: np.asarray(a, dtype=np.float64)
    out = project(f64(scene.means3d), f64(scene.scales), f64(scene.quats), f64(scene.opacities),
                  f64(scene.sh), scene.sh_degree, cam, alpha_min, eps2d)
    vis = out["visible"]
    out["keys"] = depth_keys(out["tz"], vis)
    out["depth"] = np.where(vis, out["tz"], 0.0)
    for k in ("means2d", "conic", "rgb"):
        out[k] = np.where(vis[:, None], out[k], 0.0)
    out["opacities"] = f64(scene.opacities)
    return out


def preprocess_vjp(scene, cam, alpha_min, eps2d, g_means2d, g_conics, g_rgb, g_opac):
    """Vector-Jacobian product of the projection by complex step.

    Given dL/d(means2d [N,2], conic [N,3], rgb [N,3], opacity [N]) returns dL/d(means3d,
    scales, quats, opacities, sh) for the scene's raw inputs (zero for culled splats)."""
    f64 = lambda a: np.asarray(a, dtype=np.float64)
    base = [f64(scene.means3d), f64(scene.scales), f64(scene.quats), f64(scene.opacities),
            f64(scene.sh)]
    ref = project(*base, scene.sh_degree, cam, alpha_min, eps2d)
    vis = ref["visible"]
    gm, gc, gr = f64(g_means2d), f64(g_conics), f64(g_rgb)
    h = 1e-30
    grads = [np.zeros_like(b) for b in base]
    for idx in (0, 1, 2, 4):
        X = base[idx]
        flat_shape = X.shape[1:]
        for comp in np.ndindex(*flat_shape):
            args = [b.astype(np.complex128) for b in base]
            sl = (slice(None),) + comp
            args[idx][sl] += 1j * h
            out = project(*args, scene.sh_degree, cam, alpha_min, eps2d, visible=vis)
            d = (np.sum(gm * out["means2d"].imag, axis=1) + np.sum(gc * out["conic"].imag, axis=1)
                 + np.sum(gr * out["rgb"].imag, axis=1)) / h
            grads[idx][sl] = d
    grads[3] = f64(g_opac).copy()      # opacity passes through the projection unchanged
    for g in grads:
        g[~vis] = 0.0
    return dict(means3d=grads[0], scales=grads[1], quats=grads[2], opacities=grads[3],
                sh=grads[4])
