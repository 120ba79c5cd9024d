"""FP64 CPU oracle for the differentiable splat rasterizer.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package. The product path (the HIP library and its
Python binding) never imports it and shares no code with it; both read only the seeded inputs
of the ``synth`` package.

Parts:
  * ``raster.c`` (built to ``liboracle.so``): per-pixel front-to-back compositing (Eq. 2) and the
    front-to-back gradient procedure (Procedure 1 with Eqs. 3, 5, 6, 7), FP64, with optional
    render-target format emulation (Sec. 3.3) and ambiguity flags.
  * ``projection.py``: the projection (Sec. 2.1.1-2.1.2) in FP64 and its exact vector-Jacobian
    product by complex step.
  * ``depth_order``: the depth sort as its plain definition, a stable sort by (key, index).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

from . import projection as _pre

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

FMT = {"f32": 0, "f16": 1, "unorm16": 2, "bf16": 3, "unorm8": 4}


def _f32(x: float) -> float:
    return float(np.float32(x))


@dataclasses.dataclass
class OracleConfig:
    """The method's constants (Sec. 2.1.2: alpha >= 1/255; Sec. 2.1.4 / Procedure 1: T >= 1e-4)
    and the readings for what the paper leaves open (alpha clamp 0.99, eps2d 0.3, z_near 0.2).
    Thresholds are the FP32 values the GPU path compares against."""
    alpha_min: float = _f32(1.0 / 255.0)
    alpha_max: float = _f32(0.99)
    t_min_fwd: float = 0.0
    t_min_bwd: float = _f32(1e-4)
    eps2d: float = _f32(0.3)
    fb_format: str = "f32"
    emulate: bool = False
    fb_round: str = "at_rest"      # or "per_fragment"
    saturate: bool | None = None   # default: True for the unorm formats
    prefilter: bool = True
    beta: float = 1e-6
    beta_abs: float = 0.0
    tau: float = 1e-4
    nthreads: int = 0              # 0: all cores
    background: tuple = (0.0, 0.0, 0.0)   # C += T_final bg (zero: Eq. 2 as printed)


class _OCfg(ctypes.Structure):
    _fields_ = [("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("t_min_fwd", ctypes.c_double), ("t_min_bwd", ctypes.c_double),
                ("beta", ctypes.c_double), ("beta_abs", ctypes.c_double),
                ("tau", ctypes.c_double), ("fb_format", ctypes.c_int32),
                ("emulate", ctypes.c_int32), ("fb_round", ctypes.c_int32),
                ("saturate", ctypes.c_int32), ("prefilter", ctypes.c_int32),
                ("nthreads", ctypes.c_int32), ("background", ctypes.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH} (run oracle/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.oracle_raster.restype = ctypes.c_int
        L.oracle_raster.argtypes = [ctypes.POINTER(_OCfg), ctypes.c_int32, P, P, P, P, P,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, P, P, P, P, P, P, P, P, P]
        L.oracle_round_array.restype = None
        L.oracle_round_array.argtypes = [P, ctypes.c_int64, ctypes.c_int32]
        L.oracle_pixel_trace.restype = ctypes.c_int32
        L.oracle_pixel_trace.argtypes = [ctypes.POINTER(_OCfg), ctypes.c_int32, P, P, P, P, P,
                                         ctypes.c_int32, ctypes.c_double, ctypes.c_double, P,
                                         ctypes.c_int32, P, P]
        L.oracle_version.restype = ctypes.c_int32
        _lib = L
    return _lib


def _ccfg(cfg: OracleConfig) -> _OCfg:
    sat = cfg.saturate
    if sat is None:
        sat = cfg.fb_format in ("unorm16", "unorm8")
    nth = cfg.nthreads if cfg.nthreads > 0 else (os.cpu_count() or 1)
    return _OCfg(cfg.alpha_min, cfg.alpha_max, cfg.t_min_fwd, cfg.t_min_bwd, cfg.beta,
                 cfg.beta_abs, cfg.tau, FMT[cfg.fb_format], int(cfg.emulate),
                 1 if cfg.fb_round == "per_fragment" else 0, int(sat), int(cfg.prefilter), nth,
                 (ctypes.c_double * 3)(*[float(v) for v in cfg.background]))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def round_fmt(x, fmt: str) -> np.ndarray:
    """Round FP64 values to a framebuffer format (round to nearest even; unorm clamps to [0,1])."""
    a = np.array(x, dtype=np.float64, copy=True)
    flat = np.ascontiguousarray(a.reshape(-1))
    lib().oracle_round_array(_ptr(flat), flat.size, FMT[fmt])
    return flat.reshape(a.shape)


def depth_order(keys: np.ndarray) -> np.ndarray:
    """Depth order: a stable ascending sort of the keys, ties kept in index order (Sec. 4.1's
    depth sort has no stated tie rule; stability is the reading)."""
    return np.argsort(np.asarray(keys), kind="stable").astype(np.int32)


def visible_order(keys: np.ndarray) -> np.ndarray:
    """Stable depth order of the splats whose key is not the culled sentinel."""
    o = depth_order(keys)
    return o[np.asarray(keys)[o] != np.uint32(0xFFFFFFFF)].astype(np.int32)


def raster(means2d, conics, opacities, rgb, order, width, height, crop=None, dL_dimg=None,
           cfg: OracleConfig | None = None, want_grad=True, dL_dT=None):
    """Composite the splats listed in ``order`` (front to back) over the crop
    (x0, y0, w, h) of a width x height image; with ``dL_dimg`` ([3, H, W]) also run the
    backward procedure (and with ``dL_dT`` [H, W] the final transmittance's gradient). Returns
    img [3,h,w], T [h,w], cov/live/amb [h,w] int32 and, when requested, grad [N, 9] = (dmean x,
    y, dconic a, b, c, dopacity, drgb r, g, b) and grad_bg [3] (w.r.t. the background)."""
    cfg = cfg or OracleConfig()
    m = _c(means2d, np.float64)
    cn = _c(conics, np.float64)
    op = _c(opacities, np.float64)
    cl = _c(rgb, np.float64)
    od = _c(order, np.int32)
    n = int(m.shape[0])
    x0, y0, cw, ch = crop if crop is not None else (0, 0, width, height)
    img = np.zeros((3, ch, cw))
    T = np.zeros((ch, cw))
    cov = np.zeros((ch, cw), np.int32)
    live = np.zeros((ch, cw), np.int32)
    amb = np.zeros((ch, cw), np.int32)
    G = _c(dL_dimg, np.float64) if dL_dimg is not None else None
    grad = np.zeros((n, 9)) if (G is not None and want_grad) else None
    gT = _c(dL_dT, np.float64) if dL_dT is not None else None
    gbg = np.zeros(3) if G is not None else None
    c = _ccfg(cfg)
    rc = lib().oracle_raster(ctypes.byref(c), n, _ptr(m), _ptr(cn), _ptr(op), _ptr(cl), _ptr(od),
                             int(od.size), int(width), int(height), int(x0), int(y0), int(cw),
                             int(ch), _ptr(G), _ptr(img), _ptr(T), _ptr(cov), _ptr(live),
                             _ptr(amb), _ptr(grad), _ptr(gT), _ptr(gbg))
    if rc != 0:
        raise ValueError("oracle_raster: invalid arguments")
    out = dict(img=img, T=T, cov=cov, live=live, amb=amb)
    if grad is not None:
        out["grad"] = grad
    if gbg is not None:
        out["grad_bg"] = gbg
    return out


def pixel_trace(means2d, conics, opacities, rgb, order, px, py, G, cfg=None, max_frag=4096):
    """Per-fragment record of one pixel: rows (order position, alpha, T_i, C'_i (3),
    dL/dalpha_i, live), plus the forward colour C used as C'_1."""
    cfg = cfg or OracleConfig()
    m = _c(means2d, np.float64)
    cn = _c(conics, np.float64)
    op = _c(opacities, np.float64)
    cl = _c(rgb, np.float64)
    od = _c(order, np.int32)
    g = _c(G, np.float64)
    out = np.zeros((max_frag, 8))
    Cf = np.zeros(3)
    c = _ccfg(cfg)
    k = lib().oracle_pixel_trace(ctypes.byref(c), int(m.shape[0]), _ptr(m), _ptr(cn), _ptr(op),
                                 _ptr(cl), _ptr(od), int(od.size), float(px), float(py), _ptr(g),
                                 int(max_frag), _ptr(out), _ptr(Cf))
    return out[:k], Cf


# ---- projection ------------------------------------------------------------------------------

def preprocess(scene, cam, cfg: OracleConfig | None = None):
    cfg = cfg or OracleConfig()
    return _pre.preprocess(scene, cam, cfg.alpha_min, cfg.eps2d)


def preprocess_vjp(scene, cam, g_means2d, g_conics, g_rgb, g_opac, cfg=None):
    cfg = cfg or OracleConfig()
    return _pre.preprocess_vjp(scene, cam, cfg.alpha_min, cfg.eps2d, g_means2d, g_conics, g_rgb,
                               g_opac)


def render_scene(scene, cam, dL_dimg=None, crop=None, cfg=None):
    """Whole oracle pipeline on a 3D scene in FP64: projection, stable depth order (by the fp32
    depth key), raster. No intermediate is rounded, so the chain is smooth for finite
    differences."""
    cfg = cfg or OracleConfig()
    pre = preprocess(scene, cam, cfg)
    order = visible_order(pre["keys"])
    out = raster(pre["means2d"], pre["conic"], np.asarray(scene.opacities, np.float64),
                 pre["rgb"], order, cam.width, cam.height, crop=crop, dL_dimg=dL_dimg, cfg=cfg)
    out["pre"] = pre
    out["order"] = order
    return out
