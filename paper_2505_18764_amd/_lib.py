"""ctypes binding of libgsr.so: the C-ABI entry points under the same names.

Argument marshalling only: every function takes torch tensors (device memory) or None, passes
their data pointers and the stream handle to the library, and raises GsrError on a nonzero
status. Nothing here computes any part of the method, and there is no fallback: if the library is
not built, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsr.so")

c_f = ctypes.c_float
c_i = ctypes.c_int32
c_p = ctypes.c_void_p
c_sz = ctypes.c_size_t

FB_FORMATS = {"f32": 0, "f16": 1, "unorm16": 2, "bf16": 3, "unorm8": 4}
FB_ROUND = {"at_rest": 0, "per_fragment": 1}
REDUCE_MODES = {"naive": 0, "quad": 1, "wave": 2, "hybrid": 3, "hybrid_lane": 4, "tile": 5}
OPS = {"preprocess": 0, "sort": 1, "raster_fwd": 2, "raster_bwd": 3, "preprocess_bwd": 4,
       "prepare_2d": 5, "all": 6}
STATUS = {0: "GS_OK", 1: "GS_ERR_INVALID_ARGUMENT", 2: "GS_ERR_CAPACITY", 3: "GS_ERR_UNSUPPORTED",
          4: "GS_ERR_HIP", 5: "GS_ERR_STATE"}
STATUS_BITS = {1: "GS_STATUS_BAD_ID", 2: "GS_STATUS_FWD_SCHEDULE", 4: "GS_STATUS_BWD_SCHEDULE",
               8: "GS_STATUS_STALE_RECORD"}


class GsCamera(ctypes.Structure):
    _fields_ = [("viewmat", c_f * 12), ("fx", c_f), ("fy", c_f), ("cx", c_f), ("cy", c_f),
                ("width", c_i), ("height", c_i), ("znear", c_f), ("reserved", c_f)]


class GsConfig(ctypes.Structure):
    _fields_ = [("alpha_min", c_f), ("alpha_max", c_f), ("t_min_fwd", c_f), ("t_min_bwd", c_f),
                ("eps2d", c_f), ("sh_degree", c_i), ("fb_format", c_i), ("fb_round", c_i),
                ("reduce_mode", c_i), ("reduce_threshold", c_i), ("flags", c_i),
                ("background", c_f * 3), ("n_views", c_i), ("reserved", c_i * 1)]


MAX_VIEWS = 16


def camera_array(cams) -> ctypes.Array:
    """A C array of gs_camera for the view-batched entry points (cam points to n_views cameras)."""
    arr = (GsCamera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = c
    return arr


STATS_FIELDS = ["fwd_queued", "fwd_evaluated", "fwd_covered", "bwd_queued", "bwd_evaluated",
                "bwd_live", "bwd_atomic_sets", "bwd_wave_reductions", "bwd_quad_reductions",
                "bwd_cohesive", "fwd_walked", "fwd_empty_blocks", "fwd_chunks", "fwd_batches"]


class GsStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_ulonglong) for f in STATS_FIELDS] + [("reserved", ctypes.c_ulonglong * 2)]


class GsrError(RuntimeError):
    def __init__(self, name, status, message):
        super().__init__(f"{name} failed with {STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None

_SIGS = {
    "gs_last_error": (ctypes.c_char_p, []),
    "gs_version": (c_i, []),
    "gs_config_default": (None, [ctypes.POINTER(GsConfig)]),
    "gs_workspace_size": (c_sz, [c_i, c_i, c_i, c_i, ctypes.POINTER(GsConfig)]),
    "gs_framebuffer_size": (c_sz, [c_i, c_i, c_i]),
    "gs_preprocess": (ctypes.c_int, [ctypes.POINTER(GsCamera), ctypes.POINTER(GsConfig), c_i,
                                     c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p,
                                     c_p, c_sz, c_p]),
    "gs_prepare_2d": (ctypes.c_int, [ctypes.POINTER(GsCamera), ctypes.POINTER(GsConfig), c_i,
                                     c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_sz, c_p]),
    "gs_sort": (ctypes.c_int, [c_i, c_p, c_p, c_p, c_p, c_sz, c_p]),
    "gs_sort_views": (ctypes.c_int, [c_i, c_i, c_p, c_p, c_p, c_p, c_sz, c_p]),
    "gs_sort_noalloc": (ctypes.c_int, [c_i, c_p, c_p, c_p, c_p]),
    "gs_raster_setup": (ctypes.c_int, [ctypes.POINTER(GsCamera), ctypes.POINTER(GsConfig), c_i,
                                       c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_sz, c_p]),
    "gs_raster_fwd": (ctypes.c_int, [ctypes.POINTER(GsCamera), ctypes.POINTER(GsConfig), c_i,
                                     c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p,
                                     c_sz, c_p]),
    "gs_raster_bwd": (ctypes.c_int, [ctypes.POINTER(GsCamera), ctypes.POINTER(GsConfig), c_i,
                                     c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p,
                                     c_p, c_p, c_p, c_p, c_p, c_sz, c_p]),
    "gs_preprocess_bwd": (ctypes.c_int, [ctypes.POINTER(GsCamera), ctypes.POINTER(GsConfig), c_i,
                                         c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p,
                                         c_p, c_p, c_p, c_p]),
    "gs_raster_status": (ctypes.c_int, [ctypes.POINTER(GsConfig), c_i, c_i, c_i, c_p, c_sz,
                                        ctypes.POINTER(ctypes.c_uint32), c_p]),
    "gs_raster_debug_schedule": (ctypes.c_int, [ctypes.POINTER(GsConfig), c_i, c_i, c_i, c_p,
                                                c_sz, c_p, c_p, c_p, c_p, c_p, c_p]),
    "gs_micro_copy": (ctypes.c_int, [c_p, c_p, c_sz, c_p]),
    "gs_micro_atomic_f32": (ctypes.c_int, [c_p, ctypes.c_int64, c_i, c_i, c_p]),
    "gs_tile_workspace_size": (c_sz, [c_i, ctypes.c_int64, c_i, c_i]),
    "gs_tile_prepare": (ctypes.c_int, [ctypes.POINTER(GsCamera), ctypes.POINTER(GsConfig), c_i,
                                       c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_sz, c_p]),
    "gs_tile_raster_fwd": (ctypes.c_int, [ctypes.POINTER(GsCamera), ctypes.POINTER(GsConfig), c_i,
                                          c_p, c_p, c_p, c_p, c_p, c_p, c_p, ctypes.c_int64, c_p,
                                          c_p, c_p, c_p, c_sz, c_p]),
    "gs_tile_raster_bwd": (ctypes.c_int, [ctypes.POINTER(GsCamera), ctypes.POINTER(GsConfig), c_i,
                                          c_p, c_p, c_p, c_p, c_p, c_p, c_p, ctypes.c_int64, c_p,
                                          c_p, c_p, c_p, c_p, c_sz, c_p]),
}


def lib():
    """Load libgsr.so (built in-tree by ``paper_2505_18764_amd/build.py``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"the HIP library is not built: {LIB_PATH} is missing; run "
                               "python -c 'import __graft_entry__ as g; g.build()'")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _cam(cam):
    """A gs_camera* argument from one GsCamera or a camera_array()."""
    return cam if isinstance(cam, ctypes.Array) else ctypes.byref(cam)


def _check(name, rc):
    if rc != 0:
        msg = lib().gs_last_error()
        raise GsrError(name, rc, msg.decode() if msg else "")


def gs_version() -> int:
    return int(lib().gs_version())


def gs_last_error() -> str:
    return lib().gs_last_error().decode()


def gs_config_default() -> GsConfig:
    c = GsConfig()
    lib().gs_config_default(ctypes.byref(c))
    return c


def gs_workspace_size(op, n, width, height, cfg: GsConfig) -> int:
    op = OPS[op] if isinstance(op, str) else op
    return int(lib().gs_workspace_size(op, n, width, height, ctypes.byref(cfg)))


def gs_framebuffer_size(width, height, fb_format) -> int:
    f = FB_FORMATS[fb_format] if isinstance(fb_format, str) else fb_format
    return int(lib().gs_framebuffer_size(width, height, f))


def gs_preprocess(cam: GsCamera, cfg: GsConfig, n, means3d, scales, quats, opacities, sh,
                  means2d, conics, rgb, depth, keys, ids, n_visible, ws, ws_bytes, stream):
    _check("gs_preprocess", lib().gs_preprocess(
        _cam(cam), ctypes.byref(cfg), n, _ptr(means3d), _ptr(scales), _ptr(quats),
        _ptr(opacities), _ptr(sh), _ptr(means2d), _ptr(conics), _ptr(rgb), _ptr(depth),
        _ptr(keys), _ptr(ids), _ptr(n_visible), _ptr(ws), ws_bytes, stream))


def gs_prepare_2d(cam: GsCamera, cfg: GsConfig, n, means2d, conics, opacities, depth, keys, ids,
                  n_visible, ws, ws_bytes, stream):
    _check("gs_prepare_2d", lib().gs_prepare_2d(
        ctypes.byref(cam), ctypes.byref(cfg), n, _ptr(means2d), _ptr(conics), _ptr(opacities),
        _ptr(depth), _ptr(keys), _ptr(ids), _ptr(n_visible), _ptr(ws), ws_bytes, stream))


def gs_sort(n, keys, ids, n_visible, ws, ws_bytes, stream):
    _check("gs_sort", lib().gs_sort(n, _ptr(keys), _ptr(ids), _ptr(n_visible), _ptr(ws),
                                    ws_bytes, stream))


def gs_sort_noalloc(n, keys, ids, n_visible, stream):
    _check("gs_sort_noalloc", lib().gs_sort_noalloc(n, _ptr(keys), _ptr(ids), _ptr(n_visible),
                                                    stream))


NOALLOC_SORT_MAX_N = 1 << 22


def gs_sort_views(n_views, n, keys, ids, n_visible, ws, ws_bytes, stream):
    _check("gs_sort_views", lib().gs_sort_views(n_views, n, _ptr(keys), _ptr(ids), _ptr(n_visible),
                                                _ptr(ws), ws_bytes, stream))


def gs_raster_setup(cam: GsCamera, cfg: GsConfig, n, sorted_ids, n_visible, means2d, conics,
                    opacities, rgb, ws, ws_bytes, stream):
    _check("gs_raster_setup", lib().gs_raster_setup(
        ctypes.byref(cam), ctypes.byref(cfg), n, _ptr(sorted_ids), _ptr(n_visible),
        _ptr(means2d), _ptr(conics), _ptr(opacities), _ptr(rgb), _ptr(ws), ws_bytes, stream))


def gs_raster_fwd(cam: GsCamera, cfg: GsConfig, n, sorted_ids, n_visible, means2d, conics,
                  opacities, rgb, fb, out_rgb, out_T, out_coverage, stats, ws, ws_bytes, stream):
    _check("gs_raster_fwd", lib().gs_raster_fwd(
        ctypes.byref(cam), ctypes.byref(cfg), n, _ptr(sorted_ids), _ptr(n_visible),
        _ptr(means2d), _ptr(conics), _ptr(opacities), _ptr(rgb), _ptr(fb), _ptr(out_rgb),
        _ptr(out_T), _ptr(out_coverage), _ptr(stats), _ptr(ws), ws_bytes, stream))


def gs_raster_bwd(cam: GsCamera, cfg: GsConfig, n, sorted_ids, n_visible, means2d, conics,
                  opacities, rgb, fb, dL_dimage, dL_dmeans2d, dL_dconics, dL_dopacities, dL_drgb,
                  dL_dT, dL_dbackground, out_live, stats, ws, ws_bytes, stream):
    _check("gs_raster_bwd", lib().gs_raster_bwd(
        ctypes.byref(cam), ctypes.byref(cfg), n, _ptr(sorted_ids), _ptr(n_visible),
        _ptr(means2d), _ptr(conics), _ptr(opacities), _ptr(rgb), _ptr(fb), _ptr(dL_dimage),
        _ptr(dL_dmeans2d), _ptr(dL_dconics), _ptr(dL_dopacities), _ptr(dL_drgb), _ptr(dL_dT),
        _ptr(dL_dbackground), _ptr(out_live), _ptr(stats), _ptr(ws), ws_bytes, stream))


def gs_preprocess_bwd(cam: GsCamera, cfg: GsConfig, n, means3d, scales, quats, opacities, sh,
                      dL_dmeans2d, dL_dconics, dL_drgb, dL_dopacities2d, dL_dmeans3d, dL_dscales,
                      dL_dquats, dL_dopacities, dL_dsh, stream):
    _check("gs_preprocess_bwd", lib().gs_preprocess_bwd(
        _cam(cam), ctypes.byref(cfg), n, _ptr(means3d), _ptr(scales), _ptr(quats),
        _ptr(opacities), _ptr(sh), _ptr(dL_dmeans2d), _ptr(dL_dconics), _ptr(dL_drgb),
        _ptr(dL_dopacities2d), _ptr(dL_dmeans3d), _ptr(dL_dscales), _ptr(dL_dquats),
        _ptr(dL_dopacities), _ptr(dL_dsh), stream))


def gs_raster_status(cfg: GsConfig, n, width, height, ws, ws_bytes, stream) -> int:
    """The raster's device status word (waits for the stream); raises GsrError when non-zero."""
    word = ctypes.c_uint32(0)
    _check("gs_raster_status", lib().gs_raster_status(ctypes.byref(cfg), n, width, height,
                                                      _ptr(ws), ws_bytes, ctypes.byref(word),
                                                      stream))
    return int(word.value)


def gs_raster_debug_schedule(cfg: GsConfig, n, width, height, ws, ws_bytes, fwd_order, bwd_order,
                             item_order, items, n_items, stream):
    _check("gs_raster_debug_schedule", lib().gs_raster_debug_schedule(
        ctypes.byref(cfg), n, width, height, _ptr(ws), ws_bytes, _ptr(fwd_order), _ptr(bwd_order),
        _ptr(item_order), _ptr(items), _ptr(n_items), stream))


MICRO_THREADS = 1 << 20
MICRO_ATOMIC = {"spread": 0, "spread_return": 1, "wave_same": 2}


def gs_micro_copy(src, dst, nbytes, stream):
    _check("gs_micro_copy", lib().gs_micro_copy(_ptr(src), _ptr(dst), nbytes, stream))


def gs_micro_atomic_f32(slots, nslots, adds_per_thread, mode, stream):
    m = MICRO_ATOMIC[mode] if isinstance(mode, str) else mode
    _check("gs_micro_atomic_f32", lib().gs_micro_atomic_f32(_ptr(slots), nslots, adds_per_thread,
                                                            m, stream))


def gs_tile_workspace_size(n, pair_capacity, width, height) -> int:
    return int(lib().gs_tile_workspace_size(n, pair_capacity, width, height))


def gs_tile_prepare(cam: GsCamera, cfg: GsConfig, n, ids, n_visible, means2d, conics, opacities,
                    n_pairs, ws, ws_bytes, stream):
    _check("gs_tile_prepare", lib().gs_tile_prepare(
        ctypes.byref(cam), ctypes.byref(cfg), n, _ptr(ids), _ptr(n_visible), _ptr(means2d),
        _ptr(conics), _ptr(opacities), _ptr(n_pairs), _ptr(ws), ws_bytes, stream))


def gs_tile_raster_fwd(cam: GsCamera, cfg: GsConfig, n, ids, keys, means2d, conics, opacities, rgb,
                       n_pairs, pair_capacity, out_rgb, out_T, n_contrib, ws, ws_bytes, stream):
    _check("gs_tile_raster_fwd", lib().gs_tile_raster_fwd(
        ctypes.byref(cam), ctypes.byref(cfg), n, _ptr(ids), _ptr(keys), _ptr(means2d),
        _ptr(conics), _ptr(opacities), _ptr(rgb), _ptr(n_pairs), pair_capacity, _ptr(out_rgb),
        _ptr(out_T), _ptr(n_contrib), _ptr(ws), ws_bytes, stream))


def gs_tile_raster_bwd(cam: GsCamera, cfg: GsConfig, n, means2d, conics, opacities, rgb,
                       dL_dimage, T_final, n_contrib, pair_capacity, dL_dmeans2d, dL_dconics,
                       dL_dopacities, dL_drgb, ws, ws_bytes, stream):
    _check("gs_tile_raster_bwd", lib().gs_tile_raster_bwd(
        ctypes.byref(cam), ctypes.byref(cfg), n, _ptr(means2d), _ptr(conics), _ptr(opacities),
        _ptr(rgb), _ptr(dL_dimage), _ptr(T_final), _ptr(n_contrib), pair_capacity,
        _ptr(dL_dmeans2d), _ptr(dL_dconics), _ptr(dL_dopacities), _ptr(dL_drgb), _ptr(ws),
        ws_bytes, stream))
