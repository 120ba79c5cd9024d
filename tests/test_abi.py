"""C-ABI checks that need no GPU: the library loads, exports every function include/gsr.h
declares, reports the paper's defaults, sizes its buffers by closed forms, and rejects invalid
arguments on the host before any HIP call (so these calls never touch a device)."""
import ctypes
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsr.h")
LIB = os.path.join(ROOT, "paper_2505_18764_amd", "libgsr.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libgsr.so not built")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    from paper_2505_18764_amd import _lib as L
    names = _declared()
    assert len(names) >= 14
    cdll = ctypes.CDLL(LIB)
    for nm in names:
        assert hasattr(cdll, nm), nm
    assert set(names) == set(L.exported_symbols())    # the binding covers the same names


_CSIZE = {"float": 4, "int32_t": 4, "uint32_t": 4, "double": 8, "unsigned long long": 8}


def _header_structs():
    """{struct name: [(field, bytes)]} for the header's plain typedef structs."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"typedef struct (\w+) \{(.*?)\} \1;", src, flags=re.S):
        fields = []
        for stmt in m.group(2).split(";"):
            stmt = " ".join(stmt.split())
            if not stmt:
                continue
            tm = re.match(r"(unsigned long long|float|int32_t|uint32_t|double) (.*)", stmt)
            assert tm, stmt
            for part in tm.group(2).split(","):
                am = re.fullmatch(r"(\w+)(?:\[(\d+)\])?", part.strip())
                assert am, part
                fields.append((am.group(1), _CSIZE[tm.group(1)] * int(am.group(2) or 1)))
        out[m.group(1)] = fields
    return out


def test_ctypes_structs_match_the_header():
    from paper_2505_18764_amd import _lib as L
    hs = _header_structs()
    for cname, py in (("gs_camera", L.GsCamera), ("gs_config", L.GsConfig),
                      ("gs_stats", L.GsStats)):
        got = [(name, ctypes.sizeof(t)) for name, t in py._fields_]
        assert got == hs[cname], cname
        assert ctypes.sizeof(py) == sum(b for _, b in hs[cname]), cname
    assert ctypes.sizeof(L.GsStats) == 16 * 8


def test_defaults_are_the_papers_constants():
    from paper_2505_18764_amd import _lib as L
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_constants.json")))
    c = L.gs_config_default()
    assert c.alpha_min == pytest.approx(g["alpha_min"]["value"], rel=1e-7)
    assert c.t_min_bwd == pytest.approx(g["t_min_bwd"]["value"], rel=1e-6)
    assert c.reduce_threshold == g["reduce_threshold_hybrid"]["value"]
    assert c.t_min_fwd == 0.0 and c.reduce_mode == L.REDUCE_MODES["hybrid"]
    assert L.gs_version() == 1


def test_sizes_are_closed_forms():
    from paper_2505_18764_amd import _lib as L
    c = L.gs_config_default()
    assert L.gs_framebuffer_size(100, 70, "f32") == 100 * 70 * 16
    assert L.gs_framebuffer_size(100, 70, "f16") == 100 * 70 * 8
    assert L.gs_framebuffer_size(100, 70, "unorm8") == 100 * 70 * 4
    assert L.gs_framebuffer_size(0, 70, "f16") == 0
    for op in ("preprocess", "sort", "raster_fwd", "raster_bwd", "all"):
        prev = -1
        for n in (0, 1, 1000, 200_000, 1_000_000, 3_000_000):
            v = L.gs_workspace_size(op, n, 1600, 1064, c)
            assert v >= prev
            prev = v
        a = L.gs_workspace_size(op, 10_000, 640, 480, c)
        b = L.gs_workspace_size(op, 10_000, 1920, 1080, c)
        assert b >= a
    allb = L.gs_workspace_size("all", 1_000_000, 1600, 1064, c)
    for op in ("preprocess", "sort", "raster_fwd", "raster_bwd"):
        assert L.gs_workspace_size(op, 1_000_000, 1600, 1064, c) <= allb
    assert L.gs_workspace_size("raster_fwd", -1, 10, 10, c) == 0
    assert L.gs_workspace_size("raster_fwd", 10, 0, 10, c) == 0
    # fixed O(N + pixels) memory at the 1M / 1600x1064 view (records and gradient slots per splat,
    # bitmap, depth-split partial states): under 256 MiB
    assert allb < 256 << 20
    assert L.gs_tile_workspace_size(1000, 5000, 128, 128) > L.gs_tile_workspace_size(1000, 0, 128, 128)


def _cam(L, w=64, h=48):
    c = L.GsCamera()
    c.viewmat[0] = c.viewmat[5] = c.viewmat[10] = 1.0
    c.fx = c.fy = 50.0
    c.cx, c.cy, c.width, c.height, c.znear = w / 2, h / 2, w, h, 0.2
    return c


def test_invalid_arguments_rejected_on_host():
    from paper_2505_18764_amd import _lib as L
    cfg = L.gs_config_default()
    cam = _cam(L)
    fake = 0x1000    # never dereferenced: validation fails first
    buf = (ctypes.c_char * 4096)()
    ws = ctypes.addressof(buf) + (-ctypes.addressof(buf)) % 256

    def raster(cam_, cfg_, n=10, nvis=fake, fb=fake, ws_=ws, wsb=16):
        return L.lib().gs_raster_fwd(ctypes.byref(cam_) if cam_ is not None else None,
                                     ctypes.byref(cfg_), n, fake, nvis, fake, fake, fake, fake, fb,
                                     None, None, None, None, ws_, wsb, None)

    assert raster(None, cfg) == 1 and "camera" in L.gs_last_error()
    bad = _cam(L, w=0)
    assert raster(bad, cfg) == 1 and "image" in L.gs_last_error()
    for field, val in (("fb_format", 9), ("fb_round", 5), ("reduce_mode", 11),
                       ("reduce_threshold", 65), ("sh_degree", 4), ("flags", 8)):
        c2 = L.gs_config_default()
        setattr(c2, field, val)
        assert raster(cam, c2) == 1, field
    c2 = L.gs_config_default()
    c2.alpha_min = 0.0
    assert raster(cam, c2) == 1
    c2 = L.gs_config_default()
    c2.alpha_max = 1.5
    assert raster(cam, c2) == 1
    assert raster(cam, cfg, n=-3) == 1
    assert raster(cam, cfg, nvis=None) == 1 and "n_visible" in L.gs_last_error()
    assert raster(cam, cfg, fb=None) == 1
    assert raster(cam, cfg, ws_=None, wsb=0) == 1
    assert raster(cam, cfg, wsb=16) == 2 and "workspace" in L.gs_last_error()  # GS_ERR_CAPACITY
    assert raster(cam, cfg, ws_=ws + 4, wsb=1 << 30) == 1                       # misaligned
    assert L.lib().gs_sort(-1, None, None, fake, None, 0, None) == 1
    assert L.lib().gs_preprocess(ctypes.byref(cam), ctypes.byref(cfg), 5, None, None, None, None,
                                 None, None, None, None, None, None, None, fake, ws, 1 << 20,
                                 None) == 1
    f = fake
    assert L.lib().gs_preprocess(ctypes.byref(cam), ctypes.byref(cfg), 5, f, f, f, f, f + 4, f, f, f,
                                 f, f, f, f, ws, 1 << 20, None) == 1
    assert "aligned" in L.gs_last_error()                  # sh: 16-byte aligned
    cz = _cam(L)
    cz.znear = 0.0
    assert L.lib().gs_preprocess_bwd(ctypes.byref(cz), ctypes.byref(cfg), 0, *([None] * 14),
                                     None) == 1
    # the status query and the schedule copy validate before touching the device
    word = ctypes.c_uint32(7)
    assert L.lib().gs_raster_status(ctypes.byref(cfg), 10, 64, 48, ws, 16, ctypes.byref(word),
                                    None) == 2                    # workspace too small
    assert L.lib().gs_raster_status(ctypes.byref(cfg), 10, 64, 48, ws, 1 << 30, None, None) == 1
    assert L.lib().gs_raster_status(ctypes.byref(cfg), 10, 0, 48, ws, 1 << 30, ctypes.byref(word),
                                    None) == 1
    assert word.value == 7                                        # untouched on failure
    assert L.lib().gs_raster_debug_schedule(ctypes.byref(cfg), 10, 64, 48, None, 0, f, f, None,
                                            None, None, None) == 1
    big = 100 * 32                                                # > 4096 tiles: no depth split
    assert L.lib().gs_raster_debug_schedule(ctypes.byref(cfg), 10, big, big, ws, 1 << 40, None,
                                            None, f, None, None, None) == 3


def test_view_batches_checked_on_host():
    """Several views per call: the view count, the cameras' common image size, the per-view
    workspace slabs and the entry points that take one view only are checked before any launch."""
    from paper_2505_18764_amd import _lib as L
    c1 = L.gs_config_default()
    for V in (2, 5, 16):
        cv = L.gs_config_default()
        cv.n_views = V
        for op in ("preprocess", "sort", "raster_fwd", "raster_bwd", "all"):
            one = L.gs_workspace_size(op, 12_345, 640, 480, c1)
            assert L.gs_workspace_size(op, 12_345, 640, 480, cv) == V * ((one + 255) // 256 * 256)
    cv = L.gs_config_default()
    cv.n_views = 17
    assert L.gs_workspace_size("raster_fwd", 100, 64, 48, cv) == 0
    fake = 0x1000
    buf = (ctypes.c_char * 8192)()
    ws = ctypes.addressof(buf) + (-ctypes.addressof(buf)) % 256
    f = fake
    # too many views
    assert L.lib().gs_raster_fwd(ctypes.byref(_cam(L)), ctypes.byref(cv), 10, f, f, f, f, f, f, f,
                                 None, None, None, None, ws, 4096, None) == 1
    assert "n_views" in L.gs_last_error()
    assert L.lib().gs_sort_views(0, 10, f, f, f, ws, 4096, None) == 1
    assert L.lib().gs_sort_views(17, 10, f, f, f, ws, 4096, None) == 1
    # each view's slab must hold the one-view size
    need = L.gs_workspace_size("sort", 5000, 64, 48, c1)
    assert L.lib().gs_sort_views(4, 5000, f, f, f, ws, 4 * need - 4096, None) == 2
    assert "slab" in L.gs_last_error()
    # cameras of one call share the image size
    cv.n_views = 2
    cams = L.camera_array([_cam(L, 64, 48), _cam(L, 64, 40)])
    assert L.lib().gs_preprocess(cams, ctypes.byref(cv), 5, f, f, f, f, f, f, f, f,
                                 f, f, f, f, ws, 1 << 30, None) == 1
    assert "image size" in L.gs_last_error()
    cams = L.camera_array([_cam(L), _cam(L)])
    cams[1].znear = 0.0
    assert L.lib().gs_preprocess_bwd(cams, ctypes.byref(cv), 0, *([None] * 14),
                                     None) == 1
    # one view only: the 2D entry and the tile-based baseline
    cam = _cam(L)
    assert L.lib().gs_prepare_2d(ctypes.byref(cam), ctypes.byref(cv), 5, f, f, f, f, f, f, f, ws,
                                 1 << 20, None) == 3
    assert L.lib().gs_tile_prepare(ctypes.byref(cam), ctypes.byref(cv), 5, f, f, f, f, f, f, ws,
                                   1 << 20, None) == 3
