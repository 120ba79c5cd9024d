"""Torch-facing layer over the C ABI: configuration, workspaces, the five pipeline stages and the
autograd Functions.

PyTorch only supplies device memory and the current stream; every step of the method runs in the
HIP library. Passing a list of cameras renders those views of one scene in the same launches
(the library's view batching): per-view tensors then carry a leading view dimension, and the
backward sums the views' gradients w.r.t. the shared 3D parameters. The forward state kept for the backward is O(N) splat records plus the O(W H)
framebuffer: nothing per fragment is stored, the backward rematerialises each fragment from the
framebuffer state (Procedure 1).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import _lib as L


def _f32(x):
    return float(np.float32(x))


@dataclasses.dataclass
class RasterConfig:
    """Method constants and switches (mirrors gs_config). Defaults are the paper's: alpha_min
    1/255, backward T-cull 1e-4, no forward T-cull, hybrid reduction with X = 8, FP32 state."""
    fb_format: str = "f32"            # f32 | f16 | unorm16 | bf16 | unorm8
    fb_round: str = "at_rest"         # at_rest | per_fragment
    reduce_mode: str = "hybrid"       # naive | quad | wave | hybrid | hybrid_lane | tile
    reduce_threshold: int = 8
    t_min_fwd: float = 0.0
    t_min_bwd: float = _f32(1e-4)
    alpha_min: float = _f32(1.0 / 255.0)
    alpha_max: float = _f32(0.99)
    eps2d: float = _f32(0.3)
    sh_degree: int = 3
    stats: bool = False
    background: tuple = (0.0, 0.0, 0.0)   # C += T_final background (zero: Eq. 2 as printed)
    composite_all: bool = False           # forward: no saturation exit (GS_FLAG_COMPOSITE_ALL)

    def c(self, n_views: int = 1) -> L.GsConfig:
        c = L.GsConfig()
        c.alpha_min = self.alpha_min
        c.alpha_max = self.alpha_max
        c.t_min_fwd = self.t_min_fwd
        c.t_min_bwd = self.t_min_bwd
        c.eps2d = self.eps2d
        c.sh_degree = self.sh_degree
        c.fb_format = L.FB_FORMATS[self.fb_format]
        c.fb_round = L.FB_ROUND[self.fb_round]
        c.reduce_mode = L.REDUCE_MODES[self.reduce_mode]
        c.reduce_threshold = self.reduce_threshold
        c.flags = (1 if self.stats else 0) | (4 if self.composite_all else 0)
        for k in range(3):
            c.background[k] = float(self.background[k])
        c.n_views = int(n_views)
        return c


def is_views(cam) -> bool:
    """A list or tuple of cameras (several views per call) rather than one camera."""
    return isinstance(cam, (list, tuple))


def cameras_c(cam):
    """(gs_camera or an array of them, number of views) for one camera or a list of cameras."""
    if is_views(cam):
        if not 1 <= len(cam) <= L.MAX_VIEWS:
            raise ValueError(f"1..{L.MAX_VIEWS} views per call, got {len(cam)}")
        return L.camera_array([camera_c(c) for c in cam]), len(cam)
    return camera_c(cam), 1


def camera_c(cam) -> L.GsCamera:
    """gs_camera from any object with viewmat (3x4), fx, fy, cx, cy, width, height, znear."""
    c = L.GsCamera()
    vm = np.asarray(cam.viewmat, dtype=np.float32).reshape(-1)
    for i in range(12):
        c.viewmat[i] = float(vm[i])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.znear = float(getattr(cam, "znear", 0.2))
    return c


class _Size:
    def __init__(self, width, height):
        self.width, self.height = int(width), int(height)


def image_camera(width, height) -> L.GsCamera:
    """A camera that carries only the image size (for the 2D entry points)."""
    c = L.GsCamera()
    c.viewmat[0] = c.viewmat[5] = c.viewmat[10] = 1.0
    c.fx = c.fy = 1.0
    c.width, c.height, c.znear = int(width), int(height), 0.2
    return c


class Workspace:
    """A growing device scratch buffer (256-byte aligned). Reused across calls on one stream;
    its size only depends on (n, width, height, format), see gs_workspace_size."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.buf = None
        self.setup_owner = None     # who built the raster setup the buffer holds (see own_setup)

    def get(self, nbytes: int, keep: bool = False):
        """A buffer of at least nbytes; with keep, a grown buffer starts with the old contents."""
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes:
            new = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            if keep and self.buf is not None:
                new[: self.buf.numel()].copy_(self.buf)
            else:
                self.setup_owner = None
            self.buf = new
        return self.buf

    def own_setup(self):
        """A token for the raster setup about to be built in this buffer; holds_setup(token)
        stays true until another setup is built here or the buffer is replaced."""
        self.setup_owner = object()
        return self.setup_owner

    def holds_setup(self, token) -> bool:
        return token is not None and self.setup_owner is token

    @property
    def nbytes(self) -> int:
        return 0 if self.buf is None else self.buf.numel()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ws_args(ws: Workspace, need: int, keep_setup: bool = False):
    """The workspace buffer for a call that needs `need` bytes. Every call writes scratch over the
    buffer's front, where a raster setup lives, so the setup's ownership ends here unless the
    call reads that setup (keep_setup)."""
    b = ws.get(need)
    if not keep_setup:
        ws.setup_owner = None
    return b, b.numel()


@dataclasses.dataclass
class Projected:
    """Splats in screen space plus the depth-sorted (keys, ids) and the device-side count of
    visible splats. For V views of one scene every per-view tensor has a leading dimension V
    (means2d [V,n,2], keys [V,n], n_visible [V], ...); opacities stay [n]."""
    means2d: torch.Tensor
    conics: torch.Tensor
    rgb: torch.Tensor
    opacities: torch.Tensor
    depth: torch.Tensor
    keys: torch.Tensor
    ids: torch.Tensor
    n_visible: torch.Tensor
    width: int
    height: int

    @property
    def n(self) -> int:
        return int(self.means2d.shape[-2])

    @property
    def n_views(self) -> int:
        return 1 if self.means2d.dim() == 2 else int(self.means2d.shape[0])

    def lead(self):
        """Leading shape of per-view tensors: () for one view, (V,) for several."""
        return () if self.means2d.dim() == 2 else (self.n_views,)


def _c32(t):
    assert t.is_cuda and t.dtype == torch.float32, "expected a float32 CUDA tensor"
    return t.contiguous()


def project(means3d, scales, quats, opacities, sh, cam, cfg: RasterConfig, ws: Workspace,
            sort: bool = True) -> Projected:
    """gs_preprocess (projection, SH colour, culling, keys) then gs_sort. cam: one camera, or a
    list of cameras of equal image size (one batched call; outputs [V, n, ..])."""
    dev = means3d.device
    n = int(means3d.shape[0])
    cm, V = cameras_c(cam)
    cc = cfg.c(V)
    lead = (V,) if is_views(cam) else ()
    means3d, scales, quats, opacities, sh = map(_c32, (means3d, scales, quats, opacities, sh))
    out = dict(means2d=torch.empty(*lead, n, 2, device=dev),
               conics=torch.empty(*lead, n, 3, device=dev),
               rgb=torch.empty(*lead, n, 3, device=dev), depth=torch.empty(*lead, n, device=dev),
               keys=torch.empty(*lead, n, dtype=torch.int32, device=dev),
               ids=torch.empty(*lead, n, dtype=torch.int32, device=dev),
               n_visible=torch.empty(V, dtype=torch.int32, device=dev))   # written by the call
    cm0 = cm[0] if is_views(cam) else cm
    b, nb = _ws_args(ws, max(L.gs_workspace_size("preprocess", n, cm0.width, cm0.height, cc), 256))
    L.gs_preprocess(cm, cc, n, means3d, scales, quats, opacities, sh, out["means2d"],
                    out["conics"], out["rgb"], out["depth"], out["keys"], out["ids"],
                    out["n_visible"], b, nb, _stream(dev))
    p = Projected(opacities=opacities, width=cm0.width, height=cm0.height, **out)
    if sort:
        sort_(p, ws)
    return p


def prepare_2d(means2d, conics, opacities, rgb, depth, width, height, cfg: RasterConfig,
               ws: Workspace, sort: bool = True) -> Projected:
    """gs_prepare_2d (keys and culling for pre-projected splats) then gs_sort."""
    dev = means2d.device
    n = int(means2d.shape[0])
    cc, cm = cfg.c(), image_camera(width, height)
    means2d, conics, opacities, rgb, depth = map(_c32, (means2d, conics, opacities, rgb, depth))
    keys = torch.empty(n, dtype=torch.int32, device=dev)
    ids = torch.empty(n, dtype=torch.int32, device=dev)
    nvis = torch.empty(1, dtype=torch.int32, device=dev)            # written by the call
    b, nb = _ws_args(ws, L.gs_workspace_size("prepare_2d", n, width, height, cc))
    L.gs_prepare_2d(cm, cc, n, means2d, conics, opacities, depth, keys, ids, nvis, b, nb,
                    _stream(dev))
    p = Projected(means2d=means2d, conics=conics, rgb=rgb, opacities=opacities, depth=depth,
                  keys=keys, ids=ids, n_visible=nvis, width=width, height=height)
    if sort:
        sort_(p, ws)
    return p


def sort_(p: Projected, ws: Workspace):
    """gs_sort (gs_sort_views for several views): stable depth sort of the visible prefix of
    (keys, ids), in place."""
    n, V = p.n, p.n_views
    cc = L.GsConfig()
    cc.n_views = V
    b, nb = _ws_args(ws, L.gs_workspace_size("sort", n, p.width, p.height, cc))
    if p.lead():
        L.gs_sort_views(V, n, p.keys, p.ids, p.n_visible, b, nb, _stream(p.keys.device))
    else:
        L.gs_sort(n, p.keys, p.ids, p.n_visible, b, nb, _stream(p.keys.device))


def new_stats(device):
    """Zeroed gs_stats block on the device (16 x uint64)."""
    return torch.zeros(16, dtype=torch.int64, device=device)


def read_stats(t) -> dict:
    v = t.cpu().numpy().astype(np.uint64)
    return {k: int(v[i]) for i, k in enumerate(L.STATS_FIELDS)}


FB_BYTES = {"f32": 16, "f16": 8, "unorm16": 8, "bf16": 8, "unorm8": 4}


def raster_setup(p: Projected, cfg: RasterConfig, ws: Workspace):
    """gs_raster_setup: builds the records, bitmap and tile schedule that a following
    raster_forward / raster_backward with reuse_setup=True on the same workspace share. The
    workspace is sized for the backward here, so those calls never regrow (and lose) it.
    Returns the workspace's ownership token of this setup (Workspace.holds_setup)."""
    dev = p.means2d.device
    W, H, n = p.width, p.height, p.n
    cc, cm = cfg.c(p.n_views), image_camera(W, H)
    b, nb = _ws_args(ws, L.gs_workspace_size("raster_bwd", n, W, H, cc))
    token = ws.own_setup()
    L.gs_raster_setup(cm, cc, n, p.ids, p.n_visible, p.means2d, p.conics, p.opacities, p.rgb, b, nb,
                      _stream(dev))
    return token


def raster_forward(p: Projected, cfg: RasterConfig, ws: Workspace, fb=None, image=None, T=None,
                   coverage=False, stats=None, reuse_setup=False):
    """gs_raster_fwd: returns dict(fb, image [3,H,W], T [H,W], coverage [H,W] or None), each with
    a leading view dimension for several views.
    reuse_setup: the workspace holds raster_setup's output for exactly these inputs."""
    dev = p.means2d.device
    W, H, n = p.width, p.height, p.n
    lead = p.lead()
    cc, cm = cfg.c(p.n_views), image_camera(W, H)
    if reuse_setup:
        cc.flags |= 2
    if fb is None:
        fb = torch.empty(*lead, L.gs_framebuffer_size(W, H, cfg.fb_format), dtype=torch.uint8,
                         device=dev)
    if image is None:
        image = torch.empty(*lead, 3, H, W, device=dev)
    if T is None:
        T = torch.empty(*lead, H, W, device=dev)
    cov = torch.empty(*lead, H, W, dtype=torch.int32, device=dev) if coverage else None
    if stats is not None:
        cc.flags |= 1
    b, nb = _ws_args(ws, L.gs_workspace_size("raster_fwd", n, W, H, cc), keep_setup=reuse_setup)
    L.gs_raster_fwd(cm, cc, n, p.ids, p.n_visible, p.means2d, p.conics, p.opacities, p.rgb, fb,
                    image, T, cov, stats, b, nb, _stream(dev))
    return dict(fb=fb, image=image, T=T, coverage=cov)


def raster_backward(p: Projected, fb, dL_dimage, cfg: RasterConfig, ws: Workspace, live=False,
                    stats=None, out=None, reuse_setup=False, dL_dT=None):
    """gs_raster_bwd: gradients w.r.t. (means2d, conics, opacities, rgb) by splat id and w.r.t.
    the background ('background' [3]); dL_dT [H, W] is an optional gradient of the final T.
    For several views the 2D gradients are per view ([V, n, ..]) and the background's is their sum.
    reuse_setup: the workspace holds raster_setup's output for exactly these inputs."""
    dev = p.means2d.device
    W, H, n = p.width, p.height, p.n
    lead = p.lead()
    cc, cm = cfg.c(p.n_views), image_camera(W, H)
    if reuse_setup:
        cc.flags |= 2
    if out is None:
        out = dict(means2d=torch.empty(*lead, n, 2, device=dev),
                   conics=torch.empty(*lead, n, 3, device=dev),
                   opacities=torch.empty(*lead, n, device=dev),
                   rgb=torch.empty(*lead, n, 3, device=dev))
    if "background" not in out:
        out["background"] = torch.empty(3, device=dev)
    lv = torch.empty(*lead, H, W, dtype=torch.int32, device=dev) if live else None
    if stats is not None:
        cc.flags |= 1
    b, nb = _ws_args(ws, L.gs_workspace_size("raster_bwd", n, W, H, cc), keep_setup=reuse_setup)
    L.gs_raster_bwd(cm, cc, n, p.ids, p.n_visible, p.means2d, p.conics, p.opacities, p.rgb, fb,
                    _c32(dL_dimage), out["means2d"], out["conics"], out["opacities"], out["rgb"],
                    None if dL_dT is None else _c32(dL_dT), out["background"], lv, stats, b, nb,
                    _stream(dev))
    out["live"] = lv
    return out


def raster_status(p: Projected, cfg: RasterConfig, ws: Workspace) -> int:
    """gs_raster_status: waits for the stream and raises GsrError (GS_ERR_STATE) if a raster
    kernel met a splat id or a schedule entry outside its range since the last raster setup on
    this workspace; returns the (zero) status word."""
    cc = cfg.c(p.n_views)
    b = ws.buf
    return L.gs_raster_status(cc, p.n, p.width, p.height, b, 0 if b is None else b.numel(),
                              _stream(p.means2d.device))


def raster_schedule(p: Projected, cfg: RasterConfig, ws: Workspace, items: bool = False) -> dict:
    """gs_raster_debug_schedule: the tile orders of the forward and the backward ([T] each, or
    [V, T]) and, with items, the depth split's work items ([4T] order, [4T, 4] items, item count)."""
    dev = p.means2d.device
    T = ((p.width + 31) // 32) * ((p.height + 31) // 32)
    lead = p.lead()
    out = dict(fwd_order=torch.empty(*lead, T, dtype=torch.int32, device=dev),
               bwd_order=torch.empty(*lead, T, dtype=torch.int32, device=dev))
    if items:
        out.update(item_order=torch.empty(*lead, 4 * T, dtype=torch.int32, device=dev),
                   items=torch.empty(*lead, 4 * T, 4, dtype=torch.int32, device=dev),
                   n_items=torch.empty(*lead, 1, dtype=torch.int64, device=dev))
    b = ws.buf
    L.gs_raster_debug_schedule(cfg.c(p.n_views), p.n, p.width, p.height, b, b.numel(),
                               out["fwd_order"], out["bwd_order"], out.get("item_order"),
                               out.get("items"), out.get("n_items"), _stream(dev))
    return out


def project_backward(means3d, scales, quats, opacities, sh, cam, cfg: RasterConfig, g2d: dict,
                     out=None):
    """gs_preprocess_bwd: gradients w.r.t. the 3D Gaussian parameters; for a list of cameras, the
    sum over the views of g2d's [V, n, ..] gradients (accumulated on the device in view order)."""
    dev = means3d.device
    n = int(means3d.shape[0])
    cm, V = cameras_c(cam)
    cc = cfg.c(V)
    if out is None:
        out = dict(means3d=torch.empty_like(means3d), scales=torch.empty_like(scales),
                   quats=torch.empty_like(quats), opacities=torch.empty_like(opacities),
                   sh=torch.empty_like(sh))
    L.gs_preprocess_bwd(cm, cc, n, _c32(means3d), _c32(scales), _c32(quats), _c32(opacities),
                        _c32(sh), g2d["means2d"], g2d["conics"], g2d["rgb"], g2d["opacities"],
                        out["means3d"], out["scales"], out["quats"], out["opacities"], out["sh"],
                        _stream(dev))
    return out


# ---- autograd -------------------------------------------------------------------------------

class GaussianRasterizeFn(torch.autograd.Function):
    """image, T = f(means3d, scales, quats, opacities, sh): projection, depth sort, ordered
    compositing (over cfg.background); the backward runs Procedures 1-2 and the projection's
    backward. Activations (exp of log-scales, sigmoid of logits) stay in torch, outside this
    function. A loss on the final T (e.g. an alpha mask) reaches the splats through dL/dT.
    With a list of cameras the views render in the same launches (image [V,3,H,W], T [V,H,W])
    and the backward returns the sum of the views' gradients."""

    @staticmethod
    def forward(ctx, means3d, scales, quats, opacities, sh, cam, cfg, ws):
        ctx.set_materialize_grads(False)
        p = project(means3d, scales, quats, opacities, sh, cam, cfg, ws)
        ctx.setup = raster_setup(p, cfg, ws)
        out = raster_forward(p, cfg, ws, reuse_setup=True)
        ctx.cam, ctx.cfg, ctx.ws, ctx.proj = cam, cfg, ws, p
        ctx.save_for_backward(means3d, scales, quats, opacities, sh, out["fb"])
        return out["image"], out["T"]

    @staticmethod
    def backward(ctx, d_image, d_T):
        means3d, scales, quats, opacities, sh, fb = ctx.saved_tensors
        if d_image is None:
            d_image = torch.zeros(*ctx.proj.lead(), 3, ctx.proj.height, ctx.proj.width,
                                  device=fb.device)
        g2 = raster_backward(ctx.proj, fb, d_image.contiguous(), ctx.cfg, ctx.ws, dL_dT=d_T,
                             reuse_setup=ctx.ws.holds_setup(ctx.setup))
        g3 = project_backward(means3d, scales, quats, opacities, sh, ctx.cam, ctx.cfg, g2)
        return g3["means3d"], g3["scales"], g3["quats"], g3["opacities"], g3["sh"], None, None, None


class Raster2DFn(torch.autograd.Function):
    """image, T = f(means2d, conics, opacities, rgb; depth) for splats that are already 2D."""

    @staticmethod
    def forward(ctx, means2d, conics, opacities, rgb, depth, width, height, cfg, ws):
        ctx.set_materialize_grads(False)
        p = prepare_2d(means2d, conics, opacities, rgb, depth, width, height, cfg, ws)
        ctx.setup = raster_setup(p, cfg, ws)
        out = raster_forward(p, cfg, ws, reuse_setup=True)
        ctx.cfg, ctx.ws, ctx.proj = cfg, ws, p
        ctx.save_for_backward(out["fb"])
        return out["image"], out["T"]

    @staticmethod
    def backward(ctx, d_image, d_T):
        (fb,) = ctx.saved_tensors
        if d_image is None:
            d_image = torch.zeros(3, ctx.proj.height, ctx.proj.width, device=fb.device)
        g = raster_backward(ctx.proj, fb, d_image.contiguous(), ctx.cfg, ctx.ws, dL_dT=d_T,
                            reuse_setup=ctx.ws.holds_setup(ctx.setup))
        return g["means2d"], g["conics"], g["opacities"], g["rgb"], None, None, None, None, None


def rasterize_gaussians(means3d, scales, quats, opacities, sh, cam, cfg=None, ws=None):
    cfg = cfg or RasterConfig()
    ws = ws or Workspace(means3d.device)
    return GaussianRasterizeFn.apply(means3d, scales, quats, opacities, sh, cam, cfg, ws)


def rasterize_2d(means2d, conics, opacities, rgb, depth, width, height, cfg=None, ws=None):
    cfg = cfg or RasterConfig()
    ws = ws or Workspace(means2d.device)
    return Raster2DFn.apply(means2d, conics, opacities, rgb, depth, width, height, cfg, ws)


# ---- tile-based comparison rasterizer --------------------------------------------------------

def tile_forward(p: Projected, cfg: RasterConfig, ws: Workspace, out=None):
    """gs_tile_prepare, host readback of the pair count (the dynamic allocation), then
    gs_tile_raster_fwd. Returns dict(image, T, n_contrib, n_pairs, capacity)."""
    dev = p.means2d.device
    W, H, n = p.width, p.height, p.n
    cc, cm = cfg.c(), image_camera(W, H)
    st = _stream(dev)
    n_pairs = torch.zeros(1, dtype=torch.int32, device=dev)
    b, _ = _ws_args(ws, L.gs_tile_workspace_size(n, 0, W, H))
    L.gs_tile_prepare(cm, cc, n, p.ids, p.n_visible, p.means2d, p.conics, p.opacities, n_pairs, b,
                      b.numel(), st)
    npairs = int(n_pairs.item())
    cap = max(npairs, 1)
    b = ws.get(L.gs_tile_workspace_size(n, cap, W, H), keep=True)
    ws.setup_owner = None
    if out is None:
        out = dict(image=torch.empty(3, H, W, device=dev), T=torch.empty(H, W, device=dev),
                   n_contrib=torch.empty(H, W, dtype=torch.int32, device=dev))
    L.gs_tile_raster_fwd(cm, cc, n, p.ids, p.keys, p.means2d, p.conics, p.opacities, p.rgb,
                         n_pairs, cap, out["image"], out["T"], out["n_contrib"], b, b.numel(), st)
    out.update(n_pairs=npairs, capacity=cap)
    return out


def tile_backward(p: Projected, fwd: dict, dL_dimage, cfg: RasterConfig, ws: Workspace, out=None):
    """gs_tile_raster_bwd with the workspace the forward filled."""
    dev = p.means2d.device
    W, H, n = p.width, p.height, p.n
    cc, cm = cfg.c(), image_camera(W, H)
    if out is None:
        out = dict(means2d=torch.empty(n, 2, device=dev), conics=torch.empty(n, 3, device=dev),
                   opacities=torch.empty(n, device=dev), rgb=torch.empty(n, 3, device=dev))
    if "background" not in out:
        out["background"] = torch.empty(3, device=dev)
    b = ws.get(L.gs_tile_workspace_size(n, fwd["capacity"], W, H), keep=True)
    ws.setup_owner = None
    L.gs_tile_raster_bwd(cm, cc, n, p.means2d, p.conics, p.opacities, p.rgb, _c32(dL_dimage),
                         fwd["T"], fwd["n_contrib"], fwd["capacity"], out["means2d"],
                         out["conics"], out["opacities"], out["rgb"], b, b.numel(), _stream(dev))
    return out
