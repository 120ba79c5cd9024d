// api.hip -- the extern "C" boundary of libgsr.so: host-side validation, workspace sizing and
// error reporting around the launchers. No exception crosses this boundary; no entry point
// allocates device memory or synchronises.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <string>

#include "device.hpp"
#include "internal.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok() {
    g_err.clear();
    return GS_OK;
}

int hip_status(hipError_t e, const char* where) {
    if (e == hipSuccess) return ok();
    return fail(GS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

constexpr int32_t MAX_N = 1 << 28;
constexpr int32_t MAX_DIM = 16384;

int check_n(int32_t n) {
    if (n < 0 || n > MAX_N) return fail(GS_ERR_INVALID_ARGUMENT, "n = %d outside 0..2^28", n);
    return GS_OK;
}

int check_cam(const gs_camera* cam) {
    if (!cam) return fail(GS_ERR_INVALID_ARGUMENT, "camera is NULL");
    if (cam->width < 1 || cam->width > MAX_DIM || cam->height < 1 || cam->height > MAX_DIM)
        return fail(GS_ERR_INVALID_ARGUMENT, "image %d x %d outside 1..16384", cam->width,
                    cam->height);
    for (int i = 0; i < 12; ++i)
        if (!isfinite(cam->viewmat[i])) return fail(GS_ERR_INVALID_ARGUMENT, "viewmat not finite");
    if (!(isfinite(cam->fx) && isfinite(cam->fy) && isfinite(cam->cx) && isfinite(cam->cy)) ||
        !(cam->fx > 0.f && cam->fy > 0.f))
        return fail(GS_ERR_INVALID_ARGUMENT, "focal lengths must be finite and > 0");
    if (!(cam->znear > 0.f) || !isfinite(cam->znear))
        return fail(GS_ERR_INVALID_ARGUMENT, "znear must be finite and > 0");
    return GS_OK;
}

int check_dims(int32_t width, int32_t height) {
    if (width < 1 || width > MAX_DIM || height < 1 || height > MAX_DIM)
        return fail(GS_ERR_INVALID_ARGUMENT, "image %d x %d outside 1..16384", width, height);
    return GS_OK;
}

int check_cfg(const gs_config* c) {
    if (!c) return fail(GS_ERR_INVALID_ARGUMENT, "config is NULL");
    if (!(c->alpha_min > 0.f && c->alpha_min < 1.f))
        return fail(GS_ERR_INVALID_ARGUMENT, "alpha_min must be in (0, 1)");
    if (!(c->alpha_max > c->alpha_min && c->alpha_max < 1.f))
        return fail(GS_ERR_INVALID_ARGUMENT, "alpha_max must be in (alpha_min, 1)");
    if (!(c->t_min_fwd >= 0.f && c->t_min_fwd < 1.f))
        return fail(GS_ERR_INVALID_ARGUMENT, "t_min_fwd must be in [0, 1)");
    if (!(c->t_min_bwd >= 0.f && c->t_min_bwd < 1.f))
        return fail(GS_ERR_INVALID_ARGUMENT, "t_min_bwd must be in [0, 1)");
    if (!(c->eps2d >= 0.f) || !isfinite(c->eps2d))
        return fail(GS_ERR_INVALID_ARGUMENT, "eps2d must be finite and >= 0");
    if (c->sh_degree < 0 || c->sh_degree > 3)
        return fail(GS_ERR_INVALID_ARGUMENT, "sh_degree %d outside 0..3", c->sh_degree);
    if (c->fb_format < GS_FB_F32 || c->fb_format > GS_FB_UNORM8)
        return fail(GS_ERR_INVALID_ARGUMENT, "unknown fb_format %d", c->fb_format);
    if (c->fb_round != GS_ROUND_AT_REST && c->fb_round != GS_ROUND_PER_FRAGMENT)
        return fail(GS_ERR_INVALID_ARGUMENT, "unknown fb_round %d", c->fb_round);
    if (c->reduce_mode < GS_REDUCE_NAIVE || c->reduce_mode > GS_REDUCE_TILE)
        return fail(GS_ERR_INVALID_ARGUMENT, "unknown reduce_mode %d", c->reduce_mode);
    if (c->reduce_threshold < 0 || c->reduce_threshold > 64)
        return fail(GS_ERR_INVALID_ARGUMENT, "reduce_threshold %d outside 0..64", c->reduce_threshold);
    if (c->flags & ~(GS_FLAG_STATS | GS_FLAG_REUSE_SETUP | GS_FLAG_COMPOSITE_ALL))
        return fail(GS_ERR_INVALID_ARGUMENT, "unknown flags 0x%x", c->flags);
    for (int k = 0; k < 3; ++k)
        if (!isfinite(c->background[k]))
            return fail(GS_ERR_INVALID_ARGUMENT, "background must be finite");
    if (c->n_views < 0 || c->n_views > GS_MAX_VIEWS)
        return fail(GS_ERR_INVALID_ARGUMENT, "n_views %d outside 0..%d", c->n_views, GS_MAX_VIEWS);
    return GS_OK;
}



#define GSR_TRY(x)                \
    do {                          \
        int _rc = (x);            \
        if (_rc != GS_OK) return _rc; \
    } while (0)

#define GSR_NEED(p)                                                              \
    do {                                                                         \
        if (!(p)) return fail(GS_ERR_INVALID_ARGUMENT, "%s is NULL", #p);       \
    } while (0)

int check_ws(void* ws, size_t have, size_t need) {
    if (need == 0) return GS_OK;
    if (!ws) return fail(GS_ERR_INVALID_ARGUMENT, "workspace is NULL (%zu bytes needed)", need);
    if (have < need)
        return fail(GS_ERR_CAPACITY, "workspace has %zu bytes, %zu needed", have, need);
    if (((uintptr_t)ws) % 256 != 0) return fail(GS_ERR_INVALID_ARGUMENT, "workspace not 256-byte aligned");
    return GS_OK;
}

int views_of(const gs_config* c) { return (c && c->n_views > 1) ? c->n_views : 1; }

int check_one_view(const gs_config* c, const char* what) {
    if (views_of(c) != 1)
        return fail(GS_ERR_UNSUPPORTED, "%s processes one view per call (n_views = %d)", what,
                    c->n_views);
    return GS_OK;
}

// V cameras of one image size, each valid.
int check_cams(const gs_camera* cam, int V) {
    if (!cam) return fail(GS_ERR_INVALID_ARGUMENT, "camera is NULL");
    for (int v = 0; v < V; ++v) {
        GSR_TRY(check_cam(cam + v));
        if (cam[v].width != cam[0].width || cam[v].height != cam[0].height)
            return fail(GS_ERR_INVALID_ARGUMENT, "camera %d is %d x %d, camera 0 %d x %d: the views "
                        "of one call share the image size", v, cam[v].width, cam[v].height,
                        cam[0].width, cam[0].height);
    }
    return GS_OK;
}

gsr::CamSet cam_set(const gs_camera* cam, int V) {
    gsr::CamSet cs{};
    for (int v = 0; v < V; ++v) cs.c[v] = gsr::make_cam(cam[v]);
    return cs;
}

// The per-view slab of a V-view call: ws_bytes / V rounded down to 256 bytes.
size_t slab_of(size_t ws_bytes, int V) { return V > 1 ? (ws_bytes / (size_t)V) / 256 * 256 : ws_bytes; }

// Checks that each of the V slabs holds `need` bytes; the views' Views descriptor.
int check_ws_views(void* ws, size_t ws_bytes, size_t need, int V, gsr::Views& out) {
    out.count = V;
    out.ws = V > 1 ? slab_of(ws_bytes, V) : 0;
    if (need == 0) return GS_OK;
    if (V == 1) return check_ws(ws, ws_bytes, need);
    if (!ws) return fail(GS_ERR_INVALID_ARGUMENT, "workspace is NULL (%d x %zu bytes needed)", V, need);
    if (slab_of(ws_bytes, V) < need)
        return fail(GS_ERR_CAPACITY, "workspace slab per view has %zu bytes, %zu needed",
                    slab_of(ws_bytes, V), need);
    if (((uintptr_t)ws) % 256 != 0) return fail(GS_ERR_INVALID_ARGUMENT, "workspace not 256-byte aligned");
    return GS_OK;
}

int check_align16(const void* p, const char* what) {
    if (((uintptr_t)p) % 16 != 0)
        return fail(GS_ERR_INVALID_ARGUMENT, "%s must be 16-byte aligned", what);
    return GS_OK;
}

int check_no_background(const gs_config* c) {
    if (c->background[0] != 0.f || c->background[1] != 0.f || c->background[2] != 0.f)
        return fail(GS_ERR_INVALID_ARGUMENT, "the tile-based baseline composites Eq. 2 without a background");
    return GS_OK;
}

size_t preprocess_ws(int32_t n) { return gsr::align_up((size_t)n * 4) + gsr::compact_ws_bytes(n); }

}  // namespace

extern "C" {

const char* gs_last_error(void) { return g_err.c_str(); }

int32_t gs_version(void) { return GSR_ABI_VERSION; }

void gs_config_default(gs_config* c) {
    if (!c) return;
    *c = gs_config{};
    c->alpha_min = 1.0f / 255.0f;
    c->alpha_max = 0.99f;
    c->t_min_fwd = 0.0f;
    c->t_min_bwd = 1e-4f;
    c->eps2d = 0.3f;
    c->sh_degree = 3;
    c->fb_format = GS_FB_F32;
    c->fb_round = GS_ROUND_AT_REST;
    c->reduce_mode = GS_REDUCE_HYBRID;
    c->reduce_threshold = 8;
    c->flags = 0;
}

size_t gs_framebuffer_size(int32_t width, int32_t height, int32_t fb_format) {
    if (width < 1 || width > MAX_DIM || height < 1 || height > MAX_DIM) return 0;
    if (fb_format < GS_FB_F32 || fb_format > GS_FB_UNORM8) return 0;
    return (size_t)width * height * gsr::fb_bytes_per_pixel(fb_format);
}

static size_t one_view_ws(int32_t op, int32_t n, int32_t width, int32_t height) {
    switch (op) {
    case GS_OP_PREPROCESS:
    case GS_OP_PREPARE_2D: return preprocess_ws(n);
    case GS_OP_SORT: return gsr::sort_ws_bytes(n, 4);
    case GS_OP_RASTER_FWD: return gsr::raster_ws_bytes(n, width, height, false);
    case GS_OP_RASTER_BWD: return gsr::raster_ws_bytes(n, width, height, true);
    case GS_OP_PREPROCESS_BWD: return 0;
    case GS_OP_ALL: {
        size_t m = preprocess_ws(n);
        size_t s = gsr::sort_ws_bytes(n, 4);
        size_t r = gsr::raster_ws_bytes(n, width, height, true);
        if (s > m) m = s;
        if (r > m) m = r;
        return m;
    }
    default: return 0;
    }
}

size_t gs_workspace_size(int32_t op, int32_t n, int32_t width, int32_t height, const gs_config* cfg) {
    if (n < 0 || n > MAX_N) return 0;
    if (width < 1 || width > MAX_DIM || height < 1 || height > MAX_DIM) return 0;
    if (cfg && (cfg->n_views < 0 || cfg->n_views > GS_MAX_VIEWS)) return 0;
    const int V = views_of(cfg);
    const size_t one = one_view_ws(op, n, width, height);
    return V == 1 ? one : (size_t)V * gsr::align_up(one);
}

int gs_preprocess(const gs_camera* cam, const gs_config* cfg, int32_t n, const float* means3d,
                  const float* scales, const float* quats, const float* opacities, const float* sh,
                  float* means2d, float* conics, float* rgb, float* depth, uint32_t* keys,
                  int32_t* ids, int32_t* n_visible, void* ws, size_t ws_bytes, void* stream) {
    GSR_TRY(check_cfg(cfg));
    const int V = views_of(cfg);
    GSR_TRY(check_cams(cam, V));
    GSR_TRY(check_n(n));
    GSR_NEED(n_visible);
    gsr::Views vs{V, 0};
    if (n > 0) {
        GSR_NEED(means3d); GSR_NEED(scales); GSR_NEED(quats); GSR_NEED(opacities); GSR_NEED(sh);
        GSR_NEED(means2d); GSR_NEED(conics); GSR_NEED(rgb); GSR_NEED(depth); GSR_NEED(keys);
        GSR_NEED(ids);
        GSR_TRY(check_align16(sh, "sh"));
        GSR_TRY(check_ws_views(ws, ws_bytes, preprocess_ws(n), V, vs));
    }
    return hip_status(gsr::launch_preprocess(cam_set(cam, V), vs, *cfg, n, means3d, scales, quats,
                                             opacities, sh, means2d, conics, rgb, depth, keys, ids,
                                             n_visible, ws, (hipStream_t)stream),
                      "gs_preprocess");
}

int gs_prepare_2d(const gs_camera* cam, const gs_config* cfg, int32_t n, const float* means2d,
                  const float* conics, const float* opacities, const float* depth, uint32_t* keys,
                  int32_t* ids, int32_t* n_visible, void* ws, size_t ws_bytes, void* stream) {
    if (!cam) return fail(GS_ERR_INVALID_ARGUMENT, "camera is NULL");
    GSR_TRY(check_dims(cam->width, cam->height));
    GSR_TRY(check_cfg(cfg));
    GSR_TRY(check_one_view(cfg, "gs_prepare_2d"));
    GSR_TRY(check_n(n));
    GSR_NEED(n_visible);
    if (n > 0) {
        GSR_NEED(means2d); GSR_NEED(conics); GSR_NEED(opacities); GSR_NEED(depth);
        GSR_NEED(keys); GSR_NEED(ids);
        GSR_TRY(check_ws(ws, ws_bytes, preprocess_ws(n)));
    }
    return hip_status(gsr::launch_prepare_2d(cam->width, cam->height, *cfg, n, means2d, conics,
                                             opacities, depth, keys, ids, n_visible, ws,
                                             (hipStream_t)stream),
                      "gs_prepare_2d");
}

int gs_sort(int32_t n, uint32_t* keys, int32_t* ids, const int32_t* n_visible, void* ws,
            size_t ws_bytes, void* stream) {
    GSR_TRY(check_n(n));
    GSR_NEED(n_visible);
    if (n == 0) return ok();
    GSR_NEED(keys);
    GSR_NEED(ids);
    GSR_TRY(check_ws(ws, ws_bytes, gsr::sort_ws_bytes(n, 4)));
    return hip_status(gsr::launch_sort_u32(n, keys, ids, n_visible, ws, (hipStream_t)stream),
                      "gs_sort");
}

int gs_sort_noalloc(int32_t n, uint32_t* keys, int32_t* ids, const int32_t* n_visible,
                    void* stream) {
    GSR_TRY(check_n(n));
    GSR_NEED(n_visible);
    if (n > gsr::NOALLOC_SORT_MAX_N)
        return fail(GS_ERR_CAPACITY, "gs_sort_noalloc sorts at most %d keys (n = %d); use gs_sort "
                    "with a workspace", gsr::NOALLOC_SORT_MAX_N, n);
    if (n == 0) return ok();
    GSR_NEED(keys);
    GSR_NEED(ids);
    return hip_status(gsr::launch_sort_u32_noalloc(n, keys, ids, n_visible, (hipStream_t)stream),
                      "gs_sort_noalloc");
}

int gs_sort_views(int32_t n_views, int32_t n, uint32_t* keys, int32_t* ids,
                  const int32_t* n_visible, void* ws, size_t ws_bytes, void* stream) {
    if (n_views < 1 || n_views > GS_MAX_VIEWS)
        return fail(GS_ERR_INVALID_ARGUMENT, "n_views %d outside 1..%d", n_views, GS_MAX_VIEWS);
    GSR_TRY(check_n(n));
    GSR_NEED(n_visible);
    if (n == 0) return ok();
    GSR_NEED(keys);
    GSR_NEED(ids);
    gsr::Views vs{n_views, 0};
    GSR_TRY(check_ws_views(ws, ws_bytes, gsr::sort_ws_bytes(n, 4), n_views, vs));
    return hip_status(gsr::launch_sort_u32(n, keys, ids, n_visible, ws, (hipStream_t)stream, vs),
                      "gs_sort_views");
}

int gs_raster_setup(const gs_camera* cam, const gs_config* cfg, int32_t n, const int32_t* sorted_ids,
                    const int32_t* n_visible, const float* means2d, const float* conics,
                    const float* opacities, const float* rgb, void* ws, size_t ws_bytes,
                    void* stream) {
    if (!cam) return fail(GS_ERR_INVALID_ARGUMENT, "camera is NULL");
    GSR_TRY(check_dims(cam->width, cam->height));
    GSR_TRY(check_cfg(cfg));
    GSR_TRY(check_n(n));
    GSR_NEED(n_visible);
    if (n > 0) {
        GSR_NEED(sorted_ids); GSR_NEED(means2d); GSR_NEED(conics); GSR_NEED(opacities); GSR_NEED(rgb);
    }
    gsr::Views vs{1, 0};
    GSR_TRY(check_ws_views(ws, ws_bytes, gsr::raster_ws_bytes(n, cam->width, cam->height, false),
                           views_of(cfg), vs));
    return hip_status(gsr::launch_raster_setup(*cfg, cam->width, cam->height, n, sorted_ids,
                                               n_visible, means2d, conics, opacities, rgb, ws,
                                               (hipStream_t)stream, vs),
                      "gs_raster_setup");
}

int gs_raster_fwd(const gs_camera* cam, const gs_config* cfg, int32_t n, const int32_t* sorted_ids,
                  const int32_t* n_visible, const float* means2d, const float* conics,
                  const float* opacities, const float* rgb, void* fb, float* out_rgb, float* out_T,
                  int32_t* out_coverage, gs_stats* stats, void* ws, size_t ws_bytes, void* stream) {
    if (!cam) return fail(GS_ERR_INVALID_ARGUMENT, "camera is NULL");
    GSR_TRY(check_dims(cam->width, cam->height));
    GSR_TRY(check_cfg(cfg));
    GSR_TRY(check_n(n));
    GSR_NEED(n_visible);
    GSR_NEED(fb);
    if (n > 0) {
        GSR_NEED(sorted_ids); GSR_NEED(means2d); GSR_NEED(conics); GSR_NEED(opacities); GSR_NEED(rgb);
    }
    gsr::Views vs{1, 0};
    GSR_TRY(check_ws_views(ws, ws_bytes, gsr::raster_ws_bytes(n, cam->width, cam->height, false),
                           views_of(cfg), vs));
    return hip_status(gsr::launch_raster_fwd(*cfg, cam->width, cam->height, n, sorted_ids,
                                             n_visible, means2d, conics, opacities, rgb, fb,
                                             out_rgb, out_T, out_coverage, stats, ws,
                                             (hipStream_t)stream, vs),
                      "gs_raster_fwd");
}

int gs_raster_bwd(const gs_camera* cam, const gs_config* cfg, int32_t n, const int32_t* sorted_ids,
                  const int32_t* n_visible, const float* means2d, const float* conics,
                  const float* opacities, const float* rgb, const void* fb, const float* dL_dimage,
                  float* dL_dmeans2d, float* dL_dconics, float* dL_dopacities, float* dL_drgb,
                  const float* dL_dT, float* dL_dbackground, int32_t* out_live, gs_stats* stats,
                  void* ws, size_t ws_bytes, void* stream) {
    if (!cam) return fail(GS_ERR_INVALID_ARGUMENT, "camera is NULL");
    GSR_TRY(check_dims(cam->width, cam->height));
    GSR_TRY(check_cfg(cfg));
    GSR_TRY(check_n(n));
    GSR_NEED(n_visible);
    GSR_NEED(fb);
    GSR_NEED(dL_dimage);
    if (n > 0) {
        GSR_NEED(sorted_ids); GSR_NEED(means2d); GSR_NEED(conics); GSR_NEED(opacities); GSR_NEED(rgb);
        GSR_NEED(dL_dmeans2d); GSR_NEED(dL_dconics); GSR_NEED(dL_dopacities); GSR_NEED(dL_drgb);
    }
    gsr::Views vs{1, 0};
    GSR_TRY(check_ws_views(ws, ws_bytes, gsr::raster_ws_bytes(n, cam->width, cam->height, true),
                           views_of(cfg), vs));
    return hip_status(gsr::launch_raster_bwd(*cfg, cam->width, cam->height, n, sorted_ids,
                                             n_visible, means2d, conics, opacities, rgb, fb,
                                             dL_dimage, dL_dmeans2d, dL_dconics, dL_dopacities,
                                             dL_drgb, dL_dT, dL_dbackground, out_live, stats, ws,
                                             (hipStream_t)stream, vs),
                      "gs_raster_bwd");
}

int gs_preprocess_bwd(const gs_camera* cam, const gs_config* cfg, int32_t n, const float* means3d,
                      const float* scales, const float* quats, const float* opacities,
                      const float* sh, const float* dL_dmeans2d, const float* dL_dconics,
                      const float* dL_drgb, const float* dL_dopacities2d, float* dL_dmeans3d,
                      float* dL_dscales, float* dL_dquats, float* dL_dopacities, float* dL_dsh,
                      void* stream) {
    GSR_TRY(check_cfg(cfg));
    const int V = views_of(cfg);
    GSR_TRY(check_cams(cam, V));
    GSR_TRY(check_n(n));
    if (n == 0) return ok();
    GSR_NEED(means3d); GSR_NEED(scales); GSR_NEED(quats); GSR_NEED(opacities); GSR_NEED(sh);
    GSR_NEED(dL_dmeans2d); GSR_NEED(dL_dconics); GSR_NEED(dL_drgb); GSR_NEED(dL_dopacities2d);
    GSR_NEED(dL_dmeans3d); GSR_NEED(dL_dscales); GSR_NEED(dL_dquats); GSR_NEED(dL_dopacities);
    GSR_NEED(dL_dsh);
    GSR_TRY(check_align16(sh, "sh"));
    GSR_TRY(check_align16(dL_dsh, "dL_dsh"));
    return hip_status(gsr::launch_preprocess_bwd(cam_set(cam, V), V, *cfg, n, means3d, scales, quats, opacities, sh,
                                                 dL_dmeans2d, dL_dconics, dL_drgb, dL_dopacities2d,
                                                 dL_dmeans3d, dL_dscales, dL_dquats, dL_dopacities,
                                                 dL_dsh, (hipStream_t)stream),
                      "gs_preprocess_bwd");
}

int gs_raster_status(const gs_config* cfg, int32_t n, int32_t width, int32_t height,
                     const void* ws, size_t ws_bytes, uint32_t* status, void* stream) {
    GSR_TRY(check_dims(width, height));
    GSR_TRY(check_cfg(cfg));
    GSR_TRY(check_n(n));
    GSR_NEED(status);
    gsr::Views vs{1, 0};
    GSR_TRY(check_ws_views(const_cast<void*>(ws), ws_bytes,
                           gsr::raster_ws_bytes(n, width, height, false), views_of(cfg), vs));
    uint32_t word = 0u;
    const int rc = hip_status(gsr::raster_status(ws, n, width, height, &word, (hipStream_t)stream, vs),
                              "gs_raster_status");
    if (rc != GS_OK) return rc;
    *status = word;
    if (word == 0u) return ok();
    return fail(GS_ERR_STATE, "raster status 0x%x:%s%s%s%s", word,
                (word & GS_STATUS_BAD_ID) ? " sorted id out of range;" : "",
                (word & GS_STATUS_FWD_SCHEDULE) ? " forward schedule entry out of range;" : "",
                (word & GS_STATUS_BWD_SCHEDULE) ? " backward schedule entry out of range;" : "",
                (word & GS_STATUS_STALE_RECORD) ? " staged record of other inputs;" : "");
}

int gs_raster_debug_schedule(const gs_config* cfg, int32_t n, int32_t width, int32_t height,
                             const void* ws, size_t ws_bytes, int32_t* fwd_order,
                             int32_t* bwd_order, int32_t* item_order, int32_t* items,
                             int64_t* n_items, void* stream) {
    GSR_TRY(check_dims(width, height));
    GSR_TRY(check_cfg(cfg));
    GSR_TRY(check_n(n));
    gsr::Views vs{1, 0};
    GSR_TRY(check_ws_views(const_cast<void*>(ws), ws_bytes,
                           gsr::raster_ws_bytes(n, width, height, false), views_of(cfg), vs));
    if ((item_order || items || n_items) && !gsr::raster_has_split(n, width, height))
        return fail(GS_ERR_UNSUPPORTED, "this workspace holds no depth-split schedule");
    return hip_status(gsr::copy_raster_schedule(ws, n, width, height, fwd_order, bwd_order,
                                                item_order, items, n_items, (hipStream_t)stream, vs),
                      "gs_raster_debug_schedule");
}

int gs_micro_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (bytes == 0) return ok();
    GSR_NEED(src);
    GSR_NEED(dst);
    if (bytes % 16 || ((uintptr_t)src) % 16 || ((uintptr_t)dst) % 16)
        return fail(GS_ERR_INVALID_ARGUMENT, "gs_micro_copy: 16-byte sizes and alignment");
    const char* a = (const char*)src;
    const char* b = (const char*)dst;
    if (a < b + bytes && b < a + bytes)
        return fail(GS_ERR_INVALID_ARGUMENT, "gs_micro_copy: overlapping buffers");
    return hip_status(gsr::launch_micro_copy(src, dst, bytes, (hipStream_t)stream), "gs_micro_copy");
}

int gs_micro_atomic_f32(float* slots, int64_t nslots, int32_t adds_per_thread, int32_t mode,
                        void* stream) {
    GSR_NEED(slots);
    if (nslots < 64 || nslots > ((int64_t)1 << 30) || (nslots & (nslots - 1)))
        return fail(GS_ERR_INVALID_ARGUMENT, "gs_micro_atomic_f32: nslots a power of two in 64..2^30");
    if (adds_per_thread < 0 || adds_per_thread > 4096)
        return fail(GS_ERR_INVALID_ARGUMENT, "gs_micro_atomic_f32: adds_per_thread in 0..4096");
    if (mode < GS_MICRO_ATOMIC_SPREAD || mode > GS_MICRO_ATOMIC_WAVE_SAME)
        return fail(GS_ERR_INVALID_ARGUMENT, "gs_micro_atomic_f32: unknown mode %d", mode);
    return hip_status(gsr::launch_micro_atomic(slots, (size_t)nslots, adds_per_thread, mode,
                                               (hipStream_t)stream),
                      "gs_micro_atomic_f32");
}

// ---- tile-based comparison rasterizer --------------------------------------------------------

size_t gs_tile_workspace_size(int32_t n, int64_t pair_capacity, int32_t width, int32_t height) {
    if (n < 0 || n > MAX_N || pair_capacity < 0 || pair_capacity > (int64_t)1 << 31) return 0;
    if (width < 1 || width > MAX_DIM || height < 1 || height > MAX_DIM) return 0;
    return gsr::tile_ws_bytes(n, (size_t)pair_capacity, width, height);
}

int gs_tile_prepare(const gs_camera* cam, const gs_config* cfg, int32_t n, const int32_t* ids,
                    const int32_t* n_visible, const float* means2d, const float* conics,
                    const float* opacities, uint32_t* n_pairs, void* ws, size_t ws_bytes,
                    void* stream) {
    if (!cam) return fail(GS_ERR_INVALID_ARGUMENT, "camera is NULL");
    GSR_TRY(check_dims(cam->width, cam->height));
    GSR_TRY(check_cfg(cfg));
    GSR_TRY(check_no_background(cfg));
    GSR_TRY(check_one_view(cfg, "the tile-based baseline"));
    GSR_TRY(check_n(n));
    GSR_NEED(n_pairs);
    if (n > 0) {
        GSR_NEED(ids); GSR_NEED(n_visible); GSR_NEED(means2d); GSR_NEED(conics); GSR_NEED(opacities);
    }
    GSR_TRY(check_ws(ws, ws_bytes, gsr::tile_ws_bytes(n, 0, cam->width, cam->height)));
    return hip_status(gsr::launch_tile_prepare(*cfg, cam->width, cam->height, n, ids, n_visible,
                                               means2d, conics, opacities, n_pairs, ws,
                                               (hipStream_t)stream),
                      "gs_tile_prepare");
}

int gs_tile_raster_fwd(const gs_camera* cam, const gs_config* cfg, int32_t n, const int32_t* ids,
                       const uint32_t* keys, const float* means2d, const float* conics,
                       const float* opacities, const float* rgb, const uint32_t* n_pairs,
                       int64_t pair_capacity, float* out_rgb, float* out_T, int32_t* n_contrib,
                       void* ws, size_t ws_bytes, void* stream) {
    if (!cam) return fail(GS_ERR_INVALID_ARGUMENT, "camera is NULL");
    GSR_TRY(check_dims(cam->width, cam->height));
    GSR_TRY(check_cfg(cfg));
    GSR_TRY(check_no_background(cfg));
    GSR_TRY(check_one_view(cfg, "the tile-based baseline"));
    GSR_TRY(check_n(n));
    if (pair_capacity < 0 || pair_capacity > (int64_t)1 << 31)
        return fail(GS_ERR_INVALID_ARGUMENT, "pair_capacity outside 0..2^31");
    GSR_NEED(n_pairs); GSR_NEED(out_rgb); GSR_NEED(out_T); GSR_NEED(n_contrib);
    if (n > 0) {
        GSR_NEED(ids); GSR_NEED(keys); GSR_NEED(means2d); GSR_NEED(conics); GSR_NEED(opacities);
        GSR_NEED(rgb);
    }
    GSR_TRY(check_ws(ws, ws_bytes, gsr::tile_ws_bytes(n, (size_t)pair_capacity, cam->width, cam->height)));
    return hip_status(gsr::launch_tile_fwd(*cfg, cam->width, cam->height, n, ids, keys, means2d,
                                           conics, opacities, rgb, n_pairs, (size_t)pair_capacity,
                                           out_rgb, out_T, n_contrib, ws, (hipStream_t)stream),
                      "gs_tile_raster_fwd");
}

int gs_tile_raster_bwd(const gs_camera* cam, const gs_config* cfg, int32_t n, const float* means2d,
                       const float* conics, const float* opacities, const float* rgb,
                       const float* dL_dimage, const float* T_final, const int32_t* n_contrib,
                       int64_t pair_capacity, float* dL_dmeans2d, float* dL_dconics,
                       float* dL_dopacities, float* dL_drgb, void* ws, size_t ws_bytes,
                       void* stream) {
    if (!cam) return fail(GS_ERR_INVALID_ARGUMENT, "camera is NULL");
    GSR_TRY(check_dims(cam->width, cam->height));
    GSR_TRY(check_cfg(cfg));
    GSR_TRY(check_no_background(cfg));
    GSR_TRY(check_one_view(cfg, "the tile-based baseline"));
    GSR_TRY(check_n(n));
    if (pair_capacity < 0 || pair_capacity > (int64_t)1 << 31)
        return fail(GS_ERR_INVALID_ARGUMENT, "pair_capacity outside 0..2^31");
    GSR_NEED(dL_dimage); GSR_NEED(T_final); GSR_NEED(n_contrib);
    if (n > 0) {
        GSR_NEED(means2d); GSR_NEED(conics); GSR_NEED(opacities); GSR_NEED(rgb);
        GSR_NEED(dL_dmeans2d); GSR_NEED(dL_dconics); GSR_NEED(dL_dopacities); GSR_NEED(dL_drgb);
    }
    GSR_TRY(check_ws(ws, ws_bytes, gsr::tile_ws_bytes(n, (size_t)pair_capacity, cam->width, cam->height)));
    return hip_status(gsr::launch_tile_bwd(*cfg, cam->width, cam->height, n, means2d, conics,
                                           opacities, rgb, dL_dimage, T_final, n_contrib,
                                           (size_t)pair_capacity, dL_dmeans2d, dL_dconics,
                                           dL_dopacities, dL_drgb, ws, (hipStream_t)stream),
                      "gs_tile_raster_bwd");
}

}  // extern "C"
