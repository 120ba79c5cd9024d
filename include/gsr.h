/*
 * gsr.h -- C ABI of libgsr.so, the MI355X (gfx950) differentiable Gaussian-splat rasterizer.
 *
 * Method: "Efficient Differentiable Hardware Rasterization for 3D Gaussian Splatting"
 * (arXiv 2505.18764). The path is: projection of 3D Gaussians to 2D splats (Sec. 2.1.2), a depth
 * sort of all splats (Sec. 1, Sec. 4.1), ordered alpha compositing into a fixed-size per-pixel
 * framebuffer (Eq. 2), the front-to-back gradient procedure that rematerialises each fragment's
 * gradient from the stored framebuffer state (Sec. 3.1, Procedure 1), the quad/wave gradient
 * reduction before global atomics (Sec. 3.2, Procedure 2), and the backward of the projection
 * (Sec. 2.1.3, the "dedicated subsequent pass").
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE pointers to caller-owned, contiguous, row-major memory
 *     (FP32 unless typed otherwise). The library never allocates device memory; scratch comes from
 *     the caller's workspace `ws` of `ws_bytes` bytes (size it with gs_workspace_size()).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream). Work is enqueued
 *     asynchronously; no entry point synchronises the device or the stream, except
 *     gs_raster_status, which waits for its stream to read the device status word back.
 *   - Arguments are validated on the host before any HIP call. On failure the call returns a
 *     nonzero status, enqueues nothing, and gs_last_error() describes the problem (thread-local).
 *     GS_ERR_HIP means a launch failed; its message carries the HIP error string.
 *   - n = 0 is valid everywhere; images are then 0 with T = 1 and gradient outputs are zero.
 *   - Gradient outputs are overwritten (zero-filled first), as the buffers in Procedure 2 start
 *     at zero.
 *   - Width and height are 1 .. 16384; n is 0 .. 2^28.
 *   - Nothing here is thread-safe across calls that share a workspace.
 *
 * Several views per launch (cfg->n_views = V, 2 .. GS_MAX_VIEWS; 0 and 1 mean one view): the
 * views are cameras of one scene with the same image size, processed by the same kernels with the
 * view as the grid's second dimension. Every per-view array is then the concatenation of the V
 * views' arrays: [V][n][..] by splat id (means2d, conics, rgb, depth, keys, ids and the 2D
 * gradients), [V] for n_visible, [V][3][H][W] / [V][H][W] images, V framebuffers back to back.
 * Per-Gaussian inputs that do not depend on the view (the 3D parameters, opacities) stay [n].
 * Gradients w.r.t. quantities shared by the views are summed over them: gs_preprocess_bwd writes
 * the sum of the V views' 3D gradients and gs_raster_bwd the sum of their dL/dbackground. The
 * workspace is cut into V equal slabs of floor(ws_bytes / V / 256) * 256 bytes, one per view; each
 * must hold the op's one-view size (gs_workspace_size returns V times that size, rounded up to
 * 256 bytes). Calls that pass state through the workspace (gs_raster_setup -> gs_raster_fwd ->
 * gs_raster_bwd with GS_FLAG_REUSE_SETUP) must pass the same ws_bytes. Only the ordered path
 * batches views: gs_prepare_2d and the tile-based baseline reject n_views > 1.
 */
#ifndef GSR_H
#define GSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSR_ABI_VERSION 1
#define GS_MAX_VIEWS 16

enum gs_status {
    GS_OK = 0,
    GS_ERR_INVALID_ARGUMENT = 1,
    GS_ERR_CAPACITY = 2,        /* workspace or pair buffer too small */
    GS_ERR_UNSUPPORTED = 3,
    GS_ERR_HIP = 4,
    GS_ERR_STATE = 5            /* gs_raster_status: a kernel found inconsistent state (see below) */
};

/* Bits of the raster's device status word (gs_raster_status). Each names an input or workspace
 * state the kernels refuse to guess about; the affected work is skipped, so the outputs of the
 * calls since the last raster setup are then incomplete. */
enum gs_status_bits {
    GS_STATUS_BAD_ID = 1,           /* sorted_ids[p] outside 0..n-1 for some p < n_visible */
    GS_STATUS_FWD_SCHEDULE = 2,     /* the forward met a tile or work-item entry outside its range */
    GS_STATUS_BWD_SCHEDULE = 4,     /* the backward met a tile entry outside its range */
    GS_STATUS_STALE_RECORD = 8      /* a staged record named a splat outside 0..n-1: the workspace
                                       holds a setup built for other inputs */
};

/* Render-target formats of the framebuffer state (Sec. 3.3, mixed-precision rendering). */
enum gs_fb_format {
    GS_FB_F32 = 0,      /* 4 x fp32 per pixel (16 B) */
    GS_FB_F16 = 1,      /* 4 x IEEE half, round to nearest even (8 B) */
    GS_FB_UNORM16 = 2,  /* 4 x round(clamp(x,0,1) * 65535) (8 B); splat colours saturate to 1 */
    GS_FB_BF16 = 3,     /* 4 x bfloat16, round to nearest even (8 B) */
    GS_FB_UNORM8 = 4    /* 4 x round(clamp(x,0,1) * 255) (4 B); splat colours saturate to 1 */
};

/* When the per-pixel state is rounded to the framebuffer format. */
enum gs_fb_round {
    GS_ROUND_AT_REST = 0,       /* state is FP32 while a tile is resident on chip; rounded when
                                   written back to the framebuffer (and read back rounded) */
    GS_ROUND_PER_FRAGMENT = 1   /* rounded after every fragment store, like a hardware render
                                   target that blends in its own format */
};

/* Gradient reduction before the global atomics (Sec. 3.2, Procedure 2, Table 1). */
enum gs_reduce_mode {
    GS_REDUCE_NAIVE = 0,        /* one atomicAdd per live fragment and parameter */
    GS_REDUCE_QUAD = 1,         /* sum over the 2x2 quad; the lowest live lane of each quad adds */
    GS_REDUCE_WAVE = 2,         /* wave sum when >= X lanes are live, else per-fragment atomics */
    GS_REDUCE_HYBRID = 3,       /* Procedure 2: wave sum when all live lanes hold one splat and
                                   >= X are live, else quad sums */
    GS_REDUCE_HYBRID_LANE = 4,  /* Procedure 2 applied once per splat per wave after each lane
                                   has summed its own pixels' fragments in registers */
    GS_REDUCE_TILE = 5          /* per splat and wave, the lanes' register sums are reduced
                                   over the whole wave at once (nine values through lane swaps;
                                   no threshold X), the four waves' totals are added in LDS, and
                                   one set of global atomics per splat and 32x32 tile commits */
};

enum gs_flags {
    GS_FLAG_STATS = 1,          /* count fragments, atomics and reductions into gs_stats */
    GS_FLAG_REUSE_SETUP = 2,    /* gs_raster_fwd / gs_raster_bwd: the workspace already holds the
                                   raster setup (see gs_raster_setup) for these exact inputs,
                                   image size, alpha_min and fb_format; skip rebuilding it */
    GS_FLAG_COMPOSITE_ALL = 4   /* gs_raster_fwd: composite every covered fragment even where the
                                   stored state can no longer change (see gs_raster_fwd); same
                                   image, T a little lower; for comparisons */
};

/* Pinhole camera. viewmat is the 3x4 world->camera matrix [R|t], row-major; the camera looks
 * along +z, x to the right, y down; fx, fy, cx, cy in pixels; pixel (x, y) has its centre at
 * (x + 0.5, y + 0.5). Splats with view depth below znear are culled. */
typedef struct gs_camera {
    float viewmat[12];
    float fx, fy, cx, cy;
    int32_t width, height;
    float znear;
    float reserved;
} gs_camera;

/* Method constants and switches. gs_config_default() fills in the paper's values. */
typedef struct gs_config {
    float alpha_min;        /* 1/255: fragments below it are discarded (Sec. 2.1.2) */
    float alpha_max;        /* 0.99: clamp that keeps 1 - alpha away from 0 (reading) */
    float t_min_fwd;        /* 0: the forward does not T-cull, as hardware blending cannot
                               (Sec. 2.1.4); > 0 enables forward T-culling */
    float t_min_bwd;        /* 1e-4: T-culling in the backward (Sec. 2.1.4, Procedure 1) */
    float eps2d;            /* 0.3 px^2 dilation of the 2D covariance (reading) */
    int32_t sh_degree;      /* 0..3; sh arrays hold (sh_degree + 1)^2 coefficients per colour */
    int32_t fb_format;      /* enum gs_fb_format */
    int32_t fb_round;       /* enum gs_fb_round */
    int32_t reduce_mode;    /* enum gs_reduce_mode */
    int32_t reduce_threshold; /* X of Procedure 2: minimum live lanes for the wave path (8) */
    int32_t flags;          /* enum gs_flags */
    float background[3];    /* colour behind the last splat, C += T_final bg; 0 (the default)
                               is Eq. 2 as printed. Not supported by the tile-based baseline. */
    int32_t n_views;        /* views per call (0 or 1: one; up to GS_MAX_VIEWS), see above */
    int32_t reserved[1];
} gs_config;

/* Device-side counters (add-only; zero them before the calls you want to count). */
typedef struct gs_stats {
    unsigned long long fwd_queued;      /* (tile, splat) pairs taken from the sorted list */
    unsigned long long fwd_evaluated;   /* (pixel, splat) alphas evaluated */
    unsigned long long fwd_covered;     /* fragments blended */
    unsigned long long bwd_queued;
    unsigned long long bwd_evaluated;
    unsigned long long bwd_live;        /* fragments that passed both culls of Procedure 1 */
    unsigned long long bwd_atomic_sets; /* leader lanes that issued one set of gradient atomics */
    unsigned long long bwd_wave_reductions;
    unsigned long long bwd_quad_reductions;
    unsigned long long bwd_cohesive;    /* reductions whose live lanes all held one splat */
    unsigned long long fwd_walked;      /* (wave, splat) entries of the forward's culled lists */
    unsigned long long fwd_empty_blocks;/* (8x8 sub-block, splat) evaluations where no alpha passed */
    unsigned long long fwd_chunks;      /* (tile, 16-splat chunk) pairs whose rectangles were tested */
    unsigned long long fwd_batches;     /* staged batches of up to 256 records */
    unsigned long long reserved[2];
} gs_stats;

/* Workspace users (argument `op` of gs_workspace_size). */
enum gs_op {
    GS_OP_PREPROCESS = 0,
    GS_OP_SORT = 1,
    GS_OP_RASTER_FWD = 2,
    GS_OP_RASTER_BWD = 3,
    GS_OP_PREPROCESS_BWD = 4,
    GS_OP_PREPARE_2D = 5,
    GS_OP_ALL = 6           /* enough for every op above (one shared workspace) */
};

/* Thread-local description of the last failure ("" when none). */
const char* gs_last_error(void);

/* GSR_ABI_VERSION of the built library. */
int32_t gs_version(void);

/* Paper defaults: alpha_min 1/255, alpha_max 0.99, t_min_fwd 0, t_min_bwd 1e-4, eps2d 0.3,
 * sh_degree 3, F32 framebuffer rounded at rest, HYBRID reduction with X = 8. */
void gs_config_default(gs_config* cfg);

/* Bytes of scratch the op needs for n splats at width x height (times cfg->n_views, each view's
 * part rounded up to 256 bytes; cfg may be NULL for one view). Pure host function of its
 * arguments (no HIP call); 0 for invalid arguments. Every buffer in the library has a size that
 * is a closed form of (n, width, height, format): this is what a server admits requests by. */
size_t gs_workspace_size(int32_t op, int32_t n, int32_t width, int32_t height,
                         const gs_config* cfg);

/* Bytes of the framebuffer (width * height pixels x 4 channels in cfg->fb_format). */
size_t gs_framebuffer_size(int32_t width, int32_t height, int32_t fb_format);

/*
 * Projection (Sec. 2.1.1-2.1.2): for each Gaussian i, Sigma_3D = R S S^T R^T from the quaternion
 * quats[i] = (w, x, y, z) (normalised here) and scales[i] (> 0); t = R_view mu + t_view;
 * mean2d = (fx tx/tz + cx, fy ty/tz + cy); Sigma_2D = J W Sigma_3D W^T J^T + eps2d I with J the
 * Jacobian of the perspective map; conic = Sigma_2D^{-1} as (a, b, c) with
 * q = a dx^2 + 2 b dx dy + c dy^2; colour = max(0, sum_k Y_k(dir) sh[i][k] + 0.5) with real SH of
 * degree cfg->sh_degree at the unit direction from the camera centre to mu.
 * Frustum culling (Sec. 4.1): a splat is culled when tz < znear, opacity < alpha_min, the 2D
 * covariance is not positive definite, or the bounding box of its alpha >= alpha_min ellipse
 * holds no pixel centre of the image.
 * Inputs [n]: means3d [n,3], scales [n,3], quats [n,4], opacities [n] (in [0,1]),
 *   sh [n, (sh_degree+1)^2, 3] (16-byte aligned; GS_ERR_INVALID_ARGUMENT otherwise).
 * Outputs by splat id: means2d [n,2], conics [n,3], rgb [n,3], depth [n] (fp32 view depth; 0 if
 *   culled; culled splats also get zero means2d/conics/rgb).
 * Sort input (GPU-driven culling, Sec. 4.1): keys [n], ids [n] hold the visible splats first, in
 *   id order, as (bits of fp32(tz) with tz evaluated in FP64, id), then the culled splats in id
 *   order as (0xFFFFFFFF, id); n_visible [1] (device int32) is the number of visible splats.
 *   The compaction is deterministic (a prefix sum, no atomics).
 * Workspace: gs_workspace_size(GS_OP_PREPROCESS, n, ...).
 * With cfg->n_views = V, cam points to V cameras (equal width and height) and the outputs are
 * [V][..] as described at the top.
 */
int gs_preprocess(const gs_camera* cam, const gs_config* cfg, int32_t n,
                  const float* means3d, const float* scales, const float* quats,
                  const float* opacities, const float* sh,
                  float* means2d, float* conics, float* rgb, float* depth,
                  uint32_t* keys, int32_t* ids, int32_t* n_visible,
                  void* ws, size_t ws_bytes, void* stream);

/*
 * Sort input for splats that are already 2D (Sec. 2.1.2 with the projection given): the key of
 * splat i is the order-preserving uint32 of fp32 depth[i]; a splat is culled when it cannot put a
 * fragment on the image (opacity < alpha_min, conic not positive definite, or the bounding box of
 * its alpha >= alpha_min ellipse holds no pixel centre). keys/ids/n_visible as gs_preprocess
 * (visible first in id order, then culled with key 0xFFFFFFFF). Only cam->width and cam->height
 * are read. Workspace: gs_workspace_size(GS_OP_PREPARE_2D, n, ...).
 */
int gs_prepare_2d(const gs_camera* cam, const gs_config* cfg, int32_t n,
                  const float* means2d, const float* conics, const float* opacities,
                  const float* depth, uint32_t* keys, int32_t* ids, int32_t* n_visible,
                  void* ws, size_t ws_bytes, void* stream);

/*
 * Depth sort (Sec. 1, Sec. 4.1): stable ascending sort of the first *n_visible (key, id) pairs in
 * place, by the full 32-bit key; equal keys keep their input order (so, after gs_preprocess,
 * ties are broken by id). The length is read on the device (dynamic-length sort after culling,
 * no host readback); entries from *n_visible to n are left in place. Afterwards ids[0..n) is
 * still a permutation of 0..n-1. Workspace: gs_workspace_size(GS_OP_SORT, n, ...).
 */
int gs_sort(int32_t n, uint32_t* keys, int32_t* ids, const int32_t* n_visible,
            void* ws, size_t ws_bytes, void* stream);

/*
 * gs_sort for callers that cannot allocate device memory or pass a workspace: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation. Same operation, result
 * and argument meaning as gs_sort; the scratch is instead a fixed array inside the library, one
 * per GPU (GS_NOALLOC_SORT_MAX_N keys' worth, about 36 MB), set up on the first call on each
 * device and held until the process ends. The call allocates nothing. n above
 * GS_NOALLOC_SORT_MAX_N is rejected with GS_ERR_CAPACITY before any launch. Calls that overlap on
 * one GPU (other streams, other threads) share that array and race: serialise them.
 */
#define GS_NOALLOC_SORT_MAX_N (1 << 22)
int gs_sort_noalloc(int32_t n, uint32_t* keys, int32_t* ids, const int32_t* n_visible,
                    void* stream);

/*
 * gs_sort for n_views views in one launch per step: keys [n_views][n], ids [n_views][n],
 * n_visible [n_views]; each view's first n_visible[v] pairs are sorted as gs_sort does. The
 * workspace is cut into n_views slabs as described at the top (each needs
 * gs_workspace_size(GS_OP_SORT, n, ...) bytes with one view). n_views is 1 .. GS_MAX_VIEWS.
 */
int gs_sort_views(int32_t n_views, int32_t n, uint32_t* keys, int32_t* ids,
                  const int32_t* n_visible, void* ws, size_t ws_bytes, void* stream);

/*
 * Raster setup, shared by the forward and the backward walk: per sorted position, the splat's
 * record (mean, conic factors, opacity, colour, pixel bounding box of the alpha >= alpha_min
 * ellipse) and its tile rectangle; per tile, an occupancy bitmap over chunks of 16 sorted splats
 * and a splat count that orders the tiles heaviest first. gs_raster_fwd and gs_raster_bwd run it
 * themselves unless cfg->flags has GS_FLAG_REUSE_SETUP; calling it once and passing that flag to
 * both lets one view's forward and backward share it. The setup depends on the inputs, the image
 * size, cfg->alpha_min and whether cfg->fb_format saturates colours; reusing a setup built for
 * anything else gives wrong images and gradients (it cannot fault: every index is bounded).
 * Inputs as gs_raster_fwd. Workspace: gs_workspace_size(GS_OP_RASTER_FWD, n, W, H, cfg); the
 * backward's workspace starts with the same layout, so one buffer sized for GS_OP_RASTER_BWD
 * serves all three calls.
 */
int gs_raster_setup(const gs_camera* cam, const gs_config* cfg, int32_t n,
                    const int32_t* sorted_ids, const int32_t* n_visible,
                    const float* means2d, const float* conics, const float* opacities,
                    const float* rgb, void* ws, size_t ws_bytes, void* stream);

/*
 * Forward rasterization (Eq. 2): for every pixel, the splats in sorted_ids[0 .. *n_visible) are
 * composited front to back: alpha = min(alpha_max, o exp(-q/2)), fragments with
 * alpha < alpha_min discarded, C += T alpha c, T *= 1 - alpha (optionally T-culled when
 * cfg->t_min_fwd > 0); at the end C += T cfg->background (T stays the splats' product). The
 * per-pixel state (C, T) is rounded to cfg->fb_format per cfg->fb_round
 * and written to the framebuffer `fb` (gs_framebuffer_size bytes, [H][W][4] in that format).
 * Saturation exit (state at rest, no counters requested, GS_FLAG_COMPOSITE_ALL not set): a
 * pixel block stops compositing once each of its pixels has T <= 1e-6 and, in FP32, no fragment
 * of the view can change its colour any more (C_ch + 2 T max|c| == C_ch): the stored colour is
 * then bit-identical to compositing every fragment, and T within 1e-6 of its product over all
 * of them. With out_coverage every covered fragment is composited and counted; stats count the
 * fragments actually composited (with the exit unless GS_FLAG_COMPOSITE_ALL is set).
 * In the unorm formats splat colours saturate to 1 (Sec. 3.3).
 * Inputs [n] by splat id: means2d [n,2], conics [n,3], opacities [n], rgb [n,3];
 *   sorted_ids [n] (a permutation of 0..n-1, as gs_sort leaves it), n_visible [1] device int32.
 * Outputs: fb; out_rgb [3,H,W] and out_T [H,W] (fp32 copies of the stored state, nullable);
 *   out_coverage [H,W] int32 fragments blended per pixel (nullable); stats (nullable, counted
 *   with GS_FLAG_STATS).
 * Workspace: gs_workspace_size(GS_OP_RASTER_FWD, n, W, H, cfg).
 */
int gs_raster_fwd(const gs_camera* cam, const gs_config* cfg, int32_t n,
                  const int32_t* sorted_ids, const int32_t* n_visible,
                  const float* means2d, const float* conics, const float* opacities,
                  const float* rgb, void* fb, float* out_rgb, float* out_T,
                  int32_t* out_coverage, gs_stats* stats, void* ws, size_t ws_bytes,
                  void* stream);

/*
 * Backward rasterization (Sec. 3.1, Procedure 1 ComputeGradient; Sec. 3.2, Procedure 2
 * ReduceGradient): the state (C', T) starts at (C from `fb`, 1); the splats are walked in the
 * forward's order; for each fragment: cull if alpha < alpha_min; cull if T < t_min_bwd (state
 * left unchanged); otherwise dL/dc = dL/dC alpha T (Eq. 3), dL/dalpha = dL/dC . (c T - C')/(1 -
 * alpha) (Eq. 7), (C', T) <- (C' - T alpha c, T (1 - alpha)) (Eqs. 5-6), and the chain rule to
 * (mean2d, conic, opacity, rgb); then the reduction of cfg->reduce_mode with threshold X and FP32
 * global atomics.
 * Inputs: as gs_raster_fwd plus fb (the forward's framebuffer, same cfg) and dL_dimage [3,H,W];
 *   dL_dT [H,W] (nullable): the gradient of a loss on the final transmittance T_final =
 *   prod (1 - alpha_i), which adds -dL_dT T_final / (1 - alpha_i) to dL/dalpha_i.
 * Outputs (overwritten) [n] by splat id: dL_dmeans2d [n,2], dL_dconics [n,3] (w.r.t. a, b, c),
 *   dL_dopacities [n], dL_drgb [n,3]; dL_dbackground [3] (nullable) = sum over pixels of
 *   dL/dC T_final; out_live [H,W] int32 live fragments per pixel (nullable); stats (nullable).
 * Workspace: gs_workspace_size(GS_OP_RASTER_BWD, n, W, H, cfg).
 */
int gs_raster_bwd(const gs_camera* cam, const gs_config* cfg, int32_t n,
                  const int32_t* sorted_ids, const int32_t* n_visible,
                  const float* means2d, const float* conics, const float* opacities,
                  const float* rgb, const void* fb, const float* dL_dimage,
                  float* dL_dmeans2d, float* dL_dconics, float* dL_dopacities, float* dL_drgb,
                  const float* dL_dT, float* dL_dbackground, int32_t* out_live,
                  gs_stats* stats, void* ws, size_t ws_bytes, void* stream);

/*
 * Backward of the projection (Sec. 2.1.3: "a dedicated subsequent pass"): from the gradients
 * w.r.t. the 2D splat (mean2d, conic, rgb, opacity) to those w.r.t. the 3D Gaussian, including
 * the view-direction term of the SH colour and the quaternion normalisation. Recomputes the
 * forward from the same inputs as gs_preprocess. Culled splats get zero gradients.
 * Outputs (overwritten): dL_dmeans3d [n,3], dL_dscales [n,3], dL_dquats [n,4],
 *   dL_dopacities [n], dL_dsh [n,(sh_degree+1)^2,3]. sh and dL_dsh must be 16-byte aligned.
 *   Workspace: none.
 * With cfg->n_views = V: cam points to V cameras, the 2D gradients are [V][n][..], and each
 *   output is the sum over the views (in view order, accumulated in registers and written once).
 */
int gs_preprocess_bwd(const gs_camera* cam, const gs_config* cfg, int32_t n,
                      const float* means3d, const float* scales, const float* quats,
                      const float* opacities, const float* sh,
                      const float* dL_dmeans2d, const float* dL_dconics, const float* dL_drgb,
                      const float* dL_dopacities2d,
                      float* dL_dmeans3d, float* dL_dscales, float* dL_dquats,
                      float* dL_dopacities, float* dL_dsh, void* stream);

/*
 * The raster's device status word: every raster setup (gs_raster_setup, or a gs_raster_fwd /
 * gs_raster_bwd that builds its own) clears it, and the setup, forward and backward kernels set
 * gs_status_bits in it when they meet a splat id or a schedule entry outside its range, instead
 * of substituting a value. This call waits for `stream`, copies the word of each of the
 * cfg->n_views workspace slabs to the host, and stores their OR in *status (host pointer).
 * Returns GS_OK when it is zero and GS_ERR_STATE otherwise (gs_last_error() names the bits).
 * n, width, height and cfg must be those of the raster calls that used the workspace.
 * Unlike every other entry point it synchronises (the stream only).
 */
int gs_raster_status(const gs_config* cfg, int32_t n, int32_t width, int32_t height,
                     const void* ws, size_t ws_bytes, uint32_t* status, void* stream);

/*
 * Diagnostics: copies the raster's schedules from the workspace into caller device buffers
 * (enqueued on `stream`, no synchronisation). With T = tiles of 32 x 32 pixels of the image and
 * V = cfg->n_views (each buffer holds V views back to back):
 *   fwd_order [V][T] int32   tiles in the forward's dispatch order (one tile per workgroup);
 *   bwd_order [V][T] int32   tiles in the backward's dispatch order (written by gs_raster_bwd);
 *   item_order [V][4T] int32 the depth-split forward's work items in dispatch order, -1 past the
 *                            item count; items [V][4T] int4 (tile, first column, end column,
 *                            partial slot or -1); n_items [V] int64 the item count.
 * Each pointer may be NULL. The item arrays exist only when the workspace holds a depth split
 * (GS_ERR_UNSUPPORTED if item_order, items or n_items is requested without one: images of more
 * than 4096 tiles), and are planned by the forward that splits (GS_FLAG_COMPOSITE_ALL with the
 * state at rest, no forward T-cull and no counters): after other calls they hold what the last
 * such forward planned, or nothing. A setup (or forward) must have run on the workspace first.
 */
int gs_raster_debug_schedule(const gs_config* cfg, int32_t n, int32_t width, int32_t height,
                             const void* ws, size_t ws_bytes, int32_t* fwd_order,
                             int32_t* bwd_order, int32_t* item_order, int32_t* items,
                             int64_t* n_items, void* stream);

/* ---- Microbenchmarks: the measured ceilings of the raster's bounds (compute nothing of the
 * method). Both enqueue one kernel on `stream` and return at once; time them with events. ---- */

/* Copies `bytes` (a multiple of 16; src and dst 16-byte aligned, not overlapping) from src to dst
 * with 16-byte loads and stores over a grid-stride loop: the HBM stream bandwidth a kernel of
 * this library can reach. */
int gs_micro_copy(const void* src, void* dst, size_t bytes, void* stream);

#define GS_MICRO_THREADS (1 << 20)
enum gs_micro_atomic_mode {
    GS_MICRO_ATOMIC_SPREAD = 0,         /* consecutive lanes add to consecutive words (the
                                           backward's gradient flush); no value returned */
    GS_MICRO_ATOMIC_SPREAD_RETURN = 1,  /* the same, each add returning the old value (the first
                                           add of the flush's compensated pair) */
    GS_MICRO_ATOMIC_WAVE_SAME = 2       /* the 64 lanes of a wave add to one word (per-fragment
                                           atomics of one splat across a wave) */
};
/* adds_per_thread x GS_MICRO_THREADS FP32 atomic adds of 1/64 into slots[0 .. nslots) (device
 * memory, nslots a power of two, 64 .. 2^30) in the pattern `mode`. The slots are not cleared:
 * each one gains (adds it received) / 64. */
int gs_micro_atomic_f32(float* slots, int64_t nslots, int32_t adds_per_thread, int32_t mode,
                        void* stream);

/* ---- Comparison design: tile-based software rasterization (Sec. 2.1.3-2.1.4) ----------------
 *
 * 16x16-pixel tiles. Each visible splat is duplicated into one (tile, depth key) pair per tile its
 * alpha >= alpha_min bounding box touches; the pairs are radix-sorted by the 64-bit key (stable,
 * so equal depths stay in input order) and cut into per-tile ranges; the forward composites each
 * pixel front to back with T-culling at cfg->t_min_bwd (a fragment is skipped when T before it
 * is below the threshold) and records the number of range entries up to its last blended
 * fragment; the backward walks each pixel's range back to front from that entry, recovering T by
 * division by (1 - alpha), and adds each fragment's 9 gradients with its own atomics (Eq. 3 and
 * Eq. 4). It computes the same function as gs_raster_fwd/bwd with t_min_fwd = t_min_bwd, in FP32
 * state (fb_format only selects colour saturation for the unorm formats).
 *
 * Protocol (the pair count is data dependent, the dynamic allocation of Sec. 1):
 *   1. gs_tile_prepare(...) with a workspace of gs_tile_workspace_size(n, 0, W, H) bytes or more
 *      writes the pair count to n_pairs [1] (device uint32);
 *   2. the caller reads n_pairs back and provides a workspace of
 *      gs_tile_workspace_size(n, capacity, W, H) bytes with capacity >= n_pairs (the first
 *      bytes must be the same workspace as in step 1: they carry the per-splat tile counts);
 *   3. gs_tile_raster_fwd(...) then gs_tile_raster_bwd(...) with the same workspace and capacity
 *      (the sorted pairs and tile ranges pass from the forward to the backward).
 * If capacity < *n_pairs the excess pairs are dropped (no out-of-bounds write; results are then
 * incomplete). ids/keys/n_visible are gs_preprocess's or gs_prepare_2d's (sorted or not).
 * Outputs: out_rgb [3,H,W], out_T [H,W], n_contrib [H,W] int32; gradients as gs_raster_bwd.
 */
size_t gs_tile_workspace_size(int32_t n, int64_t pair_capacity, int32_t width, int32_t height);

int gs_tile_prepare(const gs_camera* cam, const gs_config* cfg, int32_t n, const int32_t* ids,
                    const int32_t* n_visible, const float* means2d, const float* conics,
                    const float* opacities, uint32_t* n_pairs, void* ws, size_t ws_bytes,
                    void* stream);

int gs_tile_raster_fwd(const gs_camera* cam, const gs_config* cfg, int32_t n, const int32_t* ids,
                       const uint32_t* keys, const float* means2d, const float* conics,
                       const float* opacities, const float* rgb, const uint32_t* n_pairs,
                       int64_t pair_capacity, float* out_rgb, float* out_T, int32_t* n_contrib,
                       void* ws, size_t ws_bytes, void* stream);

int gs_tile_raster_bwd(const gs_camera* cam, const gs_config* cfg, int32_t n,
                       const float* means2d, const float* conics, const float* opacities,
                       const float* rgb, const float* dL_dimage, const float* T_final,
                       const int32_t* n_contrib, int64_t pair_capacity, float* dL_dmeans2d,
                       float* dL_dconics, float* dL_dopacities, float* dL_drgb, void* ws,
                       size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GSR_H */
