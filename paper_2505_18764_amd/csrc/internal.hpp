// internal.hpp -- host-side launcher declarations shared by the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/gsr.h"

namespace gsr {

// Camera in the form the kernels take by value.
struct CamDev {
    float R[9];      // world->camera rotation, row-major
    float t[3];
    float campos[3]; // -R^T t
    float fx, fy, cx, cy;
    int width, height;
    float znear;
};

CamDev make_cam(const gs_camera& c);

// ---- batched launches over views --------------------------------------------------------------
// A launch over V views of one scene has grid y = V. Each per-view array of the batch is the
// concatenation of the views' arrays ([V][n][..] by splat, [V][3][H][W] images, [V] framebuffers);
// each view's scratch is its own slab of `ws` bytes of the workspace. Kernels move every pointer
// by blockIdx.y times that array's per-view size (view 0 of a one-view launch moves nothing).
constexpr int MAX_VIEWS = 16;

struct CamSet {
    CamDev c[MAX_VIEWS];
};

struct Views {
    int count;         // V >= 1
    uint64_t ws;       // bytes between two views' workspace slabs
};

inline Views one_view() { return Views{1, 0}; }

// ---- layout of the raster workspace -------------------------------------------------------
constexpr int TILE = 32;              // pixels per side of the tile one workgroup owns
constexpr int REC_BYTES = 48;         // one staged splat record
// floats per splat in the gradient accumulation buffer: the nine sums [0, 9), the rounding errors
// of the tile reduction's compensated adds to them [9, 18) (zero in the per-fragment modes), pad
constexpr int GRAD_STRIDE = 20;
constexpr int GRAD_LO = 9;

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

struct RasterWs {
    void* rec;         // [n] records in sorted order
    void* rect;        // [n] uint2 tile rectangles
    void* idrec;       // [n] 64-byte per-id records, the setup's staging in id order
    float* grad;       // [n * GRAD_STRIDE] (backward only)
    float* bgpart;     // [tiles][4] per-tile dL/dbackground partial sums (backward only)
    unsigned long long* counters;  // [16] planner scratch: [0] the work-item count, [1] the status word
    uint32_t* status;  // device status word (gs_status_bits), cleared by every raster setup;
                       // status[2] holds the bits of the view's largest |colour| (the forward's
                       // saturation exit)
    uint32_t* weights; // [tiles] splat count per tile
    int32_t* order;    // [tiles] tiles, heaviest first
    uint32_t* bwd_w;   // [tiles] the backward's walk length per tile (forward's estimate)
    int32_t* bwd_order; // [tiles] tiles by bwd_w, heaviest first
    uint32_t* bits;    // [tiles][wpr] occupancy bitmap: one bit per 64 sorted splats
    int wpr;           // words per bitmap row (0: no bitmap)
    // depth-split forward (split != 0): per-tile splat counts of each 2048-position column,
    // work items (tile, first column, end column, partial slot), their order, per-tile segment
    // count and first item, and FP32 partial states of the split tiles' segments
    int split;
    uint16_t* colcnt;  // [tiles][wpr]
    int4* items;       // [4 tiles]
    uint32_t* item_w;  // [4 tiles]
    int32_t* item_order; // [4 tiles], -1 past the item count
    int32_t* tile_first; // [tiles]
    int32_t* tile_k;     // [tiles]
    float4* partial;     // [4 tiles][TILE * TILE]
};
size_t raster_ws_bytes(int n, int width, int height, bool bwd);
RasterWs carve_raster_ws(void* ws, int n, int width, int height, bool bwd);
// The status words of the views' slabs, OR-ed (synchronises the stream).
hipError_t raster_status(const void* ws, int n, int width, int height, uint32_t* out,
                         hipStream_t s, const Views& vs);
bool raster_has_split(int n, int width, int height);
hipError_t copy_raster_schedule(const void* ws, int n, int width, int height, int32_t* fwd_order,
                                int32_t* bwd_order, int32_t* item_order, int32_t* items,
                                int64_t* n_items, hipStream_t s, const Views& vs);

size_t sort_ws_bytes(int n, int key_bytes);
size_t compact_ws_bytes(int n);

// ---- launchers (return hipError_t of the last launch) -------------------------------------
hipError_t launch_preprocess(const CamSet& cams, const Views& vs, const gs_config& cfg, int n,
                             const float* means3d, const float* scales, const float* quats,
                             const float* opac, const float* sh, float* means2d, float* conics,
                             float* rgb, float* depth, uint32_t* keys, int32_t* ids,
                             int32_t* n_visible, void* ws, hipStream_t s);
// Sums the views' gradients: the 3D outputs are written once, after all V views.
hipError_t launch_preprocess_bwd(const CamSet& cams, int nviews, const gs_config& cfg, int n,
                                 const float* means3d, const float* scales, const float* quats,
                                 const float* opac, const float* sh, const float* g_means2d,
                                 const float* g_conics, const float* g_rgb, const float* g_opac2d,
                                 float* d_means3d, float* d_scales, float* d_quats, float* d_opac,
                                 float* d_sh, hipStream_t s);
hipError_t launch_prepare_2d(int width, int height, const gs_config& cfg, int n,
                             const float* means2d, const float* conics, const float* opac,
                             const float* depth, uint32_t* keys, int32_t* ids, int32_t* n_visible,
                             void* ws, hipStream_t s);
hipError_t launch_sort_u32(int n, uint32_t* keys, int32_t* vals, const int32_t* n_dev, void* ws,
                           hipStream_t s, const Views& vs = one_view());
hipError_t launch_sort_u64(int n, uint64_t* keys, int32_t* vals, const int32_t* n_dev,
                           int end_bit, void* ws, hipStream_t s);
// The depth sort with its scratch in the library's fixed per-device array (no workspace):
// n <= NOALLOC_SORT_MAX_N.
constexpr int NOALLOC_SORT_MAX_N = GS_NOALLOC_SORT_MAX_N;
constexpr int MAX_DEVICES = 64;
hipError_t launch_sort_u32_noalloc(int n, uint32_t* keys, int32_t* vals, const int32_t* n_dev,
                                   hipStream_t s);
// Fills `count` words at p in each of `views` slabs `stride` bytes apart.
hipError_t launch_fill_u32(void* p, size_t count, uint32_t value, hipStream_t s, int views = 1,
                           uint64_t stride = 0);
hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, size_t count, uint32_t* sums,
                                 hipStream_t s, const Views& vs = one_view());
hipError_t launch_compact(int n, const uint32_t* key_by_id, uint32_t* keys, int32_t* ids,
                          int32_t* n_visible, void* ws, hipStream_t s, const Views& vs = one_view());
hipError_t launch_raster_setup(const gs_config& cfg, int width, int height, int n,
                               const int32_t* sorted_ids, const int32_t* n_visible,
                               const float* means2d, const float* conics, const float* opac,
                               const float* rgb, void* ws, hipStream_t s,
                               const Views& vs = one_view());
hipError_t launch_raster_fwd(const gs_config& cfg, int width, int height, int n,
                             const int32_t* sorted_ids, const int32_t* n_visible,
                             const float* means2d, const float* conics, const float* opac,
                             const float* rgb, void* fb, float* out_rgb, float* out_T,
                             int32_t* out_cov, gs_stats* stats, void* ws, hipStream_t s,
                             const Views& vs = one_view());
hipError_t launch_raster_bwd(const gs_config& cfg, int width, int height, int n,
                             const int32_t* sorted_ids, const int32_t* n_visible,
                             const float* means2d, const float* conics, const float* opac,
                             const float* rgb, const void* fb, const float* dL_dimg,
                             float* g_means2d, float* g_conics, float* g_opac, float* g_rgb, const float* dL_dT, float* dL_dbg,
                             int32_t* out_live, gs_stats* stats, void* ws, hipStream_t s,
                             const Views& vs = one_view());


// ---- microbenchmarks ---------------------------------------------------------------------------
hipError_t launch_micro_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
hipError_t launch_micro_atomic(float* slots, size_t nslots, int per, int mode, hipStream_t s);

// ---- tile-based comparison rasterizer ------------------------------------------------------
size_t tile_ws_bytes(int n, size_t cap, int W, int H);
hipError_t launch_tile_prepare(const gs_config& cfg, int W, int H, int n, const int32_t* ids,
                               const int32_t* n_visible, const float* means2d,
                               const float* conics, const float* opac, uint32_t* n_pairs,
                               void* ws, hipStream_t s);
hipError_t launch_tile_fwd(const gs_config& cfg, int W, int H, int n, const int32_t* ids,
                           const uint32_t* keys, const float* means2d, const float* conics,
                           const float* opac, const float* rgb, const uint32_t* n_pairs,
                           size_t cap, float* out_rgb, float* out_T, int32_t* n_contrib, void* ws,
                           hipStream_t s);
hipError_t launch_tile_bwd(const gs_config& cfg, int W, int H, int n, const float* means2d,
                           const float* conics, const float* opac, const float* rgb,
                           const float* dL_dimg, const float* T_final, const int32_t* n_contrib,
                           size_t cap, float* g_m, float* g_c, float* g_o, float* g_rgb, void* ws,
                           hipStream_t s);

}  // namespace gsr
