// tile.hip -- the tile-based software rasterizer used as the comparison design (Sec. 2.1.3-2.1.4):
// 16x16-pixel tiles; every splat is duplicated into a (tile, depth) key per tile its footprint
// touches; the variable-size pair list is sorted by that key and cut into per-tile ranges; the
// forward composites each pixel front to back with T-culling and records its last contributor;
// the backward walks each pixel's list back to front, recovering T by division, and adds every
// fragment's gradients with its own atomics.
//
// The pair count is data dependent: gs_tile_prepare leaves it on the device and the caller reads
// it back to size the pair buffers before gs_tile_raster_fwd (the dynamic allocation the paper
// contrasts with a fixed framebuffer, Sec. 1).
#include "device.hpp"
#include "internal.hpp"

namespace gsr {

constexpr int BT = 16;          // tile side in pixels
constexpr int BT_THREADS = 256; // one pixel per thread

__device__ __forceinline__ bool splat_box(float mx, float my, float a, float b, float c, float o,
                                          float amin, int W, int H, uint32_t& x0, uint32_t& x1,
                                          uint32_t& y0, uint32_t& y1) {
    // det in FP64: the products of FP32 values are exact (thin splats cancel a c against b^2)
    const double det = (double)a * c - (double)b * b;
    if (!(a > 0.f && c > 0.f && det > 0.0 && o >= amin && isfinite(mx) && isfinite(my))) return false;
    const float detf = (float)det;
    const float r2 = 2.0f * logf(o / amin);
    const float hx = sqrtf(fmaxf(r2 * c / detf, 0.f)) * 1.001f + 0.01f;
    const float hy = sqrtf(fmaxf(r2 * a / detf, 0.f)) * 1.001f + 0.01f;
    const float fx0 = fminf(fmaxf(floorf(mx - hx - 0.5f), 0.f), (float)W);
    const float fx1 = fminf(fmaxf(floorf(mx + hx - 0.5f) + 1.f, 0.f), (float)W);
    const float fy0 = fminf(fmaxf(floorf(my - hy - 0.5f), 0.f), (float)H);
    const float fy1 = fminf(fmaxf(floorf(my + hy - 0.5f) + 1.f, 0.f), (float)H);
    if (!(fx0 < fx1 && fy0 < fy1)) return false;
    x0 = (uint32_t)fx0; x1 = (uint32_t)fx1; y0 = (uint32_t)fy0; y1 = (uint32_t)fy1;
    return true;
}

// Tiles touched by each visible splat (entries p < n_visible of the compacted list).
__global__ __launch_bounds__(256) void k_tile_count(
    int n, const int32_t* __restrict__ ids, const int32_t* __restrict__ nvis_ptr,
    const float* __restrict__ means2d, const float* __restrict__ conics,
    const float* __restrict__ opac, int W, int H, float amin, uint32_t* __restrict__ counts,
    uint2* __restrict__ rects) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int nvis = *nvis_ptr;
    nvis = nvis < 0 ? 0 : (nvis > n ? n : nvis);
    uint32_t cnt = 0;
    uint2 rr = make_uint2(0u, 0u);
    if (p < nvis) {
        const int id = ids[p];
        uint32_t x0, x1, y0, y1;
        if ((unsigned)id < (unsigned)n &&
            splat_box(means2d[2 * (size_t)id], means2d[2 * (size_t)id + 1], conics[3 * (size_t)id],
                      conics[3 * (size_t)id + 1], conics[3 * (size_t)id + 2], opac[id], amin, W, H,
                      x0, x1, y0, y1)) {
            const uint32_t tx0 = x0 / BT, tx1 = (x1 - 1) / BT, ty0 = y0 / BT, ty1 = (y1 - 1) / BT;
            cnt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
            rr = make_uint2(tx0 | (tx1 << 16), ty0 | (ty1 << 16));
        }
    }
    counts[p] = cnt;
    rects[p] = rr;
}

__global__ void k_tile_total(int n, const uint32_t* __restrict__ counts,
                             const uint32_t* __restrict__ offs, uint32_t* __restrict__ n_pairs) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *n_pairs = n > 0 ? offs[n - 1] + counts[n - 1] : 0u;
}

// One (tile << 32 | depth key) pair per touched tile; pairs beyond `cap` are dropped.
__global__ __launch_bounds__(256) void k_tile_dup(
    int n, const int32_t* __restrict__ ids, const uint32_t* __restrict__ keys,
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ offs,
    const uint2* __restrict__ rects, int tiles_x, uint32_t cap, uint64_t* __restrict__ pkeys,
    int32_t* __restrict__ pvals) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n || counts[p] == 0) return;
    const uint2 r = rects[p];
    const uint32_t tx0 = r.x & 0xFFFF, tx1 = r.x >> 16, ty0 = r.y & 0xFFFF, ty1 = r.y >> 16;
    uint32_t o = offs[p];
    const uint64_t k = keys[p];
    const int32_t id = ids[p];
    for (uint32_t ty = ty0; ty <= ty1; ++ty)
        for (uint32_t tx = tx0; tx <= tx1; ++tx, ++o)
            if (o < cap) {
                pkeys[o] = ((uint64_t)(ty * (uint32_t)tiles_x + tx) << 32) | k;
                pvals[o] = id;
            }
}

__global__ __launch_bounds__(256) void k_tile_ranges(const uint32_t* __restrict__ n_pairs,
                                                     uint32_t cap, const uint64_t* __restrict__ pkeys,
                                                     uint2* __restrict__ ranges) {
    const uint32_t np = min(*n_pairs, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
        const uint32_t t = (uint32_t)(pkeys[i] >> 32);
        if (i == 0 || (uint32_t)(pkeys[i - 1] >> 32) != t) ranges[t].x = i;
        if (i == np - 1 || (uint32_t)(pkeys[i + 1] >> 32) != t) ranges[t].y = i + 1;
    }
}

// A staged splat. The conic is kept in its LDL^T factors, q = a (dx + k dy)^2 + d dy^2 with
// k = b / a and d = det / a: two non-negative terms, where the expanded a dx^2 + 2b dx dy + c dy^2
// cancels large terms on long thin splats in FP32.
struct TRec {
    float mx, my, a, k, d, o, r, g, bl;
    int id;
};

__device__ __forceinline__ void load_trec(TRec& t, int id, const float* __restrict__ means2d,
                                          const float* __restrict__ conics,
                                          const float* __restrict__ opac,
                                          const float* __restrict__ rgb, int saturate) {
    t.id = id;
    t.mx = means2d[2 * (size_t)id];
    t.my = means2d[2 * (size_t)id + 1];
    const float a = conics[3 * (size_t)id], b = conics[3 * (size_t)id + 1],
                c = conics[3 * (size_t)id + 2];
    t.a = a;
    t.k = b / a;
    t.d = (float)((double)a * c - (double)b * b) / a;
    t.o = opac[id];
    t.r = rgb[3 * (size_t)id];
    t.g = rgb[3 * (size_t)id + 1];
    t.bl = rgb[3 * (size_t)id + 2];
    if (saturate) { t.r = fminf(t.r, 1.f); t.g = fminf(t.g, 1.f); t.bl = fminf(t.bl, 1.f); }
}

__global__ __launch_bounds__(BT_THREADS) void k_tile_fwd(
    const uint2* __restrict__ ranges, const int32_t* __restrict__ pvals,
    const float* __restrict__ means2d, const float* __restrict__ conics,
    const float* __restrict__ opac, const float* __restrict__ rgb, int W, int H, int tiles_x,
    float amin, float amax, float tmin, int saturate, float* __restrict__ out_rgb,
    float* __restrict__ out_T, int32_t* __restrict__ n_contrib) {
    __shared__ TRec s_rec[BT_THREADS];
    const int tile = blockIdx.x;
    const int X = (tile % tiles_x) * BT + (threadIdx.x % BT);
    const int Y = (tile / tiles_x) * BT + (threadIdx.x / BT);
    const bool valid = X < W && Y < H;
    const float px = X + 0.5f, py = Y + 0.5f;
    const uint2 rg = ranges[tile];
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;
    bool done = !valid;
    uint32_t last = 0;
    for (uint32_t b0 = rg.x; b0 < rg.y; b0 += BT_THREADS) {
        if (__syncthreads_count(!done) == 0) break;
        if (b0 + threadIdx.x < rg.y)
            load_trec(s_rec[threadIdx.x], pvals[b0 + threadIdx.x], means2d, conics, opac, rgb,
                      saturate);
        __syncthreads();
        const uint32_t m = min((uint32_t)BT_THREADS, rg.y - b0);
        for (uint32_t k = 0; k < m && !done; ++k) {
            const TRec& s = s_rec[k];
            const float dx = px - s.mx, dy = py - s.my;
            const float u = fmaf(s.k, dy, dx);
            const float q = fmaf(s.a * u, u, s.d * dy * dy);
            const float al = fminf(amax, s.o * __expf(-0.5f * q));
            if (al < amin) continue;
            const float w = al * T;
            C0 += w * s.r;
            C1 += w * s.g;
            C2 += w * s.bl;
            T *= 1.f - al;
            last = b0 + k - rg.x + 1;
            if (T < tmin) done = true;     // every later fragment would be T-culled
        }
    }
    if (valid) {
        const size_t i = (size_t)Y * W + X, P = (size_t)W * H;
        out_rgb[i] = C0;
        out_rgb[P + i] = C1;
        out_rgb[2 * P + i] = C2;
        out_T[i] = T;
        n_contrib[i] = (int32_t)last;
    }
}

__global__ __launch_bounds__(BT_THREADS) void k_tile_bwd(
    const uint2* __restrict__ ranges, const int32_t* __restrict__ pvals,
    const float* __restrict__ means2d, const float* __restrict__ conics,
    const float* __restrict__ opac, const float* __restrict__ rgb, int W, int H, int tiles_x,
    float amin, float amax, int saturate, const float* __restrict__ dL_dimg,
    const float* __restrict__ T_final, const int32_t* __restrict__ n_contrib,
    float* __restrict__ g_m, float* __restrict__ g_c, float* __restrict__ g_o,
    float* __restrict__ g_rgb) {
    __shared__ TRec s_rec[BT_THREADS];
    __shared__ uint32_t s_max;
    const int tile = blockIdx.x;
    const int X = (tile % tiles_x) * BT + (threadIdx.x % BT);
    const int Y = (tile / tiles_x) * BT + (threadIdx.x / BT);
    const bool valid = X < W && Y < H;
    const float px = X + 0.5f, py = Y + 0.5f;
    const uint2 rg = ranges[tile];
    const size_t i = (size_t)Y * W + X, P = (size_t)W * H;
    float G0 = 0.f, G1 = 0.f, G2 = 0.f, T = 1.f;
    uint32_t last = 0;
    if (valid) {
        G0 = dL_dimg[i]; G1 = dL_dimg[P + i]; G2 = dL_dimg[2 * P + i];
        T = T_final[i];
        last = (uint32_t)n_contrib[i];
    }
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    atomicMax(&s_max, last);
    __syncthreads();
    const uint32_t end = rg.x + s_max;
    float S0 = 0.f, S1 = 0.f, S2 = 0.f;    // contributions of the fragments behind, back to front
    for (uint32_t b1 = end; b1 > rg.x;) {
        const uint32_t b0 = b1 - min((uint32_t)BT_THREADS, b1 - rg.x);
        if (b0 + threadIdx.x < b1)
            load_trec(s_rec[threadIdx.x], pvals[b0 + threadIdx.x], means2d, conics, opac, rgb,
                      saturate);
        __syncthreads();
        for (int k = (int)(b1 - b0) - 1; k >= 0; --k) {
            if (b0 + k - rg.x >= last) continue;
            const TRec& s = s_rec[k];
            const float dx = px - s.mx, dy = py - s.my;
            const float u = fmaf(s.k, dy, dx);
            const float au = s.a * u;
            const float q = fmaf(au, u, s.d * dy * dy);
            const float e = __expf(-0.5f * q);
            const float araw = s.o * e;
            const float al = fminf(amax, araw);
            if (al < amin) continue;
            const float om = 1.f - al;
            T = T / om;                                 // T_i, transmittance before fragment i
            const float w = al * T;
            // Eq. 4 with the back-to-front running sum of the fragments behind
            const float ga = (G0 * (s.r * T - S0 / om) + G1 * (s.g * T - S1 / om) +
                              G2 * (s.bl * T - S2 / om));
            S0 += w * s.r; S1 += w * s.g; S2 += w * s.bl;
            const int id = s.id;
            atomic_add_f32(&g_rgb[3 * (size_t)id], G0 * w);
            atomic_add_f32(&g_rgb[3 * (size_t)id + 1], G1 * w);
            atomic_add_f32(&g_rgb[3 * (size_t)id + 2], G2 * w);
            if (araw < amax) {
                const float gq = -0.5f * ga * araw;
                atomic_add_f32(&g_o[id], ga * e);
                // dq/dmu = -2 Q d with Q d = (a u, k a u + d dy) in the factored form
                atomic_add_f32(&g_m[2 * (size_t)id], -2.f * gq * au);
                atomic_add_f32(&g_m[2 * (size_t)id + 1], -2.f * gq * fmaf(s.k, au, s.d * dy));
                atomic_add_f32(&g_c[3 * (size_t)id], gq * dx * dx);
                atomic_add_f32(&g_c[3 * (size_t)id + 1], 2.f * gq * dx * dy);
                atomic_add_f32(&g_c[3 * (size_t)id + 2], gq * dy * dy);
            }
        }
        __syncthreads();
        b1 = b0;
    }
}

// ---- host side -------------------------------------------------------------------------------

static int tiles16(int W, int H) { return ((W + BT - 1) / BT) * ((H + BT - 1) / BT); }

static int tile_bits(int ntiles) {
    int b = 0;
    while ((1 << b) < ntiles) ++b;
    return b;
}

struct TileWs {
    uint32_t* counts; uint32_t* offs; uint32_t* scan_sums; uint2* rects; uint2* ranges;
    uint64_t* pkeys; int32_t* pvals; void* sort_ws;
};

size_t tile_ws_bytes(int n, size_t cap, int W, int H) {
    const size_t nt = (size_t)tiles16(W, H);
    return align_up((size_t)n * 4) * 2 + align_up(((size_t)n / 4096 + 2) * 4) +
           align_up((size_t)n * 8) + align_up(nt * 8) + align_up(cap * 8) + align_up(cap * 4) +
           sort_ws_bytes((int)cap, 8);
}

static TileWs carve_tile_ws(void* ws, int n, size_t cap, int W, int H) {
    const size_t nt = (size_t)tiles16(W, H);
    TileWs t;
    char* p = (char*)ws;
    t.counts = (uint32_t*)p;    p += align_up((size_t)n * 4);
    t.offs = (uint32_t*)p;      p += align_up((size_t)n * 4);
    t.scan_sums = (uint32_t*)p; p += align_up(((size_t)n / 4096 + 2) * 4);
    t.rects = (uint2*)p;        p += align_up((size_t)n * 8);
    t.ranges = (uint2*)p;       p += align_up(nt * 8);
    t.pkeys = (uint64_t*)p;     p += align_up(cap * 8);
    t.pvals = (int32_t*)p;      p += align_up(cap * 4);
    t.sort_ws = p;
    return t;
}

hipError_t launch_tile_prepare(const gs_config& cfg, int W, int H, int n, const int32_t* ids,
                               const int32_t* n_visible, const float* means2d,
                               const float* conics, const float* opac, uint32_t* n_pairs,
                               void* ws, hipStream_t s) {
    TileWs t = carve_tile_ws(ws, n, 0, W, H);
    if (n == 0) return launch_fill_u32(n_pairs, 1, 0u, s);
    hipLaunchKernelGGL(k_tile_count, dim3((n + 255) / 256), dim3(256), 0, s, n, ids, n_visible,
                       means2d, conics, opac, W, H, cfg.alpha_min, t.counts, t.rects);
    hipError_t e = launch_exclusive_scan(t.counts, t.offs, (size_t)n, t.scan_sums, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_total, dim3(1), dim3(64), 0, s, n, t.counts, t.offs, n_pairs);
    return hipGetLastError();
}

hipError_t launch_tile_fwd(const gs_config& cfg, int W, int H, int n, const int32_t* ids,
                           const uint32_t* keys, const float* means2d, const float* conics,
                           const float* opac, const float* rgb, const uint32_t* n_pairs,
                           size_t cap, float* out_rgb, float* out_T, int32_t* n_contrib, void* ws,
                           hipStream_t s) {
    TileWs t = carve_tile_ws(ws, n, cap, W, H);
    const int tiles_x = (W + BT - 1) / BT, nt = tiles16(W, H);
    hipError_t e = launch_fill_u32(t.ranges, (size_t)nt * 2, 0u, s);
    if (e != hipSuccess) return e;
    if (n > 0 && cap > 0) {
        hipLaunchKernelGGL(k_tile_dup, dim3((n + 255) / 256), dim3(256), 0, s, n, ids, keys,
                           t.counts, t.offs, t.rects, tiles_x, (uint32_t)cap, t.pkeys, t.pvals);
        e = launch_sort_u64((int)cap, t.pkeys, t.pvals, (const int32_t*)n_pairs,
                            32 + tile_bits(nt), t.sort_ws, s);
        if (e != hipSuccess) return e;
        int blocks = (int)((cap + 255) / 256);
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(k_tile_ranges, dim3(blocks), dim3(256), 0, s, n_pairs, (uint32_t)cap,
                           t.pkeys, t.ranges);
    }
    const int sat = (cfg.fb_format == FB_UNORM16 || cfg.fb_format == FB_UNORM8) ? 1 : 0;
    hipLaunchKernelGGL(k_tile_fwd, dim3(nt), dim3(BT_THREADS), 0, s, t.ranges, t.pvals, means2d,
                       conics, opac, rgb, W, H, tiles_x, cfg.alpha_min, cfg.alpha_max,
                       cfg.t_min_bwd, sat, out_rgb, out_T, n_contrib);
    return hipGetLastError();
}

hipError_t launch_tile_bwd(const gs_config& cfg, int W, int H, int n, const float* means2d,
                           const float* conics, const float* opac, const float* rgb,
                           const float* dL_dimg, const float* T_final, const int32_t* n_contrib,
                           size_t cap, float* g_m, float* g_c, float* g_o, float* g_rgb, void* ws,
                           hipStream_t s) {
    TileWs t = carve_tile_ws(ws, n, cap, W, H);
    const int tiles_x = (W + BT - 1) / BT, nt = tiles16(W, H);
    hipError_t e = launch_fill_u32(g_m, (size_t)n * 2, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32(g_c, (size_t)n * 3, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32(g_o, (size_t)n, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32(g_rgb, (size_t)n * 3, 0u, s);
    if (e != hipSuccess) return e;
    const int sat = (cfg.fb_format == FB_UNORM16 || cfg.fb_format == FB_UNORM8) ? 1 : 0;
    hipLaunchKernelGGL(k_tile_bwd, dim3(nt), dim3(BT_THREADS), 0, s, t.ranges, t.pvals, means2d,
                       conics, opac, rgb, W, H, tiles_x, cfg.alpha_min, cfg.alpha_max, sat, dL_dimg,
                       T_final, n_contrib, g_m, g_c, g_o, g_rgb);
    return hipGetLastError();
}

}  // namespace gsr
