// raster.hip -- ordered splat compositing into a fixed-size per-pixel framebuffer (Eq. 2) and
// the front-to-back gradient procedure with quad/wave gradient reduction (Sec. 3.1-3.2,
// Procedures 1 and 2).
//
// Design (gfx950, wave64). CDNA has no rasterizer, no blend unit and no fragment interlock, so
// the ordering that programmable blending gives the paper (Sec. 3.1.1) comes from ownership:
//   * one workgroup (4 waves) owns a 32x32-pixel screen tile; each wave owns a 16x16 quadrant
//     made of four 8x8 sub-blocks; lane l holds the same position in each sub-block, and lanes
//     4k..4k+3 form a 2x2 pixel quad, so DPP quad_perm is the paper's quad;
//   * the workgroup walks the globally depth-sorted splat array in order (no per-tile lists,
//     memory O(N + pixels)) in rounds of up to 64 chunks of 64 sorted splats that the tile's
//     occupancy bitmap marks; the waves test the chunks' tile rectangles, compact the hits in
//     order into LDS and stage their records in LDS; every wave then applies the staged splats
//     one after another to its own pixels, whose state lives in VGPRs. A pixel is only ever
//     touched by one lane, in splat order, so no interlock is needed;
//   * per staged batch, each wave keeps only the splats whose alpha can reach alpha_min in one
//     of its sub-blocks, with a mask of those sub-blocks.
// Each iteration therefore processes one splat per wave across up to 64 lanes; that is the
// "subgroup" of Procedure 2, and its live lanes always share one splat id (cohesion 100 %).
#include <type_traits>

#include "device.hpp"
#include "internal.hpp"
#include "plan.hpp"

namespace gsr {

constexpr int NT = 256;            // threads per workgroup
constexpr int BATCH = 256;         // splat records staged in LDS at once
static_assert(BATCH == NT, "staging and the tile gradient flush give each thread one record");

// A staged splat: a = (mean x, mean y, a', k); b = (d', opacity, r, g);
// c = (bits of colour b, bits of log2 o, bits of p_min, splat id) where p_min = log2(alpha_min / o)
// is the least exponent whose alpha passes alpha_min.
//
// The conic Q = [[a, b], [b, c]] is stored in its LDL^T factors: q = d^T Q d =
// a (dx + k dy)^2 + (det Q / a) dy^2 with k = b / a, a sum of two non-negative terms. The
// expanded form a dx^2 + 2b dx dy + c dy^2 cancels terms of size q / (1 - rho^2) (rho the
// correlation of the footprint) down to q, which in FP32 loses several digits on long thin
// splats, e.g. those just beyond the near plane whose projected means lie thousands of pixels
// off-screen; the factored form costs the same instructions. det Q is formed in FP64 from the
// FP32 conic (products exact, one rounding), k and det Q / a in FP32, and they are stored
// pre-scaled, a' = -log2(e) a / 2 and d' = -log2(e) det Q / (2a), so that the exponent of
// alpha = o 2^p is p = a' u^2 + d' dy^2 = -q/2 log2(e), u = dx + k dy.
// Fields: a = (mean x, mean y, a', k), b = (d', opacity, r, g), c = (b colour, log2 opacity,
// p_min, splat id); the forward reads c.x and c.y together.
struct __align__(16) Rec {
    float4 a;
    float4 b;
    uint4 c;
};
static_assert(sizeof(Rec) == REC_BYTES, "record size");

constexpr float LOG2E = 1.4426950408889634f;
constexpr int WEIGHT_SAMPLE = 8;        // every 8th sorted splat votes for the tiles it touches
constexpr int CHUNK_SPLATS = 16;        // sorted splats per bit of the tile occupancy bitmap
// Occupied chunks a walk round takes. The forward walks every splat of a tile, so its rounds are
// large (fewer rounds, fuller staged batches); the backward stops where its pixels saturate, and
// a smaller round stages fewer splats past that point.
constexpr int ROUND_CHUNKS = 192;
constexpr int BWD_ROUND_CHUNKS = 64;
constexpr size_t BITMAP_BUDGET = 1024u << 20;  // the bitmap is skipped above this many bytes

// ---- schedule ------------------------------------------------------------------------------
// The work of a tile grows with the number of splats over it, which on clustered scenes varies
// by orders of magnitude across the screen. Workgroups are dispatched in block order (round-robin
// over the 8 XCDs, then to whichever CU has room), so listing the work heaviest first spreads the
// heavy tiles over all XCDs and starts them first: a longest-processing-time-first schedule. The
// order only has to be approximate, so it is a counting sort over weight buckets.
//
// Depth split. All tiles of a view are resident at once, so the forward lasts as long as its
// densest tile, whose workgroup walks its whole splat list alone. Compositing is associative:
// (C1, T1) then (C2, T2) gives (C1 + T1 C2, T1 T2). A tile heavier than the mean weight is
// therefore cut into up to MAX_SEGMENTS depth segments at 2048-position column boundaries, each
// carrying about the same number of splats (from exact per-column counts); each segment is a
// work item that composites from (0, 1) into an FP32 partial state, and k_raster_merge combines
// the segments in depth order. Only the at-rest, non-T-culled forward splits: T-culling and
// per-fragment rounding of the stored state need the segments' inputs in sequence. Shorter
// segments also keep each FP32 colour sum short.
constexpr int MAX_SPLIT_TILES = 4096;

// Exclusive scan of one value per thread over a workgroup of NBUCKETS (1024) threads: within each
// wave by shuffles, then over the 16 wave totals. Returns the prefix; *total gets the sum.
__device__ uint32_t block_scan_1024(uint32_t v, uint32_t* total) {
    __shared__ uint32_t s_wtot[NBUCKETS / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(incl, o);
        if (lane >= o) incl += u;
    }
    if (lane == 63) s_wtot[wave] = incl;
    __syncthreads();
    uint32_t before = 0u, all = 0u;
#pragma unroll
    for (int w2 = 0; w2 < NBUCKETS / 64; ++w2) {
        const uint32_t t = s_wtot[w2];
        before += w2 < wave ? t : 0u;
        all += t;
    }
    __syncthreads();                      // s_wtot may be reused by the next call
    if (total) *total = all;
    return before + incl - v;
}

// The schedulers' workgroup policy for bucket_order (plan.hpp): one workgroup of NBUCKETS threads.
struct WgBlock {
    template <class F>
    __device__ void each(F&& f) { f((int)threadIdx.x, (int)blockDim.x); }
    __device__ void sync() { __syncthreads(); }
    __device__ uint32_t atomic_inc(uint32_t* p) { return atomicAdd(p, 1u); }
    __device__ void exclusive_scan(uint32_t* h) {      // blockDim.x == NBUCKETS
        const uint32_t first = block_scan_1024(h[threadIdx.x], nullptr);
        h[threadIdx.x] = first;
    }
};

// Error bits of the device status word (gs_raster_status): a kernel that meets a schedule entry
// or a splat id outside its range records it here and skips that work instead of guessing.
__device__ __forceinline__ void flag_status(uint32_t* status, uint32_t bit) {
    if (status) atomicOr(status, bit);
}

// One workgroup: the tile order; with `split`, each tile's segment count k_t (its weight over
// the mean tile weight, rounded up, at most MAX_SEGMENTS) and the first item of each tile (an
// exclusive scan of k_t); counters[0] = number of items.
__global__ __launch_bounds__(NBUCKETS) void k_plan_tiles(
    const uint32_t* __restrict__ weights, int ntiles, int32_t* __restrict__ order, int split,
    int32_t* __restrict__ tile_k, int32_t* __restrict__ tile_first,
    unsigned long long* __restrict__ counters, uint32_t* __restrict__ bwd_w, uint64_t vws) {
    __shared__ uint32_t s_hist[NBUCKETS];
    __shared__ unsigned long long s_tot;
    __shared__ uint32_t s_max;
    weights = view_bytes(weights, vws);
    order = view_bytes(order, vws);
    tile_k = view_bytes(tile_k, vws);
    tile_first = view_bytes(tile_first, vws);
    counters = view_bytes(counters, vws);
    bwd_w = view_bytes(bwd_w, vws);
    const int tid = threadIdx.x;
    for (int t = tid; t < ntiles; t += blockDim.x) bwd_w[t] = weights[t];   // see k_raster_fwd
    if (tid == 0) { s_tot = 0ull; s_max = 0u; }
    __syncthreads();
    unsigned long long tot = 0ull;
    uint32_t mx = 0u;
    for (int t = tid; t < ntiles; t += blockDim.x) { tot += weights[t]; mx = max(mx, weights[t]); }
    atomicAdd(&s_tot, tot);
    atomicMax(&s_max, mx);
    __syncthreads();
    const unsigned long long total = s_tot;
    const uint32_t wmax = s_max;
    WgBlock blk;
    bucket_order(blk, weights, ntiles, wmax, order, ntiles, s_hist);
    if (!split) return;
    __syncthreads();
    // k_t segments per tile (segment_count), their exclusive scan the first item of each tile;
    // the items number at most ITEMS_PER_TILE ntiles (segment_cap)
    const uint32_t cap = segment_cap(total, ntiles);
    // exclusive scan of k_t over tiles: thread tid owns tiles [4 tid, 4 tid + 4) (ntiles <= 4096)
    int kk[4], loc = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int t = 4 * tid + r;
        int k = 0;
        if (t < ntiles) {
            k = segment_count(weights[t], cap);
            tile_k[t] = k;
        }
        kk[r] = k;
        loc += k;
    }
    uint32_t nitems = 0u;
    int run = (int)block_scan_1024((uint32_t)loc, &nitems);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int t = 4 * tid + r;
        if (t < ntiles) tile_first[t] = run;
        run += kk[r];
    }
    if (tid == 0) counters[0] = (unsigned long long)nitems;
}

// One wave per tile: the tile's work items. A tile with k_t = 1 is one item over all columns
// writing the framebuffer directly (slot -1); otherwise the column counts are scanned and cut
// where the running count first reaches j w_t / k_t.
__global__ __launch_bounds__(64) void k_plan_cuts(
    const uint32_t* __restrict__ weights, const uint16_t* __restrict__ colcnt, int ncol, int ntiles,
    const int32_t* __restrict__ tile_k, const int32_t* __restrict__ tile_first,
    int4* __restrict__ items, uint32_t* __restrict__ item_w, uint64_t vws) {
    weights = view_bytes(weights, vws);
    colcnt = view_bytes(colcnt, vws);
    tile_k = view_bytes(tile_k, vws);
    tile_first = view_bytes(tile_first, vws);
    items = view_bytes(items, vws);
    item_w = view_bytes(item_w, vws);
    const int t = blockIdx.x, lane = threadIdx.x;
    const int k = tile_k[t], f = tile_first[t];
    const uint32_t w = weights[t];
    if (k < 1 || f < 0 || f + k > ITEMS_PER_TILE * ntiles) return;
    if (k == 1) {
        if (lane == 0) { items[f] = make_int4(t, 0, ncol, -1); item_w[f] = w; }
        return;
    }
    __shared__ int cut[MAX_SEGMENTS + 1];            // in LDS: indexed by a runtime j below
    __shared__ uint32_t cum[MAX_SEGMENTS + 1];
    __shared__ uint32_t tgt[MAX_SEGMENTS];           // cut j where the count first reaches tgt[j]
    if (lane <= MAX_SEGMENTS) { cut[lane] = lane ? ncol : 0; cum[lane] = lane ? w : 0u; }
    if (lane < MAX_SEGMENTS) tgt[lane] = cut_target(w, lane, k);
    __syncthreads();
    int found = 1;                                   // next cut to find
    uint32_t base = 0u;
    const uint16_t* row = colcnt + (size_t)t * ncol;
    // the first PRE chunks of 64 columns are loaded together, later ones one at a time
    constexpr int PRE = 16;
    uint32_t pre[PRE];
#pragma unroll
    for (int i = 0; i < PRE; ++i) pre[i] = (i * 64 + lane < ncol) ? row[i * 64 + lane] : 0u;
    auto chunk = [&](int c0, uint32_t v) {
        for (int o = 1; o < 64; o <<= 1) {          // inclusive prefix over the wave
            const uint32_t u = __shfl_up(v, o);
            if (lane >= o) v += u;
        }
        const uint32_t incl = base + v;
        for (int j = found; j < k; ++j) {
            const uint64_t m = ballot(incl >= tgt[j] && c0 + lane < ncol);
            if (!m) break;                          // later targets are larger still
            const int l = __builtin_ctzll(m);
            if (lane == l) { cut[j] = c0 + l + 1; cum[j] = incl; }
            found = j + 1;
        }
        base = __shfl(incl, 63);
    };
#pragma unroll
    for (int i = 0; i < PRE; ++i)
        if (i * 64 < ncol && found < k) chunk(i * 64, pre[i]);
    for (int c0 = PRE * 64; c0 < ncol && found < k; c0 += 64)
        chunk(c0, (c0 + lane < ncol) ? row[c0 + lane] : 0u);
    __syncthreads();
    if (lane == 0) {
        cut[k] = ncol; cum[k] = w;
        for (int j = 0; j < k; ++j) {
            const int a = cut[j], b = max(cut[j], cut[j + 1]);
            items[f + j] = make_int4(t, a, b, f + j);
            item_w[f + j] = cum[j + 1] >= cum[j] ? cum[j + 1] - cum[j] : 0u;
        }
    }
}

// One workgroup: items heaviest first; item_order padded with -1 to 2 ntiles.
__global__ __launch_bounds__(NBUCKETS) void k_plan_items(
    const uint32_t* __restrict__ item_w, int ntiles, const unsigned long long* __restrict__ counters,
    int32_t* __restrict__ item_order, uint64_t vws) {
    __shared__ uint32_t s_hist[NBUCKETS];
    __shared__ uint32_t s_max;
    item_w = view_bytes(item_w, vws);
    counters = view_bytes(counters, vws);
    item_order = view_bytes(item_order, vws);
    const int cap = ITEMS_PER_TILE * ntiles;
    const int count = (int)min((unsigned long long)cap, counters[0]);
    if (threadIdx.x == 0) s_max = 0u;
    __syncthreads();
    uint32_t mx = 0u;
    for (int i = threadIdx.x; i < count; i += blockDim.x) mx = max(mx, item_w[i]);
    atomicMax(&s_max, mx);
    __syncthreads();
    WgBlock blk;
    bucket_order(blk, item_w, count, s_max, item_order, cap, s_hist);
}

// One workgroup: the backward's tile order, heaviest first by bwd_w (the forward's estimate of
// each tile's backward walk, else its whole weight).
__global__ __launch_bounds__(NBUCKETS) void k_plan_bwd(const uint32_t* __restrict__ bwd_w,
                                                       int ntiles, int32_t* __restrict__ order,
                                                       uint64_t vws) {
    __shared__ uint32_t s_hist[NBUCKETS];
    __shared__ uint32_t s_max;
    bwd_w = view_bytes(bwd_w, vws);
    order = view_bytes(order, vws);
    if (threadIdx.x == 0) s_max = 0u;
    __syncthreads();
    uint32_t mx = 0u;
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) mx = max(mx, bwd_w[t]);
    atomicMax(&s_max, mx);
    __syncthreads();
    WgBlock blk;
    bucket_order(blk, bwd_w, ntiles, s_max, order, ntiles, s_hist);
}

__device__ __forceinline__ bool rect_hit(uint2 r, uint32_t tx, uint32_t ty) {
    return (r.x & 0xFFFFu) <= tx && tx <= (r.x >> 16) && (r.y & 0xFFFFu) <= ty && ty <= (r.y >> 16);
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ---- setup: records, tile rectangles, occupancy bitmap and tile weights ---------------------
// Two kernels. k_raster_pack runs in splat-id order: it reads the caller's arrays coalesced and
// writes each splat's record fields and tile rectangle as one 64-byte IdRec. k_raster_setup runs
// in sorted order: one workgroup per SETUP_SPAN consecutive sorted positions = one column of
// the bitmap (COL_WORDS words, 128 chunks of 16 splats); each of its 1024 threads gathers its two
// splats' IdRecs by id (one cache line each, both in flight), writes the sorted records, and the
// workgroup gathers, in LDS, the column's chunk bits and a 16-bit splat count per tile, then
// writes its bitmap column with plain stores and adds its counts to the tile weights: one global
// atomic per (workgroup, touched tile), none contended within an instruction. The LDS arrays are
// sized to the image's tiles at launch (18 B per tile). The (splat, tile) pairs of each round of
// 1024 splats are spread evenly over the threads: a scan of the splats' pair counts gives each
// thread an equal run of consecutive pairs, whose first owner a binary search finds; the thread
// then walks the run tile by tile. One splat may cover every tile of the image, and a thread
// walking its own splats' tiles would leave the workgroup waiting on it.
constexpr int SETUP_SPAN = 2048;                // sorted positions per workgroup = one column
constexpr int SETUP_NT = 1024;                  // threads: 16 waves keep the gathers in flight
constexpr int SETUP_PER_THREAD = SETUP_SPAN / SETUP_NT;
constexpr int COL_CHUNKS = SETUP_SPAN / CHUNK_SPLATS;   // 128 chunks per column
constexpr int COL_WORDS = COL_CHUNKS / 32;              // 4 bitmap words per (tile, column)
static_assert(COL_WORDS == 4, "a column of a tile's bitmap row is stored as one uint4");
// 18 B of LDS per tile (4 words of bits, a 16-bit count) and 12.1 KB of fixed arrays in 160 KB
constexpr int MAX_LDS_TILES = 8192;
constexpr uint32_t NO_TILE_X = 0xFFFFu;         // rect.x of a splat that touches no tile

struct IdRec {
    Rec r;          // c.w (the splat id) is filled in by k_raster_setup
    uint2 rect;     // tile rectangle (tx0 | tx1 << 16, ty0 | ty1 << 16)
    uint2 pad;
};
static_assert(sizeof(IdRec) == 64, "one cache line per splat");

// Also clears the tile weights (the first workgroup; k_raster_setup adds to them after it).
__global__ __launch_bounds__(256) void k_raster_pack(
    int n, const float* __restrict__ means2d, const float* __restrict__ conics,
    const float* __restrict__ opac, const float* __restrict__ rgb, int W, int H, float amin,
    int saturate, IdRec* __restrict__ out, uint32_t* __restrict__ weights, int ntiles,
    uint32_t* __restrict__ status, uint64_t vws) {
    means2d = view_at(means2d, 2ull * n);
    conics = view_at(conics, 3ull * n);
    rgb = view_at(rgb, 3ull * n);          // opacities are the views' shared [n]
    out = view_bytes(out, vws);
    if (blockIdx.x == 0) {               // a new setup: weights and the status word start at 0
        weights = view_bytes(weights, vws);
        for (int t = threadIdx.x; t < ntiles; t += blockDim.x) weights[t] = 0u;
        if (threadIdx.x == 0) {
            *view_bytes(status, vws) = 0u;
            *view_bytes(status + 2, vws) = 0u;      // the largest |colour| (k_raster_setup)
        }
    }
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    const float mx = means2d[2 * (size_t)id], my = means2d[2 * (size_t)id + 1];
    const float a = conics[3 * (size_t)id], b = conics[3 * (size_t)id + 1],
                c = conics[3 * (size_t)id + 2];
    const float o = opac[id];
    float cr = rgb[3 * (size_t)id], cg = rgb[3 * (size_t)id + 1], cb = rgb[3 * (size_t)id + 2];
    if (saturate) { cr = fminf(cr, 1.f); cg = fminf(cg, 1.f); cb = fminf(cb, 1.f); }
    IdRec q;
    q.r.a = make_float4(0.f, 0.f, 0.f, 0.f);
    q.r.b = make_float4(0.f, 0.f, 0.f, 0.f);
    q.r.c = make_uint4(0u, 0u, 0u, 0u);
    q.rect = make_uint2(NO_TILE_X, 0u);
    q.pad = make_uint2(0u, 0u);
    // det in FP64: the products of FP32 values are exact, so its sign is exact and its one
    // rounding leaves it accurate to FP32 even when a c and b^2 nearly cancel
    const double det = (double)a * c - (double)b * b;
    if (a > 0.f && c > 0.f && det > 0.0 && o >= amin && isfinite(mx) && isfinite(my)) {
        const float detf = (float)det;
        // alpha >= alpha_min  <=>  q <= r2 = 2 ln(o / alpha_min): the ellipse's half extents are
        // sqrt(r2 Sigma_xx), sqrt(r2 Sigma_yy) with Sigma = conic^-1; padded so FP32 rounding
        // never puts a passing pixel outside the box.
        const float r2 = 2.0f * logf(o / amin);
        const float hx = sqrtf(fmaxf(r2 * c / detf, 0.f)) * 1.001f + 0.01f;
        const float hy = sqrtf(fmaxf(r2 * a / detf, 0.f)) * 1.001f + 0.01f;
        const float fx0 = fminf(fmaxf(floorf(mx - hx - 0.5f), 0.f), (float)W);
        const float fx1 = fminf(fmaxf(floorf(mx + hx - 0.5f) + 1.f, 0.f), (float)W);
        const float fy0 = fminf(fmaxf(floorf(my - hy - 0.5f), 0.f), (float)H);
        const float fy1 = fminf(fmaxf(floorf(my + hy - 0.5f) + 1.f, 0.f), (float)H);
        if (fx0 < fx1 && fy0 < fy1) {
            const uint32_t x0 = (uint32_t)fx0, x1 = (uint32_t)fx1;
            const uint32_t y0 = (uint32_t)fy0, y1 = (uint32_t)fy1;
            q.r.a = make_float4(mx, my, -0.5f * LOG2E * a, b / a);
            q.r.b = make_float4(-0.5f * LOG2E * (detf / a), o, cr, cg);
            const float lo = log2f(o);
            const float pmin = log2f(amin) - lo;
            q.r.c = make_uint4(__float_as_uint(cb), __float_as_uint(lo), __float_as_uint(pmin), 0u);
            q.rect = make_uint2((x0 / TILE) | (((x1 - 1) / TILE) << 16),
                                (y0 / TILE) | (((y1 - 1) / TILE) << 16));
        }
    }
    out[id] = q;
}

__global__ __launch_bounds__(SETUP_NT) void k_raster_setup(
    int n, const int32_t* __restrict__ sorted_ids, const int32_t* __restrict__ nvis_ptr,
    const IdRec* __restrict__ idrec, int tiles_x, int ntiles, Rec* __restrict__ rec,
    uint2* __restrict__ rect, uint32_t* __restrict__ weights,
    uint32_t* __restrict__ bits, int wpr, uint16_t* __restrict__ colcnt,
    uint32_t* __restrict__ status, uint64_t vws) {
    // when ntiles <= MAX_LDS_TILES: [ntiles][COL_WORDS] chunk bits, then the tiles' 16-bit
    // counts two to a word (a count is at most SETUP_SPAN, so an add never carries across)
    extern __shared__ uint32_t s_dyn[];
    uint32_t* s_bits = s_dyn;
    uint32_t* s_cnt = s_dyn + (size_t)ntiles * COL_WORDS;
    sorted_ids = view_at(sorted_ids, (uint64_t)n);
    nvis_ptr = view_at(nvis_ptr, 1);
    idrec = view_bytes(idrec, vws);
    rec = view_bytes(rec, vws);
    rect = view_bytes(rect, vws);
    weights = view_bytes(weights, vws);
    bits = view_bytes(bits, vws);
    colcnt = view_bytes(colcnt, vws);
    const bool in_lds = ntiles <= MAX_LDS_TILES;
    const int ncol = wpr / COL_WORDS;
    if (in_lds)
        for (int t = threadIdx.x; t < ntiles * COL_WORDS + (ntiles + 1) / 2; t += blockDim.x)
            s_dyn[t] = 0u;
    __syncthreads();
    int nvis = *nvis_ptr;
    nvis = nvis < 0 ? 0 : (nvis > n ? n : nvis);
    const int p0 = blockIdx.x * SETUP_SPAN;
    int ids[SETUP_PER_THREAD];
#pragma unroll
    for (int j = 0; j < SETUP_PER_THREAD; ++j) {
        const int p = p0 + j * SETUP_NT + threadIdx.x;
        const int id = p < nvis ? sorted_ids[p] : -1;
        ids[j] = (unsigned)id < (unsigned)n ? id : -1;
        if (p < nvis && ids[j] < 0) flag_status(view_bytes(status, vws), GS_STATUS_BAD_ID);
    }
    IdRec q[SETUP_PER_THREAD];
#pragma unroll
    for (int j = 0; j < SETUP_PER_THREAD; ++j)
        if (ids[j] >= 0) q[j] = idrec[ids[j]];
    float cmax_l = 0.f;
    __shared__ uint32_t s_first[SETUP_NT + 1];   // exclusive scan of the round's pair counts
    __shared__ uint2 s_rect[SETUP_NT];
    __shared__ uint32_t s_wtot[SETUP_NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int j = 0; j < SETUP_PER_THREAD; ++j) {
        const int p = p0 + j * SETUP_NT + tid;
        uint2 rr = make_uint2(NO_TILE_X, 0u);
        if (p < n && ids[j] >= 0 && q[j].rect.x != NO_TILE_X) {
            Rec r = q[j].r;
            r.c.w = (uint32_t)ids[j];  // the splat's gradient slot
            rec[p] = r;
            rr = q[j].rect;
        }
        if (p < n) rect[p] = rr;
        if (rr.x != NO_TILE_X) {             // the view's largest |colour| (saturation exit)
            const float cm = fmaxf(fmaxf(fabsf(q[j].r.b.z), fabsf(q[j].r.b.w)),
                                   fabsf(__uint_as_float(q[j].r.c.x)));
            cmax_l = fmaxf(cmax_l, cm);
        }
        const uint32_t tx0 = rr.x & 0xFFFFu, tx1 = rr.x >> 16;
        const uint32_t ty0 = rr.y & 0xFFFFu, ty1 = rr.y >> 16;
        const uint32_t cnt = rr.x != NO_TILE_X ? (tx1 - tx0 + 1) * (ty1 - ty0 + 1) : 0u;
        if (!in_lds) {                     // sampled weights only: each thread walks its own pairs
            if (p % WEIGHT_SAMPLE == 0 && cnt)
                for (uint32_t ty = ty0; ty <= ty1; ++ty)
                    for (uint32_t tx = tx0; tx <= tx1; ++tx)
                        atomicAdd(&weights[ty * (uint32_t)tiles_x + tx], 1u);
            continue;
        }
        uint32_t incl = cnt;               // inclusive scan over the wave, then over the waves
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(incl, o);
            if (lane >= o) incl += u;
        }
        if (lane == 63) s_wtot[wave] = incl;
        __syncthreads();
        uint32_t before = 0u;
        for (int w2 = 0; w2 < wave; ++w2) before += s_wtot[w2];
        s_first[tid] = before + incl - cnt;
        s_rect[tid] = rr;
        if (tid == SETUP_NT - 1) s_first[SETUP_NT] = before + incl;
        __syncthreads();
        const uint32_t total = s_first[SETUP_NT];
        const uint32_t per = (total + SETUP_NT - 1u) / SETUP_NT;
        const uint32_t k0 = min((uint32_t)tid * per, total), k1 = min(k0 + per, total);
        if (k0 < k1) {
            int i = 0;                     // owner of pair k0: the last entry whose first pair <= k0
#pragma unroll
            for (int step = SETUP_NT / 2; step > 0; step >>= 1)
                if (s_first[i + step] <= k0) i += step;
            uint2 ro = s_rect[i];
            uint32_t w = (ro.x >> 16) - (ro.x & 0xFFFFu) + 1u;
            const uint32_t local = k0 - s_first[i];
            uint32_t ty = (ro.y & 0xFFFFu) + local / w, tx = (ro.x & 0xFFFFu) + local % w;
            uint32_t next = s_first[i + 1];   // first pair of the next entry
            for (uint32_t k = k0; k < k1; ++k) {
                while (k >= next) {           // the run moves on to the next splat with pairs
                    ++i;
                    next = s_first[i + 1];
                    ro = s_rect[i];
                    w = (ro.x >> 16) - (ro.x & 0xFFFFu) + 1u;
                    tx = ro.x & 0xFFFFu;
                    ty = ro.y & 0xFFFFu;
                }
                const uint32_t t = ty * (uint32_t)tiles_x + tx;
                const uint32_t c = (uint32_t)(j * SETUP_NT + i) / CHUNK_SPLATS;   // < COL_CHUNKS
                atomicOr(&s_bits[t * COL_WORDS + (c >> 5)], 1u << (c & 31u));
                atomicAdd(&s_cnt[t >> 1], 1u << ((t & 1u) << 4));
                if (++tx > (ro.x >> 16)) { tx = ro.x & 0xFFFFu; ++ty; }
            }
        }
        __syncthreads();                   // s_first / s_rect are rewritten by the next round
    }
    {   // the workgroup's largest |colour|, one atomic per workgroup (non-negative floats order
        // as their bits)
        __shared__ float s_cm[SETUP_NT / 64];
        float m = cmax_l;
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        if (lane == 0) s_cm[wave] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w2 = 1; w2 < SETUP_NT / 64; ++w2) m = fmaxf(m, s_cm[w2]);
            if (m > 0.f) atomicMax(view_bytes(status, vws) + 2, __float_as_uint(m));
        }
    }
    if (in_lds)
        for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
            const uint32_t cnt = (s_cnt[t >> 1] >> ((t & 1) << 4)) & 0xFFFFu;
            if (wpr > 0) {
                const uint32_t* sb = s_bits + (size_t)t * COL_WORDS;
                reinterpret_cast<uint4*>(bits + (size_t)t * wpr)[blockIdx.x] =
                    make_uint4(sb[0], sb[1], sb[2], sb[3]);
            }
            if (colcnt) colcnt[(size_t)t * ncol + blockIdx.x] = (uint16_t)cnt;
            if (cnt) atomicAdd(&weights[t], cnt);
        }
}

// ---- the shared walk ------------------------------------------------------------------------
// Rounds of up to RC occupied chunks (chunk = 16 consecutive sorted splats; occupied = its bit is
// set in the tile's occupancy bitmap). Wave w tests the splats of the round's chunks
// [RC/4 w, RC/4 (w + 1)) against the tile, so the four waves' hit lists concatenate in sorted
// order; the hits are staged into LDS in batches. A dense tile's round is 16 RC splats; a
// sparse tile skips the chunks none of whose splats touch it. Most (tile, splat) pairs are
// sparse: a tile's splats lie far apart in depth order, so an occupied chunk holds one or two
// hits, and the chunk size sets how many rectangles the walk tests per hit. The LDS state is sized
// for the round length RC.
template <int RC>
struct Walk {
    static constexpr int SPAN = RC / 4 * CHUNK_SPLATS;   // hits one wave can hold per round
    Rec rec[BATCH];             // first: its reads take small immediate offsets
    uint16_t seg[4][SPAN];      // per wave: hits as chunk slot * CHUNK_SPLATS + splat
    uint16_t list[4][BATCH];
    int chunk[RC];              // the round's chunks, increasing
    int nchunk;
    int segn[4];
    int alive[4];
};

// alpha = o exp(-q/2) = exp2(log2 o + p) with p = a' u^2 + d' dy^2, u = dx + k dy (the record's
// pre-scaled LDL^T factors). A lane's four pixels share two columns and two rows, so the row part
// log2 o + d' dy^2 is formed once per row; each pixel then costs u, a' u, one FMA and the exp2.
// The forward and the backward evaluate alpha with these same operations, so they take the same
// alpha_min decisions.
__device__ __forceinline__ void alpha_rows(const float4& A, const float4& B, float lo,
                                           const float (&px)[4], const float (&py)[4],
                                           float (&dx)[2], float (&dy)[2], float (&er)[2]) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        dx[j] = px[j] - A.x;          // columns: sub-blocks 0 and 1
        dy[j] = py[2 * j] - A.y;      // rows: sub-blocks 0 and 2
        er[j] = fmaf(B.x * dy[j], dy[j], lo);
    }
}
__device__ __forceinline__ float alpha_raw(const float4& A, float dx, float dy, float er) {
    const float u = fmaf(A.w, dy, dx);
    return __builtin_amdgcn_exp2f(fmaf(A.z * u, u, er));
}
// min(alpha_max, raw) for raw >= 0, as one median-of-three that takes alpha_max from a scalar
// register (fminf would re-canonicalise it every iteration)
__device__ __forceinline__ float clamp_alpha(float raw, float amax) {
    return __builtin_amdgcn_fmed3f(raw, 0.f, amax);
}

// Per-wave culling of a staged batch. Lane j takes staged splat k0 + j and bounds its exponent
// over each of the wave's four 8x8 sub-blocks: with c the sub-block centre and g the gradient of
// p there, p(c + d) = p(c) + g.d + d^T Q' d <= p(c) + 3.5 (|g_x| + |g_y|) over the pixel centres
// (|d_x|, |d_y| <= 3.5), since Q' (the pre-scaled conic, negative definite) adds nothing positive.
// A sub-block whose bound stays below p_min (with a margin far above the FP32 error of the
// bound) holds no fragment with alpha >= alpha_min. The splats that reach at least one
// sub-block are compacted in order into w.list[wave] as k | mask << 8; returns their count.
template <int RC>
__device__ __forceinline__ int cull_batch(Walk<RC>& w, int m, int wave, int lane, uint64_t lt,
                                          float cx0, float cy0) {
    int cnt = 0;
    for (int k0 = 0; k0 < m; k0 += 64) {
        const int k = k0 + lane;
        uint32_t mask = 0u;
        if (k < m) {
            const float4 A = w.rec[k].a;
            const float4 B = w.rec[k].b;
            const float pmin = __uint_as_float(w.rec[k].c.z);
            const float dx0 = cx0 - A.x, dy0 = cy0 - A.y;
#pragma unroll
            for (int sb = 0; sb < 4; ++sb) {
                const float dx = dx0 + (float)((sb & 1) * 8), dy = dy0 + (float)((sb >> 1) * 8);
                const float u = fmaf(A.w, dy, dx);
                const float au = A.z * u, dd = B.x * dy;
                const float p0 = fmaf(au, u, dd * dy);
                const float slack = 7.0f * (fabsf(au) + fabsf(fmaf(A.w, au, dd)));
                const float margin = 1e-3f + 1e-5f * (slack - p0);
                if (p0 + slack >= pmin - margin) mask |= 1u << sb;
            }
        }
        const uint64_t hit = ballot(mask != 0u);
        if (mask) w.list[wave][cnt + popc(hit & lt)] = (uint16_t)(k | (mask << 8));
        cnt += popc(hit);
    }
    // the list is written and read by this wave only: order its LDS traffic
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return cnt;
}

// Wave 0: the next (up to) RC occupied chunks in [cursor, cend) into w.chunk / w.nchunk, and the
// cursor moved past them (every chunk counts as occupied without a bitmap). One bitmap word per
// lane; a wave prefix sum of the words' popcounts places each lane's chunks.
template <int RC>
__device__ __forceinline__ void next_round(Walk<RC>& w, const uint32_t* __restrict__ trow,
                                           int cend, int lane, int& cursor) {
    int cc = cursor, got = 0;
    if (!trow) {
        got = min(RC, max(0, cend - cc));
        for (int l = lane; l < got; l += 64) w.chunk[l] = cc + l;
        cc += got;
    } else {
        while (got < RC && cc < cend) {
            const int wi = (cc >> 5) + lane;
            uint32_t word = wi * 32 < cend ? trow[wi] : 0u;
            if (lane == 0) word &= ~0u << (cc & 31);           // chunks before the cursor
            const int left = cend - wi * 32;                   // chunks from cend on
            if (left < 32) word &= left > 0 ? (1u << left) - 1u : 0u;
            const int pc = popc(word);
            int incl = pc;
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(incl, o);
                if (lane >= o) incl += u;
            }
            const int excl = incl - pc, need = RC - got;
            const int take = max(0, min(pc, need - excl));
            int last = -1;
            for (int t = 0; t < take; ++t) {
                const int bit = __builtin_ctz(word);
                word &= word - 1u;
                last = wi * 32 + bit;
                w.chunk[got + excl + t] = last;
            }
            const int total = __shfl(incl, 63);
            if (total >= need) {                              // the round is full
                const uint64_t edge = ballot(excl < need && incl >= need);
                cc = __shfl(last, (int)__builtin_ctzll(edge)) + 1;
                got = RC;
            } else {
                got += total;
                cc = ((cc >> 5) + 64) * 32;                    // all 64 words consumed
            }
        }
    }
    cursor = cc;
    if (lane == 0) w.nchunk = got;
}

// Wave `wave`: tests the splats of the round's chunk slots [RC/4 wave, RC/4 (wave + 1)) against
// the tile, four chunks per step (lane = 16 x slot offset + splat), two steps' loads in flight;
// writes the in-order hits to w.seg[wave] (slot * CHUNK_SPLATS + splat) and their count to
// w.segn.
template <int RC>
__device__ __forceinline__ void scan_round(Walk<RC>& w, const uint2* __restrict__ rect, int nvis,
                                           uint32_t ttx, uint32_t tty, int wave, int lane,
                                           uint64_t lt) {
    constexpr int PER_STEP = 64 / CHUNK_SPLATS, WAVE_CHUNKS = RC / 4;
    int cnt = 0;
    const int s0 = wave * WAVE_CHUNKS, s1 = min(w.nchunk, s0 + WAVE_CHUNKS);
    const int sub = lane / CHUNK_SPLATS, idx = lane % CHUNK_SPLATS;
    for (int sl = s0; sl < s1; sl += 2 * PER_STEP) {
        const int sa = sl + sub, sb = sl + PER_STEP + sub;
        const int o0 = sa < s1 ? w.chunk[sa] * CHUNK_SPLATS + idx : nvis;
        const int o1 = sb < s1 ? w.chunk[sb] * CHUNK_SPLATS + idx : nvis;
        const uint2 r0 = o0 < nvis ? rect[o0] : make_uint2(0xFFFFu, 0u);
        const uint2 r1 = o1 < nvis ? rect[o1] : make_uint2(0xFFFFu, 0u);
        const bool h0 = rect_hit(r0, ttx, tty);
        const uint64_t m0 = ballot(h0);
        if (h0) w.seg[wave][cnt + popc(m0 & lt)] = (uint16_t)(sa * CHUNK_SPLATS + idx);
        cnt += popc(m0);
        const bool h1 = rect_hit(r1, ttx, tty);
        const uint64_t m1 = ballot(h1);
        if (h1) w.seg[wave][cnt + popc(m1 & lt)] = (uint16_t)(sb * CHUNK_SPLATS + idx);
        cnt += popc(m1);
    }
    if (lane == 0) w.segn[wave] = cnt;
}

// Stages hits [b0, b0 + BATCH) of the round (in order across the four waves' lists).
// The record's c.w is the splat id, which names its gradient slot: an id outside [0, n) (a setup
// that does not belong to these inputs) is flagged in the status word and kept in bounds.
template <int RC>
__device__ __forceinline__ void stage(Walk<RC>& w, const Rec* __restrict__ rec, int n, int b0,
                                      int total, int tid, uint32_t* __restrict__ status) {
    const int e = b0 + tid;
    if (e < total) {
        int off = e, ws = 0;
        if (off >= w.segn[0]) {
            off -= w.segn[0]; ws = 1;
            if (off >= w.segn[1]) {
                off -= w.segn[1]; ws = 2;
                if (off >= w.segn[2]) { off -= w.segn[2]; ws = 3; }
            }
        }
        const uint32_t v = w.seg[ws][off];
        const int pos = w.chunk[v / CHUNK_SPLATS] * CHUNK_SPLATS + (int)(v % CHUNK_SPLATS);
        Rec r = rec[pos];
        if (r.c.w >= (uint32_t)n) {
            flag_status(status, GS_STATUS_STALE_RECORD);
            r.c.w = (uint32_t)(n - 1);
        }
        w.rec[tid] = r;
    }
}

// ---- forward -------------------------------------------------------------------------------
// A half-precision value in a 32-bit slot of its own: arrays of these are not packed two to a
// register, which would cost a merge after every half-word update.
struct Half32 {
    _Float16 h;
    uint16_t pad;
    __device__ Half32() = default;
    __device__ Half32(float x) : h((_Float16)x) {}
    __device__ explicit operator float() const { return (float)h; }
};

// One workgroup per work item: a whole tile (items == nullptr: block b takes tile order[b]) or,
// in the depth-split forward, one depth segment of a tile (columns [c_begin, c_end) of 2048
// sorted positions), which writes its FP32 (C, T) to partial[slot] instead of the framebuffer.
// Occupancy: LDS (21.3 KB per workgroup) allows 7 workgroups per CU; the second bound asks the
// compiler for 7 waves per SIMD (<= 72 VGPRs), which measured faster than 6 with fewer spills.
// MULTI: a launch over several views (grid y). Its per-view pointers cost scalar registers that
// the one-view instances, whose walk pointers stay plain kernel arguments, do not pay.
//
// Saturation exit (at-rest state, no counters, `freeze` set): after each staged batch a wave
// drops the sub-blocks in which no pixel's stored state can change any more: T <= 1e-6 and, in
// FP32, C_ch + 2 T c_max == C_ch for each channel, c_max the view's largest |colour|. A later
// fragment adds T alpha c with |T alpha c| <= T c_max, which rounds to C under that condition
// (rounding is monotone in the addend), so C is bit-identical to compositing every covered
// fragment and T is within 1e-6 of its final value. The walk of a tile ends when all its
// sub-blocks are done. A call that asks for per-pixel coverage walks every fragment (exact
// counts); one that only counts statistics counts the fragments the exit composites.
template <int RFMT, bool TCULL, bool INSTR, bool MULTI>
__global__ __launch_bounds__(NT, 7) void k_raster_fwd(
    int n, const int32_t* __restrict__ nvis_ptr, const Rec* __restrict__ rec,
    const uint2* __restrict__ rect, const int32_t* __restrict__ order,
    const uint32_t* __restrict__ bits, int wpr, int W, int H, int tiles_x, int ntiles,
    const int4* __restrict__ items, const int32_t* __restrict__ item_order,
    float4* __restrict__ partial,
    float amin, float amax, float tmin, float tsat, float bg0, float bg1, float bg2, int fb_fmt,
    void* __restrict__ fb, float* __restrict__ out_rgb, float* __restrict__ out_T,
    int32_t* __restrict__ out_cov, unsigned long long* __restrict__ stats,
    uint32_t* __restrict__ bwd_w, uint32_t* __restrict__ status, int freeze_on, uint64_t vws) {
    __shared__ Walk<ROUND_CHUNKS> w;
    status = view_bytes(status, vws);
    constexpr bool FREEZE = RFMT < 0 && !TCULL;
    constexpr bool ALIVE = TCULL || FREEZE;        // sub-blocks can drop out of the walk
    const bool freeze = FREEZE && freeze_on;
    const float cm2 = freeze ? 2.f * __uint_as_float(status[2]) : 0.f;
    if constexpr (MULTI) {   // this view's walk state (its outputs are located at the write-back)
        nvis_ptr = view_at(nvis_ptr, 1);
        bwd_w = view_bytes(bwd_w, vws);
        rec = view_bytes(rec, vws);
        rect = view_bytes(rect, vws);
        order = view_bytes(order, vws);
        bits = view_bytes(bits, vws);
        items = view_bytes(items, vws);
        item_order = view_bytes(item_order, vws);
    }
    const int ncol = wpr / COL_WORDS;               // columns of SETUP_SPAN sorted positions
    int tile, c_begin = 0, c_end = ncol, slot = -1;
    // A schedule entry outside its range (a schedule not built for this launch) is recorded in the
    // status word and its work is skipped: each tile must be composited exactly once.
    if (items) {
        const int it = item_order[blockIdx.x];
        if (it < 0) return;                                        // past the item count
        if (it >= ITEMS_PER_TILE * ntiles) {
            if (threadIdx.x == 0) flag_status(status, GS_STATUS_FWD_SCHEDULE);
            return;
        }
        const int4 v = items[it];
        tile = v.x; c_begin = v.y; c_end = v.z; slot = v.w;
        if ((unsigned)tile >= (unsigned)ntiles || slot >= ITEMS_PER_TILE * ntiles ||
            c_begin < 0 || c_end < c_begin) {
            if (threadIdx.x == 0) flag_status(status, GS_STATUS_FWD_SCHEDULE);
            return;
        }
    } else {
        tile = order[blockIdx.x];
        if ((unsigned)tile >= (unsigned)ntiles) {
            if (threadIdx.x == 0) flag_status(status, GS_STATUS_FWD_SCHEDULE);
            return;
        }
    }
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = uniform(tid >> 6);
    const uint32_t ttx = (uint32_t)(tile % tiles_x), tty = (uint32_t)(tile / tiles_x);
    const int wx0 = (int)ttx * TILE + (wave & 1) * 16, wy0 = (int)tty * TILE + (wave >> 1) * 16;
    const int qd = lane >> 2;
    const int lx = ((qd & 3) << 1) | (lane & 1), ly = ((qd >> 2) << 1) | ((lane >> 1) & 1);
    const uint64_t lt = mask_lt(lane);
    const float cx0 = (float)wx0 + 4.f, cy0 = (float)wy0 + 4.f;   // centre of sub-block 0

    // The running (C, T) as the framebuffer holds it. A half-precision framebuffer's state stays
    // in half registers: the blend's mixed-precision FMAs read it and round their results to it
    // directly, with no widening after every update.
    using St = typename std::conditional<RFMT == FB_F16, Half32, float>::type;
    float px[4], py[4];
    St C[4][3], T[4];
    bool valid[4];
    uint32_t nev[4], ncov[4];
    uint32_t alive = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int X = wx0 + (s & 1) * 8 + lx, Y = wy0 + (s >> 1) * 8 + ly;
        valid[s] = X < W && Y < H;
        px[s] = (float)X + 0.5f;
        py[s] = (float)Y + 0.5f;
        C[s][0] = C[s][1] = C[s][2] = (St)0.f;
        T[s] = (St)1.f;
        nev[s] = ncov[s] = 0;
        if (ballot(valid[s])) alive |= 1u << s;
    }
    int nvis = *nvis_ptr;
    nvis = nvis < 0 ? 0 : (nvis > n ? n : nvis);
    uint32_t nq = 0;
    // chunks [COL_CHUNKS c_begin, cend) of this item
    const uint32_t* trow = wpr > 0 ? bits + (size_t)tile * wpr : nullptr;
    const int nch = (nvis + CHUNK_SPLATS - 1) / CHUNK_SPLATS;
    const int cend = c_end >= ncol ? nch : min(nch, c_end * COL_CHUNKS);
    int cursor = c_begin * COL_CHUNKS;            // wave 0's position in the walk
    // The backward's schedule: each wave counts the splats of its culled lists until every one of
    // its pixels has T below the backward's T-cull threshold, which is the work the backward's
    // wave will do on this tile (it walks the same lists and stops there).
    uint32_t wl = 0, nwalk = 0, nempty = 0, nchk = 0, nbat = 0;
    bool wsat = false;
    for (;;) {
        if (wave == 0) next_round<ROUND_CHUNKS>(w, trow, cend, lane, cursor);
        __syncthreads();
        if (w.nchunk == 0) break;
        scan_round<ROUND_CHUNKS>(w, rect, nvis, ttx, tty, wave, lane, lt);
        __syncthreads();
        const int total = w.segn[0] + w.segn[1] + w.segn[2] + w.segn[3];
        if (INSTR) { nq += total; nchk += w.nchunk; nbat += (total + BATCH - 1) / BATCH; }
        bool stop = false;
        for (int b0 = 0; b0 < total; b0 += BATCH) {
            stage(w, rec, n, b0, total, tid, status);
            __syncthreads();
            const int m = min(BATCH, total - b0);
            if (!ALIVE || alive) {
                const int nlist = cull_batch(w, m, wave, lane, lt, cx0, cy0);
                if (!wsat) wl += (uint32_t)nlist;
                if (INSTR) nwalk += (uint32_t)nlist;
                // the list is read 64 entries at a time, one per lane, and each entry is taken
                // from its lane by readlane (no LDS round trip per entry)
                for (int i0 = 0; i0 < nlist; i0 += 64) {
                    const int ents = i0 + lane < nlist ? (int)w.list[wave][i0 + lane] : 0;
                    // a scalar bound: as a min the compiler forms it as a vector median and spends
                    // two VALU operations per entry on the loop test
                    const int iend = __builtin_amdgcn_readfirstlane(min(64, nlist - i0));
                    for (int i = 0; i < iend; ++i) {
                        const uint32_t ent = (uint32_t)__builtin_amdgcn_readlane(ents, i);
                        const int k = (int)(ent & 0xFFu);
                        const float4 A = w.rec[k].a;
                        const float4 B = w.rec[k].b;
                        const uint4 Cw = w.rec[k].c;
                        const float cb = __uint_as_float(Cw.x);
                        // the exponent's row part (log2 o folded in) for the lane's two pixel rows
                        float dxs[2], dys[2], er[2];
                        const uint32_t sb = (ent >> 8) & (ALIVE ? alive : 0xFu);
                        alpha_rows(A, B, __uint_as_float(Cw.y), px, py, dxs, dys, er);
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            if ((sb >> s) & 1u) {
                                // the test on the unclamped alpha: alpha_max > alpha_min, so
                                // min(alpha_max, raw) >= alpha_min exactly when raw >= alpha_min
                                const float raw = alpha_raw(A, dxs[s & 1], dys[s >> 1], er[s >> 1]);
                                bool pass = raw >= amin;
                                if (TCULL) pass = pass && (float)T[s] >= tmin;
                                if (pass) {
                                    const float al = clamp_alpha(raw, amax);
                                    const float Ts = (float)T[s];
                                    const float wt = al * Ts;
                                    if constexpr (RFMT == FB_F16) {   // one rounding to half each
                                        C[s][0] = (St)fmaf(wt, B.z, (float)C[s][0]);
                                        C[s][1] = (St)fmaf(wt, B.w, (float)C[s][1]);
                                        C[s][2] = (St)fmaf(wt, cb, (float)C[s][2]);
                                        T[s] = (St)fmaf(-Ts, al, Ts);   // T (1 - alpha), Eq. 5
                                    } else {
                                        C[s][0] = fmaf(wt, B.z, C[s][0]);
                                        C[s][1] = fmaf(wt, B.w, C[s][1]);
                                        C[s][2] = fmaf(wt, cb, C[s][2]);
                                        T[s] = Ts - wt;                 // T (1 - alpha), Eq. 5
                                        if constexpr (RFMT >= 0) {
                                            C[s][0] = fb_round<RFMT>(C[s][0]);
                                            C[s][1] = fb_round<RFMT>(C[s][1]);
                                            C[s][2] = fb_round<RFMT>(C[s][2]);
                                            T[s] = fb_round<RFMT>(T[s]);
                                        }
                                    }
                                }
                                if (INSTR) {
                                    nev[s] += valid[s];
                                    ncov[s] += (pass && valid[s]);
                                    nempty += ballot(pass && valid[s]) == 0ull;
                                }
                                if (TCULL && !ballot(valid[s] && (float)T[s] >= tmin))
                                    alive &= ~(1u << s);
                            }
                        }
                    }
                }
            }
            if (!wsat) {
                bool a = false;
#pragma unroll
                for (int s = 0; s < 4; ++s) a = a || (valid[s] && (float)T[s] >= tsat);
                wsat = ballot(a) == 0ull;
            }
            if (FREEZE && freeze) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    if (!((alive >> s) & 1u)) continue;
                    const float Ts = (float)T[s];
                    const float inc = cm2 * Ts;
                    const bool done = !valid[s] ||
                                      (Ts <= 1e-6f && (float)C[s][0] + inc == (float)C[s][0] &&
                                       (float)C[s][1] + inc == (float)C[s][1] &&
                                       (float)C[s][2] + inc == (float)C[s][2]);
                    if (!ballot(!done)) alive &= ~(1u << s);
                }
            }
            if (ALIVE && lane == 0) w.alive[wave] = (int)alive;
            __syncthreads();
            if (ALIVE && !(w.alive[0] | w.alive[1] | w.alive[2] | w.alive[3])) { stop = true; break; }
        }
        if (ALIVE && stop) break;
    }
    // A walk from the front of the tile knows the backward's work on it: the largest wave count
    // (the waves run side by side). A first depth segment that leaves some wave unsaturated
    // keeps the setup's whole tile weight, which is larger.
    if (bwd_w && c_begin == 0) {
        __syncthreads();
        if (lane == 0) w.alive[wave] = (int)(wl | (wsat ? 0u : 0x80000000u));
        __syncthreads();
        if (tid == 0) {
            uint32_t mx = 0u;
            bool all_sat = true;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t x = (uint32_t)w.alive[v];
                mx = max(mx, x & 0x7FFFFFFFu);
                all_sat = all_sat && !(x >> 31);
            }
            if (slot < 0 || all_sat) bwd_w[tile] = mx;
        }
    }

    if (slot >= 0) {                              // a depth segment: FP32 partial state
        float4* part = (MULTI ? view_bytes(partial, vws) : partial) + (size_t)slot * (TILE * TILE);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int lxp = (wave & 1) * 16 + (s & 1) * 8 + lx, lyp = (wave >> 1) * 16 + (s >> 1) * 8 + ly;
            part[lyp * TILE + lxp] = make_float4((float)C[s][0], (float)C[s][1], (float)C[s][2],
                                                 (float)T[s]);
        }
        return;
    }
    const size_t P = (size_t)W * H;
    const size_t vp = MULTI ? (size_t)blockIdx.y * P : 0;   // first pixel of this view's images
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (!valid[s]) continue;
        const int X = wx0 + (s & 1) * 8 + lx, Y = wy0 + (s >> 1) * 8 + ly;
        const size_t i = vp + (size_t)Y * W + X;
        const size_t ic = 2 * vp + i;             // channel 0 of out_rgb's [3][H][W] view
        // the background behind the last splat (a final blend in per-fragment mode)
        const float Ts = (float)T[s];
        float4 v = make_float4(fmaf(Ts, bg0, (float)C[s][0]), fmaf(Ts, bg1, (float)C[s][1]),
                               fmaf(Ts, bg2, (float)C[s][2]), Ts);
        if constexpr (RFMT >= 0) {
            v.x = fb_round<RFMT>(v.x); v.y = fb_round<RFMT>(v.y); v.z = fb_round<RFMT>(v.z);
        }
        fb_store(fb, fb_fmt, i, v);
        if (out_rgb) {
            out_rgb[ic] = v.x;
            out_rgb[P + ic] = v.y;
            out_rgb[2 * P + ic] = v.z;
        }
        if (out_T) out_T[i] = v.w;
        if (INSTR && out_cov) out_cov[i] = (int32_t)ncov[s];
    }
    if (INSTR && stats) {
        uint32_t e = nev[0] + nev[1] + nev[2] + nev[3];
        uint32_t c = ncov[0] + ncov[1] + ncov[2] + ncov[3];
        e = wave_sum_u32(e);
        c = wave_sum_u32(c);
        if (lane == 0) {
            if (wave == 0) atomicAdd(&stats[0], (unsigned long long)nq);
            atomicAdd(&stats[1], (unsigned long long)e);
            atomicAdd(&stats[2], (unsigned long long)c);
            atomicAdd(&stats[10], (unsigned long long)nwalk);
            atomicAdd(&stats[11], (unsigned long long)nempty);
            if (wave == 0) {
                atomicAdd(&stats[12], (unsigned long long)nchk);
                atomicAdd(&stats[13], (unsigned long long)nbat);
            }
        }
    }
}

// Depth-split forward: combines a split tile's segment states in depth order,
// (C, T) <- (C + T C_j, T T_j), and writes the framebuffer and the FP32 copies.
__global__ __launch_bounds__(256) void k_raster_merge(
    int ntiles, int tiles_x, int W, int H, const int32_t* __restrict__ tile_k,
    const int32_t* __restrict__ tile_first, const float4* __restrict__ partial, float bg0,
    float bg1, float bg2, int fb_fmt, void* __restrict__ fb, float* __restrict__ out_rgb,
    float* __restrict__ out_T, uint64_t vws) {
    const uint64_t PV = (uint64_t)W * H;
    tile_k = view_bytes(tile_k, vws);
    tile_first = view_bytes(tile_first, vws);
    partial = view_bytes(partial, vws);
    fb = view_bytes(fb, PV * fb_bytes_per_pixel(fb_fmt));
    out_rgb = view_at(out_rgb, 3 * PV);
    out_T = view_at(out_T, PV);
    const int t = blockIdx.x;
    const int k = tile_k[t], f = tile_first[t];
    if (k <= 1 || f < 0 || f + k > ITEMS_PER_TILE * ntiles) return;
    const int tx = t % tiles_x, ty = t / tiles_x;
    const size_t P = (size_t)W * H;
    for (int lp = threadIdx.x; lp < TILE * TILE; lp += blockDim.x) {
        const int X = tx * TILE + (lp % TILE), Y = ty * TILE + (lp / TILE);
        if (X >= W || Y >= H) continue;
        float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;
        for (int j = 0; j < k; ++j) {
            const float4 v = partial[(size_t)(f + j) * (TILE * TILE) + lp];
            C0 = fmaf(T, v.x, C0);
            C1 = fmaf(T, v.y, C1);
            C2 = fmaf(T, v.z, C2);
            T *= v.w;
        }
        const size_t i = (size_t)Y * W + X;
        float4 v = make_float4(fmaf(T, bg0, C0), fmaf(T, bg1, C1), fmaf(T, bg2, C2), T);
        fb_store(fb, fb_fmt, i, v);                 // v becomes the stored (rounded) state
        if (out_rgb) { out_rgb[i] = v.x; out_rgb[P + i] = v.y; out_rgb[2 * P + i] = v.z; }
        if (out_T) out_T[i] = v.w;
    }
}

// ---- backward ------------------------------------------------------------------------------

struct BwdCounts {
    uint32_t evaluated, live, sets, wave_red, quad_red, cohesive;
};

// Procedure 2 (ReduceGradient) for one splat and one wave: `g` holds this lane's gradient
// contribution (zero when not live); `gp` is the splat's slot in the accumulation buffer.
template <bool INSTR>
__device__ __forceinline__ void reduce_commit(float (&g)[9], bool live, float* __restrict__ gp,
                                              int mode, int X, int lane, BwdCounts& cnt) {
    const uint64_t m = ballot(live);
    if (m == 0) return;
    const int nl = popc(m);
    if (mode == GS_REDUCE_NAIVE) {
        if (live)
#pragma unroll
            for (int j = 0; j < 9; ++j) atomic_add_f32(gp + j, g[j]);
        if (INSTR && lane == 0) cnt.sets += nl;
        return;
    }
    // All live lanes of the wave hold the same splat (one splat per wave iteration), so
    // subgroupAllEqual(i) holds; the wave path needs only the live-lane threshold X.
    if (mode != GS_REDUCE_QUAD && nl >= X) {
        float tot[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) tot[j] = wave_sum(g[j]);
        if (lane == __builtin_ctzll(m))          // subgroupBallotFindLSB(reduceMask)
#pragma unroll
            for (int j = 0; j < 9; ++j) atomic_add_f32(gp + j, tot[j]);
        if (INSTR && lane == 0) { cnt.sets += 1; cnt.wave_red += 1; cnt.cohesive += 1; }
        return;
    }
    if (mode == GS_REDUCE_WAVE) {                // standalone subgroup reduction: no quad path
        if (live)
#pragma unroll
            for (int j = 0; j < 9; ++j) atomic_add_f32(gp + j, g[j]);
        if (INSTR && lane == 0) cnt.sets += nl;
        return;
    }
#pragma unroll
    for (int j = 0; j < 9; ++j) g[j] = quad_sum(g[j]);
    const uint32_t qm = (uint32_t)(m >> (lane & ~3)) & 0xFu;   // reduceMask restricted to the quad
    const bool leader = qm != 0u && (uint32_t)(lane & 3) == (uint32_t)__builtin_ctz(qm | 0x10u);
    if (leader)
#pragma unroll
        for (int j = 0; j < 9; ++j) atomic_add_f32(gp + j, g[j]);
    if (INSTR) {
        const uint64_t lm = ballot(leader);
        if (lane == 0) { cnt.sets += popc(lm); cnt.quad_red += 1; cnt.cohesive += 1; }
    }
}

// GS_REDUCE_TILE: adds the staged batch's LDS accumulator (9 sums per entry) to the splats'
// gradient slots, one set of compensated global atomics per splat and tile (a splat's slot
// collects one add per tile it covers; compensation keeps that sum independent of the order in
// which the tiles arrive, FP32 throughout), and clears it. Thread t takes
// values t, t + NT, ..., so consecutive lanes add consecutive values of a slot and one wave's
// atomics touch about 7 slots' cache lines instead of 64. Reads other entries' records: the caller
// waits at a barrier before restaging them. Called before each restage and once after the walk.
template <bool INSTR, int RC>
__device__ __forceinline__ void flush_tile_grad(float* __restrict__ tg, const Walk<RC>& w,
                                                int pend, int tid, float* __restrict__ grad,
                                                BwdCounts& cnt) {
    if (INSTR) {                                  // sets committed: entries with a non-zero sum
        bool any = false;
        if (tid < pend)
            for (int j = 0; j < 9; ++j) any = any || tg[tid * 9 + j] != 0.f;
        cnt.sets += any;
        __syncthreads();                          // before any value below is cleared
    }
#pragma unroll 1
    for (int k = 0; k < 9; ++k) {
        const int q = tid + k * NT;               // value q: entry q / 9, gradient q % 9
        if (q < pend * 9) {
            const float v = tg[q];
            if (v != 0.f) {
                const int e = q / 9;
                float* hi = grad + (size_t)w.rec[e].c.w * GRAD_STRIDE + (q - 9 * e);
                atomic_add_f32_comp(hi, hi + GRAD_LO, v);
            }
        }
        tg[q] = 0.f;
    }
}

// TILEM: an instance for GS_REDUCE_TILE alone, without the per-fragment reduction paths of the
// paper's modes (the instances with TILEM = false take every mode from `mode`). It runs six
// workgroups per CU (80 VGPRs, 25.9 KB of LDS each): with a few registers spilled that measured
// faster than five without spills.
template <int RFMT, bool INSTR, bool MULTI, bool TILEM>
__global__ __launch_bounds__(NT, TILEM ? 6 : 1) void k_raster_bwd(
    int n, const int32_t* __restrict__ nvis_ptr, const Rec* __restrict__ rec,
    const uint2* __restrict__ rect, const int32_t* __restrict__ order,
    const uint32_t* __restrict__ bits, int wpr, int W, int H, int tiles_x,
    float amin, float amax, float tmin, int fb_fmt, const void* __restrict__ fb,
    const float* __restrict__ dL_dimg, const float* __restrict__ dL_dT,
    int mode, int X, float* __restrict__ grad, float* __restrict__ bgpart,
    int32_t* __restrict__ out_live, unsigned long long* __restrict__ stats,
    uint32_t* __restrict__ status, uint64_t vws) {
    __shared__ Walk<BWD_ROUND_CHUNKS> w;
    status = view_bytes(status, vws);
    __shared__ float tg[BATCH * 9];     // GS_REDUCE_TILE: per staged splat, the tile's gradient
    if constexpr (MULTI) {
        const uint64_t PV = (uint64_t)W * H;
        nvis_ptr = view_at(nvis_ptr, 1);
        rec = view_bytes(rec, vws);
        rect = view_bytes(rect, vws);
        order = view_bytes(order, vws);
        bits = view_bytes(bits, vws);
        grad = view_bytes(grad, vws);
        bgpart = view_bytes(bgpart, vws);
        fb = view_bytes(fb, PV * fb_bytes_per_pixel(fb_fmt));
        dL_dimg = view_at(dL_dimg, 3 * PV);
        dL_dT = view_at(dL_dT, PV);
        out_live = view_at(out_live, PV);
    }
    const int tile = order[blockIdx.x];
    if ((unsigned)tile >= gridDim.x) {     // a schedule not built for this grid: recorded, skipped
        if (threadIdx.x == 0) flag_status(status, GS_STATUS_BWD_SCHEDULE);
        return;
    }
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = uniform(tid >> 6);
    const uint32_t ttx = (uint32_t)(tile % tiles_x), tty = (uint32_t)(tile / tiles_x);
    const int wx0 = (int)ttx * TILE + (wave & 1) * 16, wy0 = (int)tty * TILE + (wave >> 1) * 16;
    const int qd = lane >> 2;
    const int lx = ((qd & 3) << 1) | (lane & 1), ly = ((qd >> 2) << 1) | ((lane >> 1) & 1);
    const uint64_t lt = mask_lt(lane);
    const float cx0 = (float)wx0 + 4.f, cy0 = (float)wy0 + 4.f;   // centre of sub-block 0
    const size_t P = (size_t)W * H;
    const bool tile_acc = TILEM || (mode == GS_REDUCE_TILE);
    int pend = 0;                       // staged entries whose LDS gradients are not yet flushed
    if (tile_acc)
#pragma unroll
        for (int j = 0; j < 9; ++j) tg[tid * 9 + j] = 0.f;

    // Procedure 1's per-pixel state (C', T), initialised to (C, 1) from the framebuffer, the
    // read-only dL/dC and, for a loss on the final transmittance, gTT = dL/dT_final T_final
    // (T_final = prod (1 - alpha_j) contributes -gTT / (1 - alpha_i) to dL/dalpha_i).
    float px[4], py[4], Cp[4][3], T[4], G[4][3], gTT[4];
    // The tile instance with the state at rest carries only D = dL/dC . C' + gTT per pixel:
    // Eq. 7 needs C' only through that dot product, and Eqs. 5-6 update it as D -= w (dL/dC . c).
    float D[4];
    float gbg[3] = {0.f, 0.f, 0.f};     // this lane's share of dL/dbackground = sum dL/dC T_final
    bool valid[4];
    uint32_t nlive[4];
    uint32_t alive = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int X = wx0 + (s & 1) * 8 + lx, Y = wy0 + (s >> 1) * 8 + ly;
        valid[s] = X < W && Y < H;
        px[s] = (float)X + 0.5f;
        py[s] = (float)Y + 0.5f;
        T[s] = 1.f;
        nlive[s] = 0;
        Cp[s][0] = Cp[s][1] = Cp[s][2] = 0.f;
        G[s][0] = G[s][1] = G[s][2] = 0.f;
        gTT[s] = 0.f;
        D[s] = 0.f;
        if (valid[s]) {
            const size_t i = (size_t)Y * W + X;
            const float4 v = fb_load(fb, fb_fmt, i);
            Cp[s][0] = v.x; Cp[s][1] = v.y; Cp[s][2] = v.z;
            G[s][0] = dL_dimg[i]; G[s][1] = dL_dimg[P + i]; G[s][2] = dL_dimg[2 * P + i];
            if (dL_dT) gTT[s] = dL_dT[i] * v.w;
            D[s] = fmaf(G[s][2], v.z, fmaf(G[s][1], v.y, fmaf(G[s][0], v.x, gTT[s])));
            gbg[0] = fmaf(G[s][0], v.w, gbg[0]);
            gbg[1] = fmaf(G[s][1], v.w, gbg[1]);
            gbg[2] = fmaf(G[s][2], v.w, gbg[2]);
        }
        if (ballot(valid[s])) alive |= 1u << s;
    }
    int nvis = *nvis_ptr;
    nvis = nvis < 0 ? 0 : (nvis > n ? n : nvis);
    BwdCounts cnt = {0, 0, 0, 0, 0, 0};
    uint32_t nq = 0;
    // tile_scale: the factors the tile instance at rest leaves out of its per-fragment sums, for
    // the totals that row r's first lane holds after wave_sum9 (gradients j0 and j0 + 4 with
    // j0 = 0, 2, 1, 3 for r = 0..3; gradient 5, row 2's, takes the entry's 1/o)
    const int lrow = lane >> 4;
    const float sa = lrow == 1 ? -0.5f : (lrow == 3 ? -1.f : -2.f * (1.0f / LOG2E));
    const float sb = lrow == 0 ? -0.5f : 1.f;
    const bool lane_acc = TILEM || (mode == GS_REDUCE_HYBRID_LANE || mode == GS_REDUCE_TILE);

    const uint32_t* trow = wpr > 0 ? bits + (size_t)tile * wpr : nullptr;
    const int nch = (nvis + CHUNK_SPLATS - 1) / CHUNK_SPLATS;
    int cursor = 0;                               // wave 0's position in the walk
    for (;;) {
        if (wave == 0) next_round<BWD_ROUND_CHUNKS>(w, trow, nch, lane, cursor);
        __syncthreads();
        if (w.nchunk == 0) break;
        scan_round<BWD_ROUND_CHUNKS>(w, rect, nvis, ttx, tty, wave, lane, lt);
        __syncthreads();
        const int total = w.segn[0] + w.segn[1] + w.segn[2] + w.segn[3];
        if (INSTR) nq += total;
        bool stop = false;
        for (int b0 = 0; b0 < total; b0 += BATCH) {
            if (tile_acc) {
                flush_tile_grad<INSTR>(tg, w, pend, tid, grad, cnt);
                pend = 0;
                __syncthreads();                  // the flush read other threads' records
            }
            stage(w, rec, n, b0, total, tid, status);
            __syncthreads();
            const int m = min(BATCH, total - b0);
            pend = m;
            const int nlist = alive ? cull_batch(w, m, wave, lane, lt, cx0, cy0) : 0;
            // the list is read 64 entries at a time, one per lane (readlane takes each entry)
            for (int i0 = 0; i0 < nlist && alive; i0 += 64) {
                const int ents = i0 + lane < nlist ? (int)w.list[wave][i0 + lane] : 0;
                const int iend = __builtin_amdgcn_readfirstlane(min(64, nlist - i0));
                for (int i = 0; i < iend && alive; ++i) {
                    const uint32_t ent = (uint32_t)__builtin_amdgcn_readlane(ents, i);
                    const int k = (int)(ent & 0xFFu);
                    const float4 A = w.rec[k].a;
                    const float4 B = w.rec[k].b;
                    const uint4 Cw = w.rec[k].c;
                    const float cr = B.z, cg = B.w, cb = __uint_as_float(Cw.x);
                    float* gp = grad + (size_t)uniform(Cw.w) * GRAD_STRIDE;
                    float dxs[2], dys[2], er[2];
                    alpha_rows(A, B, __uint_as_float(Cw.y), px, py, dxs, dys, er);
                    const float inv_o = __builtin_amdgcn_rcpf(B.y);
                    float acc[9];
#pragma unroll
                    for (int j = 0; j < 9; ++j) acc[j] = 0.f;
                    bool acc_live = false;
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        if (!((ent >> (8 + s)) & 1u) || !((alive >> s) & 1u)) continue;
                        const float dx = dxs[s & 1], dy = dys[s >> 1];
                        const float u = fmaf(A.w, dy, dx);
                        const float au = A.z * u;
                        // the forward's alpha (alpha_raw), with a' u kept for the gradient
                        const float araw = __builtin_amdgcn_exp2f(fmaf(au, u, er[s >> 1]));
                        const float al = clamp_alpha(araw, amax);
                        // cullingFlag: splat boundary (alpha < 1/255, tested on the unclamped alpha
                        // as in the forward), then T-Culling (T < 1e-4)
                        const bool live = valid[s] && araw >= amin && T[s] >= tmin;
                        if constexpr (TILEM) {
                            // Straight-line body: a lane that is not live takes alpha = 0 and a
                            // zero dL/dalpha, so every sum and the state update leave it as it is.
                            // (Behind divergent branches the compiler copied the nine sums at
                            // every join.) Live lanes do the operations of the paper modes below.
                            if (ballot(live)) {
                                acc_live = true;
                                const float Ti = T[s];
                                const float alm = live ? al : 0.f;
                                const float wt = alm * Ti;
                                // Eq. 3: dL/dc = dL/dC alpha T
                                acc[6] = fmaf(G[s][0], wt, acc[6]);
                                acc[7] = fmaf(G[s][1], wt, acc[7]);
                                acc[8] = fmaf(G[s][2], wt, acc[8]);
                                if constexpr (RFMT < 0) {
                                    // Eq. 7 as dL/dC . c T - D, and Eqs. 5-6 applied to D
                                    const float gc =
                                        fmaf(G[s][2], cb, fmaf(G[s][1], cg, G[s][0] * cr));
                                    const float ga = fmaf(gc, Ti, -D[s]) *
                                                     __builtin_amdgcn_rcpf(1.f - al);
                                    D[s] = fmaf(-wt, gc, D[s]);
                                    T[s] = Ti - wt;
                                    // h = dL/dalpha alpha (zero through a clamped alpha); the
                                    // sums below leave out factors that are the same for every
                                    // fragment of the entry: dL/do = (1/o) sum h; dL/dq =
                                    // -1/2 h, so the conic sums carry -1/2 (the cross term -1)
                                    // and the mean sums -2 / log2(e) (the pre-scaled factors).
                                    // They are applied to the wave's totals (tile_scale).
                                    const float h = (live && araw < amax) ? ga * araw : 0.f;
                                    acc[5] += h;
                                    const float gy = fmaf(A.w, au, B.x * dy);
                                    acc[0] = fmaf(h, au, acc[0]);
                                    acc[1] = fmaf(h, gy, acc[1]);
                                    const float hdx = h * dx;
                                    acc[2] = fmaf(hdx, dx, acc[2]);
                                    acc[3] = fmaf(hdx, dy, acc[3]);
                                    acc[4] = fmaf(h * dy, dy, acc[4]);
                                } else {
                                    // Eq. 7, and the final transmittance's share
                                    const float ga = (G[s][0] * (cr * Ti - Cp[s][0]) +
                                                      G[s][1] * (cg * Ti - Cp[s][1]) +
                                                      G[s][2] * (cb * Ti - Cp[s][2]) - gTT[s]) *
                                                     __builtin_amdgcn_rcpf(1.f - al);
                                    // Eqs. 5, 6
                                    Cp[s][0] = fmaf(-wt, cr, Cp[s][0]);
                                    Cp[s][1] = fmaf(-wt, cg, Cp[s][1]);
                                    Cp[s][2] = fmaf(-wt, cb, Cp[s][2]);
                                    if constexpr (RFMT == FB_F16) T[s] = fmaf(-Ti, alm, Ti);
                                    else T[s] = Ti - wt;
                                    if constexpr (RFMT >= 0) {   // idempotent on unchanged lanes
                                        Cp[s][0] = fb_round<RFMT>(Cp[s][0]);
                                        Cp[s][1] = fb_round<RFMT>(Cp[s][1]);
                                        Cp[s][2] = fb_round<RFMT>(Cp[s][2]);
                                        T[s] = fb_round<RFMT>(T[s]);
                                    }
                                    // bwd_diff (zero through a clamped alpha), as in the paper
                                    // modes: h = dL/dalpha alpha; dalpha/do = exp(-q/2);
                                    // dL/dq = -h / 2; dp/dd in the factored form
                                    // (a' u, k a' u + d' dy)
                                    const float h = (live && araw < amax) ? ga * araw : 0.f;
                                    acc[5] = fmaf(h, inv_o, acc[5]);
                                    const float gq = -0.5f * h;
                                    const float gm = -2.f * (h * (1.0f / LOG2E));
                                    const float gy = fmaf(A.w, au, B.x * dy);
                                    acc[0] = fmaf(gm, au, acc[0]);
                                    acc[1] = fmaf(gm, gy, acc[1]);
                                    const float gdx = gq * dx;
                                    acc[2] = fmaf(gdx, dx, acc[2]);
                                    acc[3] = fmaf(2.f * gdx, dy, acc[3]);
                                    acc[4] = fmaf(gq * dy, dy, acc[4]);
                                }
                            }
                            if (INSTR) {
                                cnt.evaluated += valid[s];
                                cnt.live += live;
                                nlive[s] += live;
                            }
                            if ((i & 3) == 3 || i0 + i + 1 == nlist)
                                if (!ballot(valid[s] && T[s] >= tmin)) alive &= ~(1u << s);
                            continue;
                        }
                        // the fragment's nine gradients, kept for the per-fragment reduction
                        float g[9];
                        if constexpr (!TILEM) {
#pragma unroll
                            for (int j = 0; j < 9; ++j) g[j] = 0.f;
                        }
                        if (live) {
                            const float Ti = T[s];
                            const float wt = al * Ti;
                            // Eq. 3: dL/dc = dL/dC alpha T
                            if constexpr (TILEM) {
                                acc[6] = fmaf(G[s][0], wt, acc[6]);
                                acc[7] = fmaf(G[s][1], wt, acc[7]);
                                acc[8] = fmaf(G[s][2], wt, acc[8]);
                                acc_live = true;
                            } else {
                                g[6] = G[s][0] * wt;
                                g[7] = G[s][1] * wt;
                                g[8] = G[s][2] * wt;
                            }
                            // Eq. 7: dL/dalpha = dL/dC . (c T - C') / (1 - alpha), and the final
                            // transmittance's share
                            const float ga = (G[s][0] * (cr * Ti - Cp[s][0]) +
                                              G[s][1] * (cg * Ti - Cp[s][1]) +
                                              G[s][2] * (cb * Ti - Cp[s][2]) - gTT[s]) *
                                             __builtin_amdgcn_rcpf(1.f - al);
                            // Eqs. 5, 6: the state update, stored back
                            Cp[s][0] = fmaf(-wt, cr, Cp[s][0]);
                            Cp[s][1] = fmaf(-wt, cg, Cp[s][1]);
                            Cp[s][2] = fmaf(-wt, cb, Cp[s][2]);
                            // Eq. 5, with the forward's arithmetic: per-fragment FP16 state
                            // is T (1 - alpha) as one FMA rounded once to half, as the forward's
                            // half-precision blend stores it; the other formats round T - T alpha
                            if constexpr (RFMT == FB_F16) T[s] = fmaf(-Ti, al, Ti);
                            else T[s] = Ti - wt;
                            if constexpr (RFMT >= 0) {
                                Cp[s][0] = fb_round<RFMT>(Cp[s][0]);
                                Cp[s][1] = fb_round<RFMT>(Cp[s][1]);
                                Cp[s][2] = fb_round<RFMT>(Cp[s][2]);
                                T[s] = fb_round<RFMT>(T[s]);
                            }
                            // bwd_diff: alpha = o exp(-q/2) (zero gradient where clamped);
                            // dq/dmu = -2 Q d, in the factored form:
                            // Q d = (a u, k a u + (det/a) dy), so
                            // dp/dd = (2 a' u, k 2 a' u + 2 d' dy) with the pre-scaled factors
                            if (araw < amax) {
                                const float gq = -0.5f * ga * araw;          // dL/dq
                                const float gm = -2.f * ga * araw * (1.0f / LOG2E);
                                const float gy = fmaf(A.w, au, B.x * dy);
                                if constexpr (TILEM) {
                                    // dalpha/do = exp(-q/2)
                                    acc[5] = fmaf(ga * araw, inv_o, acc[5]);
                                    acc[0] = fmaf(gm, au, acc[0]);
                                    acc[1] = fmaf(gm, gy, acc[1]);
                                    const float gdx = gq * dx;
                                    acc[2] = fmaf(gdx, dx, acc[2]);
                                    acc[3] = fmaf(2.f * gdx, dy, acc[3]);
                                    acc[4] = fmaf(gq * dy, dy, acc[4]);
                                } else {
                                    g[5] = ga * araw * inv_o;           // dalpha/do = exp(-q/2)
                                    g[0] = gm * au;
                                    g[1] = gm * gy;
                                    g[2] = gq * dx * dx;
                                    g[3] = 2.f * gq * dx * dy;
                                    g[4] = gq * dy * dy;
                                }
                            }
                        }
                        if (INSTR) {
                            cnt.evaluated += valid[s];
                            cnt.live += live;
                            nlive[s] += live;
                        }
                        if constexpr (!TILEM) {
                            if (lane_acc) {
#pragma unroll
                                for (int j = 0; j < 9; ++j) acc[j] += g[j];
                                acc_live = acc_live || live;
                            } else {
                                reduce_commit<INSTR>(g, live, gp, mode, X, lane, cnt);
                            }
                        }
                        // sub-blocks whose pixels are all T-culled drop out; checked every fourth
                        // list entry (a later check only costs a few fragments that the T test
                        // already rejects)
                        if ((i & 3) == 3 || i + 1 == nlist)
                            if (!ballot(valid[s] && T[s] >= tmin)) alive &= ~(1u << s);
                    }
                    if (tile_acc) {
                        // the wave's lane sums reduced at once; the first lane of each 16-lane row
                        // adds its two (row 0: three) totals to the tile's LDS accumulator
                        if (ballot(acc_live)) {
                            float ra, rb, rc;
                            wave_sum9(acc, ra, rb, rc);
                            if ((lane & 15) == 0) {
                                const int row = lane >> 4, j0 = ((row & 1) << 1) | (row >> 1);
                                if constexpr (TILEM && RFMT < 0) {   // tile_scale
                                    ra *= sa;
                                    rb *= row == 2 ? inv_o : sb;
                                }
                                atomicAdd(tg + k * 9 + j0, ra);
                                atomicAdd(tg + k * 9 + j0 + 4, rb);
                                if (row == 0) atomicAdd(tg + k * 9 + 8, rc);
                            }
                            if (INSTR && lane == 0) { cnt.wave_red += 1; cnt.cohesive += 1; }
                        }
                    } else if (lane_acc) {
                        reduce_commit<INSTR>(acc, acc_live, gp, GS_REDUCE_HYBRID, X, lane, cnt);
                    }
                }
            }
            if (lane == 0) w.alive[wave] = (int)alive;
            __syncthreads();
            if (!(w.alive[0] | w.alive[1] | w.alive[2] | w.alive[3])) { stop = true; break; }
        }
        if (stop) break;
    }
    if (tile_acc) flush_tile_grad<INSTR>(tg, w, pend, tid, grad, cnt);
    if (bgpart) {                       // the tile's dL/dbackground, summed in a fixed order
        __syncthreads();
        float* red = &tg[0];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float v = wave_sum(gbg[c]);
            if (lane == 0) red[wave * 3 + c] = v;
        }
        __syncthreads();
        if (tid < 3) bgpart[(size_t)tile * 4 + tid] = red[tid] + red[3 + tid] + red[6 + tid] + red[9 + tid];
    }

    if (INSTR && out_live) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (!valid[s]) continue;
            const int X = wx0 + (s & 1) * 8 + lx, Y = wy0 + (s >> 1) * 8 + ly;
            out_live[(size_t)Y * W + X] = (int32_t)nlive[s];
        }
    }
    if (INSTR && stats) {
        const uint32_t e = wave_sum_u32(cnt.evaluated), l = wave_sum_u32(cnt.live);
        const uint32_t sets = wave_sum_u32(cnt.sets);   // flushes count on every lane
        if (lane == 0) {
            if (wave == 0) atomicAdd(&stats[3], (unsigned long long)nq);
            atomicAdd(&stats[4], (unsigned long long)e);
            atomicAdd(&stats[5], (unsigned long long)l);
            atomicAdd(&stats[6], (unsigned long long)sets);
            atomicAdd(&stats[7], (unsigned long long)cnt.wave_red);
            atomicAdd(&stats[8], (unsigned long long)cnt.quad_red);
            atomicAdd(&stats[9], (unsigned long long)cnt.cohesive);
        }
    }
}

// dL/dbackground: the tiles' partial sums of every view added in a fixed order by one workgroup
// of 256 threads (all of them call it).
__device__ void bg_reduce(int ntiles, int nviews, const float* __restrict__ bgpart, uint64_t vws,
                          float* __restrict__ out) {
    __shared__ float s[3][256];
    float a[3] = {0.f, 0.f, 0.f};
    for (int v = 0; v < nviews; ++v) {
        const float* bp = reinterpret_cast<const float*>(
            reinterpret_cast<uintptr_t>(bgpart) + (uint64_t)v * vws);
        for (int t = threadIdx.x; t < ntiles; t += blockDim.x)
            for (int c = 0; c < 3; ++c) a[c] += bp[(size_t)t * 4 + c];
    }
    for (int c = 0; c < 3; ++c) s[c][threadIdx.x] = a[c];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int c = 0; c < 3; ++c) s[c][threadIdx.x] += s[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_bg_reduce(int ntiles, int nviews,
                                                   const float* __restrict__ bgpart, uint64_t vws,
                                                   float* __restrict__ out) {
    bg_reduce(ntiles, nviews, bgpart, vws, out);
}

// The accumulated gradients from their slots (one per splat id, cleared before the backward, so
// zero for culled splats) to the output arrays, one thread per id, both read and written in id
// order. With `dbg`, the first workgroup also reduces dL/dbackground (bg_reduce).
__global__ __launch_bounds__(256) void k_grad_finalize(
    int n, const float* __restrict__ grad, const float* __restrict__ rgb, int saturate,
    float* __restrict__ g_m, float* __restrict__ g_c, float* __restrict__ g_o,
    float* __restrict__ g_rgb, uint64_t vws, int ntiles, int nviews,
    const float* __restrict__ bgpart, float* __restrict__ dbg) {
    if (dbg && blockIdx.x == 0 && blockIdx.y == 0) bg_reduce(ntiles, nviews, bgpart, vws, dbg);
    grad = view_bytes(grad, vws);
    rgb = view_at(rgb, 3ull * n);
    g_m = view_at(g_m, 2ull * n);
    g_c = view_at(g_c, 3ull * n);
    g_o = view_at(g_o, (uint64_t)n);
    g_rgb = view_at(g_rgb, 3ull * n);
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    // each sum is hi + lo (lo: the compensated adds' rounding errors; zero in the per-fragment
    // reduction modes), rounded once
    float raw[20];
    const float4* gp = reinterpret_cast<const float4*>(grad + (size_t)id * GRAD_STRIDE);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const float4 u = gp[k];
        raw[4 * k] = u.x; raw[4 * k + 1] = u.y; raw[4 * k + 2] = u.z; raw[4 * k + 3] = u.w;
    }
    float v[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) v[j] = raw[j] + raw[GRAD_LO + j];
    if (saturate)
        for (int ch = 0; ch < 3; ++ch)
            if (rgb[3 * (size_t)id + ch] > 1.f) v[6 + ch] = 0.f;
    g_m[2 * (size_t)id] = v[0];
    g_m[2 * (size_t)id + 1] = v[1];
    g_c[3 * (size_t)id] = v[2];
    g_c[3 * (size_t)id + 1] = v[3];
    g_c[3 * (size_t)id + 2] = v[4];
    g_o[id] = v[5];
    g_rgb[3 * (size_t)id] = v[6];
    g_rgb[3 * (size_t)id + 1] = v[7];
    g_rgb[3 * (size_t)id + 2] = v[8];
}

// dL/dbackground: the per-tile partial sums of every view, added in a fixed order
// (deterministic). The background is one colour shared by the views, so its gradient is their sum.
// ---- host side -------------------------------------------------------------------------------

static int tiles_of(int width, int height) {
    return ((width + TILE - 1) / TILE) * ((height + TILE - 1) / TILE);
}

// Words per tile row of the occupancy bitmap (0: no bitmap, every chunk is tested): COL_WORDS
// per column of SETUP_SPAN sorted positions, one column per setup block.
static int bitmap_wpr(int n, int width, int height) {
    const size_t nt = (size_t)tiles_of(width, height);
    const size_t wpr = ((size_t)n + SETUP_SPAN - 1) / SETUP_SPAN * COL_WORDS;
    return (n > 0 && nt <= (size_t)MAX_LDS_TILES && nt * wpr * 4 <= BITMAP_BUDGET) ? (int)wpr : 0;
}

static bool split_ok(int n, int width, int height) {
    return bitmap_wpr(n, width, height) > 0 && tiles_of(width, height) <= MAX_SPLIT_TILES;
}

size_t raster_ws_bytes(int n, int width, int height, bool bwd) {
    const size_t nt = (size_t)tiles_of(width, height);
    const size_t wpr = (size_t)bitmap_wpr(n, width, height);
    size_t b = align_up((size_t)n * REC_BYTES) + align_up((size_t)n * 8) +
               align_up(16 * 8) + align_up(nt * 4) * 4 + align_up(nt * wpr * 4);
    if (split_ok(n, width, height))
        b += align_up(nt * (wpr / COL_WORDS) * 2) + align_up(ITEMS_PER_TILE * nt * 16) +
             2 * align_up(ITEMS_PER_TILE * nt * 4) + 2 * align_up(nt * 4) +
             align_up(ITEMS_PER_TILE * nt * TILE * TILE * 16);
    // the setup's per-id staging (64 B per splat) and the backward's gradient slots (80 B per
    // splat) share one region: the staging is dead once the setup has run, before the gradients
    // are cleared
    static_assert(GRAD_STRIDE * 4 >= sizeof(IdRec) && GRAD_STRIDE % 4 == 0, "shared region");
    static_assert(GRAD_LO + 9 <= GRAD_STRIDE, "slot layout");
    b += align_up((size_t)n * GRAD_STRIDE * 4);
    if (bwd) b += align_up(nt * 16);
    return b;
}

RasterWs carve_raster_ws(void* ws, int n, int width, int height, bool bwd) {
    const size_t nt = (size_t)tiles_of(width, height);
    RasterWs r;
    char* p = (char*)ws;
    r.rec = p;      p += align_up((size_t)n * REC_BYTES);
    r.rect = p;     p += align_up((size_t)n * 8);
    r.counters = (unsigned long long*)p; p += align_up(16 * 8);
    r.status = (uint32_t*)(r.counters + 1);
    r.weights = (uint32_t*)p; p += align_up(nt * 4);
    r.order = (int32_t*)p;    p += align_up(nt * 4);
    r.bwd_w = (uint32_t*)p;   p += align_up(nt * 4);
    r.bwd_order = (int32_t*)p; p += align_up(nt * 4);
    r.wpr = bitmap_wpr(n, width, height);
    r.bits = (uint32_t*)p;    p += align_up(nt * (size_t)r.wpr * 4);
    r.split = split_ok(n, width, height) ? 1 : 0;
    r.colcnt = nullptr; r.items = nullptr; r.item_w = nullptr; r.item_order = nullptr;
    r.tile_first = nullptr; r.tile_k = nullptr; r.partial = nullptr;
    if (r.split) {
        r.colcnt = (uint16_t*)p;    p += align_up(nt * (size_t)(r.wpr / COL_WORDS) * 2);
        r.items = (int4*)p;         p += align_up(ITEMS_PER_TILE * nt * 16);
        r.item_w = (uint32_t*)p;    p += align_up(ITEMS_PER_TILE * nt * 4);
        r.item_order = (int32_t*)p; p += align_up(ITEMS_PER_TILE * nt * 4);
        r.tile_first = (int32_t*)p; p += align_up(nt * 4);
        r.tile_k = (int32_t*)p;     p += align_up(nt * 4);
        r.partial = (float4*)p;     p += align_up(ITEMS_PER_TILE * nt * TILE * TILE * 16);
    }
    r.idrec = p;
    r.grad = bwd ? (float*)p : nullptr;
    p += align_up((size_t)n * GRAD_STRIDE * 4);
    r.bgpart = nullptr;
    if (bwd) {
        r.bgpart = (float*)p; p += align_up(nt * 16);
    }
    return r;
}

// Records, tile rectangles, tile weights, the occupancy bitmap and the schedule (tile order, the
// column and segment counts from which a forward that splits tiles plans its work items).
static hipError_t raster_setup(const gs_config& cfg, int width, int height, int n,
                               const int32_t* sorted_ids, const int32_t* n_visible,
                               const float* means2d, const float* conics, const float* opac,
                               const float* rgb, const RasterWs& r, hipStream_t s,
                               const Views& vs) {
    const int tiles_x = (width + TILE - 1) / TILE;
    const int ntiles = tiles_of(width, height);
    const int V = vs.count;
    if (n == 0) {
        hipError_t e = launch_fill_u32(r.weights, (size_t)ntiles, 0u, s, V, vs.ws);
        if (e == hipSuccess) e = launch_fill_u32(r.status, 3, 0u, s, V, vs.ws);
        if (e != hipSuccess) return e;
    } else {
        const int sat = (cfg.fb_format == FB_UNORM16 || cfg.fb_format == FB_UNORM8) ? 1 : 0;
        hipLaunchKernelGGL(k_raster_pack, dim3((n + 255) / 256, V), dim3(256), 0, s, n, means2d,
                           conics, opac, rgb, width, height, cfg.alpha_min, sat, (IdRec*)r.idrec,
                           r.weights, ntiles, r.status, vs.ws);
        const size_t lds =
            ntiles <= MAX_LDS_TILES ? ((size_t)ntiles * COL_WORDS + (ntiles + 1) / 2) * 4 : 0;
        hipLaunchKernelGGL(k_raster_setup, dim3((n + SETUP_SPAN - 1) / SETUP_SPAN, V),
                           dim3(SETUP_NT), lds, s, n, sorted_ids, n_visible,
                           (const IdRec*)r.idrec, tiles_x, ntiles, (Rec*)r.rec, (uint2*)r.rect,
                           r.weights, r.bits, r.wpr, r.colcnt, r.status, vs.ws);
    }
    hipLaunchKernelGGL(k_plan_tiles, dim3(1, V), dim3(NBUCKETS), 0, s, r.weights, ntiles, r.order,
                       r.split, r.tile_k, r.tile_first, r.counters, r.bwd_w, vs.ws);
    return hipGetLastError();
}

// The depth split's work items (cuts at equal splat counts, then their heaviest-first order), from
// the setup's column counts and segment counts. Planned by the forward that uses them: with the
// saturation exit (the default) the forward composites each tile in one item.
static hipError_t plan_items(const RasterWs& r, int ntiles, hipStream_t s, const Views& vs) {
    hipLaunchKernelGGL(k_plan_cuts, dim3(ntiles, vs.count), dim3(64), 0, s, r.weights,
                       (const uint16_t*)r.colcnt, r.wpr / COL_WORDS, ntiles,
                       (const int32_t*)r.tile_k, (const int32_t*)r.tile_first, r.items, r.item_w,
                       vs.ws);
    hipLaunchKernelGGL(k_plan_items, dim3(1, vs.count), dim3(NBUCKETS), 0, s,
                       (const uint32_t*)r.item_w, ntiles, (const unsigned long long*)r.counters,
                       r.item_order, vs.ws);
    return hipGetLastError();
}

static bool saturating(int fmt) { return fmt == FB_UNORM16 || fmt == FB_UNORM8; }

hipError_t raster_status(const void* ws, int n, int width, int height, uint32_t* out,
                         hipStream_t s, const Views& vs) {
    const RasterWs r = carve_raster_ws(const_cast<void*>(ws), n, width, height, false);
    uint32_t acc = 0u;
    for (int v = 0; v < vs.count; ++v) {
        uint32_t word = 0u;
        const char* src = reinterpret_cast<const char*>(r.status) + (size_t)v * vs.ws;
        hipError_t e = hipMemcpyAsync(&word, src, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        acc |= word;
    }
    *out = acc;
    return hipSuccess;
}

bool raster_has_split(int n, int width, int height) { return split_ok(n, width, height); }

hipError_t copy_raster_schedule(const void* ws, int n, int width, int height, int32_t* fwd_order,
                                int32_t* bwd_order, int32_t* item_order, int32_t* items,
                                int64_t* n_items, hipStream_t s, const Views& vs) {
    const RasterWs r = carve_raster_ws(const_cast<void*>(ws), n, width, height, false);
    const size_t nt = (size_t)tiles_of(width, height);
    for (int v = 0; v < vs.count; ++v) {
        const size_t off = (size_t)v * vs.ws;
        auto at = [&](const void* p) { return reinterpret_cast<const char*>(p) + off; };
        hipError_t e = hipSuccess;
        if (fwd_order)
            e = hipMemcpyAsync(fwd_order + v * nt, at(r.order), nt * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && bwd_order)
            e = hipMemcpyAsync(bwd_order + v * nt, at(r.bwd_order), nt * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && item_order)
            e = hipMemcpyAsync(item_order + v * ITEMS_PER_TILE * nt, at(r.item_order),
                               ITEMS_PER_TILE * nt * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && items)
            e = hipMemcpyAsync(items + v * 4 * ITEMS_PER_TILE * nt, at(r.items),
                               ITEMS_PER_TILE * nt * 16, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && n_items)
            e = hipMemcpyAsync(n_items + v, at(r.counters), 8, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_raster_setup(const gs_config& cfg, int width, int height, int n,
                               const int32_t* sorted_ids, const int32_t* n_visible,
                               const float* means2d, const float* conics, const float* opac,
                               const float* rgb, void* ws, hipStream_t s, const Views& vs) {
    const RasterWs r = carve_raster_ws(ws, n, width, height, false);
    return raster_setup(cfg, width, height, n, sorted_ids, n_visible, means2d, conics, opac, rgb,
                        r, s, vs);
}

using FwdKernel = void (*)(int, const int32_t*, const Rec*, const uint2*, const int32_t*,
                          const uint32_t*, int, int, int, int, int, const int4*, const int32_t*,
                          float4*, float, float, float, float, float, float, float, int, void*,
                          float*, float*, int32_t*, unsigned long long*, uint32_t*, uint32_t*,
                          int, uint64_t);

template <bool TC, bool IN, bool MU>
static FwdKernel fwd_by_fmt(int rfmt) {
    switch (rfmt) {
    case FB_F32: return k_raster_fwd<FB_F32, TC, IN, MU>;
    case FB_F16: return k_raster_fwd<FB_F16, TC, IN, MU>;
    case FB_UNORM16: return k_raster_fwd<FB_UNORM16, TC, IN, MU>;
    case FB_BF16: return k_raster_fwd<FB_BF16, TC, IN, MU>;
    case FB_UNORM8: return k_raster_fwd<FB_UNORM8, TC, IN, MU>;
    default: return k_raster_fwd<-1, TC, IN, MU>;
    }
}

template <bool MU>
static FwdKernel fwd_kernel(int rfmt, bool tcull, bool instr) {
    return tcull ? (instr ? fwd_by_fmt<true, true, MU>(rfmt) : fwd_by_fmt<true, false, MU>(rfmt))
                 : (instr ? fwd_by_fmt<false, true, MU>(rfmt) : fwd_by_fmt<false, false, MU>(rfmt));
}

hipError_t launch_raster_fwd(const gs_config& cfg, int width, int height, int n,
                             const int32_t* sorted_ids, const int32_t* n_visible,
                             const float* means2d, const float* conics, const float* opac,
                             const float* rgb, void* fb, float* out_rgb, float* out_T,
                             int32_t* out_cov, gs_stats* stats, void* ws, hipStream_t s,
                             const Views& vs) {
    const RasterWs r = carve_raster_ws(ws, n, width, height, false);
    const int V = vs.count;
    if (!(cfg.flags & GS_FLAG_REUSE_SETUP)) {
        hipError_t e0 = raster_setup(cfg, width, height, n, sorted_ids, n_visible, means2d, conics,
                                     opac, rgb, r, s, vs);
        if (e0 != hipSuccess) return e0;
    }
    const int tiles_x = (width + TILE - 1) / TILE;
    const int ntiles = tiles_of(width, height);
    const int rfmt = cfg.fb_round == GS_ROUND_PER_FRAGMENT ? cfg.fb_format : -1;
    const bool tcull = cfg.t_min_fwd > 0.f;
    const bool instr = (stats && (cfg.flags & GS_FLAG_STATS)) || out_cov;
    // the saturation exit ends a tile's walk early, so it composites each tile in one item; the
    // depth split (at-rest state, no T-culling, no counters) serves the full walk
    const bool freeze = rfmt < 0 && !tcull && !out_cov && !(cfg.flags & GS_FLAG_COMPOSITE_ALL);
    const bool split = r.split && rfmt < 0 && !tcull && !instr && !freeze;
    if (split) {
        const hipError_t e0 = plan_items(r, ntiles, s, vs);
        if (e0 != hipSuccess) return e0;
    }
    FwdKernel k = V > 1 ? fwd_kernel<true>(rfmt, tcull, instr) : fwd_kernel<false>(rfmt, tcull, instr);
    hipLaunchKernelGGL(k, dim3(split ? ITEMS_PER_TILE * ntiles : ntiles, V), dim3(NT), 0, s, n,
                       n_visible,
                       (const Rec*)r.rec, (const uint2*)r.rect, (const int32_t*)r.order,
                       (const uint32_t*)r.bits, r.wpr, width, height, tiles_x, ntiles,
                       split ? (const int4*)r.items : nullptr,
                       split ? (const int32_t*)r.item_order : nullptr, split ? r.partial : nullptr,
                       cfg.alpha_min, cfg.alpha_max, cfg.t_min_fwd, cfg.t_min_bwd, cfg.background[0],
                       cfg.background[1], cfg.background[2], cfg.fb_format, fb, out_rgb, out_T,
                       out_cov,
                       (stats && (cfg.flags & GS_FLAG_STATS)) ? (unsigned long long*)stats : nullptr,
                       r.bwd_w, r.status, freeze ? 1 : 0,
                       vs.ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !split) return e;
    hipLaunchKernelGGL(k_raster_merge, dim3(ntiles, V), dim3(256), 0, s, ntiles, tiles_x, width,
                       height, (const int32_t*)r.tile_k, (const int32_t*)r.tile_first,
                       (const float4*)r.partial, cfg.background[0], cfg.background[1],
                       cfg.background[2], cfg.fb_format, fb, out_rgb, out_T, vs.ws);
    return hipGetLastError();
}

hipError_t launch_raster_bwd(const gs_config& cfg, int width, int height, int n,
                             const int32_t* sorted_ids, const int32_t* n_visible,
                             const float* means2d, const float* conics, const float* opac,
                             const float* rgb, const void* fb, const float* dL_dimg,
                             float* g_means2d, float* g_conics, float* g_opac, float* g_rgb, const float* dL_dT, float* dL_dbg,
                             int32_t* out_live, gs_stats* stats, void* ws, hipStream_t s,
                             const Views& vs) {
    const RasterWs r = carve_raster_ws(ws, n, width, height, true);
    const int sat = (int)saturating(cfg.fb_format);
    const int V = vs.count;
    if (!(cfg.flags & GS_FLAG_REUSE_SETUP)) {
        hipError_t e0 = raster_setup(cfg, width, height, n, sorted_ids, n_visible, means2d, conics,
                                     opac, rgb, r, s, vs);
        if (e0 != hipSuccess) return e0;
    }
    if (n > 0) {   // after the setup: the gradient slots reuse its staging region
        hipError_t e = launch_fill_u32(r.grad, (size_t)n * GRAD_STRIDE, 0u, s, V, vs.ws);
        if (e != hipSuccess) return e;
    }
    const int tiles_x = (width + TILE - 1) / TILE;
    const int nblocks = tiles_of(width, height);
    hipLaunchKernelGGL(k_plan_bwd, dim3(1, V), dim3(NBUCKETS), 0, s, (const uint32_t*)r.bwd_w,
                       nblocks, r.bwd_order, vs.ws);
    const int rfmt = cfg.fb_round == GS_ROUND_PER_FRAGMENT ? cfg.fb_format : -1;
    const bool instr = (stats && (cfg.flags & GS_FLAG_STATS)) || out_live;
    void (*k)(int, const int32_t*, const Rec*, const uint2*, const int32_t*, const uint32_t*, int,
              int, int, int, float, float, float, int, const void*, const float*, const float*, int,
              int, float*, float*, int32_t*, unsigned long long*, uint32_t*, uint64_t) = nullptr;
#define GSR_BWD_PICK(IN, MU, TM)                                             \
    switch (rfmt) {                                                          \
    case FB_F32: k = k_raster_bwd<FB_F32, IN, MU, TM>; break;                \
    case FB_F16: k = k_raster_bwd<FB_F16, IN, MU, TM>; break;                \
    case FB_UNORM16: k = k_raster_bwd<FB_UNORM16, IN, MU, TM>; break;        \
    case FB_BF16: k = k_raster_bwd<FB_BF16, IN, MU, TM>; break;              \
    case FB_UNORM8: k = k_raster_bwd<FB_UNORM8, IN, MU, TM>; break;          \
    default: k = k_raster_bwd<-1, IN, MU, TM>; break;                        \
    }
#define GSR_BWD_PICK2(MU, TM)                                                \
    if (instr) { GSR_BWD_PICK(true, MU, TM) } else { GSR_BWD_PICK(false, MU, TM) }
    const bool tm = cfg.reduce_mode == GS_REDUCE_TILE;
    if (V > 1) {
        if (tm) { GSR_BWD_PICK2(true, true) } else { GSR_BWD_PICK2(true, false) }
    } else {
        if (tm) { GSR_BWD_PICK2(false, true) } else { GSR_BWD_PICK2(false, false) }
    }
#undef GSR_BWD_PICK2
#undef GSR_BWD_PICK
    hipLaunchKernelGGL(k, dim3(nblocks, V), dim3(NT), 0, s, n, n_visible, (const Rec*)r.rec,
                       (const uint2*)r.rect, (const int32_t*)r.bwd_order, (const uint32_t*)r.bits,
                       r.wpr, width, height, tiles_x,
                       cfg.alpha_min, cfg.alpha_max, cfg.t_min_bwd, cfg.fb_format, fb, dL_dimg,
                       dL_dT, cfg.reduce_mode, cfg.reduce_threshold, r.grad,
                       dL_dbg ? r.bgpart : nullptr, out_live,
                       (stats && (cfg.flags & GS_FLAG_STATS)) ? (unsigned long long*)stats : nullptr,
                       r.status, vs.ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (n == 0) {                        // no gradients to finalise: the background alone
        if (dL_dbg)
            hipLaunchKernelGGL(k_bg_reduce, dim3(1), dim3(256), 0, s, nblocks, V,
                               (const float*)r.bgpart, vs.ws, dL_dbg);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_grad_finalize, dim3((n + 255) / 256, V), dim3(256), 0, s, n, r.grad, rgb,
                       sat, g_means2d, g_conics, g_opac, g_rgb, vs.ws, nblocks, V,
                       (const float*)r.bgpart, dL_dbg);
    return hipGetLastError();
}

}  // namespace gsr
