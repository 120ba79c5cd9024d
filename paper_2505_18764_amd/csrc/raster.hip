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
//     memory O(N + pixels)): each fill, its waves test 4096 consecutive splats' tile rectangles,
//     compact the hits in order into LDS, stage their records in LDS, and then every wave applies
//     the staged splats one after another to its own pixels, whose state lives in VGPRs. A pixel
//     is only ever touched by one lane, in splat order, so no interlock is needed;
//   * a splat is skipped for a sub-block its pixel bounding box misses (one scalar branch).
// Each fill iteration therefore processes one splat per wave across up to 64 lanes; that is the
// "subgroup" of Procedure 2, and its live lanes always share one splat id (cohesion 100 %).
#include "device.hpp"
#include "internal.hpp"

namespace gsr {

constexpr int NT = 256;            // threads per workgroup
constexpr int SPAN = 1024;         // sorted splats one wave tests per fill
constexpr int CHUNK = 4 * SPAN;    // sorted splats the workgroup tests per fill
constexpr int BATCH = 256;         // splat records staged in LDS at once

// A staged splat: a = (mean x, mean y, a', k); b = (d', opacity, r, g);
// c = (bits of colour b, sorted position, bits of p_min, 0) where p_min = log2(alpha_min / o) is
// the least exponent whose alpha passes alpha_min.
//
// The conic Q = [[a, b], [b, c]] is stored in its LDL^T factors: q = d^T Q d =
// a (dx + k dy)^2 + (det Q / a) dy^2 with k = b / a, a sum of two non-negative terms. The
// expanded form a dx^2 + 2b dx dy + c dy^2 cancels terms of size q / (1 - rho^2) (rho the
// correlation of the footprint) down to q, which in FP32 loses several digits on long thin
// splats, e.g. those just beyond the near plane whose projected means lie thousands of pixels
// off-screen; the factored form costs the same instructions. k and det Q / a are formed in FP64
// from the FP32 conic and stored pre-scaled, a' = -log2(e) a / 2 and d' = -log2(e) det Q / (2a),
// so that the exponent of alpha = o 2^p is p = a' u^2 + d' dy^2 = -q/2 log2(e), u = dx + k dy.
struct __align__(16) Rec {
    float4 a;
    float4 b;
    uint4 c;
};
static_assert(sizeof(Rec) == REC_BYTES, "record size");

constexpr float LOG2E = 1.4426950408889634f;
constexpr int WEIGHT_SAMPLE = 8;        // every 8th sorted splat votes for the tiles it touches
constexpr int CHUNK_SPLATS = 64;        // sorted splats per bit of the tile occupancy bitmap
constexpr size_t BITMAP_BUDGET = 256u << 20;  // the bitmap is skipped above this many bytes
constexpr int MAX_ORDERED_TILES = 8192; // tiles ordered by weight in one workgroup (LDS sort)

// Tile schedule. The work of a tile grows with the number of splats over it, which on clustered
// scenes varies by orders of magnitude across the screen. Workgroups are dispatched in block
// order (round-robin over the 8 XCDs, then to whichever CU has room), so listing the tiles by
// decreasing estimated work starts the heaviest tiles first and spreads them over all XCDs:
// a longest-processing-time-first schedule.
__global__ __launch_bounds__(1024) void k_tile_order(const uint32_t* __restrict__ weights,
                                                     int ntiles, int32_t* __restrict__ order) {
    __shared__ unsigned long long key[MAX_ORDERED_TILES];
    const int tid = threadIdx.x;
    if (ntiles > MAX_ORDERED_TILES) {
        for (int i = tid; i < ntiles; i += blockDim.x) order[i] = i;
        return;
    }
    int m = 1;
    while (m < ntiles) m <<= 1;
    for (int i = tid; i < m; i += blockDim.x)
        key[i] = i < ntiles ? ((unsigned long long)(0xFFFFFFFFu - weights[i]) << 32) | (uint32_t)i
                            : ~0ull;
    __syncthreads();
    for (int k = 2; k <= m; k <<= 1) {          // bitonic sort, ascending
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < m; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const unsigned long long a = key[i], b = key[l];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) { key[i] = b; key[l] = a; }
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < ntiles; i += blockDim.x) order[i] = (int32_t)(key[i] & 0xFFFFFFFFu);
}

__device__ __forceinline__ bool rect_hit(uint2 r, uint32_t tx, uint32_t ty) {
    return (r.x & 0xFFFFu) <= tx && tx <= (r.x >> 16) && (r.y & 0xFFFFu) <= ty && ty <= (r.y >> 16);
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ---- setup: records, tile rectangles, occupancy bitmap and tile weights ---------------------
// One workgroup per SETUP_SPAN consecutive sorted positions = one 32-bit column of the bitmap
// (32 chunks of 64 splats). The workgroup gathers, in LDS, one word of chunk bits and one splat
// count per tile, then writes its bitmap column with plain stores and adds its counts to the tile
// weights: one global atomic per (workgroup, touched tile), none contended within an instruction.
constexpr int SETUP_SPAN = 32 * CHUNK_SPLATS;   // 2048 sorted positions per workgroup
constexpr int MAX_LDS_TILES = 8192;

__global__ __launch_bounds__(256) void k_raster_setup(
    int n, const int32_t* __restrict__ sorted_ids, const int32_t* __restrict__ nvis_ptr,
    const float* __restrict__ means2d, const float* __restrict__ conics,
    const float* __restrict__ opac, const float* __restrict__ rgb, int W, int H, float amin,
    int saturate, int tiles_x, int ntiles, Rec* __restrict__ rec, uint2* __restrict__ rect,
    uint32_t* __restrict__ weights, uint32_t* __restrict__ bits, int wpr) {
    __shared__ uint32_t s_bits[MAX_LDS_TILES];
    __shared__ uint32_t s_cnt[MAX_LDS_TILES];
    const bool in_lds = ntiles <= MAX_LDS_TILES;
    if (in_lds)
        for (int t = threadIdx.x; t < ntiles; t += blockDim.x) { s_bits[t] = 0u; s_cnt[t] = 0u; }
    __syncthreads();
    int nvis = *nvis_ptr;
    nvis = nvis < 0 ? 0 : (nvis > n ? n : nvis);
    const int p0 = blockIdx.x * SETUP_SPAN;
    for (int j = 0; j < SETUP_SPAN / 256; ++j) {
        const int p = p0 + j * 256 + threadIdx.x;
        if (p >= n) break;
        uint2 rr = make_uint2(0xFFFFu, 0u);   // matches no tile
        if (p < nvis) {
            const int id = sorted_ids[p];
            if ((unsigned)id < (unsigned)n) {
                const float mx = means2d[2 * (size_t)id], my = means2d[2 * (size_t)id + 1];
                const float a = conics[3 * (size_t)id], b = conics[3 * (size_t)id + 1],
                            c = conics[3 * (size_t)id + 2];
                const float o = opac[id];
                float cr = rgb[3 * (size_t)id], cg = rgb[3 * (size_t)id + 1],
                      cb = rgb[3 * (size_t)id + 2];
                if (saturate) { cr = fminf(cr, 1.f); cg = fminf(cg, 1.f); cb = fminf(cb, 1.f); }
                // det in FP64: the products of FP32 values are exact, so its sign is exact
                const double ad = a, bd = b, cd = c;
                const double det = ad * cd - bd * bd;
                if (a > 0.f && c > 0.f && det > 0.0 && o >= amin && isfinite(mx) && isfinite(my)) {
                    // alpha >= alpha_min  <=>  q <= r2 = 2 ln(o / alpha_min): the ellipse's half
                    // extents are sqrt(r2 Sigma_xx), sqrt(r2 Sigma_yy) with Sigma = conic^-1;
                    // padded so FP32 rounding never puts a passing pixel outside the box.
                    const float r2 = 2.0f * logf(o / amin);
                    const float hx = (float)sqrt(fmax((double)r2 * cd / det, 0.0)) * 1.001f + 0.01f;
                    const float hy = (float)sqrt(fmax((double)r2 * ad / det, 0.0)) * 1.001f + 0.01f;
                    const float fx0 = fminf(fmaxf(floorf(mx - hx - 0.5f), 0.f), (float)W);
                    const float fx1 = fminf(fmaxf(floorf(mx + hx - 0.5f) + 1.f, 0.f), (float)W);
                    const float fy0 = fminf(fmaxf(floorf(my - hy - 0.5f), 0.f), (float)H);
                    const float fy1 = fminf(fmaxf(floorf(my + hy - 0.5f) + 1.f, 0.f), (float)H);
                    if (fx0 < fx1 && fy0 < fy1) {
                        const uint32_t x0 = (uint32_t)fx0, x1 = (uint32_t)fx1;
                        const uint32_t y0 = (uint32_t)fy0, y1 = (uint32_t)fy1;
                        Rec r;
                        const double l2e = 1.4426950408889634;
                        r.a = make_float4(mx, my, -0.5f * LOG2E * a, (float)(bd / ad));
                        r.b = make_float4((float)(-0.5 * l2e * det / ad), o, cr, cg);
                        const float pmin = (float)(log2((double)amin) - log2((double)o));
                        r.c = make_uint4(__float_as_uint(cb), (uint32_t)p, __float_as_uint(pmin), 0u);
                        rec[p] = r;
                        const uint32_t tx0 = x0 / TILE, tx1 = (x1 - 1) / TILE;
                        const uint32_t ty0 = y0 / TILE, ty1 = (y1 - 1) / TILE;
                        rr = make_uint2(tx0 | (tx1 << 16), ty0 | (ty1 << 16));
                        const uint32_t bit = 1u << ((uint32_t)(p - p0) / CHUNK_SPLATS);
                        for (uint32_t ty = ty0; ty <= ty1; ++ty)
                            for (uint32_t tx = tx0; tx <= tx1; ++tx) {
                                const uint32_t t = ty * (uint32_t)tiles_x + tx;
                                if (in_lds) {
                                    atomicOr(&s_bits[t], bit);
                                    atomicAdd(&s_cnt[t], 1u);
                                } else if (p % WEIGHT_SAMPLE == 0) {
                                    atomicAdd(&weights[t], 1u);
                                }
                            }
                    }
                }
            }
        }
        rect[p] = rr;
    }
    __syncthreads();
    if (in_lds)
        for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
            if (wpr > 0) bits[(size_t)t * wpr + blockIdx.x] = s_bits[t];
            if (s_cnt[t]) atomicAdd(&weights[t], s_cnt[t]);
        }
}

// ---- the shared walk: scan 4096 sorted splats, compact hits in order, stage records ----------
struct Walk {
    uint16_t seg[4][SPAN];
    uint16_t list[4][BATCH];
    int segn[4];
    int alive[4];
    Rec rec[BATCH];
};

// Per-wave culling of a staged batch. Lane j takes staged splat k0 + j and bounds its exponent
// over each of the wave's four 8x8 sub-blocks: with c the sub-block centre and g the gradient of
// p there, p(c + d) = p(c) + g.d + d^T Q' d <= p(c) + 3.5 (|g_x| + |g_y|) over the pixel centres
// (|d_x|, |d_y| <= 3.5), since Q' (the pre-scaled conic, negative definite) adds nothing positive.
// A sub-block whose bound stays below p_min (with a margin far above the FP32 error of the
// bound) holds no fragment with alpha >= alpha_min. The splats that reach at least one
// sub-block are compacted in order into w.list[wave] as k | mask << 8; returns their count.
__device__ __forceinline__ int cull_batch(Walk& w, int m, int wave, int lane, uint64_t lt,
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

// Tests the wave's 1024 splats of this fill against the tile, one 64-splat chunk per set bit of
// `chunks` (16 bits, from the occupancy bitmap); writes the in-order offsets of the hits to
// w.seg[wave] and their count to w.segn[wave].
__device__ __forceinline__ void scan_span(Walk& w, const uint2* __restrict__ rect, int wb, int nvis,
                                          uint32_t ttx, uint32_t tty, int wave, int lane,
                                          uint64_t lt, uint32_t chunks) {
    int cnt = 0;
    if (wb >= nvis) chunks = 0;
    while (chunks) {
        const int b0 = __builtin_ctz(chunks);
        chunks &= chunks - 1u;
        const int b1 = chunks ? __builtin_ctz(chunks) : -1;   // two chunks per round
        if (b1 >= 0) chunks &= chunks - 1u;
        const int o0 = b0 * 64 + lane, o1 = b1 * 64 + lane;
        const uint2 r0 = wb + o0 < nvis ? rect[wb + o0] : make_uint2(0xFFFFu, 0u);
        const uint2 r1 = (b1 >= 0 && wb + o1 < nvis) ? rect[wb + o1] : make_uint2(0xFFFFu, 0u);
        const bool h0 = rect_hit(r0, ttx, tty);
        const uint64_t m0 = ballot(h0);
        if (h0) w.seg[wave][cnt + popc(m0 & lt)] = (uint16_t)o0;
        cnt += popc(m0);
        const bool h1 = rect_hit(r1, ttx, tty);
        const uint64_t m1 = ballot(h1);
        if (h1) w.seg[wave][cnt + popc(m1 & lt)] = (uint16_t)o1;
        cnt += popc(m1);
    }
    if (lane == 0) w.segn[wave] = cnt;
}

// The tile's 64 chunk bits for the fill starting at sorted position `base` (all ones without a
// bitmap).
__device__ __forceinline__ uint64_t window_bits(const uint32_t* __restrict__ trow, int wpr, int base) {
    if (!trow) return ~0ull;
    const int wi = (base / CHUNK) * 2;
    const uint32_t lo = wi < wpr ? trow[wi] : 0u;
    const uint32_t hi = wi + 1 < wpr ? trow[wi + 1] : 0u;
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Stages hits [b0, b0 + BATCH) of the fill (in order across the four waves' segments).
__device__ __forceinline__ void stage(Walk& w, const Rec* __restrict__ rec, int base, int b0,
                                      int total, int tid) {
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
        const int pos = base + ws * SPAN + w.seg[ws][off];
        Rec r = rec[pos];
        r.c.y = (uint32_t)pos;      // the gradient slot comes from the walk, never from memory
        w.rec[tid] = r;
    }
}

// ---- forward -------------------------------------------------------------------------------
template <int RFMT, bool TCULL, bool INSTR>
__global__ __launch_bounds__(NT) void k_raster_fwd(
    int n, const int32_t* __restrict__ nvis_ptr, const Rec* __restrict__ rec,
    const uint2* __restrict__ rect, const int32_t* __restrict__ order,
    const uint32_t* __restrict__ bits, int wpr, int W, int H, int tiles_x,
    float amin, float amax, float tmin, int fb_fmt, void* __restrict__ fb, float* __restrict__ out_rgb,
    float* __restrict__ out_T, int32_t* __restrict__ out_cov,
    unsigned long long* __restrict__ stats) {
    __shared__ Walk w;
    int tile = order[blockIdx.x];
    if ((unsigned)tile >= gridDim.x) tile = (int)blockIdx.x;   // a schedule not built for this grid
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = uniform(tid >> 6);
    const uint32_t ttx = (uint32_t)(tile % tiles_x), tty = (uint32_t)(tile / tiles_x);
    const int wx0 = (int)ttx * TILE + (wave & 1) * 16, wy0 = (int)tty * TILE + (wave >> 1) * 16;
    const int qd = lane >> 2;
    const int lx = ((qd & 3) << 1) | (lane & 1), ly = ((qd >> 2) << 1) | ((lane >> 1) & 1);
    const uint64_t lt = mask_lt(lane);
    const float cx0 = (float)wx0 + 4.f, cy0 = (float)wy0 + 4.f;   // centre of sub-block 0

    // C accumulates Eq. 2; with the state kept on chip, each staged batch's contributions are
    // first summed in Cb and folded into C at the batch end, so deep pixels (thousands of
    // fragments) take far fewer full-magnitude FP32 additions.
    float px[4], py[4], C[4][3], Cb[4][3], T[4];
    bool valid[4];
    uint32_t nev[4], ncov[4];
    uint32_t alive = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int X = wx0 + (s & 1) * 8 + lx, Y = wy0 + (s >> 1) * 8 + ly;
        valid[s] = X < W && Y < H;
        px[s] = (float)X + 0.5f;
        py[s] = (float)Y + 0.5f;
        C[s][0] = C[s][1] = C[s][2] = 0.f;
        Cb[s][0] = Cb[s][1] = Cb[s][2] = 0.f;
        T[s] = 1.f;
        nev[s] = ncov[s] = 0;
        if (ballot(valid[s])) alive |= 1u << s;
    }
    int nvis = *nvis_ptr;
    nvis = nvis < 0 ? 0 : (nvis > n ? n : nvis);
    uint32_t nq = 0;

    const uint32_t* trow = wpr > 0 ? bits + (size_t)tile * wpr : nullptr;
    for (int base = 0; base < nvis; base += CHUNK) {
        const uint64_t wbits = window_bits(trow, wpr, base);
        if (wbits == 0) continue;                 // no splat of this fill touches the tile
        scan_span(w, rect, base + wave * SPAN, nvis, ttx, tty, wave, lane, lt,
                  (uint32_t)(wbits >> (16 * wave)) & 0xFFFFu);
        __syncthreads();
        const int total = w.segn[0] + w.segn[1] + w.segn[2] + w.segn[3];
        if (INSTR) nq += total;
        bool stop = false;
        for (int b0 = 0; b0 < total; b0 += BATCH) {
            stage(w, rec, base, b0, total, tid);
            __syncthreads();
            const int m = min(BATCH, total - b0);
            if (!TCULL || alive) {
                const int nlist = cull_batch(w, m, wave, lane, lt, cx0, cy0);
                for (int i = 0; i < nlist; ++i) {
                    const uint32_t ent = uniform((uint32_t)w.list[wave][i]);
                    const int k = (int)(ent & 0xFFu);
                    const float4 A = w.rec[k].a;
                    const float4 B = w.rec[k].b;
                    const float cb = __uint_as_float(w.rec[k].c.x);
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        if (((ent >> (8 + s)) & 1u) && (!TCULL || ((alive >> s) & 1u))) {
                            const float dx = px[s] - A.x, dy = py[s] - A.y;
                            const float u = fmaf(A.w, dy, dx);
                            const float pw = fmaf(A.z * u, u, B.x * dy * dy);
                            const float al = fminf(amax, B.y * __builtin_amdgcn_exp2f(pw));
                            bool pass = al >= amin;
                            if (TCULL) pass = pass && T[s] >= tmin;
                            if (pass) {
                                const float wt = al * T[s];
                                if constexpr (RFMT >= 0) {      // a render target stores every blend
                                    C[s][0] = fmaf(wt, B.z, C[s][0]);
                                    C[s][1] = fmaf(wt, B.w, C[s][1]);
                                    C[s][2] = fmaf(wt, cb, C[s][2]);
                                } else {
                                    Cb[s][0] = fmaf(wt, B.z, Cb[s][0]);
                                    Cb[s][1] = fmaf(wt, B.w, Cb[s][1]);
                                    Cb[s][2] = fmaf(wt, cb, Cb[s][2]);
                                }
                                T[s] = T[s] - wt;                // T (1 - alpha), Eq. 5
                                if constexpr (RFMT >= 0) {
                                    C[s][0] = fb_round<RFMT>(C[s][0]);
                                    C[s][1] = fb_round<RFMT>(C[s][1]);
                                    C[s][2] = fb_round<RFMT>(C[s][2]);
                                    T[s] = fb_round<RFMT>(T[s]);
                                }
                            }
                            if (INSTR) {
                                nev[s] += valid[s];
                                ncov[s] += (pass && valid[s]);
                            }
                            if (TCULL && !ballot(valid[s] && T[s] >= tmin)) alive &= ~(1u << s);
                        }
                    }
                }
            }
            if constexpr (RFMT < 0) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    C[s][0] += Cb[s][0]; C[s][1] += Cb[s][1]; C[s][2] += Cb[s][2];
                    Cb[s][0] = Cb[s][1] = Cb[s][2] = 0.f;
                }
            }
            if (TCULL && lane == 0) w.alive[wave] = (int)alive;
            __syncthreads();
            if (TCULL && !(w.alive[0] | w.alive[1] | w.alive[2] | w.alive[3])) { stop = true; break; }
        }
        if (TCULL && stop) break;
    }

    const size_t P = (size_t)W * H;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (!valid[s]) continue;
        const int X = wx0 + (s & 1) * 8 + lx, Y = wy0 + (s >> 1) * 8 + ly;
        const size_t i = (size_t)Y * W + X;
        float4 v = make_float4(C[s][0], C[s][1], C[s][2], T[s]);
        fb_store(fb, fb_fmt, i, v);
        if (out_rgb) {
            out_rgb[i] = v.x;
            out_rgb[P + i] = v.y;
            out_rgb[2 * P + i] = v.z;
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
        }
    }
}

// ---- backward ------------------------------------------------------------------------------

struct BwdCounts {
    uint32_t evaluated, live, sets, wave_red, quad_red, cohesive;
};

// Procedure 2 (ReduceGradient) for one splat and one wave: `g` holds this lane's gradient
// contribution (zero when not live); `gp` is the splat's slot in the accumulation buffer.
template <bool INSTR, bool TO_LDS = false>
__device__ __forceinline__ void reduce_commit(float (&g)[9], bool live, float* __restrict__ gp,
                                              int mode, int X, int lane, BwdCounts& cnt) {
    // TO_LDS: gp points into the workgroup's LDS accumulator (the atomics there are ds_add_f32
    // and the global commit is counted when the accumulator is flushed)
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
            for (int j = 0; j < 9; ++j) {
                if constexpr (TO_LDS) atomicAdd(gp + j, tot[j]);
                else atomic_add_f32(gp + j, tot[j]);
            }
        if (INSTR && lane == 0) { cnt.sets += TO_LDS ? 0 : 1; cnt.wave_red += 1; cnt.cohesive += 1; }
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
        for (int j = 0; j < 9; ++j) {
            if constexpr (TO_LDS) atomicAdd(gp + j, g[j]);
            else atomic_add_f32(gp + j, g[j]);
        }
    if (INSTR) {
        const uint64_t lm = ballot(leader);
        if (lane == 0) { cnt.sets += TO_LDS ? 0 : popc(lm); cnt.quad_red += 1; cnt.cohesive += 1; }
    }
}

// GS_REDUCE_TILE: thread t owns entry t of the staged batch's LDS accumulator; it adds the
// entry to the splat's gradient slot (one set of global atomics per splat and tile) and clears it.
// Called before entry t is restaged and once after the walk.
template <bool INSTR>
__device__ __forceinline__ void flush_tile_grad(float* __restrict__ tg, const Walk& w, int pend,
                                                int tid, float* __restrict__ grad, BwdCounts& cnt) {
    if (tid < pend) {
        float v[9];
        bool any = false;
#pragma unroll
        for (int j = 0; j < 9; ++j) { v[j] = tg[tid * 9 + j]; any = any || v[j] != 0.f; }
        if (any) {
            float* gp = grad + (size_t)w.rec[tid].c.y * GRAD_STRIDE;
#pragma unroll
            for (int j = 0; j < 9; ++j) atomic_add_f32(gp + j, v[j]);
            if (INSTR) cnt.sets += 1;
        }
    }
#pragma unroll
    for (int j = 0; j < 9; ++j) tg[tid * 9 + j] = 0.f;
}

template <int RFMT, bool INSTR>
__global__ __launch_bounds__(NT) void k_raster_bwd(
    int n, const int32_t* __restrict__ nvis_ptr, const Rec* __restrict__ rec,
    const uint2* __restrict__ rect, const int32_t* __restrict__ order,
    const uint32_t* __restrict__ bits, int wpr, int W, int H, int tiles_x,
    float amin, float amax, float tmin, int fb_fmt, const void* __restrict__ fb,
    const float* __restrict__ dL_dimg,
    int mode, int X, float* __restrict__ grad, int32_t* __restrict__ out_live,
    unsigned long long* __restrict__ stats) {
    __shared__ Walk w;
    __shared__ float tg[BATCH * 9];     // GS_REDUCE_TILE: per staged splat, the tile's gradient
    int tile = order[blockIdx.x];
    if ((unsigned)tile >= gridDim.x) tile = (int)blockIdx.x;   // a schedule not built for this grid
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = uniform(tid >> 6);
    const uint32_t ttx = (uint32_t)(tile % tiles_x), tty = (uint32_t)(tile / tiles_x);
    const int wx0 = (int)ttx * TILE + (wave & 1) * 16, wy0 = (int)tty * TILE + (wave >> 1) * 16;
    const int qd = lane >> 2;
    const int lx = ((qd & 3) << 1) | (lane & 1), ly = ((qd >> 2) << 1) | ((lane >> 1) & 1);
    const uint64_t lt = mask_lt(lane);
    const float cx0 = (float)wx0 + 4.f, cy0 = (float)wy0 + 4.f;   // centre of sub-block 0
    const size_t P = (size_t)W * H;
    const bool tile_acc = (mode == GS_REDUCE_TILE);
    int pend = 0;                       // staged entries whose LDS gradients are not yet flushed
    if (tile_acc)
#pragma unroll
        for (int j = 0; j < 9; ++j) tg[tid * 9 + j] = 0.f;

    // Procedure 1's per-pixel state (C', T), initialised to (C, 1) from the framebuffer, and the
    // read-only dL/dC.
    float px[4], py[4], Cp[4][3], T[4], G[4][3];
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
        if (valid[s]) {
            const size_t i = (size_t)Y * W + X;
            const float4 v = fb_load(fb, fb_fmt, i);
            Cp[s][0] = v.x; Cp[s][1] = v.y; Cp[s][2] = v.z;
            G[s][0] = dL_dimg[i]; G[s][1] = dL_dimg[P + i]; G[s][2] = dL_dimg[2 * P + i];
        }
        if (ballot(valid[s])) alive |= 1u << s;
    }
    int nvis = *nvis_ptr;
    nvis = nvis < 0 ? 0 : (nvis > n ? n : nvis);
    BwdCounts cnt = {0, 0, 0, 0, 0, 0};
    uint32_t nq = 0;
    const bool lane_acc = (mode == GS_REDUCE_HYBRID_LANE || mode == GS_REDUCE_TILE);

    const uint32_t* trow = wpr > 0 ? bits + (size_t)tile * wpr : nullptr;
    for (int base = 0; base < nvis; base += CHUNK) {
        const uint64_t wbits = window_bits(trow, wpr, base);
        if (wbits == 0) continue;                 // no splat of this fill touches the tile
        scan_span(w, rect, base + wave * SPAN, nvis, ttx, tty, wave, lane, lt,
                  (uint32_t)(wbits >> (16 * wave)) & 0xFFFFu);
        __syncthreads();
        const int total = w.segn[0] + w.segn[1] + w.segn[2] + w.segn[3];
        if (INSTR) nq += total;
        bool stop = false;
        for (int b0 = 0; b0 < total; b0 += BATCH) {
            if (tile_acc) { flush_tile_grad<INSTR>(tg, w, pend, tid, grad, cnt); pend = 0; }
            stage(w, rec, base, b0, total, tid);
            __syncthreads();
            const int m = min(BATCH, total - b0);
            pend = m;
            const int nlist = alive ? cull_batch(w, m, wave, lane, lt, cx0, cy0) : 0;
            for (int i = 0; i < nlist && alive; ++i) {
                const uint32_t ent = uniform((uint32_t)w.list[wave][i]);
                const int k = (int)(ent & 0xFFu);
                const float4 A = w.rec[k].a;
                const float4 B = w.rec[k].b;
                const uint4 Cw = w.rec[k].c;
                const float cr = B.z, cg = B.w, cb = __uint_as_float(Cw.x);
                float* gp = grad + (size_t)uniform(Cw.y) * GRAD_STRIDE;
                float acc[9];
#pragma unroll
                for (int j = 0; j < 9; ++j) acc[j] = 0.f;
                bool acc_live = false;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    if (!((ent >> (8 + s)) & 1u) || !((alive >> s) & 1u)) continue;
                    const float dx = px[s] - A.x, dy = py[s] - A.y;
                    const float u = fmaf(A.w, dy, dx);
                    const float au = A.z * u;
                    const float pw = fmaf(au, u, B.x * dy * dy);
                    const float e = __builtin_amdgcn_exp2f(pw);       // exp(-q/2)
                    const float araw = B.y * e;
                    const float al = fminf(amax, araw);
                    // cullingFlag: splat boundary (alpha < 1/255), then T-Culling (T < 1e-4)
                    const bool live = valid[s] && al >= amin && T[s] >= tmin;
                    float g[9];
#pragma unroll
                    for (int j = 0; j < 9; ++j) g[j] = 0.f;
                    if (live) {
                        const float Ti = T[s];
                        const float wt = al * Ti;
                        // Eq. 3: dL/dc = dL/dC alpha T
                        g[6] = G[s][0] * wt;
                        g[7] = G[s][1] * wt;
                        g[8] = G[s][2] * wt;
                        // Eq. 7: dL/dalpha = dL/dC . (c T - C') / (1 - alpha)
                        const float ga = (G[s][0] * (cr * Ti - Cp[s][0]) + G[s][1] * (cg * Ti - Cp[s][1]) +
                                          G[s][2] * (cb * Ti - Cp[s][2])) *
                                         __builtin_amdgcn_rcpf(1.f - al);
                        // Eqs. 5, 6: the state update, stored back
                        Cp[s][0] = fmaf(-wt, cr, Cp[s][0]);
                        Cp[s][1] = fmaf(-wt, cg, Cp[s][1]);
                        Cp[s][2] = fmaf(-wt, cb, Cp[s][2]);
                        T[s] = Ti - wt;                                   // Eq. 5
                        if constexpr (RFMT >= 0) {
                            Cp[s][0] = fb_round<RFMT>(Cp[s][0]);
                            Cp[s][1] = fb_round<RFMT>(Cp[s][1]);
                            Cp[s][2] = fb_round<RFMT>(Cp[s][2]);
                            T[s] = fb_round<RFMT>(T[s]);
                        }
                        // bwd_diff: alpha = o exp(-q/2) (zero gradient where clamped);
                        // dq/dmu = -2 Q d, in the factored form: Q d = (a u, k a u + (det/a) dy),
                        // so dp/dd = (2 a' u, k 2 a' u + 2 d' dy) with the pre-scaled factors
                        if (araw < amax) {
                            const float gq = -0.5f * ga * araw;          // dL/dq
                            const float gm = -2.f * ga * araw * (1.0f / LOG2E);
                            g[5] = ga * e;
                            g[0] = gm * au;
                            g[1] = gm * fmaf(A.w, au, B.x * dy);
                            g[2] = gq * dx * dx;
                            g[3] = 2.f * gq * dx * dy;
                            g[4] = gq * dy * dy;
                        }
                    }
                    if (INSTR) {
                        cnt.evaluated += valid[s];
                        cnt.live += live;
                        nlive[s] += live;
                    }
                    if (lane_acc) {
#pragma unroll
                        for (int j = 0; j < 9; ++j) acc[j] += g[j];
                        acc_live = acc_live || live;
                    } else {
                        reduce_commit<INSTR>(g, live, gp, mode, X, lane, cnt);
                    }
                    if (!ballot(valid[s] && T[s] >= tmin)) alive &= ~(1u << s);
                }
                if (tile_acc) reduce_commit<INSTR, true>(acc, acc_live, tg + k * 9, GS_REDUCE_HYBRID, X, lane, cnt);
                else if (lane_acc) reduce_commit<INSTR>(acc, acc_live, gp, GS_REDUCE_HYBRID, X, lane, cnt);
            }
            if (lane == 0) w.alive[wave] = (int)alive;
            __syncthreads();
            if (!(w.alive[0] | w.alive[1] | w.alive[2] | w.alive[3])) { stop = true; break; }
        }
        if (stop) break;
    }
    if (tile_acc) flush_tile_grad<INSTR>(tg, w, pend, tid, grad, cnt);

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

// Scatter the accumulated gradients from sorted position to splat id; zero for culled splats.
__global__ __launch_bounds__(256) void k_grad_finalize(
    int n, const int32_t* __restrict__ sorted_ids, const int32_t* __restrict__ nvis_ptr,
    const float* __restrict__ grad, const float* __restrict__ rgb, int saturate,
    float* __restrict__ g_m, float* __restrict__ g_c, float* __restrict__ g_o,
    float* __restrict__ g_rgb) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int nvis = *nvis_ptr;
    nvis = nvis < 0 ? 0 : (nvis > n ? n : nvis);
    const int id = sorted_ids[p];
    if ((unsigned)id >= (unsigned)n) return;
    float v[9];
    if (p < nvis) {
        const float4* gp = reinterpret_cast<const float4*>(grad + (size_t)p * GRAD_STRIDE);
        const float4 u0 = gp[0], u1 = gp[1];
        const float u2 = grad[(size_t)p * GRAD_STRIDE + 8];
        v[0] = u0.x; v[1] = u0.y; v[2] = u0.z; v[3] = u0.w;
        v[4] = u1.x; v[5] = u1.y; v[6] = u1.z; v[7] = u1.w; v[8] = u2;
        if (saturate)
            for (int ch = 0; ch < 3; ++ch)
                if (rgb[3 * (size_t)id + ch] > 1.f) v[6 + ch] = 0.f;
    } else {
        for (int j = 0; j < 9; ++j) v[j] = 0.f;
    }
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

// ---- host side -------------------------------------------------------------------------------

static int tiles_of(int width, int height) {
    return ((width + TILE - 1) / TILE) * ((height + TILE - 1) / TILE);
}

// Words per tile row of the occupancy bitmap (0: no bitmap, every chunk is tested).
static int bitmap_wpr(int n, int width, int height) {
    const size_t nt = (size_t)tiles_of(width, height);
    const size_t wpr = ((size_t)n + SETUP_SPAN - 1) / SETUP_SPAN;   // one word per setup block
    return (n > 0 && nt <= (size_t)MAX_LDS_TILES && nt * wpr * 4 <= BITMAP_BUDGET) ? (int)wpr : 0;
}

size_t raster_ws_bytes(int n, int width, int height, bool bwd) {
    const size_t nt = (size_t)tiles_of(width, height);
    size_t b = align_up((size_t)n * REC_BYTES) + align_up((size_t)n * 8) + align_up(16 * 8) +
               align_up(nt * 4) * 2 + align_up(nt * (size_t)bitmap_wpr(n, width, height) * 4);
    if (bwd) b += align_up((size_t)n * GRAD_STRIDE * 4);
    return b;
}

RasterWs carve_raster_ws(void* ws, int n, int width, int height, bool bwd) {
    const size_t nt = (size_t)tiles_of(width, height);
    RasterWs r;
    char* p = (char*)ws;
    r.rec = p;      p += align_up((size_t)n * REC_BYTES);
    r.rect = p;     p += align_up((size_t)n * 8);
    r.counters = (unsigned long long*)p; p += align_up(16 * 8);
    r.weights = (uint32_t*)p; p += align_up(nt * 4);
    r.order = (int32_t*)p;    p += align_up(nt * 4);
    r.wpr = bitmap_wpr(n, width, height);
    r.bits = (uint32_t*)p;    p += align_up(nt * (size_t)r.wpr * 4);
    r.grad = bwd ? (float*)p : nullptr;
    return r;
}

// Records, tile rectangles, tile weights and the tile schedule.
static hipError_t raster_setup(const gs_config& cfg, int width, int height, int n,
                               const int32_t* sorted_ids, const int32_t* n_visible,
                               const float* means2d, const float* conics, const float* opac,
                               const float* rgb, const RasterWs& r, hipStream_t s) {
    const int tiles_x = (width + TILE - 1) / TILE;
    const int ntiles = tiles_of(width, height);
    hipError_t e = launch_fill_u32(r.weights, (size_t)ntiles, 0u, s);
    if (e != hipSuccess) return e;
    if (n > 0) {
        const int sat = (cfg.fb_format == FB_UNORM16 || cfg.fb_format == FB_UNORM8) ? 1 : 0;
        hipLaunchKernelGGL(k_raster_setup, dim3((n + SETUP_SPAN - 1) / SETUP_SPAN), dim3(256), 0, s,
                           n, sorted_ids, n_visible, means2d, conics, opac, rgb, width, height,
                           cfg.alpha_min, sat, tiles_x, ntiles, (Rec*)r.rec, (uint2*)r.rect,
                           r.weights, r.bits, r.wpr);
    }
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, s, r.weights, ntiles, r.order);
    return hipGetLastError();
}

static bool saturating(int fmt) { return fmt == FB_UNORM16 || fmt == FB_UNORM8; }

hipError_t launch_raster_setup(const gs_config& cfg, int width, int height, int n,
                               const int32_t* sorted_ids, const int32_t* n_visible,
                               const float* means2d, const float* conics, const float* opac,
                               const float* rgb, void* ws, hipStream_t s) {
    const RasterWs r = carve_raster_ws(ws, n, width, height, false);
    return raster_setup(cfg, width, height, n, sorted_ids, n_visible, means2d, conics, opac, rgb,
                        r, s);
}

template <bool TC, bool IN>
static void fwd_by_fmt(int rfmt, void (*&k)(int, const int32_t*, const Rec*, const uint2*,
                                             const int32_t*, const uint32_t*, int, int, int, int,
                                             float, float, float, int, void*, float*, float*,
                                             int32_t*, unsigned long long*)) {
    switch (rfmt) {
    case FB_F32: k = k_raster_fwd<FB_F32, TC, IN>; break;
    case FB_F16: k = k_raster_fwd<FB_F16, TC, IN>; break;
    case FB_UNORM16: k = k_raster_fwd<FB_UNORM16, TC, IN>; break;
    case FB_BF16: k = k_raster_fwd<FB_BF16, TC, IN>; break;
    case FB_UNORM8: k = k_raster_fwd<FB_UNORM8, TC, IN>; break;
    default: k = k_raster_fwd<-1, TC, IN>; break;
    }
}

hipError_t launch_raster_fwd(const gs_config& cfg, int width, int height, int n,
                             const int32_t* sorted_ids, const int32_t* n_visible,
                             const float* means2d, const float* conics, const float* opac,
                             const float* rgb, void* fb, float* out_rgb, float* out_T,
                             int32_t* out_cov, gs_stats* stats, void* ws, hipStream_t s) {
    const RasterWs r = carve_raster_ws(ws, n, width, height, false);
    if (!(cfg.flags & GS_FLAG_REUSE_SETUP)) {
        hipError_t e0 = raster_setup(cfg, width, height, n, sorted_ids, n_visible, means2d, conics,
                                     opac, rgb, r, s);
        if (e0 != hipSuccess) return e0;
    }
    const int tiles_x = (width + TILE - 1) / TILE;
    const int nblocks = tiles_of(width, height);
    const int rfmt = cfg.fb_round == GS_ROUND_PER_FRAGMENT ? cfg.fb_format : -1;
    const bool tcull = cfg.t_min_fwd > 0.f;
    const bool instr = (stats && (cfg.flags & GS_FLAG_STATS)) || out_cov;
    void (*k)(int, const int32_t*, const Rec*, const uint2*, const int32_t*, const uint32_t*, int,
              int, int, int, float, float, float, int, void*, float*, float*, int32_t*,
              unsigned long long*) = nullptr;
    if (tcull) { if (instr) fwd_by_fmt<true, true>(rfmt, k); else fwd_by_fmt<true, false>(rfmt, k); }
    else { if (instr) fwd_by_fmt<false, true>(rfmt, k); else fwd_by_fmt<false, false>(rfmt, k); }
    hipLaunchKernelGGL(k, dim3(nblocks), dim3(NT), 0, s, n, n_visible, (const Rec*)r.rec,
                       (const uint2*)r.rect, (const int32_t*)r.order, (const uint32_t*)r.bits,
                       r.wpr, width, height, tiles_x,
                       cfg.alpha_min, cfg.alpha_max, cfg.t_min_fwd, cfg.fb_format, fb, out_rgb, out_T,
                       out_cov,
                       (stats && (cfg.flags & GS_FLAG_STATS)) ? (unsigned long long*)stats : nullptr);
    return hipGetLastError();
}

hipError_t launch_raster_bwd(const gs_config& cfg, int width, int height, int n,
                             const int32_t* sorted_ids, const int32_t* n_visible,
                             const float* means2d, const float* conics, const float* opac,
                             const float* rgb, const void* fb, const float* dL_dimg,
                             float* g_means2d, float* g_conics, float* g_opac, float* g_rgb,
                             int32_t* out_live, gs_stats* stats, void* ws, hipStream_t s) {
    const RasterWs r = carve_raster_ws(ws, n, width, height, true);
    const int sat = (int)saturating(cfg.fb_format);
    if (n > 0) {
        hipError_t e = launch_fill_u32(r.grad, (size_t)n * GRAD_STRIDE, 0u, s);
        if (e != hipSuccess) return e;
    }
    if (!(cfg.flags & GS_FLAG_REUSE_SETUP)) {
        hipError_t e0 = raster_setup(cfg, width, height, n, sorted_ids, n_visible, means2d, conics,
                                     opac, rgb, r, s);
        if (e0 != hipSuccess) return e0;
    }
    const int tiles_x = (width + TILE - 1) / TILE;
    const int nblocks = tiles_of(width, height);
    const int rfmt = cfg.fb_round == GS_ROUND_PER_FRAGMENT ? cfg.fb_format : -1;
    const bool instr = (stats && (cfg.flags & GS_FLAG_STATS)) || out_live;
    void (*k)(int, const int32_t*, const Rec*, const uint2*, const int32_t*, const uint32_t*, int,
              int, int, int, float, float, float, int, const void*, const float*, int, int, float*,
              int32_t*, unsigned long long*) = nullptr;
#define GSR_BWD_PICK(IN)                                             \
    switch (rfmt) {                                                  \
    case FB_F32: k = k_raster_bwd<FB_F32, IN>; break;                \
    case FB_F16: k = k_raster_bwd<FB_F16, IN>; break;                \
    case FB_UNORM16: k = k_raster_bwd<FB_UNORM16, IN>; break;        \
    case FB_BF16: k = k_raster_bwd<FB_BF16, IN>; break;              \
    case FB_UNORM8: k = k_raster_bwd<FB_UNORM8, IN>; break;          \
    default: k = k_raster_bwd<-1, IN>; break;                        \
    }
    if (instr) { GSR_BWD_PICK(true) } else { GSR_BWD_PICK(false) }
#undef GSR_BWD_PICK
    hipLaunchKernelGGL(k, dim3(nblocks), dim3(NT), 0, s, n, n_visible, (const Rec*)r.rec,
                       (const uint2*)r.rect, (const int32_t*)r.order, (const uint32_t*)r.bits,
                       r.wpr, width, height, tiles_x,
                       cfg.alpha_min, cfg.alpha_max, cfg.t_min_bwd, cfg.fb_format, fb, dL_dimg,
                       cfg.reduce_mode,
                       cfg.reduce_threshold, r.grad, out_live,
                       (stats && (cfg.flags & GS_FLAG_STATS)) ? (unsigned long long*)stats : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n == 0) return e;
    hipLaunchKernelGGL(k_grad_finalize, dim3((n + 255) / 256), dim3(256), 0, s, n, sorted_ids,
                       n_visible, r.grad, rgb, sat, g_means2d, g_conics, g_opac, g_rgb);
    return hipGetLastError();
}

}  // namespace gsr
