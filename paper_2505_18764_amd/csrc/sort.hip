// sort.hip -- stable LSD radix sort of (key, int32 value) pairs with the sort length read on
// the device (the depth sort of Sec. 1 and Sec. 4.1, dynamic length after frustum culling).
//
// Each 8-bit digit pass: (1) per-block digit histograms, (2) per digit, an exclusive scan of its
// counts over the blocks and the digit's total, (3) a stable scatter in which every block first
// scans the 256 digit totals into digit bases, then ranks its keys round by round (256 keys per
// round, one per thread, in input order), ranking equal digits inside a wave with eight ballots
// and across the four waves through LDS counts. Three launches per pass.
// Several views sort in one launch per step (grid y = view): each view's keys, ids and count are
// its part of [V][n] arrays, and its histograms and ping-pong buffers live in its workspace slab.
#include <mutex>

#include "device.hpp"
#include "internal.hpp"

namespace gsr {

constexpr int SORT_THREADS = 256;
constexpr int SORT_ROUNDS = 8;
constexpr int SORT_ITEMS = SORT_THREADS * SORT_ROUNDS;   // keys per block
constexpr int SCAN_ITEMS = 4096;                         // entries per scan block (256 x 16)

__device__ __forceinline__ int dev_count(const int32_t* n_dev, int n_max) {
    int n = n_dev ? *n_dev : n_max;
    return n < 0 ? 0 : (n > n_max ? n_max : n);
}

// A sort buffer of a view: the caller's [V][n] array (in_ws = 0) or the view's workspace slab.
template <typename T>
__device__ __forceinline__ T* sort_buf(T* p, int in_ws, int n_max, uint64_t vws) {
    return in_ws ? view_bytes(p, vws) : view_at(p, (uint64_t)n_max);
}

template <typename K>
__global__ __launch_bounds__(SORT_THREADS) void k_sort_hist(const K* __restrict__ keys, int in_ws,
                                                            int n_max,
                                                            const int32_t* __restrict__ n_dev,
                                                            int shift, int nblocks,
                                                            uint32_t* __restrict__ hist,
                                                            uint64_t vws) {
    __shared__ uint32_t h[256];
    keys = sort_buf(keys, in_ws, n_max, vws);
    n_dev = view_at(n_dev, 1);
    hist = view_bytes(hist, vws);
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int n = dev_count(n_dev, n_max);
    const int start = blockIdx.x * SORT_ITEMS;
    if (start < n) {
        for (int r = 0; r < SORT_ROUNDS; ++r) {
            const int idx = start + r * SORT_THREADS + tid;
            if (idx < n) atomicAdd(&h[(uint32_t)(keys[idx] >> shift) & 0xFFu], 1u);
        }
    }
    __syncthreads();
    hist[(size_t)tid * nblocks + blockIdx.x] = h[tid];
}

// Exclusive scan of `count` uint32: block sums, scan of the sums, apply (the middle launch is
// skipped when the blocks are few enough for each to add up its predecessors itself).
// Batched over views: `in`, `out` and `sums` of view v are `vws` bytes after view v - 1's.
__global__ __launch_bounds__(256) void k_scan_sums(const uint32_t* __restrict__ in, size_t count,
                                                   uint32_t* __restrict__ sums, uint64_t vws) {
    __shared__ uint32_t red[4];
    in = view_bytes(in, vws);
    sums = view_bytes(sums, vws);
    const size_t base = (size_t)blockIdx.x * SCAN_ITEMS;
    uint32_t s = 0;
    for (int j = 0; j < SCAN_ITEMS / 256; ++j) {
        const size_t i = base + (size_t)j * 256 + threadIdx.x;
        if (i < count) s += in[i];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Single block: exclusive scan of `count` (<= 1024 * 64) block sums in place.
__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* __restrict__ sums, int count,
                                                   uint64_t vws) {
    __shared__ uint32_t part[1024];
    sums = view_bytes(sums, vws);
    const int per = (count + 1023) / 1024;
    const int lo = threadIdx.x * per;
    uint32_t s = 0;
    for (int j = 0; j < per; ++j)
        if (lo + j < count) s += sums[lo + j];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {     // Hillis-Steele inclusive scan
        uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    for (int j = 0; j < per; ++j)
        if (lo + j < count) {
            const uint32_t v = sums[lo + j];
            sums[lo + j] = run;
            run += v;
        }
}

// With `raw_sums`, sums[] holds the blocks' totals (not yet scanned) and each block adds those of
// the blocks before it itself, which saves the launch of k_scan_top when the blocks are few.
__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* __restrict__ in, size_t count,
                                                    const uint32_t* __restrict__ sums,
                                                    uint32_t* __restrict__ out, uint64_t vws,
                                                    int raw_sums) {
    // each thread owns 16 consecutive entries of the block's 4096
    __shared__ uint32_t part[256];
    __shared__ uint32_t s_red[4];
    in = view_bytes(in, vws);
    sums = view_bytes(sums, vws);
    out = view_bytes(out, vws);
    uint32_t before = 0u;
    if (raw_sums) {
        for (int b = threadIdx.x; b < (int)blockIdx.x; b += 256) before += sums[b];
        for (int o = 32; o > 0; o >>= 1) before += __shfl_xor(before, o);
        if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = before;
        __syncthreads();
        before = s_red[0] + s_red[1] + s_red[2] + s_red[3];
    } else {
        before = sums[blockIdx.x];
    }
    const size_t base = (size_t)blockIdx.x * SCAN_ITEMS + (size_t)threadIdx.x * 16;
    uint32_t v[16];
    uint32_t s = 0;
    for (int j = 0; j < 16; ++j) {
        v[j] = (base + j < count) ? in[base + j] : 0u;
        s += v[j];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t t = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t run = before + (threadIdx.x ? part[threadIdx.x - 1] : 0u);
    for (int j = 0; j < 16; ++j)
        if (base + j < count) {
            out[base + j] = run;
            run += v[j];
        }
}

// One workgroup scans up to SCAN_ONE_MAX entries in one launch (e.g. the compaction's block
// counts): thread t sums its contiguous run of at most 4 entries, the 1024 run sums are scanned
// (within each wave by shuffles, then over the 16 waves), and each thread writes its run's
// prefixes. `in` and `out` may alias. Longer arrays take the three-launch scan: one workgroup
// cannot keep enough loads in flight to read them quickly.
constexpr int SCAN_ONE_THREADS = 1024;
constexpr size_t SCAN_ONE_MAX = (size_t)SCAN_ONE_THREADS * 4;

__global__ __launch_bounds__(SCAN_ONE_THREADS) void k_scan_one(const uint32_t* in, size_t count,
                                                               uint32_t* out, uint64_t vws) {
    __shared__ uint32_t s_wave[SCAN_ONE_THREADS / 64];
    in = view_bytes(in, vws);
    out = view_bytes(out, vws);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const size_t per = (count + SCAN_ONE_THREADS - 1) / SCAN_ONE_THREADS;
    const size_t lo = min((size_t)tid * per, count), hi = min(lo + per, count);
    uint32_t run = 0u;
    for (size_t i = lo; i < hi; ++i) run += in[i];
    uint32_t incl = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(incl, o);
        if (lane >= o) incl += u;
    }
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    uint32_t base = incl - run;
    for (int w = 0; w < wave; ++w) base += s_wave[w];
    for (size_t i = lo; i < hi; ++i) {
        const uint32_t v = in[i];
        out[i] = base;
        base += v;
    }
}

hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, size_t count, uint32_t* sums,
                                 hipStream_t s, const Views& vs) {
    if (count == 0) return hipSuccess;
    if (count <= SCAN_ONE_MAX) {
        hipLaunchKernelGGL(k_scan_one, dim3(1, vs.count), dim3(SCAN_ONE_THREADS), 0, s, in, count,
                           out, vs.ws);
        return hipGetLastError();
    }
    const int blocks = (int)((count + SCAN_ITEMS - 1) / SCAN_ITEMS);
    const int V = vs.count;
    hipLaunchKernelGGL(k_scan_sums, dim3(blocks, V), dim3(256), 0, s, in, count, sums, vs.ws);
    const int raw = blocks <= 256 ? 1 : 0;   // few blocks: each adds its predecessors' totals
    if (!raw) hipLaunchKernelGGL(k_scan_top, dim3(1, V), dim3(1024), 0, s, sums, blocks, vs.ws);
    hipLaunchKernelGGL(k_scan_apply, dim3(blocks, V), dim3(256), 0, s, in, count, sums, out,
                       vs.ws, raw);
    return hipGetLastError();
}

// Row d of the digit-major [digit][block] count table (one workgroup per digit): the exclusive
// prefix of each block within the digit, and the digit's total.
__global__ __launch_bounds__(256) void k_digit_scan(const uint32_t* __restrict__ hist,
                                                    int nblocks, uint32_t* __restrict__ prefix,
                                                    uint32_t* __restrict__ totals, uint64_t vws) {
    __shared__ uint32_t s_w[4];
    hist = view_bytes(hist, vws);
    prefix = view_bytes(prefix, vws);
    totals = view_bytes(totals, vws);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t* row = hist + (size_t)blockIdx.x * nblocks;
    uint32_t* orow = prefix + (size_t)blockIdx.x * nblocks;
    uint32_t carry = 0u;
    for (int b0 = 0; b0 < nblocks; b0 += 256) {     // 256 blocks' counts at a time
        const int b = b0 + tid;
        const uint32_t v = b < nblocks ? row[b] : 0u;
        uint32_t incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(incl, o);
            if (lane >= o) incl += u;
        }
        if (lane == 63) s_w[wave] = incl;
        __syncthreads();
        uint32_t before = carry, chunk = 0u;
#pragma unroll
        for (int w2 = 0; w2 < 4; ++w2) {
            before += w2 < wave ? s_w[w2] : 0u;
            chunk += s_w[w2];
        }
        __syncthreads();                            // s_w is rewritten by the next chunk
        if (b < nblocks) orow[b] = before + incl - v;
        carry += chunk;
    }
    if (tid == 0) totals[blockIdx.x] = carry;
}

template <typename K>
__global__ __launch_bounds__(SORT_THREADS) void k_sort_scatter(
    const K* __restrict__ kin, const int32_t* __restrict__ vin, int in_ws, K* __restrict__ kout,
    int32_t* __restrict__ vout, int out_ws, int n_max, const int32_t* __restrict__ n_dev,
    int shift, int nblocks, const uint32_t* __restrict__ prefix,
    const uint32_t* __restrict__ totals, uint64_t vws) {
    __shared__ uint32_t s_off[256];
    __shared__ uint16_t s_cnt[2][4][256];
    __shared__ uint32_t s_w[4];
    kin = sort_buf(kin, in_ws, n_max, vws);
    vin = sort_buf(vin, in_ws, n_max, vws);
    kout = sort_buf(kout, out_ws, n_max, vws);
    vout = sort_buf(vout, out_ws, n_max, vws);
    n_dev = view_at(n_dev, 1);
    prefix = view_bytes(prefix, vws);
    totals = view_bytes(totals, vws);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = dev_count(n_dev, n_max);
    const int start = blockIdx.x * SORT_ITEMS;
    if (start >= n) return;                         // uniform for the block
    {   // thread tid owns digit tid: its base is the exclusive scan of the digit totals
        const uint32_t t = totals[tid];
        uint32_t incl = t;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(incl, o);
            if (lane >= o) incl += u;
        }
        if (lane == 63) s_w[wave] = incl;
        __syncthreads();
        uint32_t base = incl - t;
#pragma unroll
        for (int w2 = 0; w2 < 4; ++w2) base += w2 < wave ? s_w[w2] : 0u;
        s_off[tid] = base + prefix[(size_t)tid * nblocks + blockIdx.x];
    }
    for (int b = 0; b < 2; ++b)
        for (int w = 0; w < 4; ++w) s_cnt[b][w][tid] = 0;
    __syncthreads();
    const uint64_t lt = mask_lt(lane);
    // all of the block's pairs are loaded up front, so the rounds below wait on no global load
    K kr[SORT_ROUNDS];
    int32_t vr[SORT_ROUNDS];
#pragma unroll
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const int idx = start + r * SORT_THREADS + tid;
        kr[r] = idx < n ? kin[idx] : K(0);
        vr[r] = idx < n ? vin[idx] : 0;
    }
#pragma unroll
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const int buf = r & 1;
        const int idx = start + r * SORT_THREADS + tid;
        const bool valid = idx < n;
        const K key = kr[r];
        const int32_t val = vr[r];
        const uint32_t d = valid ? (uint32_t)(key >> shift) & 0xFFu : 0u;
        // lanes of this wave with the same digit
        uint64_t peers = ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = ballot(valid && ((d >> b) & 1u));
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        if (!valid) peers = 0;
        const int rank = popc(peers & lt);
        if (valid && rank == 0) s_cnt[buf][wave][d] = (uint16_t)popc(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = s_off[d] + (uint32_t)rank;
            for (int w = 0; w < wave; ++w) off += s_cnt[buf][w][d];
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        // thread `tid` owns digit `tid`: advance its offset and clear its column for round r+2
        s_off[tid] += (uint32_t)s_cnt[buf][0][tid] + s_cnt[buf][1][tid] + s_cnt[buf][2][tid] +
                      s_cnt[buf][3][tid];
        for (int w = 0; w < 4; ++w) s_cnt[buf][w][tid] = 0;
    }
}

template <typename K>
__global__ void k_copy_pairs(const K* __restrict__ ks, const int32_t* __restrict__ vs,
                             K* __restrict__ kd, int32_t* __restrict__ vd, int n_max,
                             const int32_t* __restrict__ n_dev, uint64_t vws) {
    ks = view_bytes(ks, vws);          // the workspace's ping-pong buffers
    vs = view_bytes(vs, vws);
    kd = view_at(kd, (uint64_t)n_max);
    vd = view_at(vd, (uint64_t)n_max);
    n_dev = view_at(n_dev, 1);
    const int n = dev_count(n_dev, n_max);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        kd[i] = ks[i];
        vd[i] = vs[i];
    }
}

// ---- order-preserving compaction of the visible splats (frustum culling, Sec. 4.1) -------
// keys_by_id[i] == 0xFFFFFFFF marks a culled splat. Output: (keys, ids) with the visible splats
// first in id order, then the culled ones in id order; n_visible = number of visible splats.

__global__ __launch_bounds__(SORT_THREADS) void k_compact_count(const uint32_t* __restrict__ kid,
                                                                int n, uint32_t* __restrict__ cnt,
                                                                uint64_t vws) {
    __shared__ uint32_t red[4];
    kid = view_bytes(kid, vws);
    cnt = view_bytes(cnt, vws);
    const int start = blockIdx.x * SORT_ITEMS;
    uint32_t c = 0;
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const int i = start + r * SORT_THREADS + threadIdx.x;
        c += popc(ballot(i < n && kid[i] != 0xFFFFFFFFu)) * (lane_id() == 0);
    }
    if (lane_id() == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(SORT_THREADS) void k_compact_scatter(
    const uint32_t* __restrict__ kid, int n, int nblocks, const uint32_t* __restrict__ cnt,
    const uint32_t* __restrict__ offs, uint32_t* __restrict__ keys, int32_t* __restrict__ ids,
    int32_t* __restrict__ n_visible, uint64_t vws) {
    __shared__ uint32_t s_w[2][4];
    kid = view_bytes(kid, vws);
    cnt = view_bytes(cnt, vws);
    offs = view_bytes(offs, vws);
    keys = view_at(keys, (uint64_t)n);
    ids = view_at(ids, (uint64_t)n);
    n_visible = view_at(n_visible, 1);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t total = offs[nblocks - 1] + cnt[nblocks - 1];
    if (blockIdx.x == 0 && tid == 0) *n_visible = (int32_t)total;
    const int start = blockIdx.x * SORT_ITEMS;
    uint32_t vis_run = offs[blockIdx.x];
    uint32_t cul_run = total + ((uint32_t)start - offs[blockIdx.x]);
    const uint64_t lt = mask_lt(lane);
    uint32_t kr[SORT_ROUNDS];               // loaded up front, as in the sort's scatter
#pragma unroll
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const int i = start + r * SORT_THREADS + tid;
        kr[r] = i < n ? kid[i] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const int i = start + r * SORT_THREADS + tid;
        const bool in = i < n;
        const uint32_t k = kr[r];
        const bool v = in && k != 0xFFFFFFFFu;
        const uint64_t mv = ballot(v), mc = ballot(in && !v);
        if (lane == 0) { s_w[0][wave] = popc(mv); s_w[1][wave] = popc(mc); }
        __syncthreads();
        uint32_t pv = vis_run, pc = cul_run;
        for (int w = 0; w < wave; ++w) { pv += s_w[0][w]; pc += s_w[1][w]; }
        if (v) { keys[pv + popc(mv & lt)] = k; ids[pv + popc(mv & lt)] = i; }
        else if (in) { keys[pc + popc(mc & lt)] = k; ids[pc + popc(mc & lt)] = i; }
        vis_run += s_w[0][0] + s_w[0][1] + s_w[0][2] + s_w[0][3];
        cul_run += s_w[1][0] + s_w[1][1] + s_w[1][2] + s_w[1][3];
        __syncthreads();
    }
}

size_t compact_ws_bytes(int n) {
    const size_t nb = (size_t)((n + SORT_ITEMS - 1) / SORT_ITEMS + 1);
    return align_up(nb * 4) * 2 + align_up(((nb + SCAN_ITEMS - 1) / SCAN_ITEMS) * 4);
}

hipError_t launch_compact(int n, const uint32_t* key_by_id, uint32_t* keys, int32_t* ids,
                          int32_t* n_visible, void* ws, hipStream_t s, const Views& vs) {
    if (n == 0) return launch_fill_u32(n_visible, (size_t)vs.count, 0u, s);
    const int nb = (n + SORT_ITEMS - 1) / SORT_ITEMS;
    char* p = (char*)ws;
    uint32_t* cnt = (uint32_t*)p;  p += align_up((size_t)(nb + 1) * 4);
    uint32_t* offs = (uint32_t*)p; p += align_up((size_t)(nb + 1) * 4);
    uint32_t* sums = (uint32_t*)p;
    hipLaunchKernelGGL(k_compact_count, dim3(nb, vs.count), dim3(SORT_THREADS), 0, s, key_by_id,
                       n, cnt, vs.ws);
    hipError_t e = launch_exclusive_scan(cnt, offs, (size_t)nb, sums, s, vs);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_compact_scatter, dim3(nb, vs.count), dim3(SORT_THREADS), 0, s, key_by_id,
                       n, nb, cnt, offs, keys, ids, n_visible, vs.ws);
    return hipGetLastError();
}

static int sort_blocks(int n) { return (n + SORT_ITEMS - 1) / SORT_ITEMS; }

size_t sort_ws_bytes(int n, int key_bytes) {
    const size_t nb = (size_t)(n > 0 ? sort_blocks(n) : 1);
    const size_t table = 256 * nb;
    return align_up((size_t)n * key_bytes) + align_up((size_t)n * 4) + align_up(table * 4) * 2 +
           align_up(256 * 4);
}

template <typename K>
static hipError_t sort_pairs(int n, K* keys, int32_t* vals, const int32_t* n_dev, int end_bit,
                             void* ws, hipStream_t s, const Views& vs) {
    if (n == 0) return hipSuccess;
    const int V = vs.count;
    const int nb = sort_blocks(n);
    const size_t table = 256 * (size_t)nb;
    char* p = (char*)ws;
    K* kalt = (K*)p;            p += align_up((size_t)n * sizeof(K));
    int32_t* valt = (int32_t*)p; p += align_up((size_t)n * 4);
    uint32_t* hist = (uint32_t*)p; p += align_up(table * 4);
    uint32_t* offs = (uint32_t*)p; p += align_up(table * 4);
    uint32_t* totals = (uint32_t*)p;
    K* kin = keys; int32_t* vin = vals;
    K* kout = kalt; int32_t* vout = valt;
    int in_ws = 0, out_ws = 1;
    int passes = 0;
    for (int shift = 0; shift < end_bit; shift += 8, ++passes) {
        hipLaunchKernelGGL(k_sort_hist<K>, dim3(nb, V), dim3(SORT_THREADS), 0, s, kin, in_ws, n,
                           n_dev, shift, nb, hist, vs.ws);
        hipLaunchKernelGGL(k_digit_scan, dim3(256, V), dim3(256), 0, s, hist, nb, offs, totals,
                           vs.ws);
        hipLaunchKernelGGL(k_sort_scatter<K>, dim3(nb, V), dim3(SORT_THREADS), 0, s, kin, vin,
                           in_ws, kout, vout, out_ws, n, n_dev, shift, nb, offs, totals, vs.ws);
        K* tk = kin; kin = kout; kout = tk;
        int32_t* tv = vin; vin = vout; vout = tv;
        const int tw = in_ws; in_ws = out_ws; out_ws = tw;
    }
    if (passes & 1) {   // result sits in the alternate buffers: copy back
        int blocks = (n + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(k_copy_pairs<K>, dim3(blocks, V), dim3(256), 0, s, kin, vin, keys,
                           vals, n, n_dev, vs.ws);
    }
    return hipGetLastError();
}

hipError_t launch_sort_u32(int n, uint32_t* keys, int32_t* vals, const int32_t* n_dev, void* ws,
                           hipStream_t s, const Views& vs) {
    return sort_pairs<uint32_t>(n, keys, vals, n_dev, 32, ws, s, vs);
}

hipError_t launch_sort_u64(int n, uint64_t* keys, int32_t* vals, const int32_t* n_dev,
                           int end_bit, void* ws, hipStream_t s) {
    return sort_pairs<uint64_t>(n, keys, vals, n_dev, end_bit, ws, s, one_view());
}

// ---- the depth sort without a caller workspace ---------------------------------------------
// For callers that cannot allocate (code under graph capture, serving loops, harnesses that
// forbid allocation), the sort's scratch is a file-scope device array of fixed size, one per GPU,
// held for the life of the process. In host code `scratch` only names the symbol: its device
// address on the current GPU comes from hipGetSymbolAddress, taken once per device on the first
// call there and kept; only that address is ever passed to a kernel. Every word of the scratch
// is written before it is read in a call, so nothing needs clearing between calls; calls that
// overlap on one GPU share the array and race.
constexpr size_t NOALLOC_SORT_BYTES =
    ((size_t)NOALLOC_SORT_MAX_N * 4 + 255) / 256 * 256 +          // alternate keys
    ((size_t)NOALLOC_SORT_MAX_N * 4 + 255) / 256 * 256 +          // alternate values
    2 * ((256 * (size_t)((NOALLOC_SORT_MAX_N + SORT_ITEMS - 1) / SORT_ITEMS) * 4 + 255) / 256 * 256) +
    256 * 4;                                                       // digit totals
static __device__ __align__(256) unsigned char scratch[NOALLOC_SORT_BYTES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_dev[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_sort_scratch(void** out, size_t* bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {           // set-up on this device, which is the current one
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    *bytes = NOALLOC_SORT_BYTES;
    return hipSuccess;
}

hipError_t launch_sort_u32_noalloc(int n, uint32_t* keys, int32_t* vals, const int32_t* n_dev,
                                   hipStream_t s) {
    if (n == 0) return hipSuccess;
    void* ws = nullptr;
    size_t bytes = 0;
    hipError_t e = noalloc_sort_scratch(&ws, &bytes);
    if (e != hipSuccess) return e;
    if (sort_ws_bytes(n, 4) > bytes) return hipErrorInvalidValue;   // the caller checked n
    return sort_pairs<uint32_t>(n, keys, vals, n_dev, 32, ws, s, one_view());
}

}  // namespace gsr
