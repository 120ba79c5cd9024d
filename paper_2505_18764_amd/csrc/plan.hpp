// plan.hpp -- the arithmetic of the raster's tile schedules, written once for a workgroup on the
// GPU and for a sequential emulation of a workgroup on the host.
//
// Every schedule of the raster (the forward's tile order, the depth-split work items and their
// order, the backward's tile order) is a longest-processing-time-first list: work items sorted by
// decreasing weight. The order only has to be approximate, so it is a counting sort over NBUCKETS
// weight buckets. The sort is written against a workgroup policy `Blk`:
//   blk.each(f)          runs f(tid, nthreads) for the calling thread (GPU) or for every thread
//                        of the emulated workgroup in some order (host);
//   blk.sync()           a workgroup barrier;
//   blk.atomic_inc(p)    returns *p and adds 1, atomically among the workgroup's threads;
//   blk.exclusive_scan(h) replaces h[0 .. NBUCKETS) by its exclusive prefix sum.
// The GPU policy lives with the kernels; the host policy with the tests, which run the same
// function over adversarial weights and check that the result is a permutation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsr {

constexpr int NBUCKETS = 1024;
// Depth split: a tile heavier than the mean is cut into up to MAX_SEGMENTS depth segments; the
// segment size is a third of the mean tile weight, so the work items of all tiles number at most
// (SEG_DIV + 1) x tiles (see segment_count).
constexpr int MAX_SEGMENTS = 32;
constexpr int SEG_DIV = 3;
constexpr int ITEMS_PER_TILE = SEG_DIV + 1;

// Buckets split [0, wmax] evenly, heaviest first: bucket 0 holds the largest weights.
__host__ __device__ inline float bucket_scale(uint32_t wmax) {
    return (float)NBUCKETS / ((float)wmax + 1.0f);
}
// The clamp happens in FP32, before the conversion, so a weight above wmax lands in bucket 0
// on any target (an out-of-range float-to-int conversion is undefined on the host).
__host__ __device__ inline int weight_bucket(uint32_t x, float scale) {
    const float f = (float)x * scale;
    return NBUCKETS - 1 - (f < (float)(NBUCKETS - 1) ? (int)f : NBUCKETS - 1);
}

// out[0 .. count) = the indices 0 .. count-1 ordered by bucket (heaviest first, any order inside
// a bucket), out[count .. pad) = -1. hist: NBUCKETS words of scratch shared by the workgroup.
// wmax must be at least every w[i] (a larger value only coarsens the buckets).
template <class Blk>
__host__ __device__ void bucket_order(Blk& blk, const uint32_t* __restrict__ w, int count,
                                      uint32_t wmax, int32_t* __restrict__ out, int pad,
                                      uint32_t* hist) {
    blk.each([&](int tid, int nt) {
        for (int b = tid; b < NBUCKETS; b += nt) hist[b] = 0u;
    });
    blk.sync();
    const float scale = bucket_scale(wmax);
    blk.each([&](int tid, int nt) {
        for (int i = tid; i < count; i += nt) blk.atomic_inc(&hist[weight_bucket(w[i], scale)]);
    });
    blk.sync();
    blk.exclusive_scan(hist);              // hist[b] = first output slot of bucket b
    blk.sync();
    blk.each([&](int tid, int nt) {
        for (int i = tid; i < count; i += nt) out[blk.atomic_inc(&hist[weight_bucket(w[i], scale)])] = i;
        for (int i = count + tid; i < pad; i += nt) out[i] = -1;
    });
}

// Segment size of the depth split: ceil(mean tile weight / SEG_DIV), at least 1. With it, the
// tiles' segment counts add up to at most total / cap + tiles <= ITEMS_PER_TILE x tiles.
__host__ __device__ inline uint32_t segment_cap(unsigned long long total, int ntiles) {
    const unsigned long long d = (unsigned long long)SEG_DIV * (unsigned long long)ntiles;
    const unsigned long long c = (total + d - 1ull) / d;
    return (uint32_t)(c > 1ull ? c : 1ull);
}

// Segments of a tile of weight w: ceil(w / cap), clamped to [1, MAX_SEGMENTS].
__host__ __device__ inline int segment_count(uint32_t w, uint32_t cap) {
    const uint32_t q = w / cap + (w % cap != 0u);
    return (int)(q < 1u ? 1u : (q > (uint32_t)MAX_SEGMENTS ? (uint32_t)MAX_SEGMENTS : q));
}

// Cut j of a tile of weight w in k segments lies where the running splat count over the tile's
// columns first reaches ceil(j w / k) (j = 1 .. k-1); the targets increase with j.
__host__ __device__ inline uint32_t cut_target(uint32_t w, int j, int k) {
    return (uint32_t)(((unsigned long long)w * (unsigned long long)j + (unsigned long long)k - 1ull) /
                      (unsigned long long)k);
}

}  // namespace gsr
