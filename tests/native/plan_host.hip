// plan_host.hip -- host build of the raster's tile schedulers (plan.hpp) for the CPU tests.
//
// The scheduling code is the GPU's own (gsr::bucket_order and the segment helpers); only the
// workgroup is emulated: each phase between two barriers runs every thread to completion, one
// after another, in an order shuffled by a seed, and the shared-memory atomics are plain
// read-modify-writes. The tests call the extern "C" functions below through ctypes.
#include <stdint.h>

#include <algorithm>
#include <random>
#include <vector>

#include "../../paper_2505_18764_amd/csrc/plan.hpp"

namespace {

struct SeqBlock {
    int nt;
    std::vector<int> order;
    std::mt19937_64 rng;
    SeqBlock(int nthreads, uint64_t seed) : nt(nthreads), order(nthreads), rng(seed) {
        for (int i = 0; i < nt; ++i) order[i] = i;
    }
    template <class F>
    void each(F&& f) {
        std::shuffle(order.begin(), order.end(), rng);   // a new interleaving per phase
        for (int t : order) f(t, nt);
    }
    void sync() {}
    uint32_t atomic_inc(uint32_t* p) { return (*p)++; }
    void exclusive_scan(uint32_t* h) {
        uint32_t run = 0u;
        for (int b = 0; b < gsr::NBUCKETS; ++b) {
            const uint32_t v = h[b];
            h[b] = run;
            run += v;
        }
    }
};

}  // namespace

extern "C" {

// gsr::bucket_order over w[0 .. count) into out[0 .. pad), as one workgroup of `nthreads`
// threads whose phases run in the order drawn from `seed`. Returns 0.
int plan_bucket_order(const uint32_t* w, int count, uint32_t wmax, int32_t* out, int pad,
                      int nthreads, uint64_t seed) {
    std::vector<uint32_t> hist(gsr::NBUCKETS, 0xDEADBEEFu);   // garbage: the function clears it
    SeqBlock blk(nthreads, seed);
    gsr::bucket_order(blk, w, count, wmax, out, pad, hist.data());
    return 0;
}

int plan_weight_bucket(uint32_t x, uint32_t wmax) {
    return gsr::weight_bucket(x, gsr::bucket_scale(wmax));
}

uint32_t plan_segment_cap(unsigned long long total, int ntiles) {
    return gsr::segment_cap(total, ntiles);
}

int plan_segment_count(uint32_t w, uint32_t cap) { return gsr::segment_count(w, cap); }

uint32_t plan_cut_target(uint32_t w, int j, int k) { return gsr::cut_target(w, j, k); }

int plan_items_per_tile(void) { return gsr::ITEMS_PER_TILE; }
int plan_max_segments(void) { return gsr::MAX_SEGMENTS; }
int plan_nbuckets(void) { return gsr::NBUCKETS; }

}  // extern "C"
