// device.hpp -- wave64 primitives, DPP reductions and framebuffer formats for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsr {

// ---- wave64 primitives ------------------------------------------------------------------

__device__ __forceinline__ int lane_id() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int popc(uint64_t m) { return __popcll(m); }
__device__ __forceinline__ uint64_t mask_lt(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float read_lane(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// ---- DPP (data-parallel primitives) ------------------------------------------------------
// Every reduction below runs with all 64 lanes active; lanes that hold nothing contribute 0.

template <int CTRL, int ROW_MASK = 0xF, int BANK_MASK = 0xF>
__device__ __forceinline__ float dpp(float old, float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                      CTRL, ROW_MASK, BANK_MASK, false));
}
template <int CTRL, int ROW_MASK = 0xF, int BANK_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp_u(uint32_t old, uint32_t src) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, CTRL, ROW_MASK, BANK_MASK,
                                                 false);
}

constexpr int DPP_QUAD_1032 = 0xB1;       // quad_perm [1,0,3,2]: horizontal neighbour in a 2x2 quad
constexpr int DPP_QUAD_2301 = 0x4E;       // quad_perm [2,3,0,1]: vertical neighbour
constexpr int DPP_ROW_MIRROR = 0x140;     // lane i <- lane 15-i within a 16-lane row
constexpr int DPP_ROW_HALF_MIRROR = 0x141;// lane i <- lane 7-i within an 8-lane half row
constexpr int DPP_ROW_BCAST15 = 0x142;    // rows 1, 3 <- lane 15 of the row before
constexpr int DPP_ROW_BCAST31 = 0x143;    // rows 2, 3 <- lane 31

// Sum over the 2x2 quad (quadAdd of Procedure 2); every lane of the quad gets the sum.
__device__ __forceinline__ float quad_sum(float v) {
    v += dpp<DPP_QUAD_1032>(v, v);
    v += dpp<DPP_QUAD_2301>(v, v);
    return v;
}

// OR over the 2x2 quad (quadOr of Procedure 2).
__device__ __forceinline__ uint32_t quad_or(uint32_t v) {
    v |= dpp_u<DPP_QUAD_1032>(v, v);
    v |= dpp_u<DPP_QUAD_2301>(v, v);
    return v;
}

// Sum over all 64 lanes (subgroupAdd); the result is returned wave-uniform.
__device__ __forceinline__ float wave_sum(float v) {
    v = quad_sum(v);
    v += dpp<DPP_ROW_HALF_MIRROR>(v, v);
    v += dpp<DPP_ROW_MIRROR>(v, v);               // every lane: sum of its 16-lane row
    v += dpp<DPP_ROW_BCAST15, 0xA>(0.0f, v);      // rows 1, 3: + previous row
    v += dpp<DPP_ROW_BCAST31, 0xC>(0.0f, v);      // rows 2, 3: + rows 0..1
    return read_lane(v, 63);
}

// ---- nine sums over the wave at once (gfx950 lane swaps) ----------------------------------
// DPP add source with bound_ctrl set: for the full-mask controls below every lane is valid, so
// the move fuses into v_add_f32_dpp.
template <int CTRL>
__device__ __forceinline__ float dpp_bc(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Every lane of each 16-lane row gets the row's sum.
__device__ __forceinline__ float row_sum16(float v) {
    v += dpp_bc<DPP_QUAD_1032>(v);
    v += dpp_bc<DPP_QUAD_2301>(v);
    v += dpp_bc<DPP_ROW_HALF_MIRROR>(v);
    v += dpp_bc<DPP_ROW_MIRROR>(v);
    return v;
}

// v_permlane32_swap: a keeps its lanes 0-31 and takes b's lanes 0-31 as lanes 32-63; b receives
// a's lanes 32-63 as lanes 0-31 and keeps its lanes 32-63. x + y then holds a's sums over the
// wave halves in lanes 0-31 and b's in lanes 32-63. v_permlane16_swap does the same between
// adjacent 16-lane rows.
__device__ __forceinline__ float swap32_add(float a, float b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap16_add(float a, float b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sums of g[0..8] over the wave (all lanes active), transposed: each pair of values shares a
// register at every halving step, so 28 VALU instructions replace nine separate reductions.
// On return every lane of 16-lane row r holds in a the total of g[{0, 2, 1, 3}[r]], in b that of
// g[{4, 6, 5, 7}[r]], and (row 0) in c that of g[8].
__device__ __forceinline__ void wave_sum9(const float (&g)[9], float& a, float& b, float& c) {
    const float p0 = swap32_add(g[0], g[1]), p1 = swap32_add(g[2], g[3]);
    const float p2 = swap32_add(g[4], g[5]), p3 = swap32_add(g[6], g[7]);
    const float p4 = swap32_add(g[8], 0.f);
    a = row_sum16(swap16_add(p0, p1));
    b = row_sum16(swap16_add(p2, p3));
    c = row_sum16(swap16_add(p4, 0.f));
}

__device__ __forceinline__ void atomic_add_f32(float* p, float v) { unsafeAtomicAdd(p, v); }

// Compensated FP32 accumulation into a (hi, lo) pair of global words: the atomic add to hi
// returns the value it added to, so the add's exact rounding error follows from Knuth's TwoSum
// and goes to lo with a second atomic. hi + lo then equals the exact sum of all the values added,
// up to the rounding of lo's own (much smaller) adds, in whatever order the adds arrive: the
// sum no longer depends on the order in which workgroups reach the word.
__device__ __forceinline__ void atomic_add_f32_comp(float* hi, float* lo, float v) {
    const float old = unsafeAtomicAdd(hi, v);
    const float s = old + v;                  // the value the atomic stored (IEEE RNE)
    const float bv = s - old;
    const float err = (old - (s - bv)) + (v - bv);
    if (err != 0.f) unsafeAtomicAdd(lo, err);
}

// View-batched launches (grid y = view): p moved to this workgroup's view, where one view's part
// of the array is `per_view` elements (view_at) or bytes (view_bytes). Null stays null.
template <class T>
__device__ __forceinline__ T* view_at(T* p, uint64_t per_view) {
    return p ? p + (uint64_t)blockIdx.y * per_view : p;
}
template <class T>
__device__ __forceinline__ T* view_bytes(T* p, uint64_t bytes) {
    return p ? reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(p) + (uint64_t)blockIdx.y * bytes)
             : p;
}

// ---- framebuffer formats (Sec. 3.3) -------------------------------------------------------

enum : int { FB_F32 = 0, FB_F16 = 1, FB_UNORM16 = 2, FB_BF16 = 3, FB_UNORM8 = 4 };

__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                            // nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint32_t f32_to_unorm(float x, float levels) {
    x = fminf(fmaxf(x, 0.0f), 1.0f);                  // NaN -> 0
    return (uint32_t)__builtin_rintf(x * levels);     // nearest even
}

// Round a state value to the format and back (a store followed by a load).
template <int FMT>
__device__ __forceinline__ float fb_round(float x) {
    if constexpr (FMT == FB_F16) {
        return (float)(_Float16)x;
    } else if constexpr (FMT == FB_BF16) {
        return bf16_to_f32(f32_to_bf16(x));
    } else if constexpr (FMT == FB_UNORM16) {
        return (float)f32_to_unorm(x, 65535.0f) / 65535.0f;
    } else if constexpr (FMT == FB_UNORM8) {
        return (float)f32_to_unorm(x, 255.0f) / 255.0f;
    } else {
        return x;
    }
}

// Store one pixel's (R, G, B, T) to the framebuffer at pixel index `i`; returns the stored
// values decoded back to fp32 in v.
__device__ __forceinline__ void fb_store(void* fb, int fmt, size_t i, float4& v) {
    switch (fmt) {
    case FB_F16: {
        _Float16 h[4] = {(_Float16)v.x, (_Float16)v.y, (_Float16)v.z, (_Float16)v.w};
        uint2 w;
        __builtin_memcpy(&w, h, 8);
        reinterpret_cast<uint2*>(fb)[i] = w;
        v = make_float4((float)h[0], (float)h[1], (float)h[2], (float)h[3]);
        break;
    }
    case FB_BF16: {
        uint16_t h0 = f32_to_bf16(v.x), h1 = f32_to_bf16(v.y), h2 = f32_to_bf16(v.z),
                 h3 = f32_to_bf16(v.w);
        reinterpret_cast<uint2*>(fb)[i] = make_uint2(h0 | ((uint32_t)h1 << 16),
                                                     h2 | ((uint32_t)h3 << 16));
        v = make_float4(bf16_to_f32(h0), bf16_to_f32(h1), bf16_to_f32(h2), bf16_to_f32(h3));
        break;
    }
    case FB_UNORM16: {
        uint32_t u0 = f32_to_unorm(v.x, 65535.f), u1 = f32_to_unorm(v.y, 65535.f),
                 u2 = f32_to_unorm(v.z, 65535.f), u3 = f32_to_unorm(v.w, 65535.f);
        reinterpret_cast<uint2*>(fb)[i] = make_uint2(u0 | (u1 << 16), u2 | (u3 << 16));
        v = make_float4((float)u0 / 65535.f, (float)u1 / 65535.f, (float)u2 / 65535.f,
                        (float)u3 / 65535.f);
        break;
    }
    case FB_UNORM8: {
        uint32_t u0 = f32_to_unorm(v.x, 255.f), u1 = f32_to_unorm(v.y, 255.f),
                 u2 = f32_to_unorm(v.z, 255.f), u3 = f32_to_unorm(v.w, 255.f);
        reinterpret_cast<uint32_t*>(fb)[i] = u0 | (u1 << 8) | (u2 << 16) | (u3 << 24);
        v = make_float4((float)u0 / 255.f, (float)u1 / 255.f, (float)u2 / 255.f,
                        (float)u3 / 255.f);
        break;
    }
    default:
        reinterpret_cast<float4*>(fb)[i] = v;
        break;
    }
}

__device__ __forceinline__ float4 fb_load(const void* fb, int fmt, size_t i) {
    switch (fmt) {
    case FB_F16: {
        uint2 w = reinterpret_cast<const uint2*>(fb)[i];
        _Float16 h[4];
        __builtin_memcpy(h, &w, 8);
        return make_float4((float)h[0], (float)h[1], (float)h[2], (float)h[3]);
    }
    case FB_BF16: {
        uint2 w = reinterpret_cast<const uint2*>(fb)[i];
        return make_float4(bf16_to_f32((uint16_t)(w.x & 0xffff)), bf16_to_f32((uint16_t)(w.x >> 16)),
                           bf16_to_f32((uint16_t)(w.y & 0xffff)), bf16_to_f32((uint16_t)(w.y >> 16)));
    }
    case FB_UNORM16: {
        uint2 w = reinterpret_cast<const uint2*>(fb)[i];
        return make_float4((float)(w.x & 0xffff) / 65535.f, (float)(w.x >> 16) / 65535.f,
                           (float)(w.y & 0xffff) / 65535.f, (float)(w.y >> 16) / 65535.f);
    }
    case FB_UNORM8: {
        uint32_t w = reinterpret_cast<const uint32_t*>(fb)[i];
        return make_float4((float)(w & 0xff) / 255.f, (float)((w >> 8) & 0xff) / 255.f,
                           (float)((w >> 16) & 0xff) / 255.f, (float)(w >> 24) / 255.f);
    }
    default:
        return reinterpret_cast<const float4*>(fb)[i];
    }
}

__host__ __device__ inline int fb_bytes_per_pixel(int fmt) {
    return fmt == FB_F32 ? 16 : (fmt == FB_UNORM8 ? 4 : 8);
}

}  // namespace gsr
