// Helpers shared by the multi-level kernels (lbm_march.hip, lbm_march_adj.hip): lane
// shifts across a wavefront, stores through buffer resources that span one row of an
// array, and the column offsets of the tiled layout.
#pragma once

#include "lbm_device.hpp"
#include "lbm_internal.hpp"

namespace lbm {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int pop_col(int x) { return (x >> 6) * (24 * kTile) + (x & (kTile - 1)); }

// The value of lane l - 1 (from_prev) or l + 1 (from_next) across the whole wavefront, by a
// DPP wave shift (one vector move instead of a permute through the LDS unit); lane 0, resp.
// 63, receives 0, a value the multi-level kernels never use.
__device__ __forceinline__ float from_prev(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_next(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double from_prev(double v) {
    const u32x2 h = __builtin_bit_cast(u32x2, v);
    const u32x2 r = {uint32_t(__builtin_amdgcn_update_dpp(0, int(h.x), 0x138, 0xf, 0xf, true)),
                       uint32_t(__builtin_amdgcn_update_dpp(0, int(h.y), 0x138, 0xf, 0xf, true))};
    return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ double from_next(double v) {
    const u32x2 h = __builtin_bit_cast(u32x2, v);
    const u32x2 r = {uint32_t(__builtin_amdgcn_update_dpp(0, int(h.x), 0x130, 0xf, 0xf, true)),
                       uint32_t(__builtin_amdgcn_update_dpp(0, int(h.y), 0x130, 0xf, 0xf, true))};
    return __builtin_bit_cast(double, r);
}

// Stores through a buffer resource that spans one row of an array: a lane whose byte offset
// is kNoStore (beyond any row) stores nothing, which the hardware's range check of raw
// buffers guarantees.  The multi-level kernels issue every store of an iteration this way,
// on every lane and in every iteration, so that all their iterations issue the same
// sequence of memory operations (see march_kernel).
constexpr uint32_t kNoStore = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* base, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, int(bytes), 0x00020000);
}

constexpr int kStoreNT = 2;     // cache policy: non-temporal, as store_stream

__device__ __forceinline__ void row_store(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, kStoreNT);
}
__device__ __forceinline__ void row_store(__amdgpu_buffer_rsrc_t r, uint32_t off, _Float16 v) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, off, 0, kStoreNT);
}
__device__ __forceinline__ void row_store(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, kStoreNT);
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void row_store16(__amdgpu_buffer_rsrc_t r, uint32_t off, u32x4 v) {
    __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, kStoreNT);
}
__device__ __forceinline__ void row_store8(__amdgpu_buffer_rsrc_t r, uint32_t off, u32x2 v) {
    __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, kStoreNT);
}

}  // namespace lbm
