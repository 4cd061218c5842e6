// Internal helpers shared by the libuvl translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "uvl.h"

namespace uvl {

constexpr int kBlock = 256;                 // threads per workgroup (4 waves of 64)
constexpr int32_t kMaxSide = 32768;         // atlas side limit (2^30 texels, int32-safe products)
constexpr int32_t kMaxDepthSide = 16384;    // depth map side limit
constexpr int32_t kEmptyOwner = 0x7fffffff; // tri_id value before ownership resolves

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Cached gfx950 check of the current device.
int32_t device_ok();

// Status after a batch of launches: UVL_E_DEVICE if the last launch failed.
inline int32_t launch_status() {
    return hipGetLastError() == hipSuccess ? UVL_OK : UVL_E_DEVICE;
}

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline bool dtype_ok(int32_t dt) { return dt == UVL_U8 || dt == UVL_U16; }

inline uint32_t dtype_max(int32_t dt) { return dt == UVL_U8 ? 0xffu : 0xffffu; }

// Bytes per texel of a layer dtype (any of the five).
inline int dtype_bytes(int32_t dt) { return dt == UVL_U8 ? 1 : (dt == UVL_U16 || dt == UVL_F16) ? 2 : 4; }

inline bool layer_ok(const uvl_layer *l) {
    return l && l->data && l->width >= 1 && l->height >= 1 && l->width <= kMaxSide &&
           l->height <= kMaxSide && aligned16(l->data);
}

inline bool numeric_ok(const uvl_numeric *l) {
    return l && l->data && l->mask && l->width >= 1 && l->height >= 1 && l->width <= kMaxSide &&
           l->height <= kMaxSide && aligned16(l->data) && aligned16(l->mask) && l->dtype >= UVL_U8 &&
           l->dtype <= UVL_F32;
}

// Mask words of a numeric layer.
inline int64_t mask_words(const uvl_numeric *l) { return ceil_div((int64_t)l->width * l->height, 32); }

// The stored bit pattern of `value` in dtype `dt` (numeric.hip): integral
// and in range for the integer dtypes, rounded to nearest even and finite
// for the float dtypes.  UVL_E_INVAL for NaN, UVL_E_DTYPE if it does not fit.
int32_t encode_value(int32_t dt, double value, uint32_t &bits);

// Validation shared by the numeric edits: geometry and layer, matching
// sizes, mode, value; fills bits.  Also checks the device.
int32_t check_numeric_edit(const uvl_geom *g, const uvl_numeric *l, int32_t mode, double value, uint32_t &bits);

// The position planes every edit reads.
inline bool geom_pos_ok(const uvl_geom *g) {
    return g && g->width >= 1 && g->height >= 1 && g->width <= kMaxSide && g->height <= kMaxSide &&
           g->pos_x && g->pos_y && g->pos_z && aligned16(g->pos_x) && aligned16(g->pos_y) &&
           aligned16(g->pos_z);
}

// 16-byte streaming load that bypasses cache residency (each position is read
// once per edit; the planes are far larger than the caches).
typedef float uvl_f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 load_stream4(const float *p) {
    const uvl_f4v v = __builtin_nontemporal_load(reinterpret_cast<const uvl_f4v *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

// Fills (device kernels in common.hip); safe inside graph capture.
void fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
void fill_bytes(void *p, int64_t nbytes, hipStream_t s);   // zero

}  // namespace uvl
