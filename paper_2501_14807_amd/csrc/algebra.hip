// Layer algebra for libuvl (§3.4.2: layer systems combine layers with logic
// operations; §4.2: database layers store unsigned keys, 0 = no data).
//
// One streaming pass, 16 texels per thread: 16-byte vector loads of each u8
// operand (two for u16), the predicate combination in registers, one vector
// store.  dst may alias a or b: every thread reads its texels before it
// writes them and no two threads share a texel.  REMAP with a u8 operand
// stages the 256-entry table in LDS; a u16 operand gathers from the 128 KiB
// table, which stays resident in L2.
#include "uvl_internal.h"

namespace uvl {
namespace {

constexpr int kPer = 16;

template <typename T>
__device__ __forceinline__ void load16(const T *p, uint32_t v[kPer]);

template <>
__device__ __forceinline__ void load16<uint8_t>(const uint8_t *p, uint32_t v[kPer]) {
    const uint4 q = *reinterpret_cast<const uint4 *>(p);
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < kPer; ++k) v[k] = (w[k >> 2] >> (8 * (k & 3))) & 0xffu;
}

template <>
__device__ __forceinline__ void load16<uint16_t>(const uint16_t *p, uint32_t v[kPer]) {
    const uint4 q0 = reinterpret_cast<const uint4 *>(p)[0];
    const uint4 q1 = reinterpret_cast<const uint4 *>(p)[1];
    const uint32_t w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
    for (int k = 0; k < kPer; ++k) v[k] = (w[k >> 1] >> (16 * (k & 1))) & 0xffffu;
}

template <typename T>
__device__ __forceinline__ void store16(T *p, const uint32_t v[kPer]);

template <>
__device__ __forceinline__ void store16<uint8_t>(uint8_t *p, const uint32_t v[kPer]) {
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        w[k] = (v[4 * k] & 0xffu) | ((v[4 * k + 1] & 0xffu) << 8) | ((v[4 * k + 2] & 0xffu) << 16) |
               ((v[4 * k + 3] & 0xffu) << 24);
    *reinterpret_cast<uint4 *>(p) = make_uint4(w[0], w[1], w[2], w[3]);
}

template <>
__device__ __forceinline__ void store16<uint16_t>(uint16_t *p, const uint32_t v[kPer]) {
    uint32_t w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = (v[2 * k] & 0xffffu) | ((v[2 * k + 1] & 0xffffu) << 16);
    reinterpret_cast<uint4 *>(p)[0] = make_uint4(w[0], w[1], w[2], w[3]);
    reinterpret_cast<uint4 *>(p)[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

__device__ __forceinline__ bool pred(uint32_t v, uint32_t sel) { return sel == 0 ? v != 0 : v == sel; }

template <int OP>
__device__ __forceinline__ uint32_t combine(uint32_t va, uint32_t vb, uint32_t sa, uint32_t sb, uint32_t out) {
    const bool pa = pred(va, sa), pb = pred(vb, sb);
    const bool p = OP == UVL_AND ? (pa && pb) : OP == UVL_OR ? (pa || pb) : (pa != pb);
    return p ? out : 0u;
}

template <typename Td, typename Ta, typename Tb, int OP>
__global__ __launch_bounds__(kBlock) void k_logic(Td *dst, const Ta *a, const Tb *b, int64_t n, uint32_t sa,
                                                  uint32_t sb, uint32_t out) {
    const int64_t t0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kPer;
    if (t0 + kPer <= n) {
        uint32_t va[kPer], vb[kPer], vd[kPer];
        load16<Ta>(a + t0, va);
        load16<Tb>(b + t0, vb);
#pragma unroll
        for (int k = 0; k < kPer; ++k) vd[k] = combine<OP>(va[k], vb[k], sa, sb, out);
        store16<Td>(dst + t0, vd);
    } else {
        for (int64_t t = t0; t < n; ++t) dst[t] = (Td)combine<OP>(a[t], b[t], sa, sb, out);
    }
}

template <typename Td, typename Ta>
__global__ __launch_bounds__(kBlock) void k_remap(Td *dst, const Ta *a, int64_t n, const uint16_t *__restrict__ lut) {
    __shared__ uint16_t s_lut[256];
    constexpr bool kSmall = sizeof(Ta) == 1;
    if (kSmall) {
        s_lut[threadIdx.x] = lut[threadIdx.x];
        __syncthreads();
    }
    auto map = [&](uint32_t v) -> uint32_t {
        const uint32_t r = kSmall ? s_lut[v & 0xffu] : lut[v];
        return v == 0 ? 0u : r;
    };
    const int64_t t0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kPer;
    if (t0 + kPer <= n) {
        uint32_t va[kPer], vd[kPer];
        load16<Ta>(a + t0, va);
#pragma unroll
        for (int k = 0; k < kPer; ++k) vd[k] = map(va[k]);
        store16<Td>(dst + t0, vd);
    } else {
        for (int64_t t = t0; t < n; ++t) dst[t] = (Td)map(a[t]);
    }
}

template <typename Td, typename Ta, typename Tb>
void launch_logic(int op, void *d, const void *a, const void *b, int64_t n, uint32_t sa, uint32_t sb, uint32_t out,
                  hipStream_t s) {
    const dim3 grid((unsigned)ceil_div(n, (int64_t)kBlock * kPer)), block(kBlock);
    Td *D = static_cast<Td *>(d);
    const Ta *A = static_cast<const Ta *>(a);
    const Tb *B = static_cast<const Tb *>(b);
    if (op == UVL_AND) hipLaunchKernelGGL((k_logic<Td, Ta, Tb, UVL_AND>), grid, block, 0, s, D, A, B, n, sa, sb, out);
    else if (op == UVL_OR) hipLaunchKernelGGL((k_logic<Td, Ta, Tb, UVL_OR>), grid, block, 0, s, D, A, B, n, sa, sb, out);
    else hipLaunchKernelGGL((k_logic<Td, Ta, Tb, UVL_XOR>), grid, block, 0, s, D, A, B, n, sa, sb, out);
}

template <typename Td, typename Ta>
void launch_remap(void *d, const void *a, int64_t n, const uint16_t *lut, hipStream_t s) {
    const dim3 grid((unsigned)ceil_div(n, (int64_t)kBlock * kPer)), block(kBlock);
    hipLaunchKernelGGL((k_remap<Td, Ta>), grid, block, 0, s, static_cast<Td *>(d), static_cast<const Ta *>(a), n, lut);
}

}  // namespace
}  // namespace uvl

using namespace uvl;

extern "C" int32_t uvl_layer_op(int32_t op, const uvl_layer *dst, const uvl_layer *a, const uvl_layer *b,
                                uint32_t sel_a, uint32_t sel_b, uint32_t out_label, const uint16_t *lut,
                                void *stream) {
    if (op < UVL_AND || op > UVL_REMAP) return UVL_E_INVAL;
    if (!layer_ok(dst) || !layer_ok(a)) return UVL_E_INVAL;
    if (!dtype_ok(dst->dtype) || !dtype_ok(a->dtype)) return UVL_E_DTYPE;
    if (dst->width != a->width || dst->height != a->height) return UVL_E_SHAPE;
    const int64_t n = (int64_t)dst->width * dst->height;
    hipStream_t s = as_stream(stream);
    const bool d8 = dst->dtype == UVL_U8, a8 = a->dtype == UVL_U8;
    if (op == UVL_REMAP) {
        if (!lut) return UVL_E_INVAL;
        if (int32_t st = device_ok()) return st;
        if (d8 && a8) launch_remap<uint8_t, uint8_t>(dst->data, a->data, n, lut, s);
        else if (d8) launch_remap<uint8_t, uint16_t>(dst->data, a->data, n, lut, s);
        else if (a8) launch_remap<uint16_t, uint8_t>(dst->data, a->data, n, lut, s);
        else launch_remap<uint16_t, uint16_t>(dst->data, a->data, n, lut, s);
        return launch_status();
    }
    if (!layer_ok(b)) return UVL_E_INVAL;
    if (!dtype_ok(b->dtype)) return UVL_E_DTYPE;
    if (b->width != a->width || b->height != a->height) return UVL_E_SHAPE;
    if (out_label > dtype_max(dst->dtype)) return UVL_E_DTYPE;
    if (int32_t st = device_ok()) return st;
    const bool b8 = b->dtype == UVL_U8;
    const void *A = a->data, *B = b->data;
    void *D = dst->data;
    if (d8) {
        if (a8 && b8) launch_logic<uint8_t, uint8_t, uint8_t>(op, D, A, B, n, sel_a, sel_b, out_label, s);
        else if (a8) launch_logic<uint8_t, uint8_t, uint16_t>(op, D, A, B, n, sel_a, sel_b, out_label, s);
        else if (b8) launch_logic<uint8_t, uint16_t, uint8_t>(op, D, A, B, n, sel_a, sel_b, out_label, s);
        else launch_logic<uint8_t, uint16_t, uint16_t>(op, D, A, B, n, sel_a, sel_b, out_label, s);
    } else {
        if (a8 && b8) launch_logic<uint16_t, uint8_t, uint8_t>(op, D, A, B, n, sel_a, sel_b, out_label, s);
        else if (a8) launch_logic<uint16_t, uint8_t, uint16_t>(op, D, A, B, n, sel_a, sel_b, out_label, s);
        else if (b8) launch_logic<uint16_t, uint16_t, uint8_t>(op, D, A, B, n, sel_a, sel_b, out_label, s);
        else launch_logic<uint16_t, uint16_t, uint16_t>(op, D, A, B, n, sel_a, sel_b, out_label, s);
    }
    return launch_status();
}
