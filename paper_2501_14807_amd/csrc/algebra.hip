// Layer algebra for libuvl (§3.4.2: layer systems combine layers with logic
// operations; §4.2: database layers store unsigned keys, 0 = no data).
//
// One streaming pass, 16 texels per thread: 16-byte vector loads of each u8
// operand (two for u16), the predicate combination in registers, one vector
// store.  dst may alias a or b: every thread reads its texels before it
// writes them and no two threads share a texel.
//
// REMAP tables come from the host and are checked there (entry 0 maps the
// null key to itself, every entry fits dst) before anything is enqueued.  A
// 256-entry table (u8 operand) travels in the kernel arguments and is staged
// in LDS.  A 65536-entry table (u16 operand) is copied into a pinned host
// slot and from there, on the caller's stream, into a slot of a static
// device ring the kernel gathers from (128 KiB, resident in L2); an event
// after the kernel frees the slot, and a call that finds its slot still in
// use waits for that event.
#include <string.h>

#include <mutex>

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

struct Lut256 {
    uint16_t v[256];
};

template <typename Td, typename Ta>
__device__ __forceinline__ void remap_body(Td *dst, const Ta *a, int64_t n, const uint16_t *tab) {
    const int64_t t0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kPer;
    if (t0 + kPer <= n) {
        uint32_t va[kPer], vd[kPer];
        load16<Ta>(a + t0, va);
#pragma unroll
        for (int k = 0; k < kPer; ++k) vd[k] = tab[va[k]];
        store16<Td>(dst + t0, vd);
    } else {
        for (int64_t t = t0; t < n; ++t) dst[t] = (Td)tab[a[t]];
    }
}

// u8 operand: the table arrives by value and is staged in LDS.
template <typename Td>
__global__ __launch_bounds__(kBlock) void k_remap8(Td *dst, const uint8_t *a, int64_t n, Lut256 lut) {
    __shared__ uint16_t s_lut[256];
    s_lut[threadIdx.x] = lut.v[threadIdx.x];
    __syncthreads();
    remap_body<Td, uint8_t>(dst, a, n, s_lut);
}

// u16 operand: gathers from the table in device memory.
template <typename Td>
__global__ __launch_bounds__(kBlock) void k_remap16(Td *dst, const uint16_t *a, int64_t n,
                                                    const uint16_t *__restrict__ lut) {
    remap_body<Td, uint16_t>(dst, a, n, lut);
}

// Ring of 65536-entry tables: the device side is a static array (no
// allocation), addressed through hipGetSymbolAddress on each device.
constexpr int kRemapSlots = 16;
constexpr size_t kRemapEntries = 65536;
__device__ __align__(256) uint16_t g_remap_ring[kRemapSlots * kRemapEntries];

struct RemapRing {
    bool ready = false;
    uint16_t *dev = nullptr;        // device address of g_remap_ring on this device
    uint16_t *host = nullptr;       // pinned staging, kRemapSlots tables
    hipEvent_t ev[kRemapSlots] = {};
    bool pending[kRemapSlots] = {};
    int next = 0;
};

std::mutex g_ring_mu;
RemapRing g_ring[64];

// The ring of the current device, set up on first use (called locked).
int32_t ring_for_device(RemapRing *&out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return UVL_E_DEVICE;
    RemapRing &r = g_ring[dev];
    if (!r.ready) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_remap_ring)) != hipSuccess || !p) return UVL_E_DEVICE;
        void *h = nullptr;
        if (hipHostMalloc(&h, kRemapSlots * kRemapEntries * sizeof(uint16_t), hipHostMallocDefault) != hipSuccess)
            return UVL_E_DEVICE;
        for (int k = 0; k < kRemapSlots; ++k) {
            if (hipEventCreateWithFlags(&r.ev[k], hipEventDisableTiming) != hipSuccess) {
                for (int q = 0; q < k; ++q) (void)hipEventDestroy(r.ev[q]);
                (void)hipHostFree(h);
                return UVL_E_DEVICE;
            }
        }
        r.dev = static_cast<uint16_t *>(p);
        r.host = static_cast<uint16_t *>(h);
        r.ready = true;
    }
    out = &r;
    return UVL_OK;
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

// Table check: the null key maps to itself and every entry fits dst.
int32_t check_lut(const uint16_t *lut, size_t n, uint32_t dst_max) {
    if (lut[0] != 0) return UVL_E_INVAL;
    uint32_t mx = 0;
    for (size_t k = 0; k < n; ++k) mx = lut[k] > mx ? lut[k] : mx;
    return mx > dst_max ? UVL_E_DTYPE : UVL_OK;
}

int32_t launch_remap(const uvl_layer *dst, const uvl_layer *a, const uint16_t *lut, hipStream_t s) {
    const int64_t n = (int64_t)dst->width * dst->height;
    const dim3 grid((unsigned)ceil_div(n, (int64_t)kBlock * kPer)), block(kBlock);
    const bool d8 = dst->dtype == UVL_U8;
    if (a->dtype == UVL_U8) {
        Lut256 L;
        memcpy(L.v, lut, sizeof(L.v));
        const uint8_t *A = static_cast<const uint8_t *>(a->data);
        if (d8) hipLaunchKernelGGL(k_remap8<uint8_t>, grid, block, 0, s, static_cast<uint8_t *>(dst->data), A, n, L);
        else hipLaunchKernelGGL(k_remap8<uint16_t>, grid, block, 0, s, static_cast<uint16_t *>(dst->data), A, n, L);
        return launch_status();
    }
    std::lock_guard<std::mutex> lock(g_ring_mu);
    RemapRing *r = nullptr;
    if (int32_t st = ring_for_device(r)) return st;
    const int k = r->next;
    if (r->pending[k]) {
        if (hipEventSynchronize(r->ev[k]) != hipSuccess) return UVL_E_DEVICE;
        r->pending[k] = false;
    }
    uint16_t *h = r->host + (size_t)k * kRemapEntries, *d = r->dev + (size_t)k * kRemapEntries;
    memcpy(h, lut, kRemapEntries * sizeof(uint16_t));
    if (hipMemcpyAsync(d, h, kRemapEntries * sizeof(uint16_t), hipMemcpyHostToDevice, s) != hipSuccess)
        return UVL_E_DEVICE;
    const uint16_t *A = static_cast<const uint16_t *>(a->data);
    if (d8) hipLaunchKernelGGL(k_remap16<uint8_t>, grid, block, 0, s, static_cast<uint8_t *>(dst->data), A, n, d);
    else hipLaunchKernelGGL(k_remap16<uint16_t>, grid, block, 0, s, static_cast<uint16_t *>(dst->data), A, n, d);
    if (launch_status() != UVL_OK) return UVL_E_DEVICE;
    if (hipEventRecord(r->ev[k], s) != hipSuccess) return UVL_E_DEVICE;
    r->pending[k] = true;
    r->next = (k + 1) % kRemapSlots;
    return UVL_OK;
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
        if (int32_t st = check_lut(lut, a8 ? 256 : kRemapEntries, dtype_max(dst->dtype))) return st;
        if (int32_t st = device_ok()) return st;
        return launch_remap(dst, a, lut, s);
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
