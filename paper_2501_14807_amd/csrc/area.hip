// Per-label surface area for libuvl.
//
// Table 1 of the paper reports the surface area one texel stands for; the
// labelled area of a layer is the sum of those texel areas over the texels
// holding the label.  The geometry image stores each texel's area as a
// uint32 multiple of a power-of-two scale, so the sums are exact uint64
// integers: independent of summation order, deterministic run to run, and
// exactly additive (area(A or B) = area(A) + area(B) - area(A and B)).
//
// One pass reads each area weight once for up to kGroup layers.  A thread
// takes 16 consecutive texels (4 x 16-byte weight loads, one 16-byte u8 label
// load); a run of equal labels collapses to one (label, sum) pair; pairs of a
// wave with the same label are summed across lanes before one atomic add.
// u8 layers accumulate in LDS bins (256 x u64 per layer) flushed once per
// workgroup; u16 layers (65536 bins) add straight into the global bins.
#include "uvl_internal.h"

namespace uvl {
namespace {

constexpr int kPer = 16;
constexpr int kGroup = 8;                 // layers per launch
constexpr int kTexPerIter = kBlock * kPer;

struct AreaArgs {
    const void *data[kGroup];
    unsigned long long *bins[kGroup];
    int32_t dtype[kGroup];
    int32_t nl;
};

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Add each pending lane's (label, sum) into bins; lanes with equal labels are
// combined first.  Must be reached by the whole wave.
__device__ __forceinline__ void flush(bool pending, uint32_t label, unsigned long long sum,
                                      unsigned long long *bins) {
    unsigned long long todo = __ballot(pending);
    const int lane = threadIdx.x & 63;
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const uint32_t l0 = __shfl(label, leader);
        const bool mine = pending && label == l0;
        const unsigned long long m = __ballot(mine);
        const unsigned long long s = wave_sum(mine ? sum : 0ull);
        if (lane == leader) atomicAdd(bins + l0, s);
        pending = pending && !mine;
        todo &= ~m;
    }
}

template <typename T>
__device__ __forceinline__ void load_labels(const T *p, uint32_t v[kPer]);

template <>
__device__ __forceinline__ void load_labels<uint8_t>(const uint8_t *p, uint32_t v[kPer]) {
    const uint4 q = *reinterpret_cast<const uint4 *>(p);
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < kPer; ++k) v[k] = (w[k >> 2] >> (8 * (k & 3))) & 0xffu;
}

template <>
__device__ __forceinline__ void load_labels<uint16_t>(const uint16_t *p, uint32_t v[kPer]) {
    const uint4 q0 = reinterpret_cast<const uint4 *>(p)[0];
    const uint4 q1 = reinterpret_cast<const uint4 *>(p)[1];
    const uint32_t w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
    for (int k = 0; k < kPer; ++k) v[k] = (w[k >> 1] >> (16 * (k & 1))) & 0xffffu;
}

// Run-length accumulation of 16 (label, weight) pairs of every lane.
__device__ __forceinline__ void accumulate(const uint32_t lab[kPer], const uint32_t w[kPer], bool valid,
                                           unsigned long long *bins) {
    bool uniform = valid;
#pragma unroll
    for (int k = 1; k < kPer; ++k) uniform = uniform && lab[k] == lab[0];
    unsigned long long total = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) total += w[k];
    // fast path: all 16 labels equal
    flush(uniform, lab[0], total, bins);
    if (__ballot(valid && !uniform) == 0) return;
    bool slow = valid && !uniform;
    uint32_t cur = lab[0];
    unsigned long long run = w[0];
#pragma unroll
    for (int k = 1; k < kPer; ++k) {
        const bool ends = slow && lab[k] != cur;
        flush(ends, cur, run, bins);
        if (slow) {
            run = ends ? (unsigned long long)w[k] : run + w[k];
            cur = lab[k];
        }
    }
    flush(slow, cur, run, bins);
}

__global__ __launch_bounds__(kBlock) void k_area(const uint32_t *__restrict__ area_w, int64_t n, AreaArgs A) {
    __shared__ unsigned long long s_bins[kGroup][256];
    for (int k = threadIdx.x; k < kGroup * 256; k += kBlock) (&s_bins[0][0])[k] = 0ull;
    __syncthreads();
    const int64_t iters = ceil_div(n, kTexPerIter);
    for (int64_t it = blockIdx.x; it < iters; it += gridDim.x) {
        const int64_t t0 = it * kTexPerIter + (int64_t)threadIdx.x * kPer;
        const bool full = t0 + kPer <= n;
        uint32_t w[kPer];
        if (full) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint4 v = reinterpret_cast<const uint4 *>(area_w + t0)[q];
                w[4 * q] = v.x; w[4 * q + 1] = v.y; w[4 * q + 2] = v.z; w[4 * q + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < kPer; ++k) w[k] = t0 + k < n ? area_w[t0 + k] : 0u;
        }
        for (int l = 0; l < A.nl; ++l) {
            uint32_t lab[kPer];
            const bool u8 = A.dtype[l] == UVL_U8;
            if (full) {
                if (u8) load_labels<uint8_t>(static_cast<const uint8_t *>(A.data[l]) + t0, lab);
                else load_labels<uint16_t>(static_cast<const uint16_t *>(A.data[l]) + t0, lab);
            } else {
#pragma unroll
                for (int k = 0; k < kPer; ++k) {
                    if (t0 + k < n)
                        lab[k] = u8 ? static_cast<const uint8_t *>(A.data[l])[t0 + k]
                                    : static_cast<const uint16_t *>(A.data[l])[t0 + k];
                    else
                        lab[k] = k > 0 ? lab[k - 1] : 0u;   // padding carries weight 0
                }
            }
            accumulate(lab, w, t0 < n, u8 ? s_bins[l] : A.bins[l]);
        }
    }
    __syncthreads();
    for (int l = 0; l < A.nl; ++l) {
        if (A.dtype[l] != UVL_U8) continue;
        const unsigned long long v = s_bins[l][threadIdx.x];
        if (v) atomicAdd(A.bins[l] + threadIdx.x, v);
    }
}

}  // namespace
}  // namespace uvl

using namespace uvl;

extern "C" int32_t uvl_area_query(const uvl_geom *geom, const uvl_layer *layers, int32_t nlayers,
                                  uint64_t *bins_dev, double *areas_host, void *stream) {
    if (!geom || !layers || !bins_dev || nlayers < 1 || nlayers > 32) return UVL_E_INVAL;
    if (!geom->area_w || !aligned16(geom->area_w) || geom->width < 1 || geom->height < 1) return UVL_E_INVAL;
    int64_t nbins = 0;
    for (int l = 0; l < nlayers; ++l) {
        if (!layer_ok(&layers[l])) return UVL_E_INVAL;
        if (!dtype_ok(layers[l].dtype)) return UVL_E_DTYPE;
        if (layers[l].width != geom->width || layers[l].height != geom->height) return UVL_E_SHAPE;
        nbins += layers[l].dtype == UVL_U8 ? 256 : 65536;
    }
    if (int32_t s = device_ok()) return s;
    hipStream_t s = as_stream(stream);
    const int64_t n = (int64_t)geom->width * geom->height;
    fill_bytes(bins_dev, nbins * 8, s);
    const int64_t iters = ceil_div(n, kTexPerIter);
    const unsigned grid = (unsigned)(iters < 2048 ? iters : 2048);
    int64_t off = 0;
    for (int l0 = 0; l0 < nlayers; l0 += kGroup) {
        AreaArgs A{};
        A.nl = nlayers - l0 < kGroup ? nlayers - l0 : kGroup;
        for (int k = 0; k < A.nl; ++k) {
            const uvl_layer &L = layers[l0 + k];
            A.data[k] = L.data;
            A.dtype[k] = L.dtype;
            A.bins[k] = reinterpret_cast<unsigned long long *>(bins_dev) + off;
            off += L.dtype == UVL_U8 ? 256 : 65536;
        }
        hipLaunchKernelGGL(k_area, dim3(grid), dim3(kBlock), 0, s, geom->area_w, n, A);
    }
    if (launch_status() != UVL_OK) return UVL_E_DEVICE;
    if (!areas_host) return UVL_OK;
    // bins -> fp64 on the host (synchronous form)
    uint64_t *tmp = static_cast<uint64_t *>(malloc((size_t)nbins * 8));
    if (!tmp) return UVL_E_NOMEM;
    hipError_t e = hipMemcpyAsync(tmp, bins_dev, (size_t)nbins * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        for (int64_t b = 0; b < nbins; ++b) areas_host[b] = (double)tmp[b] * geom->area_scale;
    free(tmp);
    return e == hipSuccess ? UVL_OK : UVL_E_DEVICE;
}
