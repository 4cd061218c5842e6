// Per-label surface area for libuvl.
//
// Table 1 of the paper reports the surface area one texel stands for; the
// labelled area of a layer is the sum of those texel areas over the texels
// holding the label.  The geometry image stores each texel's area as a
// uint32 multiple of a power-of-two scale, so the sums are exact uint64
// integers: independent of summation order, deterministic run to run, and
// exactly additive (area(A or B) = area(A) + area(B) - area(A and B)).
//
// One pass reads each area weight once for up to kGroup layers.  The atlas is
// cut into bands of 4096 columns; a workgroup owns one band over a range of
// rows and walks it row by row; lane l takes columns [16 l, 16 l + 16) of the
// band in every row (4 x 16-byte weight loads, one 16-byte u8 or two u16
// label loads per layer when the width is a multiple of 16).  Every lane
// keeps, per layer, its current label and the uint64 weight sum of its run of
// that label, carried down the rows: labelled regions are spatially coherent,
// so a run usually spans many rows and is added to a bin only when the lane's
// label changes.  u8 layers add into 256 LDS bins (native LDS atomics);
// u16 layers (65536 bins) add into an LDS hash table keyed by (layer,
// label), open addressing with linear probing, falling back to the global
// bin only if 16 probes find no slot.  Both are flushed to the global bins
// once per workgroup, so global atomics stay few and spread out.
#include "uvl_internal.h"

namespace uvl {
namespace {

constexpr int kPer = 16;
constexpr int kGroup = 8;                 // layers per launch
constexpr int kTexPerIter = kBlock * kPer;
constexpr int kHashBits = 11;
constexpr int kHash = 1 << kHashBits;     // LDS hash slots for u16 labels
constexpr uint32_t kEmptyKey = 0xffffffffu;

struct U16Table {
    uint32_t *key;                 // LDS [kHash]
    unsigned long long *val;       // LDS [kHash]
    unsigned long long *const *bins;   // global bins per layer (fallback)
};

// Add `sum` to label `label` of group layer `l` in the LDS hash table.
__device__ __forceinline__ void table_add(const U16Table &T, int l, uint32_t label, unsigned long long sum) {
    const uint32_t key = ((uint32_t)l << 16) | label;
    uint32_t h = (key * 2654435761u) >> (32 - kHashBits);
    for (int probe = 0; probe < 16; ++probe) {
        const uint32_t prev = atomicCAS(T.key + h, kEmptyKey, key);
        if (prev == kEmptyKey || prev == key) {
            atomicAdd(T.val + h, sum);
            return;
        }
        h = (h + 1) & (kHash - 1);
    }
    atomicAdd(T.bins[l] + label, sum);
}

// Bin sinks: direct LDS bins for u8 layers, the hash table for u16 layers.
struct SinkU8 {
    unsigned long long *bins;
    __device__ __forceinline__ void add(uint32_t label, unsigned long long s) const { atomicAdd(bins + label, s); }
};
struct SinkU16 {
    const U16Table *T;
    int l;
    __device__ __forceinline__ void add(uint32_t label, unsigned long long s) const { table_add(*T, l, label, s); }
};

struct AreaArgs {
    const void *data[kGroup];
    unsigned long long *bins[kGroup];
    int32_t dtype[kGroup];
    int32_t row[kGroup];      // u8 layers: their LDS bin row (rank among the group's u8 layers)
    int32_t nl;
};

__device__ __forceinline__ void label16_u8(const uint8_t *p, uint32_t v[kPer]) {
    const uint4 q = *reinterpret_cast<const uint4 *>(p);
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < kPer; ++k) v[k] = (w[k >> 2] >> (8 * (k & 3))) & 0xffu;
}

__device__ __forceinline__ void label16_u16(const uint16_t *p, uint32_t v[kPer]) {
    const uint4 q0 = reinterpret_cast<const uint4 *>(p)[0];
    const uint4 q1 = reinterpret_cast<const uint4 *>(p)[1];
    const uint32_t w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
    for (int k = 0; k < kPer; ++k) v[k] = (w[k >> 1] >> (16 * (k & 1))) & 0xffffu;
}

// Feed 16 (label, weight) pairs into a lane's run; a finished run goes to
// the sink.
template <typename Sink>
__device__ __forceinline__ void feed(const uint32_t lab[kPer], const uint32_t w[kPer], unsigned long long tot,
                                     uint32_t &cur, unsigned long long &run, const Sink &bins) {
    bool uni = true;
#pragma unroll
    for (int k = 1; k < kPer; ++k) uni = uni && lab[k] == lab[0];
    if (uni) {
        if (lab[0] != cur) {
            if (run) bins.add(cur, run);
            cur = lab[0];
            run = 0;
        }
        run += tot;
    } else {
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if (lab[k] != cur) {
                if (run) bins.add(cur, run);
                cur = lab[k];
                run = 0;
            }
            run += w[k];
        }
    }
}

// kU8 / kU16: the launch's group has u8 / u16 layers; LDS holds only the
// tables the group needs (u8 bins 2 KiB per layer, the u16 hash 24 KiB), so a
// one-layer query keeps many workgroups per CU.
template <int kNU8, bool kU16>
__global__ __launch_bounds__(kBlock) void k_area(const uint32_t *__restrict__ area_w, int W, int H, int rows_per,
                                                  AreaArgs A) {
    __shared__ unsigned long long s_bins[kNU8 > 0 ? kNU8 : 1][256];
    __shared__ uint32_t s_key[kU16 ? kHash : 1];
    __shared__ unsigned long long s_val[kU16 ? kHash : 1];
    if (kNU8 > 0)
        for (int k = threadIdx.x; k < kNU8 * 256; k += kBlock) (&s_bins[0][0])[k] = 0ull;
    if (kU16)
        for (int k = threadIdx.x; k < kHash; k += kBlock) {
            s_key[k] = kEmptyKey;
            s_val[k] = 0ull;
        }
    __syncthreads();
    const U16Table table{s_key, s_val, A.bins};
    uint32_t cur[kGroup];
    unsigned long long run[kGroup];
#pragma unroll
    for (int l = 0; l < kGroup; ++l) {
        cur[l] = 0;
        run[l] = 0;
    }
    const int col = (int)blockIdx.x * kTexPerIter + (int)threadIdx.x * kPer;   // first column of the lane
    const int ncol = W - col < kPer ? (W - col > 0 ? W - col : 0) : kPer;       // columns it owns
    const bool vec = (W % kPer) == 0 && ncol == kPer;                          // aligned 16-wide loads
    const int r0 = (int)blockIdx.y * rows_per;
    const int r1 = r0 + rows_per < H ? r0 + rows_per : H;
    for (int r = r0; r < r1; ++r) {
        const int64_t t0 = (int64_t)r * W + col;
        uint32_t w[kPer];
        if (vec) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint4 v = reinterpret_cast<const uint4 *>(area_w + t0)[q];
                w[4 * q] = v.x; w[4 * q + 1] = v.y; w[4 * q + 2] = v.z; w[4 * q + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < kPer; ++k) w[k] = k < ncol ? area_w[t0 + k] : 0u;
        }
        unsigned long long tot = 0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) tot += w[k];
#pragma unroll
        for (int l = 0; l < kGroup; ++l) {
            if (l >= A.nl) break;
            uint32_t lab[kPer];
            if (kNU8 > 0 && (!kU16 || A.dtype[l] == UVL_U8)) {
                const uint8_t *L = static_cast<const uint8_t *>(A.data[l]);
                if (vec) {
                    label16_u8(L + t0, lab);
                } else {
#pragma unroll
                    for (int k = 0; k < kPer; ++k) lab[k] = k < ncol ? L[t0 + k] : cur[l];
                }
                feed(lab, w, tot, cur[l], run[l], SinkU8{&s_bins[A.row[l]][0]});
            } else if (kU16) {
                const uint16_t *L = static_cast<const uint16_t *>(A.data[l]);
                if (vec) {
                    label16_u16(L + t0, lab);
                } else {
#pragma unroll
                    for (int k = 0; k < kPer; ++k) lab[k] = k < ncol ? L[t0 + k] : cur[l];
                }
                feed(lab, w, tot, cur[l], run[l], SinkU16{&table, l});
            }
        }
    }
#pragma unroll
    for (int l = 0; l < kGroup; ++l) {
        if (l >= A.nl) break;
        if (run[l]) {
            if (kNU8 > 0 && (!kU16 || A.dtype[l] == UVL_U8)) atomicAdd(&s_bins[A.row[l]][cur[l]], run[l]);
            else if (kU16) table_add(table, l, cur[l], run[l]);
        }
    }
    __syncthreads();
    if (kNU8 > 0)
        for (int l = 0; l < A.nl; ++l) {
            if (A.dtype[l] != UVL_U8) continue;
            const unsigned long long v = s_bins[A.row[l]][threadIdx.x];
            if (v) atomicAdd(A.bins[l] + threadIdx.x, v);
        }
    if (kU16)
        for (int k = threadIdx.x; k < kHash; k += kBlock) {
            const uint32_t key = s_key[k];
            if (key != kEmptyKey && s_val[k]) atomicAdd(A.bins[key >> 16] + (key & 0xffffu), s_val[k]);
        }
}

// Launch one group with the kernel instance sized to its u8 layer count and
// whether it has u16 layers.
template <int kNU8>
void launch_area(dim3 grid, hipStream_t s, const uint32_t *area_w, int W, int H, int rows_per, const AreaArgs &A,
                 bool u16) {
    if (u16)
        hipLaunchKernelGGL((k_area<kNU8, true>), grid, dim3(kBlock), 0, s, area_w, W, H, rows_per, A);
    else
        hipLaunchKernelGGL((k_area<kNU8, false>), grid, dim3(kBlock), 0, s, area_w, W, H, rows_per, A);
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
    fill_bytes(bins_dev, nbins * 8, s);
    // grid: column bands x row groups, about 1024 workgroups in all
    const int bands = (int)ceil_div(geom->width, kTexPerIter);
    int groups = (int)ceil_div(1024, bands);
    if (groups > geom->height) groups = geom->height;
    const int rows_per = (int)ceil_div(geom->height, groups);
    groups = (int)ceil_div(geom->height, rows_per);
    int64_t off = 0;
    for (int l0 = 0; l0 < nlayers; l0 += kGroup) {
        AreaArgs A{};
        A.nl = nlayers - l0 < kGroup ? nlayers - l0 : kGroup;
        int nu8 = 0;
        bool u16 = false;
        for (int k = 0; k < A.nl; ++k) {
            const uvl_layer &L = layers[l0 + k];
            A.data[k] = L.data;
            A.dtype[k] = L.dtype;
            A.bins[k] = reinterpret_cast<unsigned long long *>(bins_dev) + off;
            off += L.dtype == UVL_U8 ? 256 : 65536;
            if (L.dtype == UVL_U8) A.row[k] = nu8++;
            else u16 = true;
        }
        const dim3 grid((unsigned)bands, (unsigned)groups);
        const uint32_t *aw = geom->area_w;
        const int W = geom->width, H = geom->height;
        switch (nu8) {
            case 0: launch_area<0>(grid, s, aw, W, H, rows_per, A, u16); break;
            case 1: launch_area<1>(grid, s, aw, W, H, rows_per, A, u16); break;
            case 2: launch_area<2>(grid, s, aw, W, H, rows_per, A, u16); break;
            case 3:
            case 4: launch_area<4>(grid, s, aw, W, H, rows_per, A, u16); break;
            default: launch_area<kGroup>(grid, s, aw, W, H, rows_per, A, u16); break;
        }
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
