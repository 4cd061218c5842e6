// Numeric layers for libuvl (§4.2): a data texture of integers or floats
// with a mask texture of validity bits, one bit per texel (texel t in bit
// t % 32 of word t / 32).
//
// The edits themselves are the brush, lasso and tool kernels with a value
// sink (sink.h).  This file holds the host-side value conversion and the two
// passes that read numeric data:
//  - range selection, a streaming pass that turns values in [lo, hi] into a
//    label of a label layer (quantitative to qualitative data);
//  - zonal statistics, one streaming pass over tri_id, area_w, the data, the
//    mask and an optional label layer that groups the texels.  Table 1 gives
//    the surface area one texel stands for, so each group reports its count,
//    exact area (uint64 sum of area_w), area-weighted value sum, minimum and
//    maximum.
//
// Statistics walk the atlas in wave steps of 1024 consecutive texels, each
// lane taking 4 groups of 4 (the non-temporal load of a plane for one group is
// contiguous across the wave, as in the edit kernels; a group's mask bits sit
// in one word).  Range selection gives each lane 16 consecutive texels, so
// that its label writes are whole 16-byte vectors.  Statistics
// accumulate runs: a lane keeps the running totals of its current group and
// adds them to the group's bins only when the group changes, since labelled
// regions are spatially coherent.  A workgroup's bins live in LDS (native
// 64-bit LDS atomics): 256 direct bins for u8 groups, a tagged hash table for
// u16 groups; they are added to the global bins once per workgroup.  Minima
// and maxima are 64-bit atomics on an order-preserving encoding of the fp64
// value.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <type_traits>

#include "sink.h"
#include "uvl_internal.h"

namespace uvl {

// ---------------------------------------------------------------------------
// Value conversion.

namespace {

// IEEE binary16 of a double, rounded to nearest with ties to even, from the
// formats' bit layouts (binary64: 11-bit exponent, bias 1023, 52 fraction
// bits; binary16: 5-bit exponent, bias 15, 10 fraction bits, subnormals of
// spacing 2^-24 below 2^-14).  Returns false if the result is infinite.
// Used on the host (value encoding) and on the device (binary16 sums).
__host__ __device__ __forceinline__ bool f16_from_double(double v, uint16_t &out) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint16_t sign = (uint16_t)((b >> 48) & 0x8000u);
    const int ef = (int)((b >> 52) & 0x7ff);
    if (ef == 0x7ff) return false;
    if (ef == 0) {                      // zero or |v| < 2^-1022: rounds to zero
        out = sign;
        return true;
    }
    const int e = ef - 1023;
    const uint64_t m = (b & ((1ull << 52) - 1)) | (1ull << 52);   // v = m 2^(e-52)
    int he = e < -14 ? -14 : e;         // binade of the result (subnormals share 2^-14)
    const int shift = 42 + (he - e);    // bits of m below the result's last fraction bit
    uint64_t q = 0;
    if (shift < 64) {
        q = m >> shift;
        const uint64_t rem = m & ((1ull << shift) - 1), half = 1ull << (shift - 1);
        if (rem > half || (rem == half && (q & 1))) ++q;
    }
    if (q == 2048) {                    // rounding carried into the next binade
        q = 1024;
        ++he;
    }
    if (he > 15) return false;
    if (q < 1024) {                     // subnormal, he == -14
        out = sign | (uint16_t)q;
        return true;
    }
    out = sign | (uint16_t)((he + 15) << 10) | (uint16_t)(q - 1024);
    return true;
}

}  // namespace

int32_t encode_value(int32_t dt, double value, uint32_t &bits) {
    if (std::isnan(value)) return UVL_E_INVAL;
    switch (dt) {
    case UVL_U8:
    case UVL_U16:
    case UVL_I32: {
        const double lo = dt == UVL_I32 ? -2147483648.0 : 0.0;
        const double hi = dt == UVL_U8 ? 255.0 : dt == UVL_U16 ? 65535.0 : 2147483647.0;
        if (value != floor(value) || value < lo || value > hi) return UVL_E_DTYPE;
        bits = dt == UVL_I32 ? (uint32_t)(int32_t)value : (uint32_t)value;
        return UVL_OK;
    }
    case UVL_F16: {
        uint16_t h;
        if (!f16_from_double(value, h)) return UVL_E_DTYPE;
        bits = h;
        return UVL_OK;
    }
    case UVL_F32: {
        const float f = (float)value;   // round to nearest even
        if (!std::isfinite(f)) return UVL_E_DTYPE;
        memcpy(&bits, &f, sizeof bits);
        return UVL_OK;
    }
    default:
        return UVL_E_DTYPE;
    }
}

int32_t check_numeric_edit(const uvl_geom *g, const uvl_numeric *l, int32_t mode, double value, uint32_t &bits) {
    if (!geom_pos_ok(g) || !numeric_ok(l)) return UVL_E_INVAL;
    if (mode != UVL_SET && mode != UVL_ERASE) return UVL_E_INVAL;
    if (l->width != g->width || l->height != g->height) return UVL_E_SHAPE;
    bits = 0;
    if (mode == UVL_SET)
        if (int32_t s = encode_value(l->dtype, value, bits)) return s;
    return device_ok();
}

// ---------------------------------------------------------------------------
// Device side.

namespace {

constexpr int kPer = 16;                     // texels per lane per step
constexpr int kWaveStep = 64 * kPer;         // texels per wave per step
constexpr int kWaves = kBlock / 64;          // waves per workgroup
// Statistics workgroups: 2 per CU.  Each adds its LDS bins to the global
// bins once; with more workgroups those same-address atomics cost more than
// the extra waves gain (2048 workgroups: +40 us at 8192^2).
constexpr int kMaxStatBlocks = 512;

// Value of stored bits in fp64 (exact for every dtype).
template <int32_t DT>
__device__ __forceinline__ double decode(uint32_t b) {
    if constexpr (DT == UVL_I32) return (double)(int32_t)b;
    else if constexpr (DT == UVL_F32) return (double)__uint_as_float(b);
    else if constexpr (DT == UVL_F16) return (double)(float)__builtin_bit_cast(_Float16, (uint16_t)b);
    else return (double)b;
}

template <int32_t DT>
using Store = typename std::conditional<DT == UVL_U8, uint8_t,
              typename std::conditional<DT == UVL_U16 || DT == UVL_F16, uint16_t, uint32_t>::type>::type;

// Lane layout of a wave step over texels [s, s + kWaveStep): slot 4 q + j
// (q, j < 4) of lane l is texel s + 256 q + 4 l + j, so that each of the four
// loads of a plane reads one contiguous block per wave (1 KiB of a 32-bit
// plane), as in the edit kernels.
__device__ __forceinline__ int64_t slot_base(int64_t s, int lane, int q) { return s + 256 * q + 4 * lane; }

// Elements t .. t+3 of a 16-byte aligned plane (t a multiple of 4), read
// with non-temporal loads: each plane is streamed once per pass.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ void load4(const T *__restrict__ p, int64_t t, uint32_t *out) {
    if constexpr (sizeof(T) == 4) {
        const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p + t));
        out[0] = v.x;
        out[1] = v.y;
        out[2] = v.z;
        out[3] = v.w;
    } else if constexpr (sizeof(T) == 2) {
        const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p + t));
        out[0] = v.x & 0xffffu;
        out[1] = v.x >> 16;
        out[2] = v.y & 0xffffu;
        out[3] = v.y >> 16;
    } else {
        const uint32_t v = __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(p + t));
#pragma unroll
        for (int j = 0; j < 4; ++j) out[j] = (v >> (8 * j)) & 0xffu;
    }
}

template <typename T>
__device__ __forceinline__ void load4_tail(const T *__restrict__ p, int64_t t, int64_t n, uint32_t *out) {
#pragma unroll
    for (int j = 0; j < 4; ++j) out[j] = t + j < n ? (uint32_t)p[t + j] : 0u;
}

// Mask bits of texels t .. t+3 (t a multiple of 4): one word holds them.
__device__ __forceinline__ uint32_t mask4(const uint32_t *__restrict__ mask, int64_t t) {
    return (mask[t >> 5] >> (t & 31)) & 0xfu;
}

// 16 consecutive elements of a lane from a 16-byte aligned plane (range
// selection).
template <typename T>
__device__ __forceinline__ void load16(const T *__restrict__ p, int64_t t, uint32_t out[kPer]) {
    constexpr int kVec = 16 / sizeof(T);     // elements per 16-byte load
#pragma unroll
    for (int q = 0; q < kPer / kVec; ++q) {
        const uint4 v = reinterpret_cast<const uint4 *>(p + t)[q];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < kVec; ++k) {
            constexpr int kBits = 8 * sizeof(T);
            out[q * kVec + k] = kBits == 32 ? w[k * kBits / 32]
                                            : (w[k * kBits / 32] >> ((k * kBits) % 32)) & ((1u << kBits) - 1);
        }
    }
}

template <typename T>
__device__ __forceinline__ void load_tail(const T *__restrict__ p, int64_t t, int64_t n, uint32_t out[kPer]) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) out[k] = t + k < n ? (uint32_t)p[t + k] : 0u;
}

// Mask bits of texels t .. t+15 (t a multiple of 16): one word holds them.
__device__ __forceinline__ uint32_t mask16(const uint32_t *__restrict__ mask, int64_t t) {
    return (mask[t >> 5] >> (t & 31)) & 0xffffu;
}

// 16 consecutive elements to a 16-byte aligned plane of u8 or u16.
template <typename T>
__device__ __forceinline__ void store16(T *__restrict__ p, int64_t t, const uint32_t in[kPer]) {
    constexpr int kVec = 16 / sizeof(T);
    constexpr int kBits = 8 * sizeof(T);
#pragma unroll
    for (int q = 0; q < kPer / kVec; ++q) {
        uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int k = 0; k < kVec; ++k) w[k * kBits / 32] |= in[q * kVec + k] << ((k * kBits) % 32);
        reinterpret_cast<uint4 *>(p + t)[q] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// Range selection: dst[t] = label where valid and lo <= v <= hi.  Here a
// lane owns 16 consecutive texels, so that a lane with any selected texel
// rewrites its 16 labels as whole 16-byte vectors (the others unchanged): a
// selection that follows no pattern would otherwise leave partly written
// lines for the memory side to merge.  (Measured at 8192^2: 62 us, against
// 68 us with the wave-contiguous layout of the statistics, whose label
// vectors are 4 bytes per lane.)
template <int32_t DT, typename L>
__global__ __launch_bounds__(kBlock) void k_select(const Store<DT> *__restrict__ data,
                                                   const uint32_t *__restrict__ mask, int64_t n, double lo,
                                                   double hi, L *__restrict__ dst, uint32_t label) {
    const int64_t t = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kPer;
    if (t >= n) return;
    uint32_t v[kPer];
    const bool full = t + kPer <= n;
    if (full) load16(data, t, v);
    else load_tail(data, t, n, v);
    const uint32_t m = mask16(mask, t);
    uint32_t sel = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const double x = decode<DT>(v[k]);
        sel |= (uint32_t)(((m >> k) & 1u) && x >= lo && x <= hi) << k;
    }
    if (!sel) return;
    if (full) {
        uint32_t cur[kPer];
        load16(dst, t, cur);
#pragma unroll
        for (int k = 0; k < kPer; ++k)
            if ((sel >> k) & 1u) cur[k] = label;
        store16(dst, t, cur);
    } else {
        for (int k = 0; k < kPer; ++k)
            if (t + k < n && ((sel >> k) & 1u)) dst[t + k] = (L)label;
    }
}

// One wave step's planes for a lane (statistics).  wh: the high words of
// two-word area weights.
template <bool kWide>
struct StepData {
    uint32_t tr[kPer], w[kPer], wh[kWide ? kPer : 1], v[kPer], lab[kPer], m;
};

template <int32_t DT, typename R, bool kWide>
__device__ __forceinline__ void fetch_step(const int32_t *__restrict__ tri, const uint32_t *__restrict__ aw,
                                           const uint32_t *__restrict__ aw_hi, const Store<DT> *__restrict__ data,
                                           const uint32_t *__restrict__ mask, const R *__restrict__ region, int64_t n,
                                           int64_t s, int lane, StepData<kWide> &d) {
    constexpr bool kNoRegion = std::is_same<R, void>::value;
    d.m = 0;
    if (s + kWaveStep <= n) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t t = slot_base(s, lane, q);
            load4(reinterpret_cast<const uint32_t *>(tri), t, d.tr + 4 * q);
            load4(aw, t, d.w + 4 * q);
            if constexpr (kWide) load4(aw_hi, t, d.wh + 4 * q);
            load4(data, t, d.v + 4 * q);
            if constexpr (!kNoRegion) load4(region, t, d.lab + 4 * q);
            d.m |= mask4(mask, t) << (4 * q);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t t = slot_base(s, lane, q);
            load4_tail(reinterpret_cast<const uint32_t *>(tri), t, n, d.tr + 4 * q);
            load4_tail(aw, t, n, d.w + 4 * q);
            if constexpr (kWide) load4_tail(aw_hi, t, n, d.wh + 4 * q);
            load4_tail(data, t, n, d.v + 4 * q);
            if constexpr (!kNoRegion) load4_tail(region, t, n, d.lab + 4 * q);
            if (t < n) d.m |= mask4(mask, t) << (4 * q);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (t + j >= n) d.tr[4 * q + j] = 0xffffffffu;      // tri_id -1: not counted
        }
    }
}

// Statistics bins while accumulating: min and max as order-preserving keys.
struct Bin {
    unsigned long long count, aw;
    double wsum;
    unsigned long long kmin, kmax, aw_hi;
};
static_assert(sizeof(Bin) == sizeof(uvl_numstat), "bins are finalised in place");

__device__ __forceinline__ unsigned long long order_key(double d) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(d);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ __forceinline__ double from_key(unsigned long long k) {
    const unsigned long long u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)u);
}

struct Run {
    uint32_t label;
    unsigned long long count, aw, aw_hi;
    double wsum, vmin, vmax;

    __device__ __forceinline__ void reset(uint32_t l) {
        label = l;
        count = aw = aw_hi = 0;
        wsum = 0.0;
        vmin = INFINITY;
        vmax = -INFINITY;
    }
};

// Add totals to a bin: LDS (native LDS atomics) or global memory.
template <bool kGlobal, bool kWide>
__device__ __forceinline__ void add_to(Bin *b, unsigned long long count, unsigned long long aw,
                                       unsigned long long aw_hi, double wsum, unsigned long long kmin,
                                       unsigned long long kmax) {
    atomicAdd(&b->count, count);
    atomicAdd(&b->aw, aw);
    if constexpr (kWide) atomicAdd(&b->aw_hi, aw_hi);
    if constexpr (kGlobal) unsafeAtomicAdd(&b->wsum, wsum);
    else atomicAdd(&b->wsum, wsum);
    atomicMin(&b->kmin, kmin);
    atomicMax(&b->kmax, kmax);
}

// LDS slot of a u16 label: open addressing with linear probing over
// kHashSlots tagged slots; -1 when 8 probes find neither the label nor a
// free slot (the run then goes to the global bin).
constexpr int kHashBits = 9;
constexpr int kHashSlots = 1 << kHashBits;
constexpr uint32_t kNoTag = 0xffffffffu;

__device__ __forceinline__ int hash_slot(uint32_t *tags, uint32_t label) {
    uint32_t h = (label * 2654435761u) >> (32 - kHashBits);
    for (int probe = 0; probe < 8; ++probe) {
        const uint32_t prev = atomicCAS(tags + h, kNoTag, label);
        if (prev == kNoTag || prev == label) return (int)h;
        h = (h + 1) & (kHashSlots - 1);
    }
    return -1;
}

__device__ __forceinline__ void bin_clear(Bin &b) {
    b.count = b.aw = b.aw_hi = 0;
    b.wsum = 0.0;
    b.kmin = ~0ull;
    b.kmax = 0;
}

__global__ void k_stats_clear(Bin *bins, int nbins) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nbins) bin_clear(bins[i]);
}

__global__ void k_stats_final(Bin *bins, int nbins) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nbins) return;
    Bin b = bins[i];
    uvl_numstat s;
    s.count = b.count;
    s.area_w = b.aw;
    s.wsum = b.wsum;
    s.vmin = b.count ? from_key(b.kmin) : INFINITY;
    s.vmax = b.count ? from_key(b.kmax) : -INFINITY;
    s.area_w_hi = b.aw_hi;
    reinterpret_cast<uvl_numstat *>(bins)[i] = s;
}

// Zonal statistics.  R: region storage (void: no region, one group).
// Every workgroup accumulates its lanes' runs in LDS -- one bin, 256 bins
// indexed by a u8 label, or kHashSlots tagged slots for u16 labels -- and
// adds its non-empty bins to the global bins once at the end.
template <int32_t DT, typename R, bool kWide>
__global__ __launch_bounds__(kBlock) void k_stats(const int32_t *__restrict__ tri, const uint32_t *__restrict__ aw,
                                                  const uint32_t *__restrict__ aw_hi,
                                                  const Store<DT> *__restrict__ data,
                                                  const uint32_t *__restrict__ mask, const R *__restrict__ region,
                                                  int64_t n, Bin *__restrict__ bins) {
    constexpr bool kNoRegion = std::is_same<R, void>::value;
    constexpr bool kHash = std::is_same<R, uint16_t>::value;
    constexpr int kSlots = kNoRegion ? 1 : kHash ? kHashSlots : 256;
    __shared__ Bin lds[kSlots];
    __shared__ uint32_t tags[kHash ? kSlots : 1];
    for (int i = threadIdx.x; i < kSlots; i += kBlock) {
        bin_clear(lds[i]);
        if constexpr (kHash) tags[i] = kNoTag;
    }
    __syncthreads();
    auto put = [&](const Run &r) {
        if (r.count == 0) return;
        int slot = kNoRegion ? 0 : (int)r.label;
        if constexpr (kHash) slot = hash_slot(tags, r.label);
        if (slot >= 0)
            add_to<false, kWide>(lds + slot, r.count, r.aw, r.aw_hi, r.wsum, order_key(r.vmin), order_key(r.vmax));
        else
            add_to<true, kWide>(bins + r.label, r.count, r.aw, r.aw_hi, r.wsum, order_key(r.vmin),
                                order_key(r.vmax));
    };
    Run run;
    run.reset(0);
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * kWaves * kWaveStep;
    int64_t s = ((int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6)) * kWaveStep;
    // the next step's loads are issued before this step is processed
    StepData<kWide> cur, nxt;
    if (s < n) fetch_step<DT, R, kWide>(tri, aw, aw_hi, data, mask, region, n, s, lane, cur);
    for (; s < n; s += stride) {
        const bool more = s + stride < n;
        if (more) fetch_step<DT, R, kWide>(tri, aw, aw_hi, data, mask, region, n, s + stride, lane, nxt);
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if ((int32_t)cur.tr[k] < 0 || !((cur.m >> k) & 1u)) continue;
            const uint32_t l = kNoRegion ? 0u : cur.lab[k];
            if (l != run.label) {
                put(run);
                run.reset(l);
            }
            const double x = decode<DT>(cur.v[k]);
            run.count += 1;
            run.aw += cur.w[k];
            double wk = (double)cur.w[k];
            if constexpr (kWide) {
                run.aw_hi += cur.wh[k];
                wk += (double)cur.wh[k] * 4294967296.0;   // high * 2^32 + low, rounded once
            }
            run.wsum += wk * x;
            run.vmin = fmin(run.vmin, x);
            run.vmax = fmax(run.vmax, x);
        }
        if (more) cur = nxt;
    }
    put(run);
    __syncthreads();
    for (int i = threadIdx.x; i < kSlots; i += kBlock) {
        const Bin &b = lds[i];
        if (b.count == 0) continue;
        const uint32_t label = kHash ? tags[i] : (uint32_t)i;
        add_to<true, kWide>(bins + label, b.count, b.aw, b.aw_hi, b.wsum, b.kmin, b.kmax);
    }
}

// ---------------------------------------------------------------------------
// Operations between numeric layers: per texel a result validity from the
// operands' mask bits and, where it holds, a value (the operand that is
// valid for the mask operations, the smaller / larger for MIN / MAX, the
// saturating sum for ADD); elsewhere the data stay and the bit is cleared.
// A wave step covers 1024 texels; lane l takes texels 256 q + 4 l .. +3
// (q < 4) so that each plane load is one contiguous block per wave, and the
// 8 lanes that share a 32-texel mask word merge their bits with three
// shuffles before one of them writes the word.

constexpr int kNumAnd = 0, kNumOr = 1, kNumXor = 2, kNumMin = 3, kNumMax = 4, kNumAdd = 5;

template <int32_t DT>
__device__ __forceinline__ uint32_t add_sat(uint32_t xa, uint32_t xb) {
    if constexpr (DT == UVL_U8 || DT == UVL_U16) {
        const uint32_t sum = xa + xb, top = DT == UVL_U8 ? 0xffu : 0xffffu;
        return sum > top ? top : sum;
    } else if constexpr (DT == UVL_I32) {
        const long long sum = (long long)(int32_t)xa + (long long)(int32_t)xb;
        return (uint32_t)(int32_t)(sum > 2147483647LL ? 2147483647LL : sum < -2147483648LL ? -2147483648LL : sum);
    } else if constexpr (DT == UVL_F32) {
        const float sum = __uint_as_float(xa) + __uint_as_float(xb);       // one IEEE rounding
        return __float_as_uint(isinf(sum) ? copysignf(3.40282346638528859812e+38f, sum) : sum);
    } else {
        // binary16: the sum of two binary16 values is exact in fp64, then one
        // rounding to binary16; beyond the finite range the largest value
        const double sum = decode<UVL_F16>(xa) + decode<UVL_F16>(xb);
        uint16_t h;
        if (f16_from_double(sum, h)) return h;
        return sum < 0.0 ? 0xfbffu : 0x7bffu;
    }
}

template <int32_t DT, int OP>
__device__ __forceinline__ bool num_valid(bool va, bool vb) {
    return OP == kNumOr ? (va || vb) : OP == kNumXor ? (va != vb) : (va && vb);
}

template <int32_t DT, int OP>
__device__ __forceinline__ uint32_t num_value(uint32_t xa, uint32_t xb, bool va) {
    if constexpr (OP == kNumMin) return decode<DT>(xa) <= decode<DT>(xb) ? xa : xb;
    else if constexpr (OP == kNumMax) return decode<DT>(xa) >= decode<DT>(xb) ? xa : xb;
    else if constexpr (OP == kNumAdd) return add_sat<DT>(xa, xb);
    else return va ? xa : xb;
}

template <typename T>
__device__ __forceinline__ void store4(T *__restrict__ p, int64_t t, const uint32_t *in) {
    if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<uint4 *>(p + t) = make_uint4(in[0], in[1], in[2], in[3]);
    } else if constexpr (sizeof(T) == 2) {
        *reinterpret_cast<uint2 *>(p + t) = make_uint2(in[0] | (in[1] << 16), in[2] | (in[3] << 16));
    } else {
        *reinterpret_cast<uint32_t *>(p + t) = in[0] | (in[1] << 8) | (in[2] << 16) | (in[3] << 24);
    }
}

// ALIAS: 0 dst is its own layer, 1 dst is a, 2 dst is b (then a texel whose
// result is not valid keeps that operand's data, already in registers).
template <int32_t DT, int OP, int ALIAS>
__global__ __launch_bounds__(kBlock) void k_numop(Store<DT> *dst, uint32_t *dmask, const Store<DT> *a,
                                                  const uint32_t *amask, const Store<DT> *b,
                                                  const uint32_t *bmask, int64_t n) {
    const int lane = threadIdx.x & 63;
    const int64_t s = ((int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6)) * kWaveStep;
    if (s >= n) return;                                     // whole waves leave together
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t t = slot_base(s, lane, q);
        uint32_t r4 = 0;
        if (t + 4 <= n) {
            uint32_t xa[4], xb[4], out[4];
            load4(a, t, xa);
            load4(b, t, xb);
            const uint32_t ma = mask4(amask, t), mb = mask4(bmask, t);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool va = (ma >> j) & 1u, vb = (mb >> j) & 1u;
                const bool r = num_valid<DT, OP>(va, vb);
                r4 |= (uint32_t)r << j;
                out[j] = num_value<DT, OP>(xa[j], xb[j], va);
            }
            if (r4 != 0xfu) {
                uint32_t old[4];
                if constexpr (ALIAS == 1) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) old[j] = xa[j];
                } else if constexpr (ALIAS == 2) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) old[j] = xb[j];
                } else {
                    load4(dst, t, old);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (!((r4 >> j) & 1u)) out[j] = old[j];
            }
            store4(dst, t, out);
        } else if (t < n) {
            const uint32_t ma = mask4(amask, t), mb = mask4(bmask, t);
            for (int j = 0; j < 4 && t + j < n; ++j) {
                const bool va = (ma >> j) & 1u, vb = (mb >> j) & 1u;
                if (num_valid<DT, OP>(va, vb)) {
                    r4 |= 1u << j;
                    dst[t + j] = (Store<DT>)num_value<DT, OP>(a[t + j], b[t + j], va);
                }
            }
        }
        // the 8 lanes of a mask word merge their 4-bit pieces
        uint32_t word = r4 << (t & 31);
        word |= __shfl_xor(word, 1);
        word |= __shfl_xor(word, 2);
        word |= __shfl_xor(word, 4);
        const int64_t wi = t >> 5;
        if ((lane & 7) == 0 && wi * 32 < n) {
            const int64_t left = n - wi * 32;               // texels in this word
            if (left < 32) {
                const uint32_t low = (1u << left) - 1u;     // bits past the last texel stay
                word = (word & low) | (dmask[wi] & ~low);
            }
            dmask[wi] = word;
        }
    }
}

template <int32_t DT, int OP>
void launch_numop_alias(const uvl_numeric *d, const uvl_numeric *a, const uvl_numeric *b, int alias, hipStream_t s) {
    const int64_t n = (int64_t)d->width * d->height;
    const dim3 grid((unsigned)ceil_div(n, (int64_t)kWaves * kWaveStep));
    Store<DT> *D = static_cast<Store<DT> *>(d->data);
    const Store<DT> *A = static_cast<const Store<DT> *>(a->data), *B = static_cast<const Store<DT> *>(b->data);
    if (alias == 1)
        hipLaunchKernelGGL((k_numop<DT, OP, 1>), grid, dim3(kBlock), 0, s, D, d->mask, A, a->mask, B, b->mask, n);
    else if (alias == 2)
        hipLaunchKernelGGL((k_numop<DT, OP, 2>), grid, dim3(kBlock), 0, s, D, d->mask, A, a->mask, B, b->mask, n);
    else
        hipLaunchKernelGGL((k_numop<DT, OP, 0>), grid, dim3(kBlock), 0, s, D, d->mask, A, a->mask, B, b->mask, n);
}

template <int32_t DT>
void launch_numop(int op, const uvl_numeric *d, const uvl_numeric *a, const uvl_numeric *b, int alias,
                  hipStream_t s) {
    switch (op) {
    case kNumAnd: launch_numop_alias<DT, kNumAnd>(d, a, b, alias, s); break;
    case kNumOr: launch_numop_alias<DT, kNumOr>(d, a, b, alias, s); break;
    case kNumXor: launch_numop_alias<DT, kNumXor>(d, a, b, alias, s); break;
    case kNumMin: launch_numop_alias<DT, kNumMin>(d, a, b, alias, s); break;
    case kNumMax: launch_numop_alias<DT, kNumMax>(d, a, b, alias, s); break;
    default: launch_numop_alias<DT, kNumAdd>(d, a, b, alias, s); break;
    }
}

template <int32_t DT>
void launch_select(const uvl_numeric *src, double lo, double hi, const uvl_layer *dst, uint32_t label,
                   hipStream_t s) {
    const int64_t n = (int64_t)src->width * src->height;
    const dim3 grid((unsigned)ceil_div(n, (int64_t)kBlock * kPer));
    const Store<DT> *data = static_cast<const Store<DT> *>(src->data);
    if (dst->dtype == UVL_U8)
        hipLaunchKernelGGL((k_select<DT, uint8_t>), grid, dim3(kBlock), 0, s, data, src->mask, n, lo, hi,
                           static_cast<uint8_t *>(dst->data), label);
    else
        hipLaunchKernelGGL((k_select<DT, uint16_t>), grid, dim3(kBlock), 0, s, data, src->mask, n, lo, hi,
                           static_cast<uint16_t *>(dst->data), label);
}

template <int32_t DT, bool kWide>
void launch_stats_w(const uvl_geom *g, const uvl_numeric *l, const uvl_layer *region, Bin *bins, hipStream_t s) {
    const int64_t n = (int64_t)l->width * l->height;
    const dim3 grid((unsigned)std::min<int64_t>(ceil_div(n, (int64_t)kWaves * kWaveStep), kMaxStatBlocks));
    const Store<DT> *data = static_cast<const Store<DT> *>(l->data);
    const uint32_t *hi = g->area_w_hi;
    if (!region)
        hipLaunchKernelGGL((k_stats<DT, void, kWide>), grid, dim3(kBlock), 0, s, g->tri_id, g->area_w, hi, data,
                           l->mask, (const void *)nullptr, n, bins);
    else if (region->dtype == UVL_U8)
        hipLaunchKernelGGL((k_stats<DT, uint8_t, kWide>), grid, dim3(kBlock), 0, s, g->tri_id, g->area_w, hi, data,
                           l->mask, static_cast<const uint8_t *>(region->data), n, bins);
    else
        hipLaunchKernelGGL((k_stats<DT, uint16_t, kWide>), grid, dim3(kBlock), 0, s, g->tri_id, g->area_w, hi, data,
                           l->mask, static_cast<const uint16_t *>(region->data), n, bins);
}

template <int32_t DT>
void launch_stats(const uvl_geom *g, const uvl_numeric *l, const uvl_layer *region, Bin *bins, hipStream_t s) {
    if (g->area_w_hi) launch_stats_w<DT, true>(g, l, region, bins, s);
    else launch_stats_w<DT, false>(g, l, region, bins, s);
}

template <typename F>
void by_dtype(int32_t dt, F &&f) {
    switch (dt) {
    case UVL_U8: f(std::integral_constant<int32_t, UVL_U8>()); break;
    case UVL_U16: f(std::integral_constant<int32_t, UVL_U16>()); break;
    case UVL_I32: f(std::integral_constant<int32_t, UVL_I32>()); break;
    case UVL_F16: f(std::integral_constant<int32_t, UVL_F16>()); break;
    default: f(std::integral_constant<int32_t, UVL_F32>()); break;
    }
}

}  // namespace
}  // namespace uvl

using namespace uvl;

extern "C" int32_t uvl_numeric_create(const uvl_numeric *layer, void *stream) {
    if (!numeric_ok(layer)) return UVL_E_INVAL;
    if (int32_t s = device_ok()) return s;
    hipStream_t s = as_stream(stream);
    fill_bytes(layer->data, (int64_t)layer->width * layer->height * dtype_bytes(layer->dtype), s);
    fill_bytes(layer->mask, mask_words(layer) * 4, s);
    return launch_status();
}

extern "C" int32_t uvl_numeric_select(const uvl_numeric *src, double lo, double hi, const uvl_layer *dst,
                                      uint32_t label, void *stream) {
    if (!numeric_ok(src) || !layer_ok(dst) || std::isnan(lo) || std::isnan(hi)) return UVL_E_INVAL;
    if (!dtype_ok(dst->dtype) || label > dtype_max(dst->dtype)) return UVL_E_DTYPE;
    if (dst->width != src->width || dst->height != src->height) return UVL_E_SHAPE;
    if (int32_t s = device_ok()) return s;
    by_dtype(src->dtype, [&](auto dt) { launch_select<decltype(dt)::value>(src, lo, hi, dst, label, as_stream(stream)); });
    return launch_status();
}

extern "C" int32_t uvl_numeric_stats(const uvl_geom *geom, const uvl_numeric *layer, const uvl_layer *region,
                                     uvl_numstat *bins_dev, uvl_numstat *bins_host, void *stream) {
    if (!geom || !geom->tri_id || !geom->area_w || !aligned16(geom->tri_id) || !aligned16(geom->area_w))
        return UVL_E_INVAL;
    if (geom->area_w_hi && !aligned16(geom->area_w_hi)) return UVL_E_INVAL;
    if (!numeric_ok(layer) || !bins_dev || (reinterpret_cast<uintptr_t>(bins_dev) & 7)) return UVL_E_INVAL;
    if (region && !layer_ok(region)) return UVL_E_INVAL;
    if (region && !dtype_ok(region->dtype)) return UVL_E_DTYPE;
    if (layer->width != geom->width || layer->height != geom->height) return UVL_E_SHAPE;
    if (region && (region->width != geom->width || region->height != geom->height)) return UVL_E_SHAPE;
    if (int32_t s = device_ok()) return s;
    const int nbins = !region ? 1 : region->dtype == UVL_U8 ? 256 : 65536;
    hipStream_t s = as_stream(stream);
    Bin *bins = reinterpret_cast<Bin *>(bins_dev);
    hipLaunchKernelGGL(k_stats_clear, dim3((unsigned)ceil_div(nbins, kBlock)), dim3(kBlock), 0, s, bins, nbins);
    by_dtype(layer->dtype, [&](auto dt) { launch_stats<decltype(dt)::value>(geom, layer, region, bins, s); });
    hipLaunchKernelGGL(k_stats_final, dim3((unsigned)ceil_div(nbins, kBlock)), dim3(kBlock), 0, s, bins, nbins);
    if (int32_t st = launch_status()) return st;
    if (bins_host) {
        if (hipMemcpyAsync(bins_host, bins_dev, sizeof(uvl_numstat) * nbins, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return UVL_E_DEVICE;
    }
    return UVL_OK;
}

extern "C" int32_t uvl_numeric_op(int32_t op, const uvl_numeric *dst, const uvl_numeric *a, const uvl_numeric *b,
                                  void *stream) {
    if (op < UVL_NUM_AND || op > UVL_NUM_ADD) return UVL_E_INVAL;
    if (!numeric_ok(dst) || !numeric_ok(a) || !numeric_ok(b)) return UVL_E_INVAL;
    if (a->dtype != dst->dtype || b->dtype != dst->dtype) return UVL_E_DTYPE;
    if (a->width != dst->width || a->height != dst->height || b->width != dst->width || b->height != dst->height)
        return UVL_E_SHAPE;
    // dst is a or b entirely, or shares no plane with them
    for (const uvl_numeric *x : {a, b})
        if ((x->data == dst->data) != (x->mask == dst->mask)) return UVL_E_INVAL;
    if (int32_t s = device_ok()) return s;
    const int alias = dst->data == a->data ? 1 : dst->data == b->data ? 2 : 0;
    by_dtype(dst->dtype, [&](auto dt) { launch_numop<decltype(dt)::value>(op, dst, a, b, alias, as_stream(stream)); });
    return launch_status();
}
