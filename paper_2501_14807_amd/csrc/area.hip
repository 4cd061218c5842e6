// Per-label surface area for libuvl.
//
// Table 1 of the paper reports the surface area one texel stands for; the
// labelled area of a layer is the sum of those texel areas over the texels
// holding the label.  The geometry image stores each texel's area as an
// integer multiple of a power-of-two scale -- one uint32 word, or two
// (low and high) when the texel areas span too wide a range for one -- so
// the sums are exact uint64 integers: independent of summation order,
// deterministic run to run, and exactly additive (area(A or B) = area(A) +
// area(B) - area(A and B)).  With two words, the low and the high words are
// summed into separate bins (each sum stays below 2^62), and the area is
// (high sum * 2^32 + low sum) * area_scale.
//
// One pass reads every area weight from memory once for all the layers of
// a query (up to 32).  A work unit is 4 rows x 512 columns (2 rows with
// two-word weights); a wave takes units in turn, each lane holding 8
// consecutive columns: it loads the unit's weights into registers, where
// they stay while the wave walks the layers, u8 layers first, requesting
// the labels of two u8 layers (four with 1024-thread workgroups) before it
// sums any (a unit whose rows and columns all exist has every load issued
// ahead of the first wait; a ragged unit takes a path with per-row checks).  Per layer, runs of equal
// labels go to the workgroup's bins; a row whose 8 labels are equal (the
// common case: labelled regions are spatially coherent) is checked on the
// packed words and adds its row sum.  A query of one or two layers on a
// geometry image with per-block area sums (one 64-bit sum per 4 x 8
// texels, a lane's share of a unit) reads no weights where the lane's
// labels are all equal: it adds the block's sum, and a lane whose labels
// differ reads its weights then.  u8 layers add into 256 LDS bins each
// (native 64-bit LDS atomics); u16 layers (65536 bins) add into an LDS hash
// table keyed by (layer, label), open addressing with linear probing,
// falling back to the global bin only if 16 probes find no slot.  The LDS
// bins go to the global bins once per workgroup.  A workgroup (8 waves for
// queries of up to 8 u8 layers, else 16, with up to 88 KiB of LDS of the
// CU's 160 KiB) strides over the units with the others.
#include "uvl_internal.h"

namespace uvl {
namespace {

constexpr int kCols = 8;                  // columns per lane
constexpr int kChunk = 64 * kCols;        // columns per wave unit
constexpr int kMaxLayers = 32;
constexpr int kBlkMaxLayers = 2;          // queries of at most this many layers use the block sums
constexpr int kHashBits = 11;
constexpr int kHash = 1 << kHashBits;     // LDS hash slots for u16 labels
constexpr uint32_t kEmptyKey = 0xffffffffu;

// LDS of one workgroup: the u8 bins (two rows per layer with two-word
// weights) and the u16 hash.
constexpr int area_lds_bytes(int nu8, bool u16, bool wide) {
    return (nu8 > 0 ? (wide ? 2 : 1) * nu8 * 256 * 8 : 0) + (u16 ? kHash * 4 + (wide ? 2 : 1) * kHash * 8 : 0);
}

// Threads per workgroup of the one-pass query: 512 for up to 8 u8 bin rows
// where two workgroups fit the CU's 160 KiB of LDS, else 1024 (one
// workgroup of 16 waves per CU).  Measured at 8192^2: 8 u8 + 1 u16 layers
// 166-170 us with 512 threads (groups of two u8 layers, three workgroups
// per CU at most) against 190 us with 1024 (groups of four, one per CU);
// 32 u8 layers 1.70 ms with 1024 against 1.88-1.93 ms with 512.
constexpr int area_threads(int nu8, bool u16, bool wide) {
    return nu8 <= 8 && area_lds_bytes(nu8, u16, wide) <= 80 * 1024 ? 512 : 1024;
}
constexpr uint32_t kNoLabel = 0xffffffffu;

struct AreaArgs {
    const void *data[kMaxLayers];
    unsigned long long *bins[kMaxLayers];       // global low-word (or only) bins per layer
    unsigned long long *bins_hi[kMaxLayers];    // global high-word bins (two-word weights)
    int32_t nu8;                                // layers [0, nu8) are u8 (LDS bin row = index),
    int32_t nl;                                 // [nu8, nl) are u16
};

// A weight: one word, or a low and a high word.
template <bool kWide>
struct Sum {
    unsigned long long lo = 0, hi = 0;
    __device__ __forceinline__ bool nonzero() const { return kWide ? (lo | hi) != 0 : lo != 0; }
    __device__ __forceinline__ void add(const Sum &o) {
        lo += o.lo;
        if constexpr (kWide) hi += o.hi;
    }
};

template <bool kWide>
struct Bins {
    unsigned long long *u8;                // LDS [rows][256] (two-word: low rows, then high rows)
    int nu8;
    uint32_t *key;                         // LDS [kHash]
    unsigned long long *val;               // LDS [kHash] (two-word: [2][kHash])
    const AreaArgs *A;

    __device__ __forceinline__ void add_u8(int row, uint32_t label, const Sum<kWide> &s) const {
        atomicAdd(u8 + row * 256 + label, s.lo);
        if constexpr (kWide) atomicAdd(u8 + (nu8 + row) * 256 + label, s.hi);
    }
    __device__ __forceinline__ void add_u16(int l, uint32_t label, const Sum<kWide> &s) const {
        const uint32_t k = ((uint32_t)l << 16) | label;
        uint32_t h = (k * 2654435761u) >> (32 - kHashBits);
        for (int probe = 0; probe < 16; ++probe) {
            const uint32_t prev = atomicCAS(key + h, kEmptyKey, k);
            if (prev == kEmptyKey || prev == k) {
                atomicAdd(val + h, s.lo);
                if constexpr (kWide) atomicAdd(val + kHash + h, s.hi);
                return;
            }
            h = (h + 1) & (kHash - 1);
        }
        atomicAdd(A->bins[l] + label, s.lo);
        if constexpr (kWide) atomicAdd(A->bins_hi[l] + label, s.hi);
    }
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Labels of one row of a lane: the packed words (u8: 2, u16: 4).
template <typename T>
struct RowLabels {
    static constexpr int kWords = kCols * sizeof(T) / 4;
    uint32_t w[kWords];

    // streamed once: non-temporal loads of 8 (u8) or 16 (u16) bytes
    __device__ __forceinline__ void load_vec(const T *p) {
        if constexpr (kWords == 4) {
            const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
            w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
        } else {
            static_assert(kWords == 2, "8 columns of u8 or u16 labels");
            const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p));
            w[0] = v.x; w[1] = v.y;
        }
    }
    // ragged columns: labels past the row's end repeat the first one
    __device__ __forceinline__ void load_tail(const T *p, int ncol) {
        const uint32_t first = ncol > 0 ? (uint32_t)p[0] : 0u;
        constexpr int kPerWord = 4 / sizeof(T);
#pragma unroll
        for (int i = 0; i < kWords; ++i) {
            uint32_t x = 0;
#pragma unroll
            for (int b = 0; b < kPerWord; ++b) {
                const int k = i * kPerWord + b;
                x |= (k < ncol ? (uint32_t)p[k] : first) << (8 * sizeof(T) * b);
            }
            w[i] = x;
        }
    }
    __device__ __forceinline__ uint32_t at(int k) const {
        constexpr int kPerWord = 4 / sizeof(T);
        return (w[k / kPerWord] >> (8 * sizeof(T) * (k % kPerWord))) & (sizeof(T) == 1 ? 0xffu : 0xffffu);
    }
    // a word made of the first label of w, repeated
    static __device__ __forceinline__ uint32_t replicate(uint32_t w) {
        return sizeof(T) == 1 ? (w & 0xffu) * 0x01010101u : (w & 0xffffu) * 0x00010001u;
    }
    // all kCols labels equal: every word equal and made of one repeated label
    __device__ __forceinline__ bool uniform() const {
        bool eq = true;
#pragma unroll
        for (int i = 1; i < kWords; ++i) eq = eq && w[i] == w[0];
        return eq && w[0] == replicate(w[0]);
    }
};

// A unit's weights, held in registers for all the layers of the query,
// and their per-row sums.
template <bool kWide, int kRows>
struct UnitWeights {
    uint32_t lo[kRows][kCols];
    uint32_t hi[kWide ? kRows : 1][kWide ? kCols : 1];
    Sum<kWide> tot[kRows];
};

// kFull: every row of the unit exists and the lane's kCols columns are
// aligned and in the atlas (vector loads), known at compile time so that
// all the loads are issued before the first wait.
template <bool kFull, bool kWide, int kRows>
__device__ __forceinline__ void load_weights(const uint32_t *__restrict__ aw, const uint32_t *__restrict__ aw_hi,
                                             int64_t t0, int W, int nrows, int ncol, bool vec,
                                             UnitWeights<kWide, kRows> &U) {
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const int64_t t = t0 + (int64_t)r * W;
        if (kFull || (r < nrows && vec)) {
#pragma unroll
            for (int q = 0; q < kCols / 4; ++q) {
                const uint4 v = *reinterpret_cast<const uint4 *>(aw + t + 4 * q);
                U.lo[r][4 * q] = v.x; U.lo[r][4 * q + 1] = v.y; U.lo[r][4 * q + 2] = v.z; U.lo[r][4 * q + 3] = v.w;
                if constexpr (kWide) {
                    const uint4 h = *reinterpret_cast<const uint4 *>(aw_hi + t + 4 * q);
                    U.hi[r][4 * q] = h.x; U.hi[r][4 * q + 1] = h.y; U.hi[r][4 * q + 2] = h.z; U.hi[r][4 * q + 3] = h.w;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < kCols; ++k) {
                const bool in = r < nrows && k < ncol;
                U.lo[r][k] = in ? aw[t + k] : 0u;
                if constexpr (kWide) U.hi[r][k] = in ? aw_hi[t + k] : 0u;
            }
        }
        Sum<kWide> s;
#pragma unroll
        for (int k = 0; k < kCols; ++k) {
            s.lo += U.lo[r][k];
            if constexpr (kWide) s.hi += U.hi[r][k];
        }
        U.tot[r] = s;
    }
}

// A layer's labels over a unit (its rows of kCols columns).
template <bool kFull, typename T, int kRows>
__device__ __forceinline__ void load_rows(const T *__restrict__ L, int64_t t0, int W, int nrows, int ncol, bool vec,
                                          RowLabels<T> lab[kRows]) {
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        if (!kFull && r >= nrows) break;
        const T *p = L + t0 + (int64_t)r * W;
        if (kFull || vec) lab[r].load_vec(p);
        else lab[r].load_tail(p, ncol);
    }
}

// One layer over a unit: runs of equal labels go to the bins.
template <bool kFull, typename T, bool kWide, int kRows, typename Add>
__device__ __forceinline__ void unit_runs(const RowLabels<T> lab[kRows], int nrows,
                                          const UnitWeights<kWide, kRows> &U, Add &&add) {
    uint32_t cur = kNoLabel;
    Sum<kWide> run;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        if (!kFull && r >= nrows) break;
        if (lab[r].uniform()) {
            const uint32_t l0 = lab[r].at(0);
            if (l0 != cur) {
                if (run.nonzero()) add(cur, run);
                cur = l0;
                run = Sum<kWide>();
            }
            run.add(U.tot[r]);
        } else if constexpr (sizeof(T) == 2) {
            // u16: a loop, so that the hash insert is inlined once per row
            // (each inlined insert holds its probe loop's exec masks)
#pragma unroll 1
            for (int k = 0; k < kCols; ++k) {
                uint32_t word = lab[r].w[0], lo = U.lo[r][0];
#pragma unroll
                for (int q = 1; q < kCols; ++q) {
                    if (q / 2 != 0 && k / 2 == q / 2) word = lab[r].w[q / 2];
                    if (k == q) lo = U.lo[r][q];
                }
                const uint32_t lk = (word >> (16 * (k & 1))) & 0xffffu;
                if (lk != cur) {
                    if (run.nonzero()) add(cur, run);
                    cur = lk;
                    run = Sum<kWide>();
                }
                run.lo += lo;
                if constexpr (kWide) {
                    uint32_t hi = U.hi[r][0];
#pragma unroll
                    for (int q = 1; q < kCols; ++q)
                        if (k == q) hi = U.hi[r][q];
                    run.hi += hi;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < kCols; ++k) {
                const uint32_t lk = lab[r].at(k);
                if (lk != cur) {
                    if (run.nonzero()) add(cur, run);
                    cur = lk;
                    run = Sum<kWide>();
                }
                run.lo += U.lo[r][k];
                if constexpr (kWide) run.hi += U.hi[r][k];
            }
        }
    }
    if (run.nonzero()) add(cur, run);
}

// kG consecutive u8 layers from layer l over a unit: the labels of all of
// them are requested before any is used, so that kG * kRows loads are in
// flight at once rather than kRows.
template <bool kFull, int kG, bool kWide, int kRows>
__device__ __forceinline__ void u8_group(const AreaArgs &A, int l, const Bins<kWide> &bins,
                                         int64_t t0, int W, int nrows, int ncol, bool vec,
                                         const UnitWeights<kWide, kRows> &U) {
    RowLabels<uint8_t> lab[kG][kRows];
#pragma unroll
    for (int j = 0; j < kG; ++j)
        load_rows<kFull, uint8_t, kRows>(static_cast<const uint8_t *>(A.data[l + j]), t0, W, nrows, ncol, vec,
                                         lab[j]);
#pragma unroll
    for (int j = 0; j < kG; ++j) {
        const int row = l + j;
        unit_runs<kFull, uint8_t, kWide, kRows>(lab[j], nrows, U,
                                         [&](uint32_t lab_, const Sum<kWide> &s) { bins.add_u8(row, lab_, s); });
    }
}

// All of a lane's labels equal (its whole block of kRows x kCols texels).
template <typename T, int kRows>
__device__ __forceinline__ bool unit_uniform(const RowLabels<T> lab[kRows]) {
    const uint32_t rep = RowLabels<T>::replicate(lab[0].w[0]);
    bool all = true;
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int q = 0; q < RowLabels<T>::kWords; ++q) all = all && lab[r].w[q] == rep;
    return all;
}

// One layer over a full unit with the block's area sum at hand: a lane
// whose labels are all equal adds the sum; any other reads its weights
// (once per unit, only that lane) and adds its runs.
template <typename T, int kRows, typename Add>
__device__ __forceinline__ void blk_layer(const RowLabels<T> lab[kRows], const Sum<false> &bs,
                                          const uint32_t *__restrict__ aw, int64_t t0, int W,
                                          UnitWeights<false, kRows> &U, bool &have_w, Add &&add) {
    if (unit_uniform<T, kRows>(lab)) {
        if (bs.nonzero()) add(lab[0].at(0), bs);
        return;
    }
    if (!have_w) {
        load_weights<true, false, kRows>(aw, nullptr, t0, W, kRows, kCols, true, U);
        have_w = true;
    }
    unit_runs<true, T, false, kRows>(lab, kRows, U, add);
}

// A full unit of one-word weights with per-block area sums (area_blk):
// layer by layer, u8 layers first; the weights are read only by lanes whose
// labels differ within their block in some layer.
template <int kNU8, bool kU16, int kRows>
__device__ __forceinline__ void area_unit_blk(const AreaArgs &A, const Bins<false> &bins,
                                              const uint32_t *__restrict__ aw,
                                              const unsigned long long *__restrict__ blk, int64_t t0, int W,
                                              int64_t bidx) {
    Sum<false> bs;
    bs.lo = blk[bidx];
    UnitWeights<false, kRows> U;
    bool have_w = false;
    if constexpr (kNU8 > 0)
        for (int l = 0; l < A.nu8; ++l) {
            RowLabels<uint8_t> lab[kRows];
            load_rows<true, uint8_t, kRows>(static_cast<const uint8_t *>(A.data[l]), t0, W, kRows, kCols, true, lab);
            blk_layer<uint8_t, kRows>(lab, bs, aw, t0, W, U, have_w,
                                      [&](uint32_t lb, const Sum<false> &v) { bins.add_u8(l, lb, v); });
        }
    if constexpr (kU16)
        for (int l = A.nu8; l < A.nl; ++l) {
            RowLabels<uint16_t> lab[kRows];
            load_rows<true, uint16_t, kRows>(static_cast<const uint16_t *>(A.data[l]), t0, W, kRows, kCols, true, lab);
            blk_layer<uint16_t, kRows>(lab, bs, aw, t0, W, U, have_w,
                                       [&](uint32_t lb, const Sum<false> &v) { bins.add_u16(l, lb, v); });
        }
}

// One unit over every layer of the query: its weights, then the u8 layers
// (first in A) in groups of up to kG, then the u16 layers.
// kG: u8 layers whose labels are requested together.
template <bool kFull, int kNU8, bool kU16, bool kWide, int kRows, int kG>
__device__ __forceinline__ void area_unit(const AreaArgs &A, const Bins<kWide> &bins, const uint32_t *__restrict__ aw,
                                          const uint32_t *__restrict__ aw_hi, int64_t t0, int W, int nrows, int ncol,
                                          bool vec) {
    UnitWeights<kWide, kRows> U;
    load_weights<kFull, kWide, kRows>(aw, aw_hi, t0, W, nrows, ncol, vec, U);
    if constexpr (kNU8 > 0)
        for (int l = 0; l < A.nu8;) {
            const int g = A.nu8 - l >= kG ? kG : (A.nu8 - l >= 2 ? 2 : 1);
            if (g == kG) u8_group<kFull, kG, kWide, kRows>(A, l, bins, t0, W, nrows, ncol, vec, U);
            else if (g == 2) u8_group<kFull, 2, kWide, kRows>(A, l, bins, t0, W, nrows, ncol, vec, U);
            else u8_group<kFull, 1, kWide, kRows>(A, l, bins, t0, W, nrows, ncol, vec, U);
            l += g;
        }
    if constexpr (kU16)
        for (int l = A.nu8; l < A.nl; ++l) {
            RowLabels<uint16_t> lab[kRows];
            load_rows<kFull, uint16_t, kRows>(static_cast<const uint16_t *>(A.data[l]), t0, W, nrows, ncol, vec, lab);
            unit_runs<kFull, uint16_t, kWide, kRows>(lab, nrows, U,
                                                     [&](uint32_t lab_, const Sum<kWide> &s) { bins.add_u16(l, lab_, s); });
        }
}

// kNU8: LDS bin rows for u8 layers (>= the query's u8 layer count);
// kU16: the query has u16 layers; kWide: two-word weights.
// kBlk: one-word weights with per-block area sums (blk, ceil(W/8) per row).
template <int kNU8, bool kU16, bool kWide, int kRows, bool kBlk, int kT>
__global__ __launch_bounds__(kT) void k_area(const uint32_t *__restrict__ aw,
                                                      const uint32_t *__restrict__ aw_hi,
                                                      const unsigned long long *__restrict__ blk, int W, int H,
                                                      AreaArgs A) {
    static_assert(!kBlk || (!kWide && kRows == UVL_AREA_BLK_ROWS && kCols == UVL_AREA_BLK_COLS),
                  "a unit's lane covers one area block");
    constexpr int kBinRows = kNU8 > 0 ? (kWide ? 2 * kNU8 : kNU8) : 1;
    __shared__ unsigned long long s_bins[kBinRows * 256];
    __shared__ uint32_t s_key[kU16 ? kHash : 1];
    __shared__ unsigned long long s_val[kU16 ? (kWide ? 2 * kHash : kHash) : 1];
    if (kNU8 > 0)
        for (int k = threadIdx.x; k < kBinRows * 256; k += kT) s_bins[k] = 0ull;
    if (kU16) {
        for (int k = threadIdx.x; k < kHash; k += kT) s_key[k] = kEmptyKey;
        for (int k = threadIdx.x; k < (kWide ? 2 * kHash : kHash); k += kT) s_val[k] = 0ull;
    }
    __syncthreads();
    const Bins<kWide> bins{s_bins, kNU8, s_key, s_val, &A};
    const int lane = threadIdx.x & 63;
    const int chunks = (int)ceil_div(W, kChunk), rblocks = (int)ceil_div(H, kRows);
    const int64_t units = (int64_t)chunks * rblocks;
    constexpr int kWaves = kT / 64;
    // two u8 layers per request group at 8 waves per workgroup (several
    // workgroups per CU), four at 16 (one per CU)
    constexpr int kG = kT == 512 ? 2 : 4;
    for (int64_t u = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); u < units;
         u += (int64_t)gridDim.x * kWaves) {
        const int c = (int)(u % chunks), rb = (int)(u / chunks);
        const int col = c * kChunk + lane * kCols;
        const int ncol = W - col < kCols ? (W - col > 0 ? W - col : 0) : kCols;
        const int row0 = rb * kRows;
        const int nrows = H - row0 < kRows ? H - row0 : kRows;
        const bool vec = (W % kCols) == 0 && ncol == kCols;
        const int64_t t0 = (int64_t)row0 * W + col;
        if (ncol == 0) continue;
        if (nrows == kRows && vec) {
            if constexpr (kBlk)
                area_unit_blk<kNU8, kU16, kRows>(A, bins, aw, blk, t0, W,
                                                 (int64_t)rb * ((W + kCols - 1) / kCols) + col / kCols);
            else
                area_unit<true, kNU8, kU16, kWide, kRows, kG>(A, bins, aw, aw_hi, t0, W, nrows, ncol, vec);
        }
        else area_unit<false, kNU8, kU16, kWide, kRows, kG>(A, bins, aw, aw_hi, t0, W, nrows, ncol, vec);
    }
    __syncthreads();
    if (kNU8 > 0)
        for (int row = 0; row < A.nu8; ++row)
            for (int k = threadIdx.x; k < 256; k += kT) {
                const unsigned long long v = s_bins[row * 256 + k];
                if (v) atomicAdd(A.bins[row] + k, v);
                if constexpr (kWide) {
                    const unsigned long long h = s_bins[(kNU8 + row) * 256 + k];
                    if (h) atomicAdd(A.bins_hi[row] + k, h);
                }
            }
    if (kU16)
        for (int k = threadIdx.x; k < kHash; k += kT) {
            const uint32_t key = s_key[k];
            if (key == kEmptyKey) continue;
            const int l = (int)(key >> 16);
            const uint32_t lab = key & 0xffffu;
            if (s_val[k]) atomicAdd(A.bins[l] + lab, s_val[k]);
            if (kWide && s_val[kHash + k]) atomicAdd(A.bins_hi[l] + lab, s_val[kHash + k]);
        }
}

// Workgroups (area_threads): of 512 threads, three per CU at most (two are
// resident at the kernel's register use, the third takes up the slack of
// uneven units), or of 1024 threads, one per CU; fewer when there are few
// units.  The block-sum path keeps 1024 threads.
// blk: per-block area sums (one-word weights only), or null.
template <int kNU8, bool kU16, bool kWide>
void launch_area(hipStream_t s, const uint32_t *aw, const uint32_t *aw_hi, const unsigned long long *blk, int W,
                 int H, const AreaArgs &A) {
    constexpr int kRows = kWide ? 2 : 4;   // two-word weights: half the rows, the same registers
    const int64_t units = ceil_div(W, kChunk) * ceil_div(H, kRows);
    constexpr int kT = area_threads(kNU8, kU16, kWide);
    auto grid = [&](int threads) {
        int64_t g = ceil_div(units, (threads / 64) * 2);
        const int64_t cap = threads == 512 ? 768 : 256;
        g = g > cap ? cap : g;
        return (unsigned)(g < 1 ? 1 : g);
    };
    if constexpr (!kWide) {
        if (blk) {
            hipLaunchKernelGGL((k_area<kNU8, kU16, false, kRows, true, 1024>), dim3(grid(1024)), dim3(1024), 0, s,
                               aw, aw_hi, blk, W, H, A);
            return;
        }
    }
    hipLaunchKernelGGL((k_area<kNU8, kU16, kWide, kRows, false, kT>), dim3(grid(kT)), dim3(kT), 0, s, aw, aw_hi,
                       blk, W, H, A);
}

template <bool kWide>
void launch_by_layers(hipStream_t s, const uint32_t *aw, const uint32_t *aw_hi, const unsigned long long *blk, int W,
                      int H, const AreaArgs &A, int nu8, bool u16) {
    // bin rows rounded up to a power of two: fewer kernel instances
    if (u16) {
        if (nu8 == 0) launch_area<0, true, kWide>(s, aw, aw_hi, blk, W, H, A);
        else if (nu8 <= 1) launch_area<1, true, kWide>(s, aw, aw_hi, blk, W, H, A);
        else if (nu8 <= 4) launch_area<4, true, kWide>(s, aw, aw_hi, blk, W, H, A);
        else if (nu8 <= 8) launch_area<8, true, kWide>(s, aw, aw_hi, blk, W, H, A);
        else if (nu8 <= 16) launch_area<16, true, kWide>(s, aw, aw_hi, blk, W, H, A);
        else launch_area<(kWide ? 16 : 32), true, kWide>(s, aw, aw_hi, blk, W, H, A);
    } else {
        if (nu8 <= 1) launch_area<1, false, kWide>(s, aw, aw_hi, blk, W, H, A);
        else if (nu8 <= 4) launch_area<4, false, kWide>(s, aw, aw_hi, blk, W, H, A);
        else if (nu8 <= 8) launch_area<8, false, kWide>(s, aw, aw_hi, blk, W, H, A);
        else if (nu8 <= 16) launch_area<16, false, kWide>(s, aw, aw_hi, blk, W, H, A);
        else launch_area<(kWide ? 16 : 32), false, kWide>(s, aw, aw_hi, blk, W, H, A);
    }
}

int64_t bins_of(const uvl_layer *layers, int32_t nlayers) {
    int64_t n = 0;
    for (int l = 0; l < nlayers; ++l) n += layers[l].dtype == UVL_U8 ? 256 : 65536;
    return n;
}

}  // namespace
}  // namespace uvl

using namespace uvl;

extern "C" int64_t uvl_area_bin_count(const uvl_geom *geom, const uvl_layer *layers, int32_t nlayers) {
    if (!geom || !layers || nlayers < 1 || nlayers > kMaxLayers) return 0;
    for (int l = 0; l < nlayers; ++l)
        if (!dtype_ok(layers[l].dtype)) return 0;
    return bins_of(layers, nlayers) * (geom->area_w_hi ? 2 : 1);
}

extern "C" int32_t uvl_area_query(const uvl_geom *geom, const uvl_layer *layers, int32_t nlayers,
                                  uint64_t *bins_dev, double *areas_host, void *stream) {
    if (!geom || !layers || !bins_dev || nlayers < 1 || nlayers > kMaxLayers) return UVL_E_INVAL;
    if (!geom->area_w || !aligned16(geom->area_w) || geom->width < 1 || geom->height < 1) return UVL_E_INVAL;
    if (geom->area_w_hi && !aligned16(geom->area_w_hi)) return UVL_E_INVAL;
    if (reinterpret_cast<uintptr_t>(geom->area_blk) & 7) return UVL_E_INVAL;
    if (reinterpret_cast<uintptr_t>(bins_dev) & 7) return UVL_E_INVAL;
    for (int l = 0; l < nlayers; ++l) {
        if (!layer_ok(&layers[l])) return UVL_E_INVAL;
        if (!dtype_ok(layers[l].dtype)) return UVL_E_DTYPE;
        if (layers[l].width != geom->width || layers[l].height != geom->height) return UVL_E_SHAPE;
    }
    if (int32_t s = device_ok()) return s;
    const bool wide = geom->area_w_hi != nullptr;
    const int64_t nbins = bins_of(layers, nlayers);
    hipStream_t s = as_stream(stream);
    unsigned long long *lo = reinterpret_cast<unsigned long long *>(bins_dev);
    unsigned long long *hi = wide ? lo + nbins : nullptr;
    fill_bytes(bins_dev, nbins * 8 * (wide ? 2 : 1), s);
    const int W = geom->width, H = geom->height;
    // one launch for all layers (two-word weights: up to 16 u8 layers per
    // launch, to keep the bins within the workgroup's LDS)
    // bins of layer l start at off[l]
    std::vector<int64_t> off(nlayers);
    for (int l = 0, o = 0; l < nlayers; ++l) {
        off[l] = o;
        o += layers[l].dtype == UVL_U8 ? 256 : 65536;
    }
    // one launch for all layers, u8 layers first (two-word weights: up to
    // 16 u8 layers per launch, to keep the bins within the workgroup's LDS)
    std::vector<int> u8s, u16s;
    for (int l = 0; l < nlayers; ++l) (layers[l].dtype == UVL_U8 ? u8s : u16s).push_back(l);
    const size_t max_u8 = wide ? 16 : kMaxLayers;
    size_t i8 = 0, i16 = 0;
    while (i8 < u8s.size() || i16 < u16s.size()) {
        AreaArgs A{};
        int k = 0;
        auto put = [&](int l) {
            A.data[k] = layers[l].data;
            A.bins[k] = lo + off[l];
            A.bins_hi[k] = wide ? hi + off[l] : nullptr;
            ++k;
        };
        for (; i8 < u8s.size() && (size_t)k < max_u8; ++i8) put(u8s[i8]);
        A.nu8 = k;
        for (; i16 < u16s.size() && k < kMaxLayers; ++i16) put(u16s[i16]);
        A.nl = k;
        // block sums pay for one or two layers (a refresh of one layer's
        // bins reads a third of the bytes); with more, some layer is mixed
        // in most blocks and the weights read in mid-unit cost more than
        // reading them up front
        const unsigned long long *blk =
            A.nl <= kBlkMaxLayers ? reinterpret_cast<const unsigned long long *>(geom->area_blk) : nullptr;
        if (wide)
            launch_by_layers<true>(s, geom->area_w, geom->area_w_hi, nullptr, W, H, A, A.nu8, A.nl > A.nu8);
        else
            launch_by_layers<false>(s, geom->area_w, nullptr, blk, W, H, A, A.nu8, A.nl > A.nu8);
    }
    if (launch_status() != UVL_OK) return UVL_E_DEVICE;
    if (!areas_host) return UVL_OK;
    // bins -> fp64 on the host (synchronous form)
    const int64_t nwords = nbins * (wide ? 2 : 1);
    uint64_t *tmp = static_cast<uint64_t *>(malloc((size_t)nwords * 8));
    if (!tmp) return UVL_E_NOMEM;
    hipError_t e = hipMemcpyAsync(tmp, bins_dev, (size_t)nwords * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        for (int64_t b = 0; b < nbins; ++b) {
            // high sum * 2^32 + low sum, each below 2^62: exact in 128 bits
            const unsigned __int128 v = wide ? ((unsigned __int128)tmp[nbins + b] << 32) + tmp[b] : tmp[b];
            areas_host[b] = (double)v * geom->area_scale;
        }
    free(tmp);
    return e == hipSuccess ? UVL_OK : UVL_E_DEVICE;
}
