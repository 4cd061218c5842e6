// Batched edit waves for libuvl: many models' pending brush, lasso and
// screen-space tool edits applied by one persistent-kernel launch, and
// optionally their texture padding by one more.
//
// The paper applies one edit per rendering pass (§4.3.1).  Each edit's
// selection is a pure function of the texel's stored position, and the last
// selecting edit wins, so a layer's pending edits can be applied in one
// pass: read the positions of a tile once, evaluate the layer's edits in
// registers from the last to the first (a texel takes the label of the
// first that selects it; a wave stops once each of its texels is taken or
// uncovered), and store each texel's final label once.  The result is
// bit-identical to applying the edits one launch at a time in order.
// Numeric layers (§4.2) take the same path: their last selecting edit sets
// or clears the mask bit, their last selecting SET gives the data, so a
// texel stays open until a SET selects it.
//
// Work decomposition: edits are grouped by target layer into streams (each
// stream keeps its edits' order); a stream's atlas is cut into 32 x 32-texel
// tiles (row-major), and an item is `chunks` tiles of one stream (chunks per
// stream chosen per atlas size by the autotuner); a fixed grid of workgroups
// takes items from an atomic counter until none are left.  Every workgroup
// ends when the counter passes the item count, so the grid always drains.
// In a tile, lane t covers row t/8 and columns 4(t%8)..+3.
//
// Tile culling (when the geometry image has tile bounds): a first kernel
// gives every block of 8 x 8 tiles one wave and every tile one lane; each
// edit is tested against the block's bounds and, if it survives, against
// each tile's bounds (exact conservative tests, edit_texel.h); a lane stores,
// per group of 64 edits, the mask of edits that may select something in its
// tile and the mask of lassos whose polygon provably contains the whole tile
// (their polygon test is skipped).  Tiles with a live edit are appended to
// the stream's live list (one atomic per wave).  A one-workgroup kernel then
// turns the per-stream live counts into item ranges, and the wave kernel
// visits only live tiles, evaluating only their live edits.  Streams whose
// masks do not fit the workspace run without culling (every tile is an
// item).
//
// The descriptor (header with the region offsets, streams, per-stream
// counters, edits, lasso parameters) is packed densely on the host and
// copied host->device into the caller's workspace before each launch; the
// counter reset, the cull pass, the planning kernel and the persistent
// kernel are captured once per handle in a HIP graph and replayed.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

#include "edit_texel.h"
#include "tool_texel.h"
#include "uvl_internal.h"

namespace uvl {

bool make_lasso_params(const float view_proj[16], const float *poly, int32_t n, int32_t dw, int32_t dh,
                       float bias, LassoParams &p);

namespace {

static_assert(UVL_TILE_SIDE * UVL_TILE_SIDE == kBlock * 4, "a tile is 4 texels per thread");
constexpr int kMaxChunks = 8;
constexpr int kWaveGrid = 2048;            // persistent workgroups (256 CUs x 8)

#define UVL_CONST __attribute__((address_space(4)))

struct WaveStream {
    const float *px, *py, *pz;
    const float *box;   // per-tile position bounds, or null (no culling)
    void *layer;        // label layer, or a numeric layer's data
    uint32_t *vmask;    // a numeric layer's mask words (null for label layers)
    const int32_t *outline;  // padding: outline texel indices (null: no padding)
    int64_t out0;       // first padding index of this stream (running offset)
    int64_t nout;       // outline entries
    int64_t mask0;      // first cull-mask word of this stream (running offset)
    int64_t cwave0;     // first cull wave of this stream (one per block of 8 x 8 tiles)
    int64_t list0;      // first live-list entry of this stream
    int32_t W, H;       // atlas size
    int32_t tiles_x, ntiles;
    int32_t dtype;
    int32_t e0, ne;     // edits [e0, e0 + ne)
    int32_t chunks;     // tiles per item
    int32_t cull;       // 1: masks at mask0 (tiles x groups words), 0: no culling
    int32_t numeric;    // 1: a numeric layer (edits SET / ERASE with value bits)
    int32_t padk;       // padding radius
    int32_t nbins;      // label streams with bins: 256 (u8) or 65536 (u16)
    unsigned long long *bins;       // label layer's area bins kept up to date (null: none)
    const uint32_t *aw, *aw_hi;     // texel areas (low words; high words or null)
};

struct WaveEdit {
    int32_t kind;
    uint32_t label;     // label, or a numeric SET's value bits
    float cx, cy, cz, r2;
    int32_t lasso;      // index into the lasso (and, for tools, tool) parameter arrays
    int32_t erase;      // numeric layers: 1 for ERASE
    const float *depth;
    const uint8_t *shape;   // tools: the shape texture
};

// Byte offsets, within the workspace, of the regions of one packed wave.
struct WaveHeader {
    int32_t nstreams;
    int32_t any_bins;        // 1: some label stream keeps area bins
    int64_t total_cull_waves;
    int64_t total_items;     // written by k_wave_plan
    int64_t total_out;       // outline entries to pad, over all streams
    uint64_t off_streams, off_live_n, off_item0, off_edits, off_lassos, off_tools;
    unsigned int counter;
    unsigned int pad2[3];
};

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Offsets of the descriptor regions for ns streams, n edits, nl lassos:
// header | streams | live counts (uint32 per stream) | item starts (int64 per
// stream + 1) | edits | lassos | tools.  A tool edit takes the lasso slot
// of its index for a rectangle at its square's widened NDC range (used by
// the tile culling only) and the tool slot of the same index.
void descriptor_offsets(int64_t ns, int64_t n, int64_t nl, WaveHeader &h, size_t &end) {
    h.off_streams = 256;
    h.off_live_n = al256(h.off_streams + sizeof(WaveStream) * (size_t)ns);
    h.off_item0 = al256(h.off_live_n + sizeof(uint32_t) * (size_t)ns);
    h.off_edits = al256(h.off_item0 + sizeof(int64_t) * (size_t)(ns + 1));
    h.off_lassos = al256(h.off_edits + sizeof(WaveEdit) * (size_t)n);
    h.off_tools = al256(h.off_lassos + sizeof(LassoParams) * (size_t)nl);
    end = h.off_tools + sizeof(ToolParams) * (size_t)nl;
}

// Workspace layout: descriptor (at most `masks` bytes) | cull masks (uint64
// per word) | inside masks (uint64 per word: lassos whose polygon contains
// the whole tile) | live lists (uint32 tile index per entry, as many as words)
struct Layout {
    size_t masks, imasks, live, total;
    int64_t max_words;
};

Layout layout(int32_t max_edits, int32_t max_lassos, int64_t max_words) {
    Layout L;
    WaveHeader h;
    size_t end = 0;
    descriptor_offsets(max_edits, max_edits, max_lassos > 0 ? max_lassos : 0, h, end);
    L.masks = al256(end);
    const size_t words = (size_t)(max_words > 0 ? max_words : 1);
    L.imasks = L.masks + al256(sizeof(uint64_t) * words);
    L.live = L.imasks + al256(sizeof(uint64_t) * words);
    L.total = L.live + al256(sizeof(uint32_t) * words);
    L.max_words = max_words;
    return L;
}

__global__ void k_wave_reset(WaveHeader *h) {
    if (threadIdx.x == 0) h->counter = 0;
}

template <typename T>
__device__ __forceinline__ void wave_store(T *L, int64_t t, const uint32_t val[4], const bool wr[4],
                                           const bool in[4], bool full) {
    if (full && wr[0] && wr[1] && wr[2] && wr[3] && val[0] == val[1] && val[0] == val[2] && val[0] == val[3]) {
        if (sizeof(T) == 1) {
            *reinterpret_cast<uint32_t *>(L + t) = 0x01010101u * (val[0] & 0xffu);
        } else {
            const uint32_t v = 0x00010001u * (val[0] & 0xffffu);
            *reinterpret_cast<uint2 *>(L + t) = make_uint2(v, v);
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (wr[k] && in[k]) L[t + k] = (T)val[k];
}

// Numeric layers: value bits where the data is decided (wd), and the mask
// bits of texels whose mask is decided (wr) set (mset: a SET) or cleared (an
// ERASE).  With group_word the 8 lanes of a tile row hold one 32-texel mask
// word: they merge their bits with lane shuffles and one lane updates the
// word (every lane must be active); a full tile otherwise has 4-aligned t,
// so a lane's 4 bits share a word; partial tiles update texel by texel.
template <typename T>
__device__ __forceinline__ void wave_store_value(T *D, uint32_t *mask, int64_t t, const uint32_t val[4],
                                                 const bool wd[4], const bool wr[4], const bool mset[4],
                                                 const bool in[4], bool full, bool group_word) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (wd[k] && in[k]) D[t + k] = (T)val[k];
    if (!full) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!(wr[k] && in[k])) continue;
            const int64_t u = t + k;
            if (mset[k]) atomicOr(mask + (u >> 5), 1u << (u & 31));
            else atomicAnd(mask + (u >> 5), ~(1u << (u & 31)));
        }
        return;
    }
    uint32_t set = 0, clr = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        set |= (uint32_t)(wr[k] && mset[k]) << k;
        clr |= (uint32_t)(wr[k] && !mset[k]) << k;
    }
    set <<= (t & 31);
    clr <<= (t & 31);
    if (group_word) {
        set |= __shfl_xor(set, 1, 8);
        set |= __shfl_xor(set, 2, 8);
        set |= __shfl_xor(set, 4, 8);
        clr |= __shfl_xor(clr, 1, 8);
        clr |= __shfl_xor(clr, 2, 8);
        clr |= __shfl_xor(clr, 4, 8);
        if ((t & 31) != 0) return;
    }
    if (clr) atomicAnd(mask + (t >> 5), ~clr);
    if (set) atomicOr(mask + (t >> 5), set);
}

// Last stream s (of n) with key(s) <= v; keys are non-decreasing.
template <class F>
__device__ __forceinline__ int last_le(int n, int64_t v, F key) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (key(mid) <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Cull pass: one wave per block of 8 x 8 tiles of a culling stream (lane l:
// tile (l % 8, l / 8) of the block), grid-striding over the blocks.  Each
// edit is first tested against the block's bounds (the union of its tiles'
// bounds, contains every texel of the block, stored by the geometry build
// after the tile bounds); only edits that survive that are tested per tile,
// and a block no edit survives reads no tile bounds at all.  A lane's masks (one word per group of 64 edits) go
// to masks[mask0 + tile * groups + g] -- with one group, only for live tiles,
// the only ones the wave kernel reads -- and the wave's tiles with a live
// edit are appended to the stream's live list.
__global__ __launch_bounds__(kBlock) void k_wave_cull(char *__restrict__ ws, uint64_t *__restrict__ masks,
                                                       uint64_t *__restrict__ imasks, uint32_t *__restrict__ live) {
    const UVL_CONST WaveHeader *hdr = (const UVL_CONST WaveHeader *)ws;
    const UVL_CONST WaveStream *streams = (const UVL_CONST WaveStream *)(ws + hdr->off_streams);
    const UVL_CONST WaveEdit *edits = (const UVL_CONST WaveEdit *)(ws + hdr->off_edits);
    const UVL_CONST LassoParams *lassos = (const UVL_CONST LassoParams *)(ws + hdr->off_lassos);
    uint32_t *live_n = reinterpret_cast<uint32_t *>(ws + hdr->off_live_n);
    const int32_t nstreams = hdr->nstreams;
    const int64_t total = hdr->total_cull_waves;
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t cw = wave0; cw < total; cw += nwaves) {
        // streams without culling own no cull waves and every culling stream
        // owns at least one, so this is the culling stream owning the wave
        const int si = last_le(nstreams, cw, [&](int k) { return streams[k].cwave0; });
        const UVL_CONST WaveStream &S = streams[si];
        const int groups = (S.ne + 63) >> 6;
        const int tiles_y = S.ntiles / S.tiles_x;
        const int64_t blk = cw - S.cwave0;
        const int nbx = (S.tiles_x + UVL_TILE_BLOCK - 1) / UVL_TILE_BLOCK;
        const int tx = (int)(blk % nbx) * UVL_TILE_BLOCK + (lane % UVL_TILE_BLOCK);
        const int ty = (int)(blk / nbx) * UVL_TILE_BLOCK + (lane / UVL_TILE_BLOCK);
        const bool in = tx < S.tiles_x && ty < tiles_y;
        const int64_t ti = (int64_t)ty * S.tiles_x + tx;
        // the block's bounds, stored after the tiles' by the geometry build
        // (wave-uniform: scalar loads)
        float bb[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) bb[q] = S.box[6 * ((int64_t)S.ntiles + blk) + q];
        // the lane's tile bounds, read once some edit survives the block test
        float box[6];
        bool have_box = false;
        bool any = false;
        for (int g = 0; g < groups; ++g) {
            uint64_t m = 0, im = 0;
            const int lim = S.ne - 64 * g < 64 ? S.ne - 64 * g : 64;
            // block test (the same for every lane) ...
            uint64_t alive = 0;
            for (int k = 0; k < lim; ++k) {
                const UVL_CONST WaveEdit &E = edits[S.e0 + 64 * g + k];
                const bool brush = E.kind == UVL_EDIT_BRUSH;
                const BrushParams B{E.cx, E.cy, E.cz, E.r2};
                const bool block_dead = brush ? brush_culls(B, bb)
                                              : lasso_tile(lassos[E.lasso], bb, E.depth) == kTileCulled;
                alive |= (uint64_t)!block_dead << k;
            }
            // ... then the lane's tile, for the edits that survive it
            if (alive && !have_box) {
#pragma unroll
                for (int q = 0; q < 6; ++q) box[q] = in ? S.box[6 * ti + q] : (q < 3 ? INFINITY : -INFINITY);
                have_box = true;
            }
            for (uint64_t a = alive; a; a &= a - 1) {
                const int k = __builtin_ctzll(a);
                const UVL_CONST WaveEdit &E = edits[S.e0 + 64 * g + k];
                const bool brush = E.kind == UVL_EDIT_BRUSH;
                const BrushParams B{E.cx, E.cy, E.cz, E.r2};
                const int cls = brush ? (brush_culls(B, box) ? kTileCulled : kTileLive)
                                      : lasso_tile(lassos[E.lasso], box, E.depth);
                m |= (uint64_t)(cls != kTileCulled) << k;
                // a tool's shape can still exclude texels of a tile inside its square
                im |= (uint64_t)(cls == kTileInside && E.kind == UVL_EDIT_LASSO) << k;
            }
            if (in && (groups > 1 || m != 0)) {
                masks[S.mask0 + ti * groups + g] = m;
                imasks[S.mask0 + ti * groups + g] = im;
            }
            any = any || m != 0;
        }
        const uint64_t b = __ballot(any && in);
        if (b) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(live_n + si, (uint32_t)__popcll(b));
            base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
            if (any && in) {
                const uint32_t rank = (uint32_t)__popcll(b & ((1ull << lane) - 1));
                live[S.list0 + base + rank] = (uint32_t)ti;
            }
        }
    }
}

// Item ranges: stream s owns items [item0[s], item0[s + 1]), ceil(tiles /
// chunks) of them, tiles being its live-list length (culling streams) or all
// its tiles.  One workgroup: a per-thread serial range, then a block scan.
__global__ __launch_bounds__(kBlock) void k_wave_plan(char *__restrict__ ws) {
    WaveHeader *hdr = reinterpret_cast<WaveHeader *>(ws);
    const WaveStream *streams = reinterpret_cast<const WaveStream *>(ws + hdr->off_streams);
    const uint32_t *live_n = reinterpret_cast<const uint32_t *>(ws + hdr->off_live_n);
    int64_t *item0 = reinterpret_cast<int64_t *>(ws + hdr->off_item0);
    const int n = hdr->nstreams;
    const int per = (n + kBlock - 1) / kBlock;
    const int a = threadIdx.x * per, b = a + per < n ? a + per : n;
    auto items = [&](int k) {
        const WaveStream &S = streams[k];
        const int64_t tiles = S.cull ? (int64_t)live_n[k] : (int64_t)S.ntiles;
        return (tiles + S.chunks - 1) / S.chunks;
    };
    int64_t sum = 0;
    for (int k = a; k < b; ++k) sum += items(k);
    __shared__ int64_t part[kBlock];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < kBlock; d <<= 1) {
        const int64_t v = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = part[threadIdx.x] - sum;   // exclusive prefix
    for (int k = a; k < b; ++k) {
        item0[k] = run;
        run += items(k);
    }
    if (threadIdx.x == kBlock - 1) {
        item0[n] = part[kBlock - 1];
        hdr->total_items = part[kBlock - 1];
    }
}

// Area bins kept up to date by a label stream: every texel whose label the
// wave changes moves its area from the old label's bin to the new one's.
// The lanes of a wave settle one (old, new) pair at a time -- the pair of the
// first lane with a pending change -- summing the area of all texels with
// that pair and adding it with one pair of atomics (the bins are unsigned,
// a subtraction wraps and the exact totals come out).  A wave's texels
// usually share one or two pairs.  Control flow is uniform over the wave.
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned lo = __shfl_xor((unsigned)x, o), hi = __shfl_xor((unsigned)(x >> 32), o);
        x += ((unsigned long long)hi << 32) | lo;
    }
    return x;
}

// The workgroup's area changes, keyed by (stream, label), in LDS: added to
// the streams' bins once, when the persistent workgroup ends, so that the
// many tiles of an edit do not all hit the same two global bins.
constexpr int kBinSlots = 512;
constexpr uint32_t kNoBinKey = 0xffffffffu;

struct BinTable {
    uint32_t *key;
    unsigned long long *lo, *hi;

    __device__ __forceinline__ void add(const UVL_CONST WaveStream &S, int si, uint32_t label, unsigned long long dl,
                                        unsigned long long dh) const {
        const uint32_t k = ((uint32_t)si << 16) | label;
        uint32_t h = (k * 2654435761u) >> 23;         // 9 bits: kBinSlots
        for (int probe = 0; probe < 8 && si < 65535; ++probe) {
            const uint32_t prev = atomicCAS(key + h, kNoBinKey, k);
            if (prev == kNoBinKey || prev == k) {
                atomicAdd(lo + h, dl);
                if (S.aw_hi) atomicAdd(hi + h, dh);
                return;
            }
            h = (h + 1) & (kBinSlots - 1);
        }
        atomicAdd(S.bins + label, dl);
        if (S.aw_hi) atomicAdd(S.bins + S.nbins + label, dh);
    }
};

template <typename Lab>
__device__ __forceinline__ void wave_bins(const UVL_CONST WaveStream &S, int si, const BinTable &tab, int64_t t,
                                          const uint32_t val[4], const bool wr[4], const bool in[4],
                                          const bool cov[4], bool full) {
    const Lab *L = static_cast<const Lab *>(S.layer);
    bool ch[4];
    uint32_t old[4] = {0, 0, 0, 0};
    unsigned long long wl[4] = {0, 0, 0, 0}, wh[4] = {0, 0, 0, 0};
    const bool any = (wr[0] && cov[0]) || (wr[1] && cov[1]) || (wr[2] && cov[2]) || (wr[3] && cov[3]);
    if (any) {
        if (full) {
            if (sizeof(Lab) == 1) {
                const uint32_t v = *reinterpret_cast<const uint32_t *>(L + t);
#pragma unroll
                for (int k = 0; k < 4; ++k) old[k] = (v >> (8 * k)) & 0xffu;
            } else {
                const uint2 v = *reinterpret_cast<const uint2 *>(L + t);
                old[0] = v.x & 0xffffu; old[1] = v.x >> 16; old[2] = v.y & 0xffffu; old[3] = v.y >> 16;
            }
            const uint4 w = *reinterpret_cast<const uint4 *>(S.aw + t);
            wl[0] = w.x; wl[1] = w.y; wl[2] = w.z; wl[3] = w.w;
            if (S.aw_hi) {
                const uint4 h = *reinterpret_cast<const uint4 *>(S.aw_hi + t);
                wh[0] = h.x; wh[1] = h.y; wh[2] = h.z; wh[3] = h.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (in[k]) {
                    old[k] = L[t + k];
                    wl[k] = S.aw[t + k];
                    if (S.aw_hi) wh[k] = S.aw_hi[t + k];
                }
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) ch[k] = wr[k] && in[k] && cov[k] && old[k] != val[k] && (wl[k] | wh[k]) != 0;
    for (;;) {
        const bool have = ch[0] || ch[1] || ch[2] || ch[3];
        const unsigned long long lanes = __builtin_amdgcn_ballot_w64(have);
        if (lanes == 0) break;
        uint32_t key = 0;
#pragma unroll
        for (int k = 3; k >= 0; --k)
            if (ch[k]) key = (old[k] << 16) | val[k];
        const uint32_t lead = __shfl(key, __builtin_ctzll(lanes));
        unsigned long long sl = 0, sh = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (ch[k] && ((old[k] << 16) | val[k]) == lead) {
                sl += wl[k];
                sh += wh[k];
                ch[k] = false;
            }
        sl = wave_sum_u64(sl);
        sh = wave_sum_u64(sh);
        if ((threadIdx.x & 63) == 0) {
            const uint32_t o = lead >> 16, v = lead & 0xffffu;
            tab.add(S, si, o, ~sl + 1ull, ~sh + 1ull);
            tab.add(S, si, v, sl, sh);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_wave(char *__restrict__ ws, const uint64_t *__restrict__ masks_in,
                                                  const uint64_t *__restrict__ imasks_in,
                                                  const uint32_t *__restrict__ live_in) {
    // read-only descriptor, masks and live lists viewed in the constant
    // address space: uniform reads become scalar loads
    WaveHeader *hdr = reinterpret_cast<WaveHeader *>(ws);
    const UVL_CONST WaveHeader *chdr = (const UVL_CONST WaveHeader *)ws;
    const UVL_CONST WaveStream *streams = (const UVL_CONST WaveStream *)(ws + chdr->off_streams);
    const UVL_CONST WaveEdit *edits = (const UVL_CONST WaveEdit *)(ws + chdr->off_edits);
    const UVL_CONST LassoParams *lassos = (const UVL_CONST LassoParams *)(ws + chdr->off_lassos);
    const UVL_CONST ToolParams *tools = (const UVL_CONST ToolParams *)(ws + chdr->off_tools);
    const UVL_CONST uint32_t *live_n = (const UVL_CONST uint32_t *)(ws + chdr->off_live_n);
    const UVL_CONST int64_t *item0 = (const UVL_CONST int64_t *)(ws + chdr->off_item0);
    const UVL_CONST uint64_t *masks = (const UVL_CONST uint64_t *)masks_in;
    const UVL_CONST uint64_t *imasks = (const UVL_CONST uint64_t *)imasks_in;
    const UVL_CONST uint32_t *live = (const UVL_CONST uint32_t *)live_in;
    __shared__ long long s_item;
    __shared__ uint32_t s_bkey[kBinSlots];
    __shared__ unsigned long long s_blo[kBinSlots], s_bhi[kBinSlots];
    const bool any_bins = chdr->any_bins != 0;
    if (any_bins)
        for (int k = threadIdx.x; k < kBinSlots; k += kBlock) {
            s_bkey[k] = kNoBinKey;
            s_blo[k] = s_bhi[k] = 0ull;
        }
    const BinTable tab{s_bkey, s_blo, s_bhi};
    const int32_t nstreams = chdr->nstreams;
    const int64_t total = chdr->total_items;
    const int trow = threadIdx.x >> 3, tcol = (threadIdx.x & 7) * 4;
    for (;;) {
        if (threadIdx.x == 0) s_item = (long long)atomicAdd(&hdr->counter, 1u);
        __syncthreads();
        const int64_t item = s_item;
        __syncthreads();
        if (item >= total) break;
        // stream holding the item (streams owning no items share their
        // start with the next stream, which is found instead)
        const int si = last_le(nstreams, item, [&](int k) { return item0[k]; });
        const UVL_CONST WaveStream &S = streams[si];
        const int chunks = S.chunks, W = S.W, H = S.H;
        const int groups = (S.ne + 63) >> 6;
        const bool cull = S.cull != 0;
        const int64_t first = (item - item0[si]) * (int64_t)chunks;
        const int64_t ntiles = cull ? (int64_t)live_n[si] : (int64_t)S.ntiles;
        for (int c = 0; c < chunks; ++c) {
            if (first + c >= ntiles) break;
            const int64_t ti = cull ? (int64_t)live[S.list0 + first + c] : first + c;
            const UVL_CONST uint64_t *tm = masks + (cull ? S.mask0 + ti * groups : 0);
            const UVL_CONST uint64_t *tim = imasks + (cull ? S.mask0 + ti * groups : 0);
            const int tx = (int)(ti % S.tiles_x), ty = (int)(ti / S.tiles_x);
            // uniform over the workgroup: whole tile inside, rows 16-byte aligned
            const bool full = (tx + 1) * UVL_TILE_SIDE <= W && (ty + 1) * UVL_TILE_SIDE <= H && (W & 3) == 0;
            const int i = tx * UVL_TILE_SIDE + tcol, j = ty * UVL_TILE_SIDE + trow;
            const int64_t t = (int64_t)j * W + i;
            bool in[4];
            float4 X, Y, Z;
            if (full) {
                in[0] = in[1] = in[2] = in[3] = true;
                X = load_stream4(S.px + t);
                Y = load_stream4(S.py + t);
                Z = load_stream4(S.pz + t);
            } else {
                const float nan = __builtin_nanf("");
                float xs[4], ys[4], zs[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    in[k] = i + k < W && j < H;
                    xs[k] = in[k] ? S.px[t + k] : nan;
                    ys[k] = in[k] ? S.py[t + k] : nan;
                    zs[k] = in[k] ? S.pz[t + k] : nan;
                }
                X = make_float4(xs[0], xs[1], xs[2], xs[3]);
                Y = make_float4(ys[0], ys[1], ys[2], ys[3]);
                Z = make_float4(zs[0], zs[1], zs[2], zs[3]);
            }
            // live edits from the last to the first: a texel takes the
            // label of the first edit (in this order) that selects it, i.e.
            // of its last selecting edit, and a wave stops once each of its
            // texels is taken or uncovered (NaN position).  In a numeric
            // layer that edit decides the mask bit (SET: valid, ERASE:
            // invalid), while the data is the value of the last selecting
            // SET, so a texel stays open until a SET selects it.
            const bool cov[4] = {X.x == X.x, X.y == X.y, X.z == X.z, X.w == X.w};
            auto tile = [&](auto numeric_tag) {
                constexpr bool kNum = decltype(numeric_tag)::value;
                uint32_t val[4] = {0, 0, 0, 0};
                bool wr[4] = {false, false, false, false};
                bool wd[4] = {false, false, false, false}, mset[4] = {false, false, false, false};
                bool open = true;
                for (int g = groups - 1; g >= 0 && open; --g) {
                    uint64_t lm = cull ? tm[g] : ~0ull;
                    const uint64_t ins = cull ? tim[g] : 0ull;   // lassos containing the whole tile
                    const int base = g * 64;
                    const int lim = S.ne - base < 64 ? S.ne - base : 64;
                    if (lim < 64) lm &= (1ull << lim) - 1;
                    while (lm) {
                        const int b = 63 - __builtin_clzll(lm);
                        lm &= ~(1ull << b);
                        const UVL_CONST WaveEdit &E = edits[S.e0 + base + b];
                        bool sel[4];
                        if (E.kind == UVL_EDIT_BRUSH) {
                            const BrushParams B{E.cx, E.cy, E.cz, E.r2};
                            sel[0] = brush_texel(B, X.x, Y.x, Z.x);
                            sel[1] = brush_texel(B, X.y, Y.y, Z.y);
                            sel[2] = brush_texel(B, X.z, Y.z, Z.z);
                            sel[3] = brush_texel(B, X.w, Y.w, Z.w);
                        } else if (E.kind == UVL_EDIT_LASSO) {
                            lasso_quad(lassos[E.lasso], E.depth, X, Y, Z, sel, ((ins >> b) & 1) != 0);
                        } else {
                            const UVL_CONST ToolParams &T = tools[E.lasso];
                            sel[0] = tool_texel(T, E.shape, E.depth, X.x, Y.x, Z.x);
                            sel[1] = tool_texel(T, E.shape, E.depth, X.y, Y.y, Z.y);
                            sel[2] = tool_texel(T, E.shape, E.depth, X.z, Y.z, Z.z);
                            sel[3] = tool_texel(T, E.shape, E.depth, X.w, Y.w, Z.w);
                        }
                        bool pending = false;
                        if constexpr (kNum) {
                            const bool set = E.erase == 0;
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                mset[k] = sel[k] && !wr[k] ? set : mset[k];
                                wr[k] = wr[k] || sel[k];
                                val[k] = sel[k] && set && !wd[k] ? E.label : val[k];
                                wd[k] = wd[k] || (sel[k] && set);
                                pending = pending || (cov[k] && !wd[k]);
                            }
                        } else {
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                val[k] = sel[k] && !wr[k] ? E.label : val[k];
                                wr[k] = wr[k] || sel[k];
                                pending = pending || (cov[k] && !wr[k]);
                            }
                        }
                        if (__builtin_amdgcn_ballot_w64(pending) == 0) {
                            open = false;
                            break;
                        }
                    }
                }
                if constexpr (kNum) {
                    const bool group_word = full && (W & 31) == 0;
                    if (S.dtype == UVL_U8)
                        wave_store_value<uint8_t>(static_cast<uint8_t *>(S.layer), S.vmask, t, val, wd, wr, mset, in,
                                                  full, group_word);
                    else if (S.dtype == UVL_U16 || S.dtype == UVL_F16)
                        wave_store_value<uint16_t>(static_cast<uint16_t *>(S.layer), S.vmask, t, val, wd, wr, mset,
                                                   in, full, group_word);
                    else
                        wave_store_value<uint32_t>(static_cast<uint32_t *>(S.layer), S.vmask, t, val, wd, wr, mset,
                                                   in, full, group_word);
                } else {
                    if (S.bins) {
                        if (S.dtype == UVL_U8) wave_bins<uint8_t>(S, si, tab, t, val, wr, in, cov, full);
                        else wave_bins<uint16_t>(S, si, tab, t, val, wr, in, cov, full);
                    }
                    if (S.dtype == UVL_U8) wave_store<uint8_t>(static_cast<uint8_t *>(S.layer), t, val, wr, in, full);
                    else wave_store<uint16_t>(static_cast<uint16_t *>(S.layer), t, val, wr, in, full);
                }
            };
            if (S.numeric) tile(std::true_type{});
            else tile(std::false_type{});
        }
    }
    // the workgroup's area changes to the streams' bins
    if (any_bins) {
        __syncthreads();
        for (int k = threadIdx.x; k < kBinSlots; k += kBlock) {
            const uint32_t key = s_bkey[k];
            if (key == kNoBinKey) continue;
            const UVL_CONST WaveStream &S = streams[key >> 16];
            const uint32_t label = key & 0xffffu;
            if (s_blo[k]) atomicAdd(S.bins + label, s_blo[k]);
            if (S.aw_hi && s_bhi[k]) atomicAdd(S.bins + S.nbins + label, s_bhi[k]);
        }
    }
}

// Padding after a wave (§4.3.2): a lane per outline entry, over all streams
// with an outline.  The outline texel takes the decision of the last edit
// that selects a covered texel of its (2k+1)^2 window: its label, or in a
// numeric layer its mask bit (SET / ERASE) and, from the last such SET, its
// data.  Candidate edits are those live in the tiles the window touches
// (every edit without culling); mask words of tiles the cull pass found dead
// may be stale, which only adds candidates, each evaluated exactly.
constexpr int kPadGrid = 1024;
constexpr int kMaxPadRadius = 8;

__global__ __launch_bounds__(kBlock) void k_wave_pad(char *__restrict__ ws, const uint64_t *__restrict__ masks_in) {
    const UVL_CONST WaveHeader *chdr = (const UVL_CONST WaveHeader *)ws;
    const UVL_CONST WaveStream *streams = (const UVL_CONST WaveStream *)(ws + chdr->off_streams);
    const UVL_CONST WaveEdit *edits = (const UVL_CONST WaveEdit *)(ws + chdr->off_edits);
    const UVL_CONST LassoParams *lassos = (const UVL_CONST LassoParams *)(ws + chdr->off_lassos);
    const UVL_CONST ToolParams *tools = (const UVL_CONST ToolParams *)(ws + chdr->off_tools);
    const int32_t nstreams = chdr->nstreams;
    const int64_t total = chdr->total_out;
    for (int64_t gi = (int64_t)blockIdx.x * kBlock + threadIdx.x; gi < total; gi += (int64_t)gridDim.x * kBlock) {
        const int si = last_le(nstreams, gi, [&](int k) { return streams[k].out0; });
        const UVL_CONST WaveStream &S = streams[si];
        const int32_t t = S.outline[gi - S.out0];
        const int W = S.W, H = S.H, k = S.padk;
        if (t < 0 || (int64_t)t >= (int64_t)W * H) continue;   // not a texel index: ignored
        const int i = t % W, j = t / W;
        const int u0 = i - k < 0 ? 0 : i - k, u1 = i + k > W - 1 ? W - 1 : i + k;
        const int v0 = j - k < 0 ? 0 : j - k, v1 = j + k > H - 1 ? H - 1 : j + k;
        const int groups = (S.ne + 63) >> 6;
        const int tx0 = u0 / UVL_TILE_SIDE, tx1 = u1 / UVL_TILE_SIDE;
        const int ty0 = v0 / UVL_TILE_SIDE, ty1 = v1 / UVL_TILE_SIDE;
        bool wr = false, wd = false, mset = false;
        uint32_t val = 0;
        for (int g = groups - 1; g >= 0 && !wd; --g) {
            uint64_t lm = S.cull ? 0ull : ~0ull;
            if (S.cull)
                for (int ty = ty0; ty <= ty1; ++ty)
                    for (int tx = tx0; tx <= tx1; ++tx)
                        lm |= masks_in[S.mask0 + ((int64_t)ty * S.tiles_x + tx) * groups + g];
            const int lim = S.ne - 64 * g < 64 ? S.ne - 64 * g : 64;
            if (lim < 64) lm &= (1ull << lim) - 1;
            while (lm && !wd) {
                const int b = 63 - __builtin_clzll(lm);
                lm &= ~(1ull << b);
                const UVL_CONST WaveEdit &E = edits[S.e0 + 64 * g + b];
                bool hit = false;
                for (int v = v0; v <= v1 && !hit; ++v)
                    for (int u = u0; u <= u1; ++u) {
                        const int64_t q = (int64_t)v * W + u;
                        const float x = S.px[q];
                        if (x != x) continue;   // uncovered (NaN position): never edited
                        const float y = S.py[q], z = S.pz[q];
                        if (E.kind == UVL_EDIT_BRUSH) hit = brush_texel(BrushParams{E.cx, E.cy, E.cz, E.r2}, x, y, z);
                        else if (E.kind == UVL_EDIT_LASSO) hit = lasso_texel(lassos[E.lasso], E.depth, x, y, z);
                        else hit = tool_texel(tools[E.lasso], E.shape, E.depth, x, y, z);
                        if (hit) break;
                    }
                if (!hit) continue;
                if (!S.numeric) {
                    val = E.label;
                    wr = wd = true;
                } else {
                    const bool set = E.erase == 0;
                    if (!wr) {
                        wr = true;
                        mset = set;
                    }
                    if (set) {
                        wd = true;
                        val = E.label;
                    }
                }
            }
        }
        if (!S.numeric) {
            if (!wr) continue;
            if (S.dtype == UVL_U8) static_cast<uint8_t *>(S.layer)[t] = (uint8_t)val;
            else static_cast<uint16_t *>(S.layer)[t] = (uint16_t)val;
            continue;
        }
        if (wd) {
            if (S.dtype == UVL_U8) static_cast<uint8_t *>(S.layer)[t] = (uint8_t)val;
            else if (S.dtype == UVL_U16 || S.dtype == UVL_F16) static_cast<uint16_t *>(S.layer)[t] = (uint16_t)val;
            else static_cast<uint32_t *>(S.layer)[t] = val;
        }
        if (wr) {
            if (mset) atomicOr(S.vmask + (t >> 5), 1u << (t & 31));
            else atomicAnd(S.vmask + (t >> 5), ~(1u << (t & 31)));
        }
    }
}

}  // namespace
}  // namespace uvl

using namespace uvl;

constexpr int kStaging = 4;   // pinned descriptor buffers in rotation

struct uvl_wave {
    int32_t max_edits, max_lassos;
    char *ws;              // device workspace
    size_t ws_bytes;
    Layout lay;
    char *staging;         // pinned host copy of the descriptor being packed
    char *ring[kStaging];  // pinned buffers; ring[k] is free once copied[k] has fired
    hipEvent_t copied[kStaging];
    bool pending[kStaging];
    int next;
    hipStream_t cap;       // private stream for graph capture
    hipGraphExec_t exec;
    std::mutex mu;
    int32_t tuned_chunks[32];   // per log2(texels); 0 = not tuned
};

extern "C" size_t uvl_wave_workspace_bytes(int32_t max_edits, int32_t max_lassos, int64_t max_cull_words) {
    if (max_edits < 1 || max_lassos < 0 || max_cull_words < 0) return 0;
    return layout(max_edits, max_lassos, max_cull_words).total;
}

extern "C" int32_t uvl_wave_create(int32_t max_edits, int32_t max_lassos, int64_t max_cull_words, void *ws,
                                   size_t ws_bytes, uvl_wave **out) {
    if (!out || !ws || max_edits < 1 || max_edits > (1 << 20) || max_lassos < 0 || max_lassos > max_edits ||
        max_cull_words < 0)
        return UVL_E_INVAL;
    *out = nullptr;
    const Layout lay = layout(max_edits, max_lassos, max_cull_words);
    if (ws_bytes < lay.total) return UVL_E_NOMEM;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return UVL_E_INVAL;
    if (int32_t s = device_ok()) return s;
    uvl_wave *w = new uvl_wave();
    w->max_edits = max_edits;
    w->max_lassos = max_lassos;
    w->ws = static_cast<char *>(ws);
    w->ws_bytes = ws_bytes;
    w->lay = lay;
    w->staging = nullptr;
    w->next = 0;
    w->exec = nullptr;
    for (int k = 0; k < 32; ++k) w->tuned_chunks[k] = 0;
    bool ok = true;
    for (int k = 0; k < kStaging && ok; ++k) {
        w->pending[k] = false;
        ok = hipHostMalloc(reinterpret_cast<void **>(&w->ring[k]), lay.masks, hipHostMallocDefault) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&w->copied[k], hipEventDisableTiming) == hipSuccess;
    }
    ok = ok && hipStreamCreateWithFlags(&w->cap, hipStreamNonBlocking) == hipSuccess;
    if (ok) {
        // capture reset + cull masks + persistent kernel once; the
        // descriptor is data
        hipGraph_t g = nullptr;
        WaveHeader *hdr = reinterpret_cast<WaveHeader *>(w->ws);
        uint64_t *masks = reinterpret_cast<uint64_t *>(w->ws + lay.masks);
        uint64_t *imasks = reinterpret_cast<uint64_t *>(w->ws + lay.imasks);
        uint32_t *live = reinterpret_cast<uint32_t *>(w->ws + lay.live);
        ok = hipStreamBeginCapture(w->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            hipLaunchKernelGGL(k_wave_reset, dim3(1), dim3(64), 0, w->cap, hdr);
            hipLaunchKernelGGL(k_wave_cull, dim3(kWaveGrid), dim3(kBlock), 0, w->cap, w->ws, masks, imasks, live);
            hipLaunchKernelGGL(k_wave_plan, dim3(1), dim3(kBlock), 0, w->cap, w->ws);
            hipLaunchKernelGGL(k_wave, dim3(kWaveGrid), dim3(kBlock), 0, w->cap, w->ws, masks, imasks, live);
            ok = hipStreamEndCapture(w->cap, &g) == hipSuccess && g;
        }
        ok = ok && hipGraphInstantiate(&w->exec, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
    }
    if (!ok) {
        uvl_wave_destroy(w);
        return UVL_E_DEVICE;
    }
    *out = w;
    return UVL_OK;
}

extern "C" int32_t uvl_wave_destroy(uvl_wave *w) {
    if (!w) return UVL_E_INVAL;
    for (int k = 0; k < kStaging; ++k) {
        if (w->pending[k]) (void)hipEventSynchronize(w->copied[k]);
        if (w->copied[k]) (void)hipEventDestroy(w->copied[k]);
        if (w->ring[k]) (void)hipHostFree(w->ring[k]);
    }
    if (w->exec) (void)hipGraphExecDestroy(w->exec);
    if (w->cap) (void)hipStreamDestroy(w->cap);
    delete w;
    return UVL_OK;
}

namespace {

int log2_class(int64_t n) {
    int c = 0;
    while ((1LL << (c + 1)) <= n && c < 31) ++c;
    return c;
}

// Validate and pack a wave into the staging buffer.  chunks_override > 0
// forces that tile size for every stream.
int32_t pack(uvl_wave *w, const uvl_edit *edits, int32_t n, int32_t chunks_override, const uvl_wave_outline *outlines,
             int32_t noutlines, size_t &bytes) {
    // streams: one per distinct layer, in order of first appearance
    std::vector<int32_t> stream_of(n);
    std::vector<const void *> keys;
    std::vector<std::vector<int32_t>> members;
    std::vector<uint32_t> bits(n, 0);       // label, or a numeric SET's value bits
    int32_t nl = 0;
    for (int32_t i = 0; i < n; ++i) {
        const uvl_edit &e = edits[i];
        const bool num = e.numeric != nullptr;
        if (!e.geom || num == (e.layer != nullptr)) return UVL_E_INVAL;   // exactly one target
        if (!geom_pos_ok(e.geom)) return UVL_E_INVAL;
        if (num) {
            if (!numeric_ok(e.numeric) || (e.mode != UVL_SET && e.mode != UVL_ERASE)) return UVL_E_INVAL;
            if (e.mode == UVL_SET)
                if (int32_t st = encode_value(e.numeric->dtype, e.value, bits[i])) return st;
        } else {
            if (!layer_ok(e.layer)) return UVL_E_INVAL;
            if (!dtype_ok(e.layer->dtype)) return UVL_E_DTYPE;
            if (e.label > dtype_max(e.layer->dtype)) return UVL_E_DTYPE;
            bits[i] = e.label;
        }
        const int32_t tw = num ? e.numeric->width : e.layer->width, th = num ? e.numeric->height : e.layer->height;
        const int32_t tdt = num ? e.numeric->dtype : e.layer->dtype;
        const void *target = num ? e.numeric->data : e.layer->data;
        if (tw != e.geom->width || th != e.geom->height) return UVL_E_SHAPE;
        if (e.bins && (num || !e.geom->area_w || !aligned16(e.geom->area_w) ||
                       (e.geom->area_w_hi && !aligned16(e.geom->area_w_hi)) ||
                       (reinterpret_cast<uintptr_t>(e.bins) & 7)))
            return UVL_E_INVAL;
        if (e.kind == UVL_EDIT_BRUSH) {
            if (!(e.radius >= 0.0f) || !std::isfinite(e.radius)) return UVL_E_INVAL;
            if (!std::isfinite(e.center[0]) || !std::isfinite(e.center[1]) || !std::isfinite(e.center[2]))
                return UVL_E_INVAL;
        } else if (e.kind == UVL_EDIT_LASSO || e.kind == UVL_EDIT_TOOL) {
            if (!e.depth || !e.view_proj || e.dw > kMaxDepthSide || e.dh > kMaxDepthSide) return UVL_E_INVAL;
            if (e.kind == UVL_EDIT_TOOL && (!e.tool || !e.shape)) return UVL_E_INVAL;
            if (++nl > w->max_lassos) return UVL_E_NOMEM;
        } else {
            return UVL_E_INVAL;
        }
        size_t k = 0;
        while (k < keys.size() && keys[k] != target) ++k;
        if (k == keys.size()) {
            keys.push_back(target);
            members.emplace_back();
        } else {
            // every edit of one layer must read the same positions and
            // describe the layer alike
            const uvl_edit &f = edits[members[k][0]];
            const bool fnum = f.numeric != nullptr;
            if (f.geom->pos_x != e.geom->pos_x || fnum != num || f.geom->width != tw || f.geom->height != th ||
                (fnum ? f.numeric->dtype != tdt || f.numeric->mask != e.numeric->mask : f.layer->dtype != tdt) ||
                f.bins != e.bins)
                return UVL_E_INVAL;
        }
        members[k].push_back(i);
    }
    char *st = w->staging;
    WaveHeader *hdr = reinterpret_cast<WaveHeader *>(st);
    size_t end = 0;
    descriptor_offsets((int64_t)keys.size(), n, nl, *hdr, end);
    WaveStream *S = reinterpret_cast<WaveStream *>(st + hdr->off_streams);
    uint32_t *live_n = reinterpret_cast<uint32_t *>(st + hdr->off_live_n);
    WaveEdit *E = reinterpret_cast<WaveEdit *>(st + hdr->off_edits);
    LassoParams *P = reinterpret_cast<LassoParams *>(st + hdr->off_lassos);
    ToolParams *TP = reinterpret_cast<ToolParams *>(st + hdr->off_tools);
    int64_t words = 0, cwaves = 0, nout_total = 0;
    int32_t ei = 0, li = 0;
    for (size_t k = 0; k < keys.size(); ++k) {
        const uvl_edit &f = edits[members[k][0]];
        WaveStream &s = S[k];
        s.px = f.geom->pos_x;
        s.py = f.geom->pos_y;
        s.pz = f.geom->pos_z;
        s.box = f.geom->tile_box;
        s.numeric = f.numeric ? 1 : 0;
        s.layer = f.numeric ? f.numeric->data : f.layer->data;
        s.vmask = f.numeric ? f.numeric->mask : nullptr;
        s.W = f.geom->width;
        s.H = f.geom->height;
        s.tiles_x = (int32_t)ceil_div(s.W, UVL_TILE_SIDE);
        s.ntiles = s.tiles_x * (int32_t)ceil_div(s.H, UVL_TILE_SIDE);
        s.dtype = f.numeric ? f.numeric->dtype : f.layer->dtype;
        int ch = chunks_override > 0 ? chunks_override : w->tuned_chunks[log2_class((int64_t)s.W * s.H)];
        if (ch <= 0) ch = 4;
        s.chunks = std::min(std::max(ch, 1), kMaxChunks);
        // cull masks (tiles x groups words) and the live list (up to one
        // entry per tile, fewer than the words) if the geometry has tile
        // bounds and the words fit
        const int64_t nw = (int64_t)s.ntiles * ((int64_t)(members[k].size() + 63) / 64);
        s.cull = (f.geom->tile_box && words + nw <= w->lay.max_words) ? 1 : 0;
        s.mask0 = words;
        s.list0 = words;
        s.cwave0 = cwaves;
        if (s.cull) {
            words += nw;
            cwaves += ceil_div(s.tiles_x, UVL_TILE_BLOCK) * ceil_div(s.ntiles / s.tiles_x, UVL_TILE_BLOCK);
        }
        live_n[k] = 0;
        // padding: the outline of this stream's geometry image, if listed
        s.outline = nullptr;
        s.nout = 0;
        s.padk = 0;
        s.bins = f.numeric ? nullptr : reinterpret_cast<unsigned long long *>(f.bins);
        s.aw = f.geom->area_w;
        s.aw_hi = f.geom->area_w_hi;
        s.nbins = f.numeric ? 0 : (f.layer->dtype == UVL_U8 ? 256 : 65536);
        s.out0 = nout_total;
        for (int32_t q = 0; q < noutlines; ++q) {
            const uvl_wave_outline &o = outlines[q];
            if (!o.geom || o.geom->pos_x != f.geom->pos_x) continue;
            s.outline = o.outline;
            s.nout = o.n;
            s.padk = o.k;
            nout_total += o.n;
            break;
        }
        s.e0 = ei;
        s.ne = (int32_t)members[k].size();
        for (int32_t i : members[k]) {
            const uvl_edit &e = edits[i];
            WaveEdit &d = E[ei++];
            d.kind = e.kind;
            d.label = bits[i];
            d.erase = e.numeric && e.mode == UVL_ERASE ? 1 : 0;
            if (e.kind == UVL_EDIT_BRUSH) {
                d.cx = e.center[0];
                d.cy = e.center[1];
                d.cz = e.center[2];
                d.r2 = e.radius * e.radius;
                d.lasso = -1;
                d.depth = nullptr;
            } else if (e.kind == UVL_EDIT_LASSO) {
                if (!make_lasso_params(e.view_proj, e.poly_xy, e.npoly, e.dw, e.dh, e.bias, P[li])) return UVL_E_INVAL;
                for (int q = 0; q < 16; ++q)
                    if (!std::isfinite(e.view_proj[q])) return UVL_E_INVAL;
                d.cx = d.cy = d.cz = d.r2 = 0.0f;
                d.lasso = li++;
                d.depth = e.depth;
            } else {
                // the tool itself, and for culling a rectangle holding every
                // texel it can select: its square's NDC range, widened
                ToolParams &T = TP[li];
                if (!make_tool_params(e.view_proj, e.tool, e.sw, e.sh, e.dw, e.dh, e.bias, T)) return UVL_E_INVAL;
                const float rect[8] = {T.xlo_m, T.ylo_m, T.xhi_m, T.ylo_m, T.xhi_m, T.yhi_m, T.xlo_m, T.yhi_m};
                if (!make_lasso_params(e.view_proj, rect, 4, e.dw, e.dh, e.bias, P[li])) return UVL_E_INVAL;
                d.cx = d.cy = d.cz = d.r2 = 0.0f;
                d.lasso = li++;
                d.depth = e.depth;
            }
            d.shape = e.kind == UVL_EDIT_TOOL ? e.shape : nullptr;
        }
    }
    hdr->nstreams = (int32_t)keys.size();
    hdr->any_bins = 0;
    for (size_t k = 0; k < keys.size(); ++k)
        if (S[k].bins) hdr->any_bins = 1;
    hdr->total_cull_waves = cwaves;
    hdr->total_items = 0;
    hdr->total_out = nout_total;
    hdr->counter = 0;
    bytes = end;
    return UVL_OK;
}

}  // namespace

namespace {

int32_t submit(uvl_wave *w, const uvl_edit *edits, int32_t n, int32_t tile_chunks, const uvl_wave_outline *outlines,
               int32_t noutlines, void *stream) {
    if (!w || (!edits && n > 0) || n < 0 || tile_chunks < 0 || tile_chunks > kMaxChunks) return UVL_E_INVAL;
    if (noutlines < 0 || (noutlines > 0 && !outlines)) return UVL_E_INVAL;
    for (int32_t q = 0; q < noutlines; ++q) {
        const uvl_wave_outline &o = outlines[q];
        if (!o.geom || !geom_pos_ok(o.geom) || o.n < 0 || (o.n > 0 && !o.outline) || o.k < 0 || o.k > kMaxPadRadius ||
            o.n > (int64_t)o.geom->width * o.geom->height)
            return UVL_E_INVAL;
    }
    if (n > w->max_edits) return UVL_E_NOMEM;
    if (n == 0) return UVL_OK;
    std::lock_guard<std::mutex> lock(w->mu);
    // take the next pinned buffer of the ring; its previous copy must have
    // executed before it is rewritten (up to kStaging submits in flight)
    const int k = w->next;
    if (w->pending[k] && hipEventSynchronize(w->copied[k]) != hipSuccess) return UVL_E_DEVICE;
    w->pending[k] = false;
    w->staging = w->ring[k];
    size_t bytes = 0;
    if (int32_t st = pack(w, edits, n, tile_chunks, outlines, noutlines, bytes)) return st;
    const int64_t total_out = reinterpret_cast<const WaveHeader *>(w->staging)->total_out;
    hipStream_t s = as_stream(stream);
    if (hipMemcpyAsync(w->ws, w->staging, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return UVL_E_DEVICE;
    if (hipEventRecord(w->copied[k], s) != hipSuccess) return UVL_E_DEVICE;
    w->pending[k] = true;
    w->next = (k + 1) % kStaging;
    if (hipGraphLaunch(w->exec, s) != hipSuccess) return UVL_E_DEVICE;
    if (total_out > 0) {
        const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total_out, kBlock), kPadGrid);
        hipLaunchKernelGGL(k_wave_pad, dim3(grid), dim3(kBlock), 0, s, w->ws,
                           reinterpret_cast<const uint64_t *>(w->ws + w->lay.masks));
        if (hipGetLastError() != hipSuccess) return UVL_E_DEVICE;
    }
    return UVL_OK;
}

}  // namespace

extern "C" int32_t uvl_wave_submit(uvl_wave *w, const uvl_edit *edits, int32_t n, int32_t tile_chunks, void *stream) {
    return submit(w, edits, n, tile_chunks, nullptr, 0, stream);
}

extern "C" int32_t uvl_wave_submit_padded(uvl_wave *w, const uvl_edit *edits, int32_t n, int32_t tile_chunks,
                                          const uvl_wave_outline *outlines, int32_t noutlines, void *stream) {
    return submit(w, edits, n, tile_chunks, outlines, noutlines, stream);
}

extern "C" int32_t uvl_wave_tune(uvl_wave *w, const uvl_edit *edits, int32_t n, void *stream) {
    if (!w || !edits || n < 1) return UVL_E_INVAL;
    hipStream_t s = as_stream(stream);
    // size classes present in the wave
    std::vector<int> classes;
    for (int32_t i = 0; i < n; ++i) {
        if (!edits[i].geom) return UVL_E_INVAL;
        const int c = log2_class((int64_t)edits[i].geom->width * edits[i].geom->height);
        if (std::find(classes.begin(), classes.end(), c) == classes.end()) classes.push_back(c);
    }
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return UVL_E_DEVICE;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return UVL_E_DEVICE;
    }
    int32_t status = UVL_OK;
    for (int c : classes) {
        std::vector<uvl_edit> sub;
        for (int32_t i = 0; i < n; ++i)
            if (log2_class((int64_t)edits[i].geom->width * edits[i].geom->height) == c) sub.push_back(edits[i]);
        float best = INFINITY;
        int best_ch = 4;
        for (int ch : {1, 2, 4, 8}) {
            // applying a wave twice gives the same layers, so timing repeats is safe
            if ((status = uvl_wave_submit(w, sub.data(), (int32_t)sub.size(), ch, stream))) break;
            if (hipEventRecord(a, s) != hipSuccess) status = UVL_E_DEVICE;
            for (int r = 0; r < 3 && !status; ++r) status = uvl_wave_submit(w, sub.data(), (int32_t)sub.size(), ch, stream);
            if (!status && hipEventRecord(b, s) != hipSuccess) status = UVL_E_DEVICE;
            if (status || hipEventSynchronize(b) != hipSuccess) {
                status = status ? status : UVL_E_DEVICE;
                break;
            }
            float ms = INFINITY;
            if (hipEventElapsedTime(&ms, a, b) != hipSuccess) ms = INFINITY;
            if (ms < best) {
                best = ms;
                best_ch = ch;
            }
        }
        if (status) break;
        std::lock_guard<std::mutex> lock(w->mu);
        w->tuned_chunks[c] = best_ch;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return status;
}

extern "C" int32_t uvl_wave_visited_tiles(uvl_wave *w, int64_t *tiles, void *stream) {
    if (!w || !tiles) return UVL_E_INVAL;
    std::lock_guard<std::mutex> lock(w->mu);
    hipStream_t s = as_stream(stream);
    // the header (for the region offsets and stream count), then the streams
    // and their live counters
    WaveHeader h;
    if (hipMemcpyAsync(&h, w->ws, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return UVL_E_DEVICE;
    if (h.nstreams < 0 || h.nstreams > w->max_edits) return UVL_E_DEVICE;
    std::vector<WaveStream> st((size_t)h.nstreams);
    std::vector<uint32_t> live_n((size_t)h.nstreams);
    if (h.nstreams > 0 &&
        (hipMemcpyAsync(st.data(), w->ws + h.off_streams, sizeof(WaveStream) * st.size(), hipMemcpyDeviceToHost,
                        s) != hipSuccess ||
         hipMemcpyAsync(live_n.data(), w->ws + h.off_live_n, sizeof(uint32_t) * live_n.size(),
                        hipMemcpyDeviceToHost, s) != hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess))
        return UVL_E_DEVICE;
    int64_t sum = 0;
    for (size_t k = 0; k < st.size(); ++k) sum += st[k].cull ? (int64_t)live_n[k] : (int64_t)st[k].ntiles;
    *tiles = sum;
    return UVL_OK;
}

extern "C" int32_t uvl_wave_tuned_chunks(const uvl_wave *w, int64_t texels) {
    if (!w || texels < 1) return UVL_E_INVAL;
    return w->tuned_chunks[log2_class(texels)];
}
