// Batched edit waves for libuvl: many models' pending brush and lasso edits
// applied by one persistent-kernel launch.
//
// The paper applies one edit per rendering pass (§4.3.1).  Each edit is a
// pure function of the texel's stored position, and the last selecting edit
// wins, so a layer's pending edits can be applied in one pass: read the
// positions of a tile once, evaluate every edit of that layer in submission
// order in registers, and store each texel's final label once.  The result
// is bit-identical to applying the edits one launch at a time.
//
// Work decomposition: edits are grouped by target layer into streams (each
// stream keeps its edits' order); a stream's atlas is cut into 32 x 32-texel
// tiles (row-major), and an item is `chunks` consecutive tiles (chunks per
// stream chosen per atlas size by the autotuner); a fixed grid of workgroups
// takes (stream, item) pairs from an atomic counter until none are left.
// Every workgroup ends when the counter passes the item count, so the grid
// always drains.  In a tile, lane t covers row t/8 and columns 4(t%8)..+3.
//
// Tile culling (when the geometry image has tile bounds): a first kernel
// gives every (tile, group of 64 edits) one wave, each lane tests one edit
// against the tile's bounds (exact conservative tests, edit_texel.h), and the
// ballot -- the mask of edits that may select something there -- is stored in
// the workspace.  The wave kernel then reads a tile only if some edit is live
// and evaluates only the live edits.  Streams whose masks do not fit the
// workspace run without culling.
//
// The descriptor (streams, edits, lasso parameters) is copied host->device
// into the caller's workspace before each launch; the counter reset and the
// persistent kernel are captured once per handle in a HIP graph and replayed.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "edit_texel.h"
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
    void *layer;
    int64_t item0;      // first item of this stream
    int64_t mask0;      // first cull-mask word of this stream (running offset)
    int32_t W, H;       // atlas size
    int32_t tiles_x, ntiles;
    int32_t dtype;
    int32_t e0, ne;     // edits [e0, e0 + ne)
    int32_t chunks;     // tiles per item
    int32_t cull;       // 1: masks at mask0 (tiles x groups words), 0: no culling
};

struct WaveEdit {
    int32_t kind;
    uint32_t label;
    float cx, cy, cz, r2;
    int32_t lasso;      // index into the lasso parameter array
    int32_t pad;
    const float *depth;
};

struct WaveHeader {
    int32_t nstreams;
    int32_t pad;
    int64_t total_items;
    int64_t total_words;     // cull-mask words in use
    unsigned int counter;
    unsigned int pad2[3];
};

// Workspace layout: header | streams | edits | lassos | cull masks
struct Layout {
    size_t streams, edits, lassos, masks, total;
    int64_t max_words;
};

Layout layout(int32_t max_edits, int32_t max_lassos, int64_t max_words) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    Layout L;
    L.streams = 256;
    L.edits = L.streams + al(sizeof(WaveStream) * (size_t)max_edits);
    L.lassos = L.edits + al(sizeof(WaveEdit) * (size_t)max_edits);
    L.masks = L.lassos + al(sizeof(LassoParams) * (size_t)(max_lassos > 0 ? max_lassos : 1));
    L.total = L.masks + al(sizeof(uint64_t) * (size_t)(max_words > 0 ? max_words : 1));
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

// Cull masks: one wave per (tile, group of 64 edits) word, grid-striding
// over the words in use.
__global__ __launch_bounds__(kBlock) void k_wave_cull(const char *__restrict__ ws, const WaveHeader *__restrict__ hdr,
                                                       size_t off_streams, size_t off_edits, size_t off_lassos,
                                                       uint64_t *__restrict__ masks) {
    const UVL_CONST WaveStream *streams = (const UVL_CONST WaveStream *)(ws + off_streams);
    const UVL_CONST WaveEdit *edits = (const UVL_CONST WaveEdit *)(ws + off_edits);
    const UVL_CONST LassoParams *lassos = (const UVL_CONST LassoParams *)(ws + off_lassos);
    const int32_t nstreams = hdr->nstreams;
    const int64_t total = hdr->total_words;
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t word = wave0; word < total; word += nwaves) {
        // stream owning the word: the last stream with mask0 <= word (streams
        // without culling own no words, so this is a culling stream)
        int lo = 0, hi = nstreams - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (streams[mid].mask0 <= word) lo = mid;
            else hi = mid - 1;
        }
        const UVL_CONST WaveStream &S = streams[lo];
        const int groups = (S.ne + 63) >> 6;
        const int64_t rel = word - S.mask0;
        const int64_t ti = rel / groups;
        const int g = (int)(rel % groups);
        float box[6];
        const UVL_CONST float *bp = (const UVL_CONST float *)(S.box + 6 * ti);
#pragma unroll
        for (int q = 0; q < 6; ++q) box[q] = bp[q];
        const int e = g * 64 + lane;
        bool alive = false;
        if (e < S.ne) {
            const UVL_CONST WaveEdit &E = edits[S.e0 + e];
            alive = E.kind == UVL_EDIT_BRUSH ? !brush_culls(BrushParams{E.cx, E.cy, E.cz, E.r2}, box)
                                             : !lasso_culls(lassos[E.lasso], box);
        }
        const uint64_t m = __ballot(alive);
        if (lane == 0) masks[word] = m;
    }
}

__global__ __launch_bounds__(kBlock) void k_wave(const char *__restrict__ ws, WaveHeader *__restrict__ hdr,
                                                  size_t off_streams, size_t off_edits, size_t off_lassos,
                                                  const uint64_t *__restrict__ masks_in) {
    // read-only descriptor and masks viewed in the constant address space:
    // uniform reads become scalar loads
    const UVL_CONST WaveStream *streams = (const UVL_CONST WaveStream *)(ws + off_streams);
    const UVL_CONST WaveEdit *edits = (const UVL_CONST WaveEdit *)(ws + off_edits);
    const UVL_CONST LassoParams *lassos = (const UVL_CONST LassoParams *)(ws + off_lassos);
    const UVL_CONST uint64_t *masks = (const UVL_CONST uint64_t *)masks_in;
    __shared__ long long s_item;
    const int32_t nstreams = hdr->nstreams;
    const int64_t total = hdr->total_items;
    const int trow = threadIdx.x >> 3, tcol = (threadIdx.x & 7) * 4;
    for (;;) {
        if (threadIdx.x == 0) s_item = (long long)atomicAdd(&hdr->counter, 1u);
        __syncthreads();
        const int64_t item = s_item;
        __syncthreads();
        if (item >= total) break;
        // stream holding the item: last stream with item0 <= item
        int lo = 0, hi = nstreams - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (streams[mid].item0 <= item) lo = mid;
            else hi = mid - 1;
        }
        const UVL_CONST WaveStream &S = streams[lo];
        const int chunks = S.chunks, W = S.W, H = S.H;
        const int groups = (S.ne + 63) >> 6;
        const bool cull = S.cull != 0;
        const int64_t tile_first = (item - S.item0) * (int64_t)chunks;
        for (int c = 0; c < chunks; ++c) {
            const int64_t ti = tile_first + c;
            if (ti >= S.ntiles) break;
            const UVL_CONST uint64_t *tm = masks + (cull ? S.mask0 + ti * groups : 0);
            if (cull) {
                uint64_t any = 0;
                for (int g = 0; g < groups; ++g) any |= tm[g];
                if (!any) continue;
            }
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
            uint32_t val[4] = {0, 0, 0, 0};
            bool wr[4] = {false, false, false, false};
            for (int g = 0; g < groups; ++g) {
                uint64_t live = cull ? tm[g] : ~0ull;
                const int base = g * 64;
                const int lim = S.ne - base < 64 ? S.ne - base : 64;
                if (lim < 64) live &= (1ull << lim) - 1;
                while (live) {
                    const int e = base + __builtin_ctzll(live);
                    live &= live - 1;
                    const UVL_CONST WaveEdit &E = edits[S.e0 + e];
                    bool sel[4];
                    if (E.kind == UVL_EDIT_BRUSH) {
                        const BrushParams B{E.cx, E.cy, E.cz, E.r2};
                        sel[0] = brush_texel(B, X.x, Y.x, Z.x);
                        sel[1] = brush_texel(B, X.y, Y.y, Z.y);
                        sel[2] = brush_texel(B, X.z, Y.z, Z.z);
                        sel[3] = brush_texel(B, X.w, Y.w, Z.w);
                    } else {
                        lasso_quad(lassos[E.lasso], E.depth, X, Y, Z, sel);
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        val[k] = sel[k] ? E.label : val[k];
                        wr[k] = wr[k] || sel[k];
                    }
                }
            }
            if (S.dtype == UVL_U8) wave_store<uint8_t>(static_cast<uint8_t *>(S.layer), t, val, wr, in, full);
            else wave_store<uint16_t>(static_cast<uint16_t *>(S.layer), t, val, wr, in, full);
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
        ok = hipStreamBeginCapture(w->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            hipLaunchKernelGGL(k_wave_reset, dim3(1), dim3(64), 0, w->cap, hdr);
            hipLaunchKernelGGL(k_wave_cull, dim3(kWaveGrid), dim3(kBlock), 0, w->cap, w->ws, hdr, lay.streams,
                               lay.edits, lay.lassos, masks);
            hipLaunchKernelGGL(k_wave, dim3(kWaveGrid), dim3(kBlock), 0, w->cap, w->ws, hdr, lay.streams, lay.edits,
                               lay.lassos, masks);
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
int32_t pack(uvl_wave *w, const uvl_edit *edits, int32_t n, int32_t chunks_override, size_t &bytes) {
    // streams: one per distinct layer, in order of first appearance
    std::vector<int32_t> stream_of(n);
    std::vector<const void *> keys;
    std::vector<std::vector<int32_t>> members;
    int32_t nl = 0;
    for (int32_t i = 0; i < n; ++i) {
        const uvl_edit &e = edits[i];
        if (!e.geom || !e.layer) return UVL_E_INVAL;
        if (!geom_pos_ok(e.geom) || !layer_ok(e.layer)) return UVL_E_INVAL;
        if (!dtype_ok(e.layer->dtype)) return UVL_E_DTYPE;
        if (e.label > dtype_max(e.layer->dtype)) return UVL_E_DTYPE;
        if (e.layer->width != e.geom->width || e.layer->height != e.geom->height) return UVL_E_SHAPE;
        if (e.kind == UVL_EDIT_BRUSH) {
            if (!(e.radius >= 0.0f) || !std::isfinite(e.radius)) return UVL_E_INVAL;
            if (!std::isfinite(e.center[0]) || !std::isfinite(e.center[1]) || !std::isfinite(e.center[2]))
                return UVL_E_INVAL;
        } else if (e.kind == UVL_EDIT_LASSO) {
            if (!e.depth || !e.view_proj || e.dw > kMaxDepthSide || e.dh > kMaxDepthSide) return UVL_E_INVAL;
            if (++nl > w->max_lassos) return UVL_E_NOMEM;
        } else {
            return UVL_E_INVAL;
        }
        size_t k = 0;
        while (k < keys.size() && keys[k] != e.layer->data) ++k;
        if (k == keys.size()) {
            keys.push_back(e.layer->data);
            members.emplace_back();
        } else {
            // every edit of one layer must read the same positions
            const uvl_edit &f = edits[members[k][0]];
            if (f.geom->pos_x != e.geom->pos_x || f.layer->dtype != e.layer->dtype || f.layer->width != e.layer->width ||
                f.layer->height != e.layer->height)
                return UVL_E_INVAL;
        }
        members[k].push_back(i);
    }
    char *st = w->staging;
    WaveHeader *hdr = reinterpret_cast<WaveHeader *>(st);
    WaveStream *S = reinterpret_cast<WaveStream *>(st + w->lay.streams);
    WaveEdit *E = reinterpret_cast<WaveEdit *>(st + w->lay.edits);
    LassoParams *P = reinterpret_cast<LassoParams *>(st + w->lay.lassos);
    int64_t item = 0, words = 0;
    int32_t ei = 0, li = 0;
    for (size_t k = 0; k < keys.size(); ++k) {
        const uvl_edit &f = edits[members[k][0]];
        WaveStream &s = S[k];
        s.px = f.geom->pos_x;
        s.py = f.geom->pos_y;
        s.pz = f.geom->pos_z;
        s.box = f.geom->tile_box;
        s.layer = f.layer->data;
        s.W = f.layer->width;
        s.H = f.layer->height;
        s.tiles_x = (int32_t)ceil_div(s.W, UVL_TILE_SIDE);
        s.ntiles = s.tiles_x * (int32_t)ceil_div(s.H, UVL_TILE_SIDE);
        s.dtype = f.layer->dtype;
        int ch = chunks_override > 0 ? chunks_override : w->tuned_chunks[log2_class((int64_t)s.W * s.H)];
        if (ch <= 0) ch = 4;
        s.chunks = std::min(std::max(ch, 1), kMaxChunks);
        s.item0 = item;
        item += ceil_div(s.ntiles, s.chunks);
        // cull masks if the geometry has tile bounds and the words fit
        const int64_t nw = (int64_t)s.ntiles * ((int64_t)(members[k].size() + 63) / 64);
        s.mask0 = words;
        s.cull = (f.geom->tile_box && words + nw <= w->lay.max_words) ? 1 : 0;
        if (s.cull) words += nw;
        s.e0 = ei;
        s.ne = (int32_t)members[k].size();
        for (int32_t i : members[k]) {
            const uvl_edit &e = edits[i];
            WaveEdit &d = E[ei++];
            d.kind = e.kind;
            d.label = e.label;
            d.pad = 0;
            if (e.kind == UVL_EDIT_BRUSH) {
                d.cx = e.center[0];
                d.cy = e.center[1];
                d.cz = e.center[2];
                d.r2 = e.radius * e.radius;
                d.lasso = -1;
                d.depth = nullptr;
            } else {
                if (!make_lasso_params(e.view_proj, e.poly_xy, e.npoly, e.dw, e.dh, e.bias, P[li])) return UVL_E_INVAL;
                for (int q = 0; q < 16; ++q)
                    if (!std::isfinite(e.view_proj[q])) return UVL_E_INVAL;
                d.cx = d.cy = d.cz = d.r2 = 0.0f;
                d.lasso = li++;
                d.depth = e.depth;
            }
        }
    }
    hdr->nstreams = (int32_t)keys.size();
    hdr->pad = 0;
    hdr->total_items = item;
    hdr->total_words = words;
    hdr->counter = 0;
    bytes = li > 0 ? w->lay.lassos + sizeof(LassoParams) * (size_t)li : w->lay.lassos;
    return UVL_OK;
}

}  // namespace

extern "C" int32_t uvl_wave_submit(uvl_wave *w, const uvl_edit *edits, int32_t n, int32_t tile_chunks, void *stream) {
    if (!w || (!edits && n > 0) || n < 0 || tile_chunks < 0 || tile_chunks > kMaxChunks) return UVL_E_INVAL;
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
    if (int32_t st = pack(w, edits, n, tile_chunks, bytes)) return st;
    hipStream_t s = as_stream(stream);
    if (hipMemcpyAsync(w->ws, w->staging, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return UVL_E_DEVICE;
    if (hipEventRecord(w->copied[k], s) != hipSuccess) return UVL_E_DEVICE;
    w->pending[k] = true;
    w->next = (k + 1) % kStaging;
    if (hipGraphLaunch(w->exec, s) != hipSuccess) return UVL_E_DEVICE;
    return UVL_OK;
}

extern "C" int32_t uvl_wave_tune(uvl_wave *w, const uvl_edit *edits, int32_t n, void *stream) {
    if (!w || !edits || n < 1) return UVL_E_INVAL;
    hipStream_t s = as_stream(stream);
    // size classes present in the wave
    std::vector<int> classes;
    for (int32_t i = 0; i < n; ++i) {
        if (!edits[i].layer) return UVL_E_INVAL;
        const int c = log2_class((int64_t)edits[i].layer->width * edits[i].layer->height);
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
            if (log2_class((int64_t)edits[i].layer->width * edits[i].layer->height) == c) sub.push_back(edits[i]);
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

extern "C" int32_t uvl_wave_tuned_chunks(const uvl_wave *w, int64_t texels) {
    if (!w || texels < 1) return UVL_E_INVAL;
    return w->tuned_chunks[log2_class(texels)];
}
