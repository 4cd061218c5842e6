// Texture padding for libuvl (§4.3.2, the Texture Padding Algorithm).
//
// Around every texture island (the texels triangles cover) the outline is
// the band of uncovered texels within Chebyshev distance k of the island;
// after an edit, each outline texel within distance k of a texel the edit
// selected takes the edit's label (or, in a numeric layer, the edit's SET or
// ERASE), so that sampling across an island's border reads the edited value.  Both distances use the paper's square
// kernel of radius k; the paper pads one texel (k = 1).
//
// The outline is built once per geometry image, as a list of texel indices
// in ascending order (per-block counts, a block scan, an ordered write).
// Padding needs the edited-area mask of the edit; instead of storing it, a
// lane per outline texel evaluates the edit's own per-texel predicate
// (edit_texel.h) at the covered texels of its window: the predicate is a
// pure function of a texel's stored position, so this is the mask the edit
// used, bit for bit.  Outline texels are uncovered and edits write covered
// texels only, so padding and edits touch disjoint texels and a padding
// pass may run any time after its edit.
#include "edit_texel.h"
#include "sink.h"
#include "uvl_internal.h"

namespace uvl {

bool make_lasso_params(const float view_proj[16], const float *poly, int32_t n, int32_t dw, int32_t dh,
                       float bias, LassoParams &p);

namespace {

constexpr int kMaxPadRadius = 8;
constexpr int kOutlineBlock = kBlock * 4;   // texels per counting block

__device__ __forceinline__ bool is_outline(const int32_t *__restrict__ tri, int W, int H, int k, int64_t t) {
    if (tri[t] >= 0) return false;
    const int i = (int)(t % W), j = (int)(t / W);
    const int u0 = i - k < 0 ? 0 : i - k, u1 = i + k > W - 1 ? W - 1 : i + k;
    const int v0 = j - k < 0 ? 0 : j - k, v1 = j + k > H - 1 ? H - 1 : j + k;
    for (int v = v0; v <= v1; ++v)
        for (int u = u0; u <= u1; ++u)
            if (tri[(int64_t)v * W + u] >= 0) return true;
    return false;
}

// Pass 1: outline texels per block of kOutlineBlock texels.
__global__ __launch_bounds__(kBlock) void k_outline_count(const int32_t *__restrict__ tri, int W, int H, int k,
                                                          uint32_t *__restrict__ counts) {
    const int64_t N = (int64_t)W * H;
    const int64_t b0 = (int64_t)blockIdx.x * kOutlineBlock;
    unsigned c = 0;
    for (int q = 0; q < 4; ++q) {
        const int64_t t = b0 + q * kBlock + threadIdx.x;
        c += t < N && is_outline(tri, W, H, k, t);
    }
    __shared__ unsigned s[kBlock];
    s[threadIdx.x] = c;
    __syncthreads();
    for (int d = kBlock / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) s[threadIdx.x] += s[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = s[0];
}

// Pass 2 (one workgroup): exclusive prefix of the block counts, in place;
// the total goes to counts[nb].
__global__ __launch_bounds__(kBlock) void k_outline_scan(uint32_t *__restrict__ counts, int64_t nb) {
    const int64_t per = (nb + kBlock - 1) / kBlock;
    const int64_t a = threadIdx.x * per, b = a + per < nb ? a + per : nb;
    unsigned long long sum = 0;
    for (int64_t q = a; q < b; ++q) sum += counts[q];
    __shared__ unsigned long long part[kBlock];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < kBlock; d <<= 1) {
        const unsigned long long v = (int)threadIdx.x >= d ? part[threadIdx.x - d] : 0ull;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    unsigned long long run = part[threadIdx.x] - sum;
    for (int64_t q = a; q < b; ++q) {
        const unsigned c = counts[q];
        counts[q] = (uint32_t)run;
        run += c;
    }
    if (threadIdx.x == kBlock - 1) counts[nb] = (uint32_t)part[kBlock - 1];
}

// Pass 3: each block writes its outline texels, in index order, from its
// offset.  Texel order within the block: step q, then thread; ranks come
// from the wave ballots and per-wave counts in LDS.
__global__ __launch_bounds__(kBlock) void k_outline_write(const int32_t *__restrict__ tri, int W, int H, int k,
                                                          const uint32_t *__restrict__ offsets,
                                                          int32_t *__restrict__ out, int64_t capacity) {
    const int64_t N = (int64_t)W * H;
    const int64_t b0 = (int64_t)blockIdx.x * kOutlineBlock;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ unsigned wcount[4];
    unsigned base = offsets[blockIdx.x];
    for (int q = 0; q < 4; ++q) {
        const int64_t t = b0 + q * kBlock + threadIdx.x;
        const bool o = t < N && is_outline(tri, W, H, k, t);
        const uint64_t m = __ballot(o);
        if (lane == 0) wcount[wave] = (unsigned)__popcll(m);
        __syncthreads();
        unsigned before = 0;
        for (int w = 0; w < wave; ++w) before += wcount[w];
        const unsigned step_total = wcount[0] + wcount[1] + wcount[2] + wcount[3];
        const unsigned idx = base + before + (unsigned)__popcll(m & ((1ull << lane) - 1));
        if (o && (int64_t)idx < capacity) out[idx] = (int32_t)t;
        base += step_total;
        __syncthreads();
    }
}

// Padding: lane per outline texel; the covered texels of its window are
// tested with the edit's predicate until one is selected.
template <class Sink, class Pred>
__device__ __forceinline__ void pad_texel(const float *__restrict__ px, const float *__restrict__ py,
                                          const float *__restrict__ pz, const Sink &out, int W, int H, int k,
                                          int32_t t, const Pred &sel) {
    if (t < 0 || (int64_t)t >= (int64_t)W * H) return;   // not a texel index: ignored
    const int i = t % W, j = t / W;
    const int u0 = i - k < 0 ? 0 : i - k, u1 = i + k > W - 1 ? W - 1 : i + k;
    const int v0 = j - k < 0 ? 0 : j - k, v1 = j + k > H - 1 ? H - 1 : j + k;
    for (int v = v0; v <= v1; ++v)
        for (int u = u0; u <= u1; ++u) {
            const int64_t s = (int64_t)v * W + u;
            const float x = px[s];
            if (x != x) continue;   // uncovered (NaN position): never edited
            if (sel(x, py[s], pz[s])) {
                out.put1(t);
                return;
            }
        }
}

template <class Sink>
__global__ __launch_bounds__(kBlock) void k_pad_brush(const float *__restrict__ px, const float *__restrict__ py,
                                                      const float *__restrict__ pz, Sink out, int W, int H, int k,
                                                      const int32_t *__restrict__ outline, int64_t n,
                                                      BrushParams B) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= n) return;
    pad_texel(px, py, pz, out, W, H, k, outline[q],
              [&](float x, float y, float z) { return brush_texel(B, x, y, z); });
}

template <class Sink>
__global__ __launch_bounds__(kBlock) void k_pad_lasso(const float *__restrict__ px, const float *__restrict__ py,
                                                      const float *__restrict__ pz, Sink out, int W, int H, int k,
                                                      const int32_t *__restrict__ outline, int64_t n, LassoParams P,
                                                      const float *__restrict__ depth) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= n) return;
    pad_texel(px, py, pz, out, W, H, k, outline[q],
              [&](float x, float y, float z) { return lasso_texel(P, depth, x, y, z); });
}

// Outline list and radius, shared by the label and numeric calls.
int32_t check_outline(const uvl_geom *g, const int32_t *outline, int64_t n, int32_t k) {
    if (!geom_pos_ok(g)) return UVL_E_INVAL;
    if (n < 0 || (n > 0 && !outline) || k < 0 || k > kMaxPadRadius) return UVL_E_INVAL;
    if (n > (int64_t)g->width * g->height) return UVL_E_SHAPE;
    return UVL_OK;
}

int32_t check_pad(const uvl_geom *g, const uvl_layer *l, const int32_t *outline, int64_t n, int32_t k,
                  uint32_t label) {
    if (!layer_ok(l)) return UVL_E_INVAL;
    if (int32_t s = check_outline(g, outline, n, k)) return s;
    if (!dtype_ok(l->dtype)) return UVL_E_DTYPE;
    if (label > dtype_max(l->dtype)) return UVL_E_DTYPE;
    if (l->width != g->width || l->height != g->height) return UVL_E_SHAPE;
    return device_ok();
}

bool brush_ok(const float center[3], float radius) {
    return center && radius >= 0.0f && std::isfinite(radius) && std::isfinite(center[0]) &&
           std::isfinite(center[1]) && std::isfinite(center[2]);
}

bool lasso_ok(const float view_proj[16], const float *poly_xy, int32_t npoly, const float *depth, int32_t dw,
              int32_t dh, float bias, LassoParams &p) {
    if (!depth || dw > kMaxDepthSide || dh > kMaxDepthSide) return false;
    if (!make_lasso_params(view_proj, poly_xy, npoly, dw, dh, bias, p)) return false;
    for (int q = 0; q < 16; ++q)
        if (!std::isfinite(view_proj[q])) return false;
    return true;
}

template <class Sink>
void launch_pad_brush(const uvl_geom *g, const int32_t *outline, int64_t n, int32_t k, const float center[3],
                      float radius, const Sink &out, hipStream_t s) {
    const BrushParams p{center[0], center[1], center[2], radius * radius};
    hipLaunchKernelGGL(k_pad_brush<Sink>, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, s, g->pos_x,
                       g->pos_y, g->pos_z, out, g->width, g->height, k, outline, n, p);
}

template <class Sink>
void launch_pad_lasso(const uvl_geom *g, const int32_t *outline, int64_t n, int32_t k, const LassoParams &p,
                      const float *depth, const Sink &out, hipStream_t s) {
    hipLaunchKernelGGL(k_pad_lasso<Sink>, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, s, g->pos_x,
                       g->pos_y, g->pos_z, out, g->width, g->height, k, outline, n, p, depth);
}

}  // namespace
}  // namespace uvl

using namespace uvl;

extern "C" size_t uvl_outline_workspace_bytes(int32_t width, int32_t height) {
    if (width < 1 || height < 1 || width > kMaxSide || height > kMaxSide) return 0;
    const int64_t nb = ceil_div((int64_t)width * height, kOutlineBlock);
    return (size_t)(nb + 1) * sizeof(uint32_t);
}

extern "C" int32_t uvl_build_outline(const uvl_geom *geom, int32_t k, int32_t *outline, int64_t capacity,
                                     int64_t *count, void *ws, size_t ws_bytes, void *stream) {
    if (!geom || !geom->tri_id || !count || !ws || k < 0 || k > kMaxPadRadius || capacity < 0) return UVL_E_INVAL;
    if (capacity > 0 && !outline) return UVL_E_INVAL;
    if (geom->width < 1 || geom->height < 1 || geom->width > kMaxSide || geom->height > kMaxSide) return UVL_E_INVAL;
    if (ws_bytes < uvl_outline_workspace_bytes(geom->width, geom->height)) return UVL_E_NOMEM;
    if (int32_t s = device_ok()) return s;
    hipStream_t s = as_stream(stream);
    const int W = geom->width, H = geom->height;
    const int64_t nb = ceil_div((int64_t)W * H, kOutlineBlock);
    uint32_t *counts = static_cast<uint32_t *>(ws);
    hipLaunchKernelGGL(k_outline_count, dim3((unsigned)nb), dim3(kBlock), 0, s, geom->tri_id, W, H, k, counts);
    hipLaunchKernelGGL(k_outline_scan, dim3(1), dim3(kBlock), 0, s, counts, nb);
    hipLaunchKernelGGL(k_outline_write, dim3((unsigned)nb), dim3(kBlock), 0, s, geom->tri_id, W, H, k, counts,
                       outline, capacity);
    if (launch_status() != UVL_OK) return UVL_E_DEVICE;
    uint32_t total = 0;
    if (hipMemcpyAsync(&total, counts + nb, sizeof(total), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return UVL_E_DEVICE;
    *count = total;
    return (int64_t)total > capacity ? UVL_E_NOMEM : UVL_OK;
}

extern "C" int32_t uvl_pad_brush(const uvl_geom *geom, const uvl_layer *layer, const int32_t *outline, int64_t n,
                                 int32_t k, const float center[3], float radius, uint32_t label, void *stream) {
    if (!brush_ok(center, radius)) return UVL_E_INVAL;
    if (int32_t s = check_pad(geom, layer, outline, n, k, label)) return s;
    if (n == 0) return UVL_OK;
    with_label_sink(layer, label, [&](auto out) {
        launch_pad_brush(geom, outline, n, k, center, radius, out, as_stream(stream));
    });
    return launch_status();
}

extern "C" int32_t uvl_pad_lasso(const uvl_geom *geom, const uvl_layer *layer, const int32_t *outline, int64_t n,
                                 int32_t k, const float view_proj[16], const float *poly_xy, int32_t npoly,
                                 const float *depth, int32_t dw, int32_t dh, float bias, uint32_t label,
                                 void *stream) {
    LassoParams p;
    if (!lasso_ok(view_proj, poly_xy, npoly, depth, dw, dh, bias, p)) return UVL_E_INVAL;
    if (int32_t s = check_pad(geom, layer, outline, n, k, label)) return s;
    if (n == 0) return UVL_OK;
    with_label_sink(layer, label, [&](auto out) {
        launch_pad_lasso(geom, outline, n, k, p, depth, out, as_stream(stream));
    });
    return launch_status();
}

extern "C" int32_t uvl_numeric_pad_brush(const uvl_geom *geom, const uvl_numeric *layer, const int32_t *outline,
                                         int64_t n, int32_t k, const float center[3], float radius, int32_t mode,
                                         double value, void *stream) {
    if (!brush_ok(center, radius)) return UVL_E_INVAL;
    if (int32_t s = check_outline(geom, outline, n, k)) return s;
    uint32_t bits = 0;
    if (int32_t s = check_numeric_edit(geom, layer, mode, value, bits)) return s;
    if (n == 0) return UVL_OK;
    with_value_sink(layer, bits, mode, [&](auto out) {
        launch_pad_brush(geom, outline, n, k, center, radius, out, as_stream(stream));
    });
    return launch_status();
}

extern "C" int32_t uvl_numeric_pad_lasso(const uvl_geom *geom, const uvl_numeric *layer, const int32_t *outline,
                                         int64_t n, int32_t k, const float view_proj[16], const float *poly_xy,
                                         int32_t npoly, const float *depth, int32_t dw, int32_t dh, float bias,
                                         int32_t mode, double value, void *stream) {
    LassoParams p;
    if (!lasso_ok(view_proj, poly_xy, npoly, depth, dw, dh, bias, p)) return UVL_E_INVAL;
    if (int32_t s = check_outline(geom, outline, n, k)) return s;
    uint32_t bits = 0;
    if (int32_t s = check_numeric_edit(geom, layer, mode, value, bits)) return s;
    if (n == 0) return UVL_OK;
    with_value_sink(layer, bits, mode, [&](auto out) {
        launch_pad_lasso(geom, outline, n, k, p, depth, out, as_stream(stream));
    });
    return launch_status();
}
