// The paper's screen-space editing tool for libuvl (§4.3.1, TEA).
//
// The camera doubles as a slide projector whose frustum the tool transform
// of §4.3.1 narrows to the tool's square on the window: a texel's NDC
// position (the lasso's projection, edit_texel.h) maps to tool coordinates
// s = fmaf(xn, ax, bx), t = fmaf(yn, ay, by); outside [0, 1] it is
// discarded, otherwise the tool's shape texture is sampled (nearest texel)
// and must be non-zero, and the depth test with bias applies.  The
// coefficients come from the window size (Ww, Wh), the tool position
// (Tpx, Tpy, window pixels from the lower-left corner) and the tool size
// (Tw, Th) pixels: ax = Ww / (2 Tw), bx = 1/2 - (Tpx - Ww/2) / Tw (fp64,
// rounded once), so the Tw x Th square centred on the tool maps onto
// [0, 1]^2 (the reading of the printed translate factor's sign that
// centres the tool).
//
// One streaming pass over the position planes, tiled as the brush (4096
// consecutive texels per workgroup, 16-byte non-temporal loads); the tool
// covers a small part of the screen, so a reciprocal pre-test rejects most
// texels before the exact divisions and few read the depth map.
#include <math.h>

#include "edit_texel.h"
#include "sink.h"
#include "uvl_internal.h"

namespace uvl {
namespace {

constexpr int kChunk = kBlock * 4;
constexpr int kTile = 4 * kChunk;
constexpr int kMaxShape = 4096;

struct ToolParams {
    float M[16];
    float ax, bx, ay, by;                  // s = fmaf(xn, ax, bx), t = fmaf(yn, ay, by)
    float xlo_m, xhi_m, ylo_m, yhi_m;      // NDC range with s, t in [0, 1] and in the frustum, widened
    int32_t sw, sh, dw, dh;
    float bias;
};

__device__ __forceinline__ bool tool_texel(const ToolParams &P, const uint8_t *__restrict__ shape,
                                           const float *__restrict__ depth, float x, float y, float z) {
    float c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        c[k] = __builtin_fmaf(P.M[4 * k + 2], z, __builtin_fmaf(P.M[4 * k + 1], y, __builtin_fmaf(P.M[4 * k + 0], x, P.M[4 * k + 3])));
    if (!(c[3] > 0.0f)) return false;
    if (c[3] >= 1e-30f) {
        // reciprocal pre-test: within 3e-7 relative of the exact quotients,
        // far inside the margins of the bounds
        const float r = __builtin_amdgcn_rcpf(c[3]);
        const float ax = c[0] * r, ay = c[1] * r;
        if (!(ax >= P.xlo_m && ax <= P.xhi_m && ay >= P.ylo_m && ay <= P.yhi_m)) return false;
    }
    const float xn = c[0] / c[3], yn = c[1] / c[3], zn = c[2] / c[3];
    if (!(xn >= -1.0f && xn <= 1.0f && yn >= -1.0f && yn <= 1.0f && zn >= -1.0f && zn <= 1.0f)) return false;
    const float s = __builtin_fmaf(xn, P.ax, P.bx), t = __builtin_fmaf(yn, P.ay, P.by);
    if (!(s >= 0.0f && s <= 1.0f && t >= 0.0f && t <= 1.0f)) return false;
    int sx = (int)floorf(s * (float)P.sw), sy = (int)floorf(t * (float)P.sh);
    sx = sx > P.sw - 1 ? P.sw - 1 : sx;
    sy = sy > P.sh - 1 ? P.sh - 1 : sy;
    if (!shape[(int64_t)sy * P.sw + sx]) return false;
    int ix = (int)floorf(__builtin_fmaf(xn, 0.5f, 0.5f) * (float)P.dw);
    int iy = (int)floorf(__builtin_fmaf(yn, 0.5f, 0.5f) * (float)P.dh);
    ix = ix > P.dw - 1 ? P.dw - 1 : ix;
    iy = iy > P.dh - 1 ? P.dh - 1 : iy;
    const float d = __builtin_fmaf(zn, 0.5f, 0.5f);
    return d <= depth[(int64_t)iy * P.dw + ix] + P.bias;
}

template <typename Sink>
__global__ __launch_bounds__(kBlock) void k_tool(const float *__restrict__ px, const float *__restrict__ py,
                                                 const float *__restrict__ pz, Sink out, int64_t n, ToolParams p,
                                                 const uint8_t *__restrict__ shape, const float *__restrict__ depth) {
    const int64_t base = (int64_t)blockIdx.x * kTile + threadIdx.x * 4;
    if ((int64_t)(blockIdx.x + 1) * kTile > n) {
        for (int c = 0; c < 4; ++c)
            for (int k = 0; k < 4; ++k) {
                const int64_t t = base + c * kChunk + k;
                if (t < n && tool_texel(p, shape, depth, px[t], py[t], pz[t])) out.put1(t);
            }
        return;
    }
    float4 X[4], Y[4], Z[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        X[c] = load_stream4(px + base + c * kChunk);
        Y[c] = load_stream4(py + base + c * kChunk);
        Z[c] = load_stream4(pz + base + c * kChunk);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const bool s[4] = {tool_texel(p, shape, depth, X[c].x, Y[c].x, Z[c].x),
                           tool_texel(p, shape, depth, X[c].y, Y[c].y, Z[c].y),
                           tool_texel(p, shape, depth, X[c].z, Y[c].z, Z[c].z),
                           tool_texel(p, shape, depth, X[c].w, Y[c].w, Z[c].w)};
        out.put4(base + c * kChunk, s, true);      // lanes 8g..8g+7: one 32-aligned word
    }
}

// The NDC range of one axis where the tool coordinate a x + b lies in
// [0, 1], clipped to the frustum and widened for the reciprocal pre-test
// (1e-4 relative, plus the rounding of a x + b near 1 seen in x).
void tool_range(double a, double b, float &lo, float &hi) {
    double x0 = -b / a, x1 = (1.0 - b) / a;
    x0 = fmax(x0, -1.0);
    x1 = fmin(x1, 1.0);
    const double m = 1e-4 * (1.0 + fmax(fabs(x0), fabs(x1))) + 1e-6 / a;
    lo = (float)(x0 - m);
    hi = (float)(x1 + m);
}

}  // namespace
}  // namespace uvl

using namespace uvl;

namespace {

// Tool arguments shared by the label and numeric calls.
bool tool_args(const float view_proj[16], const double tool[6], const uint8_t *shape, int32_t sw, int32_t sh,
               const float *depth, int32_t dw, int32_t dh, float bias, ToolParams &p) {
    if (!view_proj || !tool || !shape || !depth) return false;
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(view_proj[k])) return false;
    for (int k = 0; k < 6; ++k)
        if (!std::isfinite(tool[k])) return false;
    if (!(tool[0] > 0.0 && tool[1] > 0.0 && tool[4] > 0.0 && tool[5] > 0.0)) return false;
    if (sw < 1 || sh < 1 || sw > kMaxShape || sh > kMaxShape) return false;
    if (dw < 1 || dh < 1 || dw > kMaxDepthSide || dh > kMaxDepthSide || !std::isfinite(bias)) return false;
    for (int k = 0; k < 16; ++k) p.M[k] = view_proj[k];
    const double ax = tool[0] / (2.0 * tool[4]), bx = 0.5 - (tool[2] - 0.5 * tool[0]) / tool[4];
    const double ay = tool[1] / (2.0 * tool[5]), by = 0.5 - (tool[3] - 0.5 * tool[1]) / tool[5];
    p.ax = (float)ax;
    p.bx = (float)bx;
    p.ay = (float)ay;
    p.by = (float)by;
    // pre-test ranges from the fp32 coefficients the predicate uses
    tool_range((double)p.ax, (double)p.bx, p.xlo_m, p.xhi_m);
    tool_range((double)p.ay, (double)p.by, p.ylo_m, p.yhi_m);
    p.sw = sw;
    p.sh = sh;
    p.dw = dw;
    p.dh = dh;
    p.bias = bias;
    return true;
}

template <typename Sink>
void launch_tool(const uvl_geom *geom, const ToolParams &p, const uint8_t *shape, const float *depth, const Sink &out,
                 hipStream_t s) {
    const int64_t n = (int64_t)geom->width * geom->height;
    hipLaunchKernelGGL(k_tool<Sink>, dim3((unsigned)ceil_div(n, kTile)), dim3(kBlock), 0, s, geom->pos_x,
                       geom->pos_y, geom->pos_z, out, n, p, shape, depth);
}

}  // namespace

extern "C" int32_t uvl_edit_tool(const uvl_geom *geom, const uvl_layer *layer, const float view_proj[16],
                                 const double tool[6], const uint8_t *shape, int32_t sw, int32_t sh,
                                 const float *depth, int32_t dw, int32_t dh, float bias, uint32_t label,
                                 void *stream) {
    ToolParams p;
    if (!tool_args(view_proj, tool, shape, sw, sh, depth, dw, dh, bias, p)) return UVL_E_INVAL;
    if (!geom_pos_ok(geom) || !layer_ok(layer)) return UVL_E_INVAL;
    if (!dtype_ok(layer->dtype) || label > dtype_max(layer->dtype)) return UVL_E_DTYPE;
    if (layer->width != geom->width || layer->height != geom->height) return UVL_E_SHAPE;
    if (int32_t s = device_ok()) return s;
    with_label_sink(layer, label, [&](auto out) { launch_tool(geom, p, shape, depth, out, as_stream(stream)); });
    return launch_status();
}

extern "C" int32_t uvl_numeric_tool(const uvl_geom *geom, const uvl_numeric *layer, const float view_proj[16],
                                    const double tool[6], const uint8_t *shape, int32_t sw, int32_t sh,
                                    const float *depth, int32_t dw, int32_t dh, float bias, int32_t mode,
                                    double value, void *stream) {
    ToolParams p;
    if (!tool_args(view_proj, tool, shape, sw, sh, depth, dw, dh, bias, p)) return UVL_E_INVAL;
    uint32_t bits = 0;
    if (int32_t s = check_numeric_edit(geom, layer, mode, value, bits)) return s;
    with_value_sink(layer, bits, mode, [&](auto out) { launch_tool(geom, p, shape, depth, out, as_stream(stream)); });
    return launch_status();
}
