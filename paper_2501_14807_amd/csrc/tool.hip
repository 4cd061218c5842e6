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
#include "tool_texel.h"
#include "uvl_internal.h"

namespace uvl {
namespace {

constexpr int kChunk = kBlock * 4;
constexpr int kTile = 4 * kChunk;
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

}  // namespace

// The NDC range of one axis where the tool coordinate a x + b lies in
// [0, 1], clipped to the frustum and widened for the reciprocal pre-test
// (1e-4 relative, plus the rounding of a x + b near 1 seen in x).
static void tool_range(double a, double b, float &lo, float &hi) {
    double x0 = -b / a, x1 = (1.0 - b) / a;
    x0 = fmax(x0, -1.0);
    x1 = fmin(x1, 1.0);
    const double m = 1e-4 * (1.0 + fmax(fabs(x0), fabs(x1))) + 1e-6 / a;
    lo = (float)(x0 - m);
    hi = (float)(x1 + m);
}

bool make_tool_params(const float view_proj[16], const double tool[6], int32_t sw, int32_t sh, int32_t dw,
                      int32_t dh, float bias, ToolParams &p) {
    if (!view_proj || !tool) return false;
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

}  // namespace uvl

using namespace uvl;

namespace {

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
    if (!shape || !depth || !make_tool_params(view_proj, tool, sw, sh, dw, dh, bias, p)) return UVL_E_INVAL;
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
    if (!shape || !depth || !make_tool_params(view_proj, tool, sw, sh, dw, dh, bias, p)) return UVL_E_INVAL;
    uint32_t bits = 0;
    if (int32_t s = check_numeric_edit(geom, layer, mode, value, bits)) return s;
    with_value_sink(layer, bits, mode, [&](auto out) { launch_tool(geom, p, shape, depth, out, as_stream(stream)); });
    return launch_status();
}
