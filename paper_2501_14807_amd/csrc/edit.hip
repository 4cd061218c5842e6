// Plain edit path of libuvl: one launch per brush or lasso edit.
//
// The paper's per-edit pass touches every texel of the layer (§4.3.1, and
// §5: the edit time does not depend on the tool size).  Here each edit is one
// streaming pass over the geometry image's position planes: 12 bytes read per
// texel, one label store per selected texel, no read of the layer.
//
// Each lane handles 4 consecutive texels of a row and reads them from each
// plane with one 16-byte non-temporal load; all 12 loads of a thread are
// issued before any predicate.  The brush walks the atlas as a flat array
// (a 256-thread workgroup owns 4096 consecutive texels as 4 chunks of 1024, a
// wave's loads are 1 KiB contiguous per plane); the lasso, which also reads
// the depth map, walks it in 2D blocks (see k_lasso).
#include <math.h>

#include "edit_texel.h"
#include "sink.h"
#include "uvl_internal.h"

namespace uvl {
namespace {

constexpr int kChunk = kBlock * 4;        // texels per chunk
constexpr int kTile = 4 * kChunk;         // texels per workgroup

template <typename Sink>
__device__ __forceinline__ void brush_tail(const float *__restrict__ px, const float *__restrict__ py,
                                           const float *__restrict__ pz, const Sink &out, int64_t n,
                                           const BrushParams &B) {
    const int64_t base = (int64_t)blockIdx.x * kTile + threadIdx.x * 4;
    for (int c = 0; c < 4; ++c)
        for (int k = 0; k < 4; ++k) {
            const int64_t t = base + c * kChunk + k;
            if (t < n && brush_texel(B, px[t], py[t], pz[t])) out.put1(t);
        }
}

// Brush: one workgroup tile of 4096 consecutive texels; the last, partial
// tile takes the per-texel path.  Lanes 8g .. 8g+7 of a wave hold 32
// consecutive texels starting at a multiple of 32 (one mask word).
template <typename Sink>
__global__ __launch_bounds__(kBlock) void k_brush(const float *__restrict__ px, const float *__restrict__ py,
                                                  const float *__restrict__ pz, Sink out, int64_t n,
                                                  BrushParams p) {
    const int64_t base = (int64_t)blockIdx.x * kTile + threadIdx.x * 4;
    if ((int64_t)(blockIdx.x + 1) * kTile > n) {
        brush_tail(px, py, pz, out, n, p);
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
        const bool s[4] = {brush_texel(p, X[c].x, Y[c].x, Z[c].x), brush_texel(p, X[c].y, Y[c].y, Z[c].y),
                           brush_texel(p, X[c].z, Y[c].z, Z[c].z), brush_texel(p, X[c].w, Y[c].w, Z[c].w)};
        out.put4(base + c * kChunk, s, true);
    }
}

// Lasso tiling: a workgroup owns a block of kLassoRows x kLassoCols texels;
// wave w covers its columns [32w, 32w + 32), in step c the rows
// [8c, 8c + 8), lane l the 4 texels at row l/8, columns 4(l%8)..+3.  One
// step of a wave is thus an 8 x 32 patch of the atlas, whose image on the
// screen is compact, so the depth reads of one instruction touch few cache
// lines (the image of a 256-texel row segment is a long screen-space curve).
// Texels beyond the atlas read as NaN positions, which no lasso selects, so
// edge blocks take the same wave-wide path with bounds-checked loads and
// stores; atlases whose width is not a multiple of 4 use those loads
// everywhere (rows are then not 16-byte aligned).  The 8 lanes of a row hold
// one mask word of a numeric layer when the width is a multiple of 32.
constexpr int kLassoRows = 32, kLassoCols = 128;

template <typename Sink>
__global__ __launch_bounds__(kBlock) void k_lasso(const float *__restrict__ px, const float *__restrict__ py,
                                                  const float *__restrict__ pz, Sink out, int32_t W,
                                                  int32_t H, LassoParams p, const float *__restrict__ depth) {
    const int lane = threadIdx.x & 63;
    const int x = blockIdx.x * kLassoCols + (threadIdx.x >> 6) * 32 + (lane & 7) * 4;
    const int y0 = blockIdx.y * kLassoRows + (lane >> 3);
    // lane-uniform over full blocks of a width that keeps rows 16-byte aligned
    const bool vec = (W & 3) == 0 && (blockIdx.x + 1) * kLassoCols <= W && (blockIdx.y + 1) * kLassoRows <= H;
    float4 X[4], Y[4], Z[4];
    if (vec) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int64_t t = (int64_t)(y0 + 8 * c) * W + x;
            X[c] = load_stream4(px + t);
            Y[c] = load_stream4(py + t);
            Z[c] = load_stream4(pz + t);
        }
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int y = y0 + 8 * c;
            const int64_t t = (int64_t)y * W + x;
            float v[3][4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool in = y < H && x + k < W;
                v[0][k] = in ? px[t + k] : NAN;
                v[1][k] = in ? py[t + k] : NAN;
                v[2][k] = in ? pz[t + k] : NAN;
            }
            X[c] = make_float4(v[0][0], v[0][1], v[0][2], v[0][3]);
            Y[c] = make_float4(v[1][0], v[1][1], v[1][2], v[1][3]);
            Z[c] = make_float4(v[2][0], v[2][1], v[2][2], v[2][3]);
        }
    }
    // all four steps' projections and polygon tests first, then all their
    // depth reads, so that a wave waits for the depth map once
    int pix[4][4];
    float d[4][4], dv[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) lasso_quad_index(p, X[c], Y[c], Z[c], pix[c], d[c]);
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int k = 0; k < 4; ++k) dv[c][k] = pix[c][k] >= 0 ? depth[pix[c][k]] : 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        bool s[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) s[k] = pix[c][k] >= 0 && lasso_depth_pass(p, d[c][k], dv[c][k]);
        const int y = y0 + 8 * c;
        const int64_t t = (int64_t)y * W + x;
        if (vec)
            out.put4(t, s, (W & 31) == 0);
        else if (y < H)
            out.put_some(t, W - x, s);
    }
}

int32_t check_edit(const uvl_geom *g, const uvl_layer *l, uint32_t label) {
    if (!geom_pos_ok(g) || !layer_ok(l)) return UVL_E_INVAL;
    if (!dtype_ok(l->dtype)) return UVL_E_DTYPE;
    if (label > dtype_max(l->dtype)) return UVL_E_DTYPE;
    if (l->width != g->width || l->height != g->height) return UVL_E_SHAPE;
    return device_ok();
}

}  // namespace

// Host-side preparation of a lasso's kernel parameters; also used by the
// batched wave path.  Returns false for an invalid polygon.
static_assert(sizeof(LassoParams) <= 3584, "lasso parameters travel as a kernel argument");

bool make_lasso_params(const float view_proj[16], const float *poly, int32_t n, int32_t dw, int32_t dh,
                       float bias, LassoParams &p) {
    if (n < 3 || n > kMaxPoly || !poly || !view_proj || dw < 1 || dh < 1 || !std::isfinite(bias)) return false;
    for (int k = 0; k < 16; ++k) p.M[k] = view_proj[k];
    p.bias = bias;
    p.dw = dw;
    p.dh = dh;
    p.n = n;
    float ylo = INFINITY, yhi = -INFINITY, xhi = -INFINITY, xlo = INFINITY;
    for (int k = 0; k < n; ++k) {
        const float x0 = poly[2 * k], y0 = poly[2 * k + 1];
        const float x1 = poly[2 * ((k + 1) % n)], y1 = poly[2 * ((k + 1) % n) + 1];
        if (!std::isfinite(x0) || !std::isfinite(y0)) return false;
        const float dx = x1 - x0, dy = y1 - y0;
        const bool up = y1 > y0;
        p.edge[k] = LassoEdge{x0, y0, y1, up ? dx : -dx, up ? dy : -dy, fmaxf(x0, x1), x1, 0.0f};
        ylo = fminf(ylo, y0);
        yhi = fmaxf(yhi, y0);
        xhi = fmaxf(xhi, x0);
        xlo = fminf(xlo, x0);
    }
    for (int k = n; k < kMaxPoly; ++k) p.edge[k] = LassoEdge{};
    p.ylo = ylo;
    p.yhi = yhi;
    p.xhi = xhi;
    p.xlo = xlo;
    p.ylo_m = ylo - 1e-4f * (1.0f + fabsf(ylo));
    p.yhi_m = yhi + 1e-4f * (1.0f + fabsf(yhi));
    p.xhi_m = xhi + 1e-4f * (1.0f + fabsf(xhi));
    {
        float xabs_v = 0.0f;
        for (int k = 0; k < n; ++k) xabs_v = fmaxf(xabs_v, fabsf(poly[2 * k]));
        p.xlo_m = xlo - (1e-4f * (1.0f + fabsf(xlo)) + 1e-5f * (2.0f + xabs_v));
    }
    // the frustum bound of the exact test, widened alike, joins each side
    p.xlo_m = fmaxf(p.xlo_m, -1.0001f);
    p.xhi_m = fminf(p.xhi_m, 1.0001f);
    p.ylo_m = fmaxf(p.ylo_m, -1.0001f);
    p.yhi_m = fminf(p.yhi_m, 1.0001f);
    // tile culling planes (see LassoCull)
    {
        const double m = 2e-3;
        const double rx0 = fmax(-1.0, (double)xlo) - m, rx1 = fmin(1.0, (double)xhi) + m;
        const double ry0 = fmax(-1.0, (double)ylo) - m, ry1 = fmin(1.0, (double)yhi) + m;
        double Md[16];
        for (int k = 0; k < 16; ++k) Md[k] = (double)view_proj[k];
        for (int j = 0; j < 4; ++j) {
            p.cull.plane[0][j] = Md[j] - rx0 * Md[12 + j];          // clip_x - rx0 clip_w
            p.cull.plane[1][j] = rx1 * Md[12 + j] - Md[j];          // rx1 clip_w - clip_x
            p.cull.plane[2][j] = Md[4 + j] - ry0 * Md[12 + j];      // clip_y - ry0 clip_w
            p.cull.plane[3][j] = ry1 * Md[12 + j] - Md[4 + j];      // ry1 clip_w - clip_y
            p.cull.wrow[j] = Md[12 + j];
            p.cull.ax[j] = fabs(Md[j]);
            p.cull.ay[j] = fabs(Md[4 + j]);
            p.cull.az[j] = fabs(Md[8 + j]);
            p.cull.aw[j] = fabs(Md[12 + j]);
        }
    }
    // y-slabs: slab s holds the edges whose y-range meets
    // [ylo + (s - 1e-3)/inv_h, ylo + (s + 1 + 1e-3)/inv_h]; horizontal edges
    // never straddle and are left out
    // (with no usable slab height every texel maps to slab 0, which then
    // holds every edge)
    const float hf = (yhi - ylo) / (float)kSlabs;
    p.inv_h = hf > 0.0f ? 1.0f / hf : 0.0f;
    if (!std::isfinite(p.inv_h)) p.inv_h = 0.0f;
    for (int s = 0; s < kSlabs; ++s) {
        uint64_t m = 0;
        const double lo = p.inv_h > 0.0f ? (double)ylo + (s - 1e-3) / (double)p.inv_h : -INFINITY;
        const double hi = p.inv_h > 0.0f ? (double)ylo + (s + 1 + 1e-3) / (double)p.inv_h : INFINITY;
        for (int k = 0; k < n; ++k) {
            const LassoEdge &E = p.edge[k];
            if (E.y0 == E.y1) continue;
            const double emin = fmin(E.y0, E.y1), emax = fmax(E.y0, E.y1);
            if (emin <= hi && emax >= lo) m |= 1ull << k;
        }
        p.slab_edges[s] = m;
        float sx0 = INFINITY, sx1 = -INFINITY;
        for (int k = 0; k < n; ++k)
            if ((m >> k) & 1) {
                const float ex1 = p.edge[k].xmax;
                const float exa = poly[2 * k], exb = poly[2 * ((k + 1) % n)];
                sx0 = fminf(sx0, fminf(exa, exb));
                sx1 = fmaxf(sx1, ex1);
            }
        p.cull.slab_x0[s] = sx0;
        p.cull.slab_x1[s] = sx1;
    }
    float xabs = 0.0f;
    for (int k = 0; k < kMaxPoly; ++k) {
        const LassoEdge &E = p.edge[k];
        p.cull.slope[k] = (k < n && E.sdy != 0.0f) ? (double)E.sdx / (double)E.sdy : 0.0;
        if (k < n) xabs = fmaxf(xabs, fabsf(E.x0));
    }
    p.cull.xabs = xabs;
    return true;
}

}  // namespace uvl

using namespace uvl;

namespace {

template <typename Sink>
void launch_brush(const uvl_geom *geom, const float center[3], float radius, const Sink &out, hipStream_t s) {
    const int64_t n = (int64_t)geom->width * geom->height;
    const BrushParams p{center[0], center[1], center[2], radius * radius};
    hipLaunchKernelGGL(k_brush<Sink>, dim3((unsigned)ceil_div(n, kTile)), dim3(kBlock), 0, s, geom->pos_x,
                       geom->pos_y, geom->pos_z, out, n, p);
}

template <typename Sink>
void launch_lasso(const uvl_geom *geom, const LassoParams &p, const float *depth, const Sink &out, hipStream_t s) {
    const int32_t W = geom->width, H = geom->height;
    const dim3 grid((unsigned)ceil_div(W, kLassoCols), (unsigned)ceil_div(H, kLassoRows));
    hipLaunchKernelGGL(k_lasso<Sink>, grid, dim3(kBlock), 0, s, geom->pos_x, geom->pos_y, geom->pos_z, out, W, H,
                       p, depth);
}

bool brush_args_ok(const float center[3], float radius) {
    return center && radius >= 0.0f && std::isfinite(radius) && std::isfinite(center[0]) &&
           std::isfinite(center[1]) && std::isfinite(center[2]);
}

// Lasso arguments shared by the label and numeric calls.
bool lasso_args(const float view_proj[16], const float *poly_xy, int32_t n, const float *depth, int32_t dw,
                int32_t dh, float bias, LassoParams &p) {
    if (!depth || dw > kMaxDepthSide || dh > kMaxDepthSide) return false;
    if (!make_lasso_params(view_proj, poly_xy, n, dw, dh, bias, p)) return false;
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(view_proj[k])) return false;
    return true;
}

}  // namespace

extern "C" int32_t uvl_edit_brush(const uvl_geom *geom, const uvl_layer *layer, const float center[3],
                                  float radius, uint32_t label, void *stream) {
    if (!brush_args_ok(center, radius)) return UVL_E_INVAL;
    if (int32_t s = check_edit(geom, layer, label)) return s;
    with_label_sink(layer, label, [&](auto out) { launch_brush(geom, center, radius, out, as_stream(stream)); });
    return launch_status();
}

extern "C" int32_t uvl_edit_lasso(const uvl_geom *geom, const uvl_layer *layer, const float view_proj[16],
                                  const float *poly_xy, int32_t n, const float *depth, int32_t dw, int32_t dh,
                                  float bias, uint32_t label, void *stream) {
    LassoParams p;
    if (!lasso_args(view_proj, poly_xy, n, depth, dw, dh, bias, p)) return UVL_E_INVAL;
    if (int32_t s = check_edit(geom, layer, label)) return s;
    with_label_sink(layer, label, [&](auto out) { launch_lasso(geom, p, depth, out, as_stream(stream)); });
    return launch_status();
}

extern "C" int32_t uvl_numeric_brush(const uvl_geom *geom, const uvl_numeric *layer, const float center[3],
                                     float radius, int32_t mode, double value, void *stream) {
    if (!brush_args_ok(center, radius)) return UVL_E_INVAL;
    uint32_t bits = 0;
    if (int32_t s = check_numeric_edit(geom, layer, mode, value, bits)) return s;
    with_value_sink(layer, bits, mode, [&](auto out) { launch_brush(geom, center, radius, out, as_stream(stream)); });
    return launch_status();
}

extern "C" int32_t uvl_numeric_lasso(const uvl_geom *geom, const uvl_numeric *layer, const float view_proj[16],
                                     const float *poly_xy, int32_t n, const float *depth, int32_t dw, int32_t dh,
                                     float bias, int32_t mode, double value, void *stream) {
    LassoParams p;
    if (!lasso_args(view_proj, poly_xy, n, depth, dw, dh, bias, p)) return UVL_E_INVAL;
    uint32_t bits = 0;
    if (int32_t s = check_numeric_edit(geom, layer, mode, value, bits)) return s;
    with_value_sink(layer, bits, mode, [&](auto out) { launch_lasso(geom, p, depth, out, as_stream(stream)); });
    return launch_status();
}
