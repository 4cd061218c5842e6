// Per-texel selection predicates of the two edit tools (device code).
//
// Both are evaluated in fp32 with every operation rounded once: fmaf where
// written, IEEE division, compiled with -ffp-contract=off so no other
// multiply-add is fused.  Their results are therefore fixed bit for bit by
// the texel's stored position and the edit's parameters.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace uvl {

constexpr int kMaxPoly = 64;

// Brush: the closed ball |p - c| <= r (a 3D stand-in for the paper's circular
// tool, §4.3.1).  NaN positions (uncovered texels) never match.
struct BrushParams {
    float cx, cy, cz, r2;   // r2 = r*r rounded to fp32
};

__device__ __forceinline__ bool brush_texel(const BrushParams &B, float x, float y, float z) {
    const float dx = x - B.cx, dy = y - B.cy, dz = z - B.cz;
    const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
    return d2 <= B.r2;
}

// Lasso: the texel projects through the camera into the unit cube, passes the
// depth test with bias, and lies inside the polygon (§4.3.1: depth test,
// projective mapping with out-of-range coordinates discarded, shape mask).
// Per edge k (from vertex k to vertex k+1): x0, y0, y1 and the edge vector
// (x1-x0, y1-y0) rounded to fp32, negated for downward edges (y1 < y0) so
// that the crossing test is always "lhs < rhs"; negation is exact, so this is
// the same comparison as "lhs > rhs" on the unnegated values.
//
// Edge culling by y-slabs: [ylo, yhi) is cut into kSlabs slabs; a texel's
// slab is floor((yn - ylo) * inv_h) (clamped), and slab_edges[s] holds every
// edge whose y-range meets slab s widened by 1e-3 of a slab on both sides,
// far more than the two fp32 roundings of the slab computation can move a
// texel.  An edge can only count for yn if min(y0,y1) <= yn < max(y0,y1), so
// testing the edges of the texel's slab (or of any set of slabs containing
// it) gives exactly the crossing count over all edges.
constexpr int kSlabs = 32;

// One polygon edge, padded to 32 bytes so that a wave loads it with a single
// scalar load.
struct alignas(32) LassoEdge {
    float x0, y0, y1, sdx, sdy, xmax, pad0, pad1;   // xmax = max(x0, x1)
};

struct LassoParams {
    float M[16];
    float bias;
    int32_t dw, dh, n;
    float ylo, yhi, xhi;        // polygon bounds: min y, max y, max x
    float ylo_m, yhi_m, xhi_m;  // the same widened by 1e-4 (1 + |v|), for the reciprocal pre-test
    float inv_h;                // slabs per unit of y
    uint64_t slab_edges[kSlabs];
    LassoEdge edge[kMaxPoly];
};

// Everything but the polygon test: true if the texel is a candidate, with
// its NDC position.
// PT is LassoParams, possibly qualified with the constant address space so
// that a parameter block in global memory is read with scalar loads.
template <class PT>
__device__ __forceinline__ bool lasso_front(const PT &P, const float *__restrict__ depth, float x, float y,
                                            float z, float &xn, float &yn) {
    float c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        c[k] = __builtin_fmaf(P.M[4 * k + 2], z, __builtin_fmaf(P.M[4 * k + 1], y, __builtin_fmaf(P.M[4 * k + 0], x, P.M[4 * k + 3])));
    if (!(c[3] > 0.0f)) return false;
    if (c[3] >= 1e-30f) {
        // Pre-test with the hardware reciprocal: x/w and y/w are within 3e-7
        // relative of the exact quotients, far inside the 1e-4 margins, so a
        // texel rejected here fails the exact tests below as well.
        const float r = __builtin_amdgcn_rcpf(c[3]);
        const float ax = c[0] * r, ay = c[1] * r;
        if (!(ax >= -1.0001f && ax <= 1.0001f && ay >= P.ylo_m && ay <= P.yhi_m && ax <= P.xhi_m)) return false;
    }
    xn = c[0] / c[3];
    yn = c[1] / c[3];
    if (!(xn >= -1.0f && xn <= 1.0f && yn >= -1.0f && yn <= 1.0f)) return false;
    // Outside [ylo, yhi) no edge straddles yn; right of xhi every straddling
    // edge fails the crossing test even after rounding (monotone rounding of
    // the differences and products): both give "outside" exactly.
    if (!(yn >= P.ylo && yn < P.yhi && xn <= P.xhi)) return false;
    const float zn = c[2] / c[3];
    if (!(zn >= -1.0f && zn <= 1.0f)) return false;
    int ix = (int)floorf(__builtin_fmaf(xn, 0.5f, 0.5f) * (float)P.dw);
    int iy = (int)floorf(__builtin_fmaf(yn, 0.5f, 0.5f) * (float)P.dh);
    ix = ix > P.dw - 1 ? P.dw - 1 : ix;
    iy = iy > P.dh - 1 ? P.dh - 1 : iy;
    const float d = __builtin_fmaf(zn, 0.5f, 0.5f);
    return d <= depth[(int64_t)iy * P.dw + ix] + P.bias;
}

template <class PT>
__device__ __forceinline__ int lasso_slab(const PT &P, float yn) {
    int s = (int)((yn - P.ylo) * P.inv_h);
    s = s < 0 ? 0 : s;
    return s > kSlabs - 1 ? kSlabs - 1 : s;
}

// Crossing test of edge e for a point; toggles `inside` when it counts.
__device__ __forceinline__ void lasso_edge(float ex0, float ey0, float ey1, float esdx, float esdy, float xn,
                                           float yn, bool &inside) {
    const bool straddle = (ey0 > yn) != (ey1 > yn);
    const float lhs = (xn - ex0) * esdy;
    const float rhs = esdx * (yn - ey0);
    inside ^= straddle && (lhs < rhs);
}

// The whole predicate for one texel (edges of its own slab).
template <class PT>
__device__ __forceinline__ bool lasso_texel(const PT &P, const float *__restrict__ depth, float x, float y,
                                            float z) {
    float xn, yn;
    if (!lasso_front(P, depth, x, y, z, xn, yn)) return false;
    uint64_t m = P.slab_edges[lasso_slab(P, yn)];
    bool inside = false;
    while (m) {
        const int e = __builtin_ctzll(m);
        m &= m - 1;
        lasso_edge(P.edge[e].x0, P.edge[e].y0, P.edge[e].y1, P.edge[e].sdx, P.edge[e].sdy, xn, yn, inside);
    }
    return inside;
}

// Wave-wide min / max of a uint32 (every lane of the wave must be active):
// rotations within each 16-lane row by DPP, then the four row results.
__device__ __forceinline__ unsigned wave_min_u32(unsigned v) {
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x121, 0xf, 0xf, false));
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x122, 0xf, 0xf, false));
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x124, 0xf, 0xf, false));
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x128, 0xf, 0xf, false));
    const unsigned a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
    const unsigned c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    return min(min(a, b), min(c, d));
}

__device__ __forceinline__ float wave_min_f32(float v) {
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x121, 0xf, 0xf, false)));
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x122, 0xf, 0xf, false)));
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x124, 0xf, 0xf, false)));
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x128, 0xf, 0xf, false)));
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return fminf(fminf(a, b), fminf(c, d));
}

__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x121, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x122, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x124, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x128, 0xf, 0xf, false));
    const unsigned a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
    const unsigned c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    return max(max(a, b), max(c, d));
}

// Lasso over 4 texels per lane, the polygon test shared by the whole wave:
// the union of the slab edge masks over the wave's candidate slabs is built
// in scalar registers and each of its edges is tested against every texel.
// An edge whose both ends lie left of every candidate (xmax < min xn) is
// skipped: for a point right of both ends the crossing test is false even
// after rounding (the same monotonicity argument as the xhi bound).
// Must be called by all 64 lanes.
template <class PT>
__device__ __forceinline__ void lasso_quad(const PT &P, const float *__restrict__ depth, const float4 &X,
                                           const float4 &Y, const float4 &Z, bool sel[4]) {
    const float xs[4] = {X.x, X.y, X.z, X.w}, ys[4] = {Y.x, Y.y, Y.z, Y.w}, zs[4] = {Z.x, Z.y, Z.z, Z.w};
    float xn[4], yn[4];
    bool cand[4], inside[4];
    unsigned smin = kSlabs, smax = 0;
    float xmin = INFINITY;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        xn[k] = 0.0f;
        yn[k] = 0.0f;
        cand[k] = lasso_front(P, depth, xs[k], ys[k], zs[k], xn[k], yn[k]);
        inside[k] = false;
        if (cand[k]) {
            const unsigned s = (unsigned)lasso_slab(P, yn[k]);
            smin = min(smin, s);
            smax = max(smax, s);
            xmin = fminf(xmin, xn[k]);
        }
    }
    const unsigned wmin = wave_min_u32(smin), wmax = wave_max_u32(smax);
    if (wmin <= wmax) {
        const float wxmin = wave_min_f32(xmin);
        uint64_t m = 0;
        for (unsigned s = wmin; s <= wmax; ++s) m |= P.slab_edges[s];
        while (m) {
            const int e = __builtin_ctzll(m);
            m &= m - 1;
            const float ex0 = P.edge[e].x0, ey0 = P.edge[e].y0, ey1 = P.edge[e].y1;
            const float esdx = P.edge[e].sdx, esdy = P.edge[e].sdy, exmax = P.edge[e].xmax;
            if (exmax < wxmin) continue;
#pragma unroll
            for (int k = 0; k < 4; ++k) lasso_edge(ex0, ey0, ey1, esdx, esdy, xn[k], yn[k], inside[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) sel[k] = cand[k] && inside[k];
}

}  // namespace uvl
