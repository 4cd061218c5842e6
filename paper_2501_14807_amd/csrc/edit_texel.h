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
struct LassoParams {
    float M[16];
    float bias;
    int32_t dw, dh, n;
    float ylo, yhi, xhi;    // polygon bounds: min y, max y, max x
    float x0[kMaxPoly], y0[kMaxPoly], y1[kMaxPoly], sdx[kMaxPoly], sdy[kMaxPoly];
};

__device__ __forceinline__ bool lasso_texel(const LassoParams &P, const float *__restrict__ depth, float x,
                                            float y, float z) {
    float c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        c[k] = __builtin_fmaf(P.M[4 * k + 2], z, __builtin_fmaf(P.M[4 * k + 1], y, __builtin_fmaf(P.M[4 * k + 0], x, P.M[4 * k + 3])));
    if (!(c[3] > 0.0f)) return false;
    const float xn = c[0] / c[3];
    const float yn = c[1] / c[3];
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
    if (!(d <= depth[(int64_t)iy * P.dw + ix] + P.bias)) return false;
    bool inside = false;
    for (int k = 0; k < P.n; ++k) {
        if ((P.y0[k] > yn) != (P.y1[k] > yn)) {
            const float lhs = (xn - P.x0[k]) * P.sdy[k];
            const float rhs = P.sdx[k] * (yn - P.y0[k]);
            inside ^= (lhs < rhs);
        }
    }
    return inside;
}

}  // namespace uvl
