// The fixed-point raster rule shared by the texture-space geometry image
// (geom.hip) and the screen-space depth texture (raster.hip).
//
// The paper renders the mesh with its texture coordinates as vertex
// positions (§4.3.1) and relies on the GPU rasteriser, which states no
// sample rule; the rule here: coordinates snapped to 1/256 cell, round half
// to even; cell centres at (256 i + 128, 256 j + 128); a centre is inside
// when every edge function of the counter-clockwise order is > 0, or == 0
// on an owning edge (t.y < s.y, or t.y == s.y and t.x > s.x).  Edge
// functions are exact int64, so the coverage is exact and independent of
// evaluation order.  (Internal header.)
#pragma once

#include <math.h>

#include "uvl_internal.h"

namespace uvl {
namespace {

struct Tri2 {
    long long X[3], Y[3];
    long long E;          // doubled area, > 0
    int ord[3];           // counter-clockwise order of the original vertices
    long long A[3], B[3], C[3];  // edge k (opposite ord[k]): e = A*px + B*py + C
    int bias[3];          // 0 if the edge owns its boundary, else 1 (inside iff e >= bias)
};

__device__ __forceinline__ long long snap256(double x) { return (long long)rint(x * 256.0); }

__device__ __forceinline__ bool tri_setup(Tri2 &T) {
    long long E = (T.X[1] - T.X[0]) * (T.Y[2] - T.Y[0]) - (T.Y[1] - T.Y[0]) * (T.X[2] - T.X[0]);
    if (E == 0) return false;
    T.ord[0] = 0;
    T.ord[1] = E > 0 ? 1 : 2;
    T.ord[2] = E > 0 ? 2 : 1;
    T.E = E > 0 ? E : -E;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int s = T.ord[(k + 1) % 3], t = T.ord[(k + 2) % 3];
        const long long dx = T.X[t] - T.X[s], dy = T.Y[t] - T.Y[s];
        T.A[k] = -dy;
        T.B[k] = dx;
        T.C[k] = dy * T.X[s] - dx * T.Y[s];
        T.bias[k] = (dy < 0 || (dy == 0 && dx > 0)) ? 0 : 1;
    }
    return true;
}

// Ownership bias of an edge with coefficients A = -dy, B = dx: 0 if it owns
// its boundary (dy < 0, or dy == 0 and dx > 0), else 1.
__device__ __forceinline__ int edge_bias(long long A, long long B) { return (A > 0 || (A == 0 && B > 0)) ? 0 : 1; }

// Cells whose centre 256 k + 128 lies in [mn, mx], clamped to [0, n).
__device__ __forceinline__ void cell_range(long long mn, long long mx, int n, int &lo, int &hi) {
    long long a = -((128 - mn) >> 8);
    long long b = (mx - 128) >> 8;
    lo = (int)(a < 0 ? 0 : a);
    hi = (int)(b > n - 1 ? n - 1 : b);
}

__device__ __forceinline__ void bbox(const Tri2 &T, int W, int H, int &i0, int &i1, int &j0, int &j1) {
    long long mnx = min(T.X[0], min(T.X[1], T.X[2])), mxx = max(T.X[0], max(T.X[1], T.X[2]));
    long long mny = min(T.Y[0], min(T.Y[1], T.Y[2])), mxy = max(T.Y[0], max(T.Y[1], T.Y[2]));
    cell_range(mnx, mxx, W, i0, i1);
    cell_range(mny, mxy, H, j0, j1);
}

// Edge functions at a cell centre, unbiased, in the original vertex order.
__device__ __forceinline__ void edge_values(const Tri2 &T, long long px, long long py, long long e[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) e[T.ord[k]] = T.A[k] * px + T.B[k] * py + T.C[k];
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ double wave_min(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o));
    return x;
}

}  // namespace
}  // namespace uvl
