// Rasterisation for libuvl on gfx950: the texture-space geometry image and
// the screen-space depth texture.
//
// Both follow one fixed-point rule (§4.3.1 renders the mesh with its texture
// coordinates as vertex positions, and renders scene depth for the depth
// test; the paper relies on the GPU rasteriser and states no sample rule):
// coordinates snapped to 1/256 cell, round half to even; cell centres at
// (256 i + 128, 256 j + 128); a centre is inside when every edge function of
// the counter-clockwise order is > 0, or == 0 on an owning edge (t.y < s.y,
// or t.y == s.y and t.x > s.x).  Edge functions are exact int64, so the
// coverage is exact and independent of evaluation order.
//
// Launch structure per raster:
//   1. one thread per triangle: set-up, and for bounding boxes of at most
//      kSmallCells cells the whole raster, with an atomicMin per covered cell
//      (lowest triangle index / nearest depth wins, order-independent);
//      larger triangles go to a queue in the caller's workspace;
//   2. a fixed grid of workgroups drains the queue, one triangle per
//      workgroup, its 256 threads striding over the bounding box;
//   3. (geometry image) one thread per texel interpolates the owner's
//      attributes and writes the structure-of-arrays planes coalesced;
//   4. (geometry image) one thread per texel quantises the area weight.
#include <math.h>

#include <mutex>

#include "uvl_internal.h"

namespace uvl {
namespace {

constexpr int kSmallCells = 64;
constexpr int kBigGrid = 2048;

// Workspace counters (first 256 bytes of the workspace).
struct Counters {
    unsigned int queue_len;
    unsigned int flags;              // bit 0: vertex index out of range, bit 1: uv out of range
    unsigned int pad0;
    unsigned int pad1;
    unsigned long long max_w_bits;   // fp64 bits of the largest texel weight (positive)
    unsigned long long min_w_bits;   // fp64 bits of the smallest weight two words hold to 2^-20
};

constexpr unsigned kFlagIndex = 1u, kFlagUV = 2u;

// Largest ratio of texel weights for which one rounding onto the scale's
// grid stays within 2^-20 relative: one word (largest weight in [2^30,
// 2^31)) and two words (in [2^62, 2^63)).
constexpr int kNarrowRatioLog2 = 11, kWideRatioLog2 = 43;

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

// ---------------------------------------------------------------------------
// geometry image

__device__ __forceinline__ bool geom_tri(const float *__restrict__ uv, const int32_t *__restrict__ tri,
                                         int64_t nv, int64_t t, int W, int H, Tri2 &T, int v[3],
                                         unsigned *flags) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[k] = tri[3 * t + k];
        if (v[k] < 0 || v[k] >= nv) {
            if (flags) atomicOr(flags, kFlagIndex);
            return false;
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float u = uv[2 * (int64_t)v[k]], w = uv[2 * (int64_t)v[k] + 1];
        if (!(fabsf(u) <= 4.0f) || !(fabsf(w) <= 4.0f)) {
            if (flags) atomicOr(flags, kFlagUV);
            return false;
        }
        T.X[k] = snap256((double)u * (double)W);
        T.Y[k] = snap256((double)w * (double)H);
    }
    return tri_setup(T);
}

__global__ __launch_bounds__(kBlock) void k_geom_tri(const float *__restrict__ uv, const float *__restrict__ pos,
                                                     const int32_t *__restrict__ tri, int64_t nv, int64_t nt,
                                                     int W, int H, int32_t *__restrict__ owner,
                                                     double *__restrict__ w_tri, unsigned *__restrict__ queue,
                                                     Counters *__restrict__ ctr) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nt) return;
    Tri2 T;
    int v[3];
    if (!geom_tri(uv, tri, nv, t, W, H, T, v, &ctr->flags)) {
        w_tri[t] = 0.0;
        return;
    }
    // texel area weight 131072 * A3 / |E| (surface area per 1/(W H) of UV area)
    double P[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) P[k][c] = (double)pos[3 * (int64_t)v[k] + c];
    double u1[3], u2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) { u1[c] = P[1][c] - P[0][c]; u2[c] = P[2][c] - P[0][c]; }
    const double f0 = u1[1] * u2[2] - u1[2] * u2[1];
    const double f1 = u1[2] * u2[0] - u1[0] * u2[2];
    const double f2 = u1[0] * u2[1] - u1[1] * u2[0];
    const double flen = sqrt(f0 * f0 + f1 * f1 + f2 * f2);
    w_tri[t] = 131072.0 * (0.5 * flen) / (double)T.E;

    int i0, i1, j0, j1;
    bbox(T, W, H, i0, i1, j0, j1);
    if (i1 < i0 || j1 < j0) return;
    const long long cells = (long long)(i1 - i0 + 1) * (j1 - j0 + 1);
    if (cells > kSmallCells) {
        queue[atomicAdd(&ctr->queue_len, 1u)] = (unsigned)t;
        return;
    }
    const long long px0 = 256LL * i0 + 128;
    for (int j = j0; j <= j1; ++j) {
        const long long py = 256LL * j + 128;
        long long e0 = T.A[0] * px0 + T.B[0] * py + T.C[0] - T.bias[0];
        long long e1 = T.A[1] * px0 + T.B[1] * py + T.C[1] - T.bias[1];
        long long e2 = T.A[2] * px0 + T.B[2] * py + T.C[2] - T.bias[2];
        const long long s0 = 256 * T.A[0], s1 = 256 * T.A[1], s2 = 256 * T.A[2];
        int32_t *row = owner + (int64_t)j * W;
        for (int i = i0; i <= i1; ++i) {
            if ((e0 | e1 | e2) >= 0) atomicMin(row + i, (int32_t)t);
            e0 += s0; e1 += s1; e2 += s2;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_geom_big(const float *__restrict__ uv, const int32_t *__restrict__ tri,
                                                     int64_t nv, int W, int H, int32_t *__restrict__ owner,
                                                     const unsigned *__restrict__ queue,
                                                     const Counters *__restrict__ ctr) {
    const unsigned n = ctr->queue_len;
    for (unsigned q = blockIdx.x; q < n; q += gridDim.x) {
        const int64_t t = queue[q];
        Tri2 T;
        int v[3];
        if (!geom_tri(uv, tri, nv, t, W, H, T, v, nullptr)) continue;
        int i0, i1, j0, j1;
        bbox(T, W, H, i0, i1, j0, j1);
        const unsigned bw = (unsigned)(i1 - i0 + 1);
        const unsigned cells = bw * (unsigned)(j1 - j0 + 1);
        for (unsigned c = threadIdx.x; c < cells; c += kBlock) {
            const int i = i0 + (int)(c % bw), j = j0 + (int)(c / bw);
            const long long px = 256LL * i + 128, py = 256LL * j + 128;
            bool in = true;
#pragma unroll
            for (int k = 0; k < 3; ++k) in &= T.A[k] * px + T.B[k] * py + T.C[k] >= T.bias[k];
            if (in) atomicMin(owner + (int64_t)j * W + i, (int32_t)t);
        }
    }
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

struct GeomPlanes {
    int32_t *owner;
    float *px, *py, *pz, *nx, *ny, *nz, *b1, *b2;
};

__global__ __launch_bounds__(kBlock) void k_geom_attr(const float *__restrict__ uv, const float *__restrict__ pos,
                                                      const float *__restrict__ nrm,
                                                      const int32_t *__restrict__ tri, int W, int H,
                                                      GeomPlanes g, const double *__restrict__ w_tri,
                                                      Counters *__restrict__ ctr) {
    const int64_t N = (int64_t)W * H;
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double wmax = 0.0;
    if (idx < N) {
        const int32_t t = g.owner[idx];
        if (t == kEmptyOwner) {
            g.owner[idx] = -1;
            g.px[idx] = g.py[idx] = g.pz[idx] = __builtin_nanf("");
            if (g.nx) g.nx[idx] = g.ny[idx] = g.nz[idx] = 0.0f;
            if (g.b1) g.b1[idx] = g.b2[idx] = 0.0f;
        } else {
            Tri2 T;
            int v[3];
            geom_tri(uv, tri, 1LL << 62, t, W, H, T, v, nullptr);
            const int i = (int)(idx % W), j = (int)(idx / W);
            long long e[3];
            edge_values(T, 256LL * i + 128, 256LL * j + 128, e);
            const double E = (double)T.E;
            const double b0 = (double)e[0] / E, b1 = (double)e[1] / E, b2 = (double)e[2] / E;
            if (g.b1) { g.b1[idx] = (float)b1; g.b2[idx] = (float)b2; }
            double P[3][3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) P[k][c] = (double)pos[3 * (int64_t)v[k] + c];
            g.px[idx] = (float)(b0 * P[0][0] + b1 * P[1][0] + b2 * P[2][0]);
            g.py[idx] = (float)(b0 * P[0][1] + b1 * P[1][1] + b2 * P[2][1]);
            g.pz[idx] = (float)(b0 * P[0][2] + b1 * P[1][2] + b2 * P[2][2]);
            if (g.nx) {
                double m[3];
                if (nrm) {
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        m[c] = b0 * (double)nrm[3 * (int64_t)v[0] + c] + b1 * (double)nrm[3 * (int64_t)v[1] + c] +
                               b2 * (double)nrm[3 * (int64_t)v[2] + c];
                } else {
                    double u1[3], u2[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) { u1[c] = P[1][c] - P[0][c]; u2[c] = P[2][c] - P[0][c]; }
                    m[0] = u1[1] * u2[2] - u1[2] * u2[1];
                    m[1] = u1[2] * u2[0] - u1[0] * u2[2];
                    m[2] = u1[0] * u2[1] - u1[1] * u2[0];
                }
                const double len = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
                g.nx[idx] = len > 0.0 ? (float)(m[0] / len) : 0.0f;
                g.ny[idx] = len > 0.0 ? (float)(m[1] / len) : 0.0f;
                g.nz[idx] = len > 0.0 ? (float)(m[2] / len) : 0.0f;
            }
            wmax = w_tri[t];
        }
    }
    // One atomic per workgroup at most: atomics on one address from every
    // wave of a 64M-texel image serialise and would dominate the kernel.
    __shared__ double s_w[kBlock / 64];
    wmax = wave_max(wmax);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = wmax;
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 1; k < kBlock / 64; ++k) wmax = fmax(wmax, s_w[k]);
        const unsigned long long b = (unsigned long long)__double_as_longlong(wmax);
        // The counter only grows, so any value read is a lower bound of its
        // final value and a weight not above it needs no atomic.
        if (wmax > 0.0 && b > __atomic_load_n(&ctr->max_w_bits, __ATOMIC_RELAXED))
            atomicMax(&ctr->max_w_bits, b);
    }
}

// One word per texel (hi == NULL): the largest weight maps into [2^30,
// 2^31); two words: into [2^62, 2^63), low and high words.  Also the
// smallest weight among the texels two words represent to 2^-20 (those of
// at least 2^-kWideRatioLog2 of the largest; lighter ones come from
// triangles of numerically zero 3D area and keep an absolute bound only):
// the host compares it with the largest to tell whether one word suffices.
__global__ __launch_bounds__(kBlock) void k_geom_quant(const int32_t *__restrict__ owner,
                                                       const double *__restrict__ w_tri,
                                                       uint32_t *__restrict__ area_w, uint32_t *__restrict__ hi,
                                                       int64_t N, Counters *__restrict__ ctr) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const double mx = __longlong_as_double((long long)ctr->max_w_bits);
    int ex;
    frexp(mx, &ex);
    double wmin = INFINITY;
    if (idx < N) {
        const int32_t t = owner[idx];
        const double w = t >= 0 ? w_tri[t] : 0.0;
        if (t >= 0 && w >= ldexp(mx, -kWideRatioLog2)) wmin = w;
        if (!hi) {
            area_w[idx] = (unsigned)rint(ldexp(w, 31 - ex));
        } else {
            const unsigned long long v = (unsigned long long)rint(ldexp(w, 63 - ex));
            area_w[idx] = (uint32_t)v;
            hi[idx] = (uint32_t)(v >> 32);
        }
    }
    __shared__ double s_w[kBlock / 64];
    wmin = wave_min(wmin);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = wmin;
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 1; k < kBlock / 64; ++k) wmin = fmin(wmin, s_w[k]);
        // positive doubles order as their bit patterns; the counter only falls
        const unsigned long long b = (unsigned long long)__double_as_longlong(wmin);
        if (wmin < INFINITY && b < __atomic_load_n(&ctr->min_w_bits, __ATOMIC_RELAXED))
            atomicMin(&ctr->min_w_bits, b);
    }
}

// ---------------------------------------------------------------------------
// depth texture

struct Mat4 { float m[16]; };

__device__ __forceinline__ bool project(const Mat4 &M, float x, float y, float z, float &xn, float &yn, float &zn) {
    float c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        c[k] = __builtin_fmaf(M.m[4 * k + 2], z, __builtin_fmaf(M.m[4 * k + 1], y, __builtin_fmaf(M.m[4 * k + 0], x, M.m[4 * k + 3])));
    if (!(c[3] > 0.0f)) return false;
    xn = c[0] / c[3];
    yn = c[1] / c[3];
    zn = c[2] / c[3];
    return true;
}

__device__ __forceinline__ bool depth_tri(const Mat4 &M, const float *__restrict__ pos,
                                          const int32_t *__restrict__ tri, int64_t nv, int64_t t, int Wd,
                                          int Hd, Tri2 &T, double d[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int32_t v = tri[3 * t + k];
        if (v < 0 || v >= nv) return false;
        float xn, yn, zn;
        if (!project(M, pos[3 * (int64_t)v], pos[3 * (int64_t)v + 1], pos[3 * (int64_t)v + 2], xn, yn, zn)) return false;
        if (!(fabsf(xn) <= 16.0f) || !(fabsf(yn) <= 16.0f)) return false;
        const float sx = __builtin_fmaf(xn, 0.5f, 0.5f) * (float)Wd;
        const float sy = __builtin_fmaf(yn, 0.5f, 0.5f) * (float)Hd;
        T.X[k] = snap256((double)sx);
        T.Y[k] = snap256((double)sy);
        d[k] = (double)__builtin_fmaf(zn, 0.5f, 0.5f);
    }
    return tri_setup(T);
}

__device__ __forceinline__ void depth_sample(const Tri2 &T, const double d[3], long long px, long long py,
                                             unsigned *cell) {
    long long e[3];
    edge_values(T, px, py, e);
    const double E = (double)T.E;
    const double z = ((double)e[0] / E) * d[0] + ((double)e[1] / E) * d[1] + ((double)e[2] / E) * d[2];
    if (!(z >= 0.0 && z <= 1.0)) return;
    const float zf = (float)z + 0.0f;   // +0.0f turns -0.0 into +0.0 for the unsigned ordering
    atomicMin(cell, __float_as_uint(zf));
}

__global__ __launch_bounds__(kBlock) void k_depth_tri(Mat4 M, const float *__restrict__ pos,
                                                      const int32_t *__restrict__ tri, int64_t nv, int64_t nt,
                                                      int Wd, int Hd, unsigned *__restrict__ depth,
                                                      unsigned *__restrict__ queue, Counters *__restrict__ ctr) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nt) return;
    Tri2 T;
    double d[3];
    if (!depth_tri(M, pos, tri, nv, t, Wd, Hd, T, d)) return;
    int i0, i1, j0, j1;
    bbox(T, Wd, Hd, i0, i1, j0, j1);
    if (i1 < i0 || j1 < j0) return;
    const long long cells = (long long)(i1 - i0 + 1) * (j1 - j0 + 1);
    if (cells > kSmallCells) {
        queue[atomicAdd(&ctr->queue_len, 1u)] = (unsigned)t;
        return;
    }
    for (int j = j0; j <= j1; ++j) {
        const long long py = 256LL * j + 128;
        for (int i = i0; i <= i1; ++i) {
            const long long px = 256LL * i + 128;
            bool in = true;
#pragma unroll
            for (int k = 0; k < 3; ++k) in &= T.A[k] * px + T.B[k] * py + T.C[k] >= T.bias[k];
            if (in) depth_sample(T, d, px, py, depth + (int64_t)j * Wd + i);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_depth_big(Mat4 M, const float *__restrict__ pos,
                                                      const int32_t *__restrict__ tri, int64_t nv, int Wd, int Hd,
                                                      unsigned *__restrict__ depth,
                                                      const unsigned *__restrict__ queue,
                                                      const Counters *__restrict__ ctr) {
    const unsigned n = ctr->queue_len;
    for (unsigned q = blockIdx.x; q < n; q += gridDim.x) {
        Tri2 T;
        double d[3];
        if (!depth_tri(M, pos, tri, nv, queue[q], Wd, Hd, T, d)) continue;
        int i0, i1, j0, j1;
        bbox(T, Wd, Hd, i0, i1, j0, j1);
        const unsigned bw = (unsigned)(i1 - i0 + 1);
        const unsigned cells = bw * (unsigned)(j1 - j0 + 1);
        for (unsigned c = threadIdx.x; c < cells; c += kBlock) {
            const int i = i0 + (int)(c % bw), j = j0 + (int)(c / bw);
            const long long px = 256LL * i + 128, py = 256LL * j + 128;
            bool in = true;
#pragma unroll
            for (int k = 0; k < 3; ++k) in &= T.A[k] * px + T.B[k] * py + T.C[k] >= T.bias[k];
            if (in) depth_sample(T, d, px, py, depth + (int64_t)j * Wd + i);
        }
    }
}

// Per-tile bounds of the covered positions: one workgroup per tile of
// UVL_TILE_SIDE x UVL_TILE_SIDE texels, a min/max over the non-NaN positions.
__global__ __launch_bounds__(kBlock) void k_tile_box(const float *__restrict__ px, const float *__restrict__ py,
                                                     const float *__restrict__ pz, int W, int H,
                                                     float *__restrict__ box) {
    __shared__ float s_red[6][kBlock / 64];
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int i0 = (int)blockIdx.x * UVL_TILE_SIDE, j0 = (int)blockIdx.y * UVL_TILE_SIDE;
    for (int k = threadIdx.x; k < UVL_TILE_SIDE * UVL_TILE_SIDE; k += kBlock) {
        const int i = i0 + (k % UVL_TILE_SIDE), j = j0 + (k / UVL_TILE_SIDE);
        if (i >= W || j >= H) continue;
        const int64_t t = (int64_t)j * W + i;
        const float v[3] = {px[t], py[t], pz[t]};
        if (v[0] == v[0]) {     // covered (uncovered texels hold NaN)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                mn[c] = fminf(mn[c], v[c]);
                mx[c] = fmaxf(mx[c], v[c]);
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            mn[c] = fminf(mn[c], __shfl_xor(mn[c], o));
            mx[c] = fmaxf(mx[c], __shfl_xor(mx[c], o));
        }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            s_red[c][wv] = mn[c];
            s_red[3 + c][wv] = mx[c];
        }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int c = threadIdx.x;
        float r = s_red[c][0];
        for (int w = 1; w < kBlock / 64; ++w) r = c < 3 ? fminf(r, s_red[c][w]) : fmaxf(r, s_red[c][w]);
        box[6 * ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) + c] = r;
    }
}

__global__ void k_counters_reset(Counters *ctr) {
    if (threadIdx.x == 0) {
        ctr->queue_len = 0;
        ctr->flags = 0;
        ctr->pad0 = 0;
        ctr->pad1 = 0;
        ctr->max_w_bits = 0;
        ctr->min_w_bits = ~0ull;
    }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace
}  // namespace uvl

using namespace uvl;

extern "C" size_t uvl_geom_bytes(int32_t width, int32_t height, uint32_t flags) {
    if (width < 1 || height < 1 || width > kMaxSide || height > kMaxSide) return 0;
    if (flags & ~(uint32_t)(UVL_GEOM_NRM | UVL_GEOM_BARY | UVL_GEOM_TILE_BOX | UVL_GEOM_AREA_HI)) return 0;
    const size_t n = (size_t)width * height;
    const size_t plane = align256(n * 4);        // every plane holds 4-byte elements
    size_t planes = 5;                            // tri_id, pos x/y/z, area_w
    if (flags & UVL_GEOM_NRM) planes += 3;
    if (flags & UVL_GEOM_BARY) planes += 2;
    if (flags & UVL_GEOM_AREA_HI) planes += 1;
    size_t bytes = planes * plane;
    if (flags & UVL_GEOM_TILE_BOX)
        bytes += align256((size_t)ceil_div(width, UVL_TILE_SIDE) * ceil_div(height, UVL_TILE_SIDE) * 6 * sizeof(float));
    return bytes;
}

extern "C" size_t uvl_build_workspace_bytes(int64_t nt) {
    if (nt < 0) return 0;
    return 256 + align256((size_t)nt * sizeof(double)) + align256((size_t)nt * sizeof(unsigned));
}

extern "C" int32_t uvl_build_geometry_image(const uvl_mesh *mesh, uvl_geom *g, void *ws, size_t ws_bytes,
                                            void *stream) {
    if (!mesh || !g || !ws) return UVL_E_INVAL;
    if (mesh->nv < 0 || mesh->nt < 0 || mesh->nv > (1LL << 31) || mesh->nt > (1LL << 31) - 1) return UVL_E_INVAL;
    if (mesh->nt > 0 && (!mesh->pos || !mesh->uv || !mesh->tri)) return UVL_E_INVAL;
    if (g->width < 1 || g->height < 1 || g->width > kMaxSide || g->height > kMaxSide) return UVL_E_INVAL;
    if (!g->tri_id || !g->pos_x || !g->pos_y || !g->pos_z || !g->area_w) return UVL_E_INVAL;
    const bool has_n = g->nrm_x || g->nrm_y || g->nrm_z, has_b = g->bary1 || g->bary2;
    if (has_n && !(g->nrm_x && g->nrm_y && g->nrm_z)) return UVL_E_INVAL;
    if (has_b && !(g->bary1 && g->bary2)) return UVL_E_INVAL;
    if (ws_bytes < uvl_build_workspace_bytes(mesh->nt)) return UVL_E_NOMEM;
    if (int32_t s = device_ok()) return s;

    hipStream_t s = as_stream(stream);
    const int W = g->width, H = g->height;
    const int64_t N = (int64_t)W * H, nt = mesh->nt;
    char *w = static_cast<char *>(ws);
    Counters *ctr = reinterpret_cast<Counters *>(w);
    double *w_tri = reinterpret_cast<double *>(w + 256);
    unsigned *queue = reinterpret_cast<unsigned *>(w + 256 + align256((size_t)nt * sizeof(double)));

    fill_u32(reinterpret_cast<uint32_t *>(g->tri_id), N, (uint32_t)kEmptyOwner, s);
    hipLaunchKernelGGL(k_counters_reset, dim3(1), dim3(64), 0, s, ctr);
    if (nt > 0) {
        hipLaunchKernelGGL(k_geom_tri, dim3((unsigned)ceil_div(nt, kBlock)), dim3(kBlock), 0, s, mesh->uv, mesh->pos,
                           mesh->tri, mesh->nv, nt, W, H, g->tri_id, w_tri, queue, ctr);
        hipLaunchKernelGGL(k_geom_big, dim3(kBigGrid), dim3(kBlock), 0, s, mesh->uv, mesh->tri, mesh->nv, W, H,
                           g->tri_id, queue, ctr);
    }
    GeomPlanes gp{g->tri_id, g->pos_x, g->pos_y, g->pos_z, has_n ? g->nrm_x : nullptr, g->nrm_y, g->nrm_z,
                  has_b ? g->bary1 : nullptr, g->bary2};
    const unsigned grid = (unsigned)ceil_div(N, kBlock);
    hipLaunchKernelGGL(k_geom_attr, dim3(grid), dim3(kBlock), 0, s, mesh->uv, mesh->pos, mesh->nrm, mesh->tri, W,
                       H, gp, w_tri, ctr);
    hipLaunchKernelGGL(k_geom_quant, dim3(grid), dim3(kBlock), 0, s, g->tri_id, w_tri, g->area_w, g->area_w_hi, N,
                       ctr);
    if (g->tile_box)
        hipLaunchKernelGGL(k_tile_box, dim3((unsigned)ceil_div(W, UVL_TILE_SIDE), (unsigned)ceil_div(H, UVL_TILE_SIDE)),
                           dim3(kBlock), 0, s, g->pos_x, g->pos_y, g->pos_z, W, H, g->tile_box);
    if (launch_status() != UVL_OK) return UVL_E_DEVICE;
    Counters host{};
    if (hipMemcpyAsync(&host, ctr, sizeof(Counters), hipMemcpyDeviceToHost, s) != hipSuccess) return UVL_E_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return UVL_E_DEVICE;
    if (host.flags & (kFlagIndex | kFlagUV)) return UVL_E_INVAL;
    const double mx = host.max_w_bits ? __builtin_bit_cast(double, host.max_w_bits) : 0.0;
    int ex = 0;
    frexp(mx, &ex);
    g->area_scale = ldexp(1.0, ex - (g->area_w_hi ? 63 : 31));
    g->area_abs_err = 0.5 * g->area_scale;
    // one word holds every texel to 2^-20 if none lies below 2^-11 of the
    // largest (among those two words would hold to 2^-20)
    if (!g->area_w_hi && host.min_w_bits != ~0ull &&
        __builtin_bit_cast(double, host.min_w_bits) < ldexp(mx, -kNarrowRatioLog2))
        return UVL_E_RANGE;
    return UVL_OK;
}

extern "C" size_t uvl_depth_workspace_bytes(int64_t nt) {
    if (nt < 0) return 0;
    return 256 + align256((size_t)nt * sizeof(unsigned));
}

namespace uvl {
namespace {

int32_t depth_args_ok(const uvl_mesh *mesh, const float *view_proj, const float *depth, int32_t dw, int32_t dh) {
    if (!mesh || !view_proj || !depth) return UVL_E_INVAL;
    if (mesh->nv < 0 || mesh->nt < 0 || mesh->nt > (1LL << 31) - 1) return UVL_E_INVAL;
    if (mesh->nt > 0 && (!mesh->pos || !mesh->tri)) return UVL_E_INVAL;
    if (dw < 1 || dh < 1 || dw > kMaxDepthSide || dh > kMaxDepthSide) return UVL_E_INVAL;
    return UVL_OK;
}

// The depth raster on a workspace of uvl_depth_workspace_bytes(nt) bytes:
// counters in the first 256 bytes, then the queue of large triangles.
int32_t launch_depth(const uvl_mesh *mesh, const float *view_proj, float *depth, int32_t dw, int32_t dh, void *ws,
                     hipStream_t s) {
    Mat4 M;
    for (int k = 0; k < 16; ++k) M.m[k] = view_proj[k];
    Counters *ctr = static_cast<Counters *>(ws);
    unsigned *queue = reinterpret_cast<unsigned *>(static_cast<char *>(ws) + 256);
    fill_u32(reinterpret_cast<uint32_t *>(depth), (int64_t)dw * dh, 0x3f800000u, s);   // 1.0f
    hipLaunchKernelGGL(k_counters_reset, dim3(1), dim3(64), 0, s, ctr);
    if (mesh->nt > 0) {
        hipLaunchKernelGGL(k_depth_tri, dim3((unsigned)ceil_div(mesh->nt, kBlock)), dim3(kBlock), 0, s, M, mesh->pos,
                           mesh->tri, mesh->nv, mesh->nt, dw, dh, reinterpret_cast<unsigned *>(depth), queue, ctr);
        hipLaunchKernelGGL(k_depth_big, dim3(kBigGrid), dim3(kBlock), 0, s, M, mesh->pos, mesh->tri, mesh->nv, dw, dh,
                           reinterpret_cast<unsigned *>(depth), queue, ctr);
    }
    return launch_status();
}

// Scratch of the allocation-free depth render: the counters and the queue
// of a mesh of up to UVL_DEPTH_NOALLOC_MAX_TRIS triangles, one static array
// per device (held from module load to process end).  Host code never
// passes the array's name to a kernel: its device address on each device
// comes from hipGetSymbolAddress.
constexpr size_t kDepthScratchBytes = 256 + (size_t)UVL_DEPTH_NOALLOC_MAX_TRIS * sizeof(unsigned);
__device__ __align__(256) unsigned char depth_scratch[kDepthScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[64];

// Device address of depth_scratch on the current device (looked up once
// per device, with that device current).
int32_t depth_scratch_ptr(void *&out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return UVL_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(depth_scratch)) != hipSuccess || !p) return UVL_E_DEVICE;
        g_scratch_ptr[dev] = p;
    }
    out = g_scratch_ptr[dev];
    return UVL_OK;
}

}  // namespace
}  // namespace uvl

extern "C" int32_t uvl_render_depth(const uvl_mesh *mesh, const float view_proj[16], float *depth, int32_t dw,
                                    int32_t dh, void *ws, size_t ws_bytes, void *stream) {
    if (int32_t st = depth_args_ok(mesh, view_proj, depth, dw, dh)) return st;
    if (!ws) return UVL_E_INVAL;
    if (ws_bytes < uvl_depth_workspace_bytes(mesh->nt)) return UVL_E_NOMEM;
    if (int32_t s = device_ok()) return s;
    return launch_depth(mesh, view_proj, depth, dw, dh, ws, as_stream(stream));
}

extern "C" int32_t uvl_render_depth_noalloc(const uvl_mesh *mesh, const float view_proj[16], float *depth,
                                            int32_t dw, int32_t dh, void *stream) {
    if (int32_t st = depth_args_ok(mesh, view_proj, depth, dw, dh)) return st;
    if (mesh->nt > UVL_DEPTH_NOALLOC_MAX_TRIS) return UVL_E_NOMEM;
    if (int32_t s = device_ok()) return s;
    void *ws = nullptr;
    if (int32_t st = depth_scratch_ptr(ws)) return st;
    return launch_depth(mesh, view_proj, depth, dw, dh, ws, as_stream(stream));
}
