// The screen-space depth texture for libuvl on gfx950 (§4.3.1: scene depth
// from the current viewpoint, for the depth test of the editing tools),
// rasterised with the fixed-point rule of raster_rule.h on screen positions.
//
// A triangle reaching beyond the near plane (z_clip + w_clip >= 0) or the
// guard band (|x_clip|, |y_clip| <= 16 w_clip) is clipped against those
// planes, as the fixed-function pipeline clips primitives, and its polygon
// drawn as a fan; one inside them is drawn as it is.
//
// Launch structure:
//   1. one thread per triangle: set-up, and for bounding boxes of at most
//      kSmallCells cells the whole raster, with an atomicMin per covered cell
//      on the fp32 bits of the (non-negative) depth, order-independent;
//      larger triangles and those to be clipped go to a queue in the
//      workspace;
//   2. a fixed grid of workgroups drains the queue, one triangle per
//      workgroup, its 256 threads striding over the bounding box (of each
//      fan triangle, for a clipped one).
#include <math.h>

#include <mutex>

#include "raster_rule.h"
#include "uvl_internal.h"

namespace uvl {
namespace {

constexpr int kSmallCells = 64;
constexpr int kBigGrid = 2048;

// Workspace counters (first 256 bytes of the workspace).
struct Counters {
    unsigned int queue_len;
    unsigned int pad[3];
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// depth texture

struct Mat4 { float m[16]; };

// A triangle's class for the depth raster: kDrop (a vertex index out of
// range or a non-finite clip coordinate), kDirect (every vertex with w > 0,
// in front of the near plane z + w >= 0 and inside the guard band
// |x|, |y| <= 16 w: drawn as it is), kClip (the rest: clipped against those
// five planes by k_depth_big, the remaining polygon drawn as a fan).
enum { kDrop = 0, kDirect = 1, kClip = 2 };
constexpr int kMaxPoly = 9;             // 3 vertices + one per clipping plane, + 1 spare

// Signed distance to clipping plane p (>= 0 inside): the near plane, then
// the guard band's right, left, top and bottom sides.
__device__ __forceinline__ double clip_dist(int p, const double c[4]) {
    switch (p) {
    case 0: return c[2] + c[3];
    case 1: return 16.0 * c[3] - c[0];
    case 2: return 16.0 * c[3] + c[0];
    case 3: return 16.0 * c[3] - c[1];
    default: return 16.0 * c[3] + c[1];
    }
}

// Clip coordinates of triangle t's vertices (fp32 fma chains, as the
// edit predicates project) and its class.
__device__ __forceinline__ int depth_vertices(const Mat4 &M, const float *__restrict__ pos,
                                              const int32_t *__restrict__ tri, int64_t nv, int64_t t,
                                              float cf[3][4]) {
    bool inside = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int32_t v = tri[3 * t + k];
        if (v < 0 || v >= nv) return kDrop;
        const float x = pos[3 * (int64_t)v], y = pos[3 * (int64_t)v + 1], z = pos[3 * (int64_t)v + 2];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            cf[k][q] = __builtin_fmaf(M.m[4 * q + 2], z,
                                      __builtin_fmaf(M.m[4 * q + 1], y, __builtin_fmaf(M.m[4 * q + 0], x, M.m[4 * q + 3])));
            if (!isfinite(cf[k][q])) return kDrop;
        }
        // the five plane tests of clip_dist, exact: 16 w is exact in fp32
        // (or +inf where the fp64 value exceeds every float, which compares
        // the same), so |x| <= 16 w needs no rounding; z + w takes fp64,
        // where the sum of two floats keeps its sign
        const float g = 16.0f * cf[k][3];
        if (!(cf[k][3] > 0.0f) || !(cf[k][0] <= g) || !(-cf[k][0] <= g) || !(cf[k][1] <= g) ||
            !(-cf[k][1] <= g) || !((double)cf[k][2] + (double)cf[k][3] >= 0.0))
            inside = false;
    }
    return inside ? kDirect : kClip;
}

// Screen set-up of a triangle from its vertices' NDC: window position
// fmaf(ndc, .5, .5) * size in fp32, snapped; window depth fmaf(z, .5, .5).
__device__ __forceinline__ bool depth_setup(const float xn[3], const float yn[3], const float zn[3], int Wd, int Hd,
                                            Tri2 &T, double d[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float sx = __builtin_fmaf(xn[k], 0.5f, 0.5f) * (float)Wd;
        const float sy = __builtin_fmaf(yn[k], 0.5f, 0.5f) * (float)Hd;
        T.X[k] = snap256((double)sx);
        T.Y[k] = snap256((double)sy);
        d[k] = (double)__builtin_fmaf(zn[k], 0.5f, 0.5f);
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

// One triangle's raster by the whole workgroup, striding over its box.
__device__ __forceinline__ void depth_block(const Tri2 &T, const double d[3], int Wd, int Hd,
                                            unsigned *__restrict__ depth) {
    int i0, i1, j0, j1;
    bbox(T, Wd, Hd, i0, i1, j0, j1);
    if (i1 < i0 || j1 < j0) return;
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

// The clipped polygon of a kClip triangle as NDC vertices x, y, z (by one
// thread, in LDS): fp64 Sutherland-Hodgman against the five planes in
// order, each cut edge split at s + t (o - s), t = f(s) / (f(s) - f(o)),
// from its inside end s to its outside end o, so that two triangles sharing
// an edge cut it at the same point; a vertex of the triangle keeps its fp32
// quotient, a cut point takes its fp64 quotient rounded to fp32, x and y
// clamped to [-16, 16].  Returns the vertex count (0: nothing left).
struct ClipPoly {
    double c[2][kMaxPoly][4];
    int orig[2][kMaxPoly];
    float x[kMaxPoly], y[kMaxPoly], z[kMaxPoly];
};

__device__ __forceinline__ float clamp16(float v) { return v < -16.0f ? -16.0f : (v > 16.0f ? 16.0f : v); }

__device__ int clip_polygon(const float cf[3][4], ClipPoly &P) {
    int n = 3, cur = 0;
    for (int k = 0; k < 3; ++k) {
        for (int q = 0; q < 4; ++q) P.c[0][k][q] = (double)cf[k][q];
        P.orig[0][k] = k;
    }
    for (int p = 0; p < 5 && n >= 3; ++p) {
        const int nxt = 1 - cur;
        int m = 0;
        for (int i = 0; i < n; ++i) {
            const int b = i + 1 < n ? i + 1 : 0;
            const double fa = clip_dist(p, P.c[cur][i]), fb = clip_dist(p, P.c[cur][b]);
            const bool ina = fa >= 0.0, inb = fb >= 0.0;
            if (ina) {
                for (int q = 0; q < 4; ++q) P.c[nxt][m][q] = P.c[cur][i][q];
                P.orig[nxt][m] = P.orig[cur][i];
                ++m;
            }
            if (ina != inb) {
                const int sv = ina ? i : b, ov = ina ? b : i;
                const double fs = ina ? fa : fb, fo = ina ? fb : fa;
                const double t = fs / (fs - fo);
                for (int q = 0; q < 4; ++q) P.c[nxt][m][q] = P.c[cur][sv][q] + t * (P.c[cur][ov][q] - P.c[cur][sv][q]);
                P.orig[nxt][m] = -1;
                ++m;
            }
        }
        n = m;
        cur = nxt;
    }
    if (n < 3) return 0;
    for (int k = 0; k < n; ++k) {
        const double *c = P.c[cur][k];
        if (!(c[3] > 0.0)) return 0;
        const int o = P.orig[cur][k];
        if (o >= 0) {
            P.x[k] = cf[o][0] / cf[o][3];
            P.y[k] = cf[o][1] / cf[o][3];
            P.z[k] = cf[o][2] / cf[o][3];
        } else {
            P.x[k] = clamp16((float)(c[0] / c[3]));
            P.y[k] = clamp16((float)(c[1] / c[3]));
            P.z[k] = (float)(c[2] / c[3]);
        }
    }
    return n;
}

__global__ __launch_bounds__(kBlock) void k_depth_tri(Mat4 M, const float *__restrict__ pos,
                                                      const int32_t *__restrict__ tri, int64_t nv, int64_t nt,
                                                      int Wd, int Hd, unsigned *__restrict__ depth,
                                                      unsigned *__restrict__ queue, Counters *__restrict__ ctr) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nt) return;
    float cf[3][4];
    const int cls = depth_vertices(M, pos, tri, nv, t, cf);
    if (cls == kDrop) return;
    if (cls == kClip) {
        queue[atomicAdd(&ctr->queue_len, 1u)] = (unsigned)t;
        return;
    }
    float xn[3], yn[3], zn[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        xn[k] = cf[k][0] / cf[k][3];
        yn[k] = cf[k][1] / cf[k][3];
        zn[k] = cf[k][2] / cf[k][3];
    }
    Tri2 T;
    double d[3];
    if (!depth_setup(xn, yn, zn, Wd, Hd, T, d)) return;
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

// Queued triangles, one per workgroup: large ones drawn directly, clipped
// ones as the fan of their polygon (the polygon built by thread 0 in LDS).
__global__ __launch_bounds__(kBlock) void k_depth_big(Mat4 M, const float *__restrict__ pos,
                                                      const int32_t *__restrict__ tri, int64_t nv, int Wd, int Hd,
                                                      unsigned *__restrict__ depth,
                                                      const unsigned *__restrict__ queue,
                                                      const Counters *__restrict__ ctr) {
    __shared__ ClipPoly s_poly;
    __shared__ int s_n;
    const unsigned n = ctr->queue_len;
    for (unsigned q = blockIdx.x; q < n; q += gridDim.x) {
        const unsigned t = queue[q];
        float cf[3][4];
        const int cls = depth_vertices(M, pos, tri, nv, t, cf);
        if (cls == kDirect) {
            float xn[3], yn[3], zn[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                xn[k] = cf[k][0] / cf[k][3];
                yn[k] = cf[k][1] / cf[k][3];
                zn[k] = cf[k][2] / cf[k][3];
            }
            Tri2 T;
            double d[3];
            if (depth_setup(xn, yn, zn, Wd, Hd, T, d)) depth_block(T, d, Wd, Hd, depth);
        } else if (cls == kClip) {
            // uniform over the workgroup (one triangle), so the barriers are too
            if (threadIdx.x == 0) s_n = clip_polygon(cf, s_poly);
            __syncthreads();
            const int m = s_n;
            for (int k = 1; k + 1 < m; ++k) {
                const float xn[3] = {s_poly.x[0], s_poly.x[k], s_poly.x[k + 1]};
                const float yn[3] = {s_poly.y[0], s_poly.y[k], s_poly.y[k + 1]};
                const float zn[3] = {s_poly.z[0], s_poly.z[k], s_poly.z[k + 1]};
                Tri2 T;
                double d[3];
                if (depth_setup(xn, yn, zn, Wd, Hd, T, d)) depth_block(T, d, Wd, Hd, depth);
            }
            __syncthreads();   // before the next triangle's polygon overwrites this one
        }
    }
}

__global__ void k_counters_reset(Counters *ctr) {
    if (threadIdx.x == 0) {
        ctr->queue_len = 0;
        ctr->pad[0] = ctr->pad[1] = ctr->pad[2] = 0;
    }
}

}  // namespace
}  // namespace uvl

using namespace uvl;

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
