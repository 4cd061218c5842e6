// The screen-space depth texture for libuvl on gfx950 (§4.3.1: scene depth
// from the current viewpoint, for the depth test of the editing tools),
// rasterised with the fixed-point rule of raster_rule.h on screen positions.
//
// Launch structure:
//   1. one thread per triangle: set-up, and for bounding boxes of at most
//      kSmallCells cells the whole raster, with an atomicMin per covered cell
//      on the fp32 bits of the (non-negative) depth, order-independent;
//      larger triangles go to a queue in the workspace;
//   2. a fixed grid of workgroups drains the queue, one triangle per
//      workgroup, its 256 threads striding over the bounding box.
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
