// The paper's screen-space editing tool (§4.3.1) for libuvl: its per-texel
// predicate and parameters, shared by the single-edit kernels (tool.hip)
// and the batched waves (wave.hip).
#pragma once

#include <math.h>

#include "uvl_internal.h"

namespace uvl {

constexpr int kMaxShape = 4096;

struct ToolParams {
    float M[16];
    float ax, bx, ay, by;                  // s = fmaf(xn, ax, bx), t = fmaf(yn, ay, by)
    float xlo_m, xhi_m, ylo_m, yhi_m;      // NDC range with s, t in [0, 1] and in the frustum, widened
    int32_t sw, sh, dw, dh;
    float bias;
};

template <class PT>
__device__ __forceinline__ bool tool_texel(const PT &P, const uint8_t *__restrict__ shape,
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

// Host: the parameters of a tool (tool = {Ww, Wh, Tpx, Tpy, Tw, Th}, shape
// sw x sh, depth map dw x dh, bias); false for invalid values.
bool make_tool_params(const float view_proj[16], const double tool[6], int32_t sw, int32_t sh, int32_t dw,
                      int32_t dh, float bias, ToolParams &p);

}  // namespace uvl
