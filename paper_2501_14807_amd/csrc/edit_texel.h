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
    float x0, y0, y1, sdx, sdy, xmax, x1, pad;   // xmax = max(x0, x1)
};

// Tile-culling data of a lasso, fp64 (filled on the host): four linear
// functions L(p) = a . p + b, one per side of the polygon's screen rectangle
// R = [max(-1, xlo), min(1, xhi)] x [max(-1, ylo), min(1, yhi)] widened by
// 2e-3, each negative exactly where a point in front of the camera projects
// beyond that side (e.g. clip_x - r clip_w for the left side); the clip w row;
// and |M| of the x, y and w rows for the conditioning check.
struct LassoCull {
    double plane[4][4];
    double wrow[4];
    double ax[4], ay[4], az[4], aw[4];
    // x-range of the edges that can straddle a point of slab s:
    // [slab_x0[s], slab_x1[s]] (min / max over the edges of slab_edges[s];
    // empty slab: x0 = +inf, x1 = -inf)
    float slab_x0[kSlabs], slab_x1[kSlabs];
    // per edge: dx/dy of its stored direction (0 for horizontal edges), and
    // the largest |x| of a vertex, for the rectangle classification
    double slope[kMaxPoly];
    float xabs;
};

struct LassoParams {
    float M[16];
    float bias;
    int32_t dw, dh, n;
    float ylo, yhi, xhi;        // polygon bounds: min y, max y, max x
    float xlo;                  // polygon min x
    float ylo_m, yhi_m, xhi_m;  // the same widened by 1e-4 (1 + |v|), for the pre-test, and clamped
                                // to the frustum [-1, 1] widened by 1e-4
    float xlo_m;                // xlo widened by 1e-4 (1 + |xlo|) + 1e-5 (2 + max |vertex x|), clamped alike
    float inv_h;                // slabs per unit of y
    uint64_t slab_edges[kSlabs];
    LassoEdge edge[kMaxPoly];
    LassoCull cull;
};

// The projective part of the test (§4.3.1: points projecting outside the
// unit cube are discarded): clip coordinates c = M [x y z 1]^T, and true if
// the texel is in front of the camera with its NDC x, y in the frustum and in
// the polygon's bounding range.  The NDC z / depth part follows in
// lasso_depth_index, so that it is evaluated only for texels inside the
// polygon.
// PT is LassoParams, possibly qualified with the constant address space so
// that a parameter block in global memory is read with scalar loads.
// mc[k] is M[4k + 3], the constant term of row k, passed apart so that a
// caller can hold it in a vector register (see lasso_quad_index).
template <class PT>
__device__ __forceinline__ bool lasso_front(const PT &P, const float mc[4], float x, float y, float z, float &xn,
                                            float &yn, float &cz, float &cw) {
    float c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        c[k] = __builtin_fmaf(P.M[4 * k + 2], z, __builtin_fmaf(P.M[4 * k + 1], y, __builtin_fmaf(P.M[4 * k + 0], x, mc[k])));
    cz = c[2];
    cw = c[3];
    if (!(c[3] > 0.0f)) return false;
    if (c[3] >= 1e-30f) {
        // Pre-test without a division: for w > 0, x / w >= a iff x >= a w.
        // The rounded product a w is within 6e-8 relative of the exact one
        // (or 1.2e-38 absolute if it underflows, 1.2e-8 of x / w at most for
        // w >= 1e-30), far inside the 1e-4 margins, so a texel rejected here
        // fails the exact tests below as well -- or, left of xlo_m, lies left
        // of every vertex by more than 1e-5 (2 + max |x|), where the fp32
        // crossing test is exact (see lasso_rect_class): it counts every edge
        // straddling y, an even number for a closed polygon, so the texel is
        // outside.  Each bound is the larger (smaller) of two such margins,
        // and rounding is monotone, so the joined test rejects a texel only
        // where one of the two would.
        if (!(c[0] >= P.xlo_m * c[3] && c[0] <= P.xhi_m * c[3] && c[1] >= P.ylo_m * c[3] &&
              c[1] <= P.yhi_m * c[3]))
            return false;
    }
    xn = c[0] / c[3];
    yn = c[1] / c[3];
    if (!(xn >= -1.0f && xn <= 1.0f && yn >= -1.0f && yn <= 1.0f)) return false;
    // Outside [ylo, yhi) no edge straddles yn; right of xhi every straddling
    // edge fails the crossing test even after rounding (monotone rounding of
    // the differences and products): both give "outside" exactly.
    return yn >= P.ylo && yn < P.yhi && xn <= P.xhi;
}

// NDC z in [-1, 1] for a texel that passed lasso_front; then its depth-map
// index and window depth, the texel being selected iff
// d <= depth[pix] + bias (lasso_depth_pass).
template <class PT>
__device__ __forceinline__ bool lasso_depth_index(const PT &P, float xn, float yn, float cz, float cw, int &pix,
                                                  float &d) {
    const float zn = cz / cw;
    if (!(zn >= -1.0f && zn <= 1.0f)) return false;
    int ix = (int)floorf(__builtin_fmaf(xn, 0.5f, 0.5f) * (float)P.dw);
    int iy = (int)floorf(__builtin_fmaf(yn, 0.5f, 0.5f) * (float)P.dh);
    ix = ix > P.dw - 1 ? P.dw - 1 : ix;
    iy = iy > P.dh - 1 ? P.dh - 1 : iy;
    pix = iy * P.dw + ix;   // < 2^28 for depth maps up to 16384 x 16384
    d = __builtin_fmaf(zn, 0.5f, 0.5f);
    return true;
}

template <class PT>
__device__ __forceinline__ bool lasso_depth_pass(const PT &P, float d, float stored) {
    return d <= stored + P.bias;
}

template <class PT>
__device__ __forceinline__ int lasso_slab(const PT &P, float yn) {
    int s = (int)((yn - P.ylo) * P.inv_h);
    s = s < 0 ? 0 : s;
    return s > kSlabs - 1 ? kSlabs - 1 : s;
}

// Crossing test of edge e (from vertex k to k+1, stored as above) for a
// wave: the mask of lanes whose point (xn, yn) has the edge counting -- one
// end above yn and the other not, and the crossing right of xn.  Each
// comparison's lane mask is taken directly.
__device__ __forceinline__ uint64_t lasso_crosses_mask(float ex0, float ey0, float ey1, float esdx, float esdy,
                                                       float xn, float yn) {
    const uint64_t a = __builtin_amdgcn_ballot_w64(ey0 > yn), b = __builtin_amdgcn_ballot_w64(ey1 > yn);
    const float lhs = (xn - ex0) * esdy;
    const float rhs = esdx * (yn - ey0);
    return (a ^ b) & __builtin_amdgcn_ballot_w64(lhs < rhs);
}

// The whole lasso predicate for one texel (a lane on its own, no wave-wide
// step): the edges of its own slab, then the depth test.  Gives the same
// result as lasso_quad for that texel.
template <class PT>
__device__ __forceinline__ bool lasso_texel(const PT &P, const float *__restrict__ depth, float x, float y,
                                            float z) {
    float xn, yn, cz, cw;
    const float mc[4] = {P.M[3], P.M[7], P.M[11], P.M[15]};
    if (!lasso_front(P, mc, x, y, z, xn, yn, cz, cw)) return false;
    uint64_t m = P.slab_edges[lasso_slab(P, yn)];
    bool inside = false;
    while (m) {
        const int e = __builtin_ctzll(m);
        m &= m - 1;
        const float ex0 = P.edge[e].x0, ey0 = P.edge[e].y0, ey1 = P.edge[e].y1;
        const float esdx = P.edge[e].sdx, esdy = P.edge[e].sdy;
        const float lhs = (xn - ex0) * esdy;
        const float rhs = esdx * (yn - ey0);
        inside ^= ((ey0 > yn) != (ey1 > yn)) && (lhs < rhs);
    }
    if (!inside) return false;
    int pix;
    float d;
    if (!lasso_depth_index(P, xn, yn, cz, cw, pix, d)) return false;
    return lasso_depth_pass(P, d, depth[pix]);
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
// after rounding (the same monotonicity argument as the xhi bound).  Texels
// inside the polygon then get their NDC z test; pix[k] is the depth-map
// index still to be tested (d[k] <= depth[pix[k]] + bias), or -1 if the
// texel is already rejected.  The depth reads are left to the caller, so
// that it can issue many of them before waiting.  all_inside: the caller
// has shown (lasso_rect_class) that every texel here lies inside the polygon
// by the fp32 test, which is then skipped.
// Must be called by all 64 lanes.
template <class PT>
__device__ __forceinline__ void lasso_quad_index(const PT &P, const float4 &X, const float4 &Y, const float4 &Z,
                                                 int pix[4], float d[4], bool all_inside = false) {
    const float xs[4] = {X.x, X.y, X.z, X.w}, ys[4] = {Y.x, Y.y, Y.z, Y.w}, zs[4] = {Z.x, Z.y, Z.z, Z.w};
    float xn[4], yn[4], cz[4], cw[4];
    bool cand[4], inside[4];
    unsigned smin = kSlabs, smax = 0;
    float xmin = INFINITY;
    // The constant terms of M in vector registers, once per call: a VALU
    // instruction reads at most one scalar register on this target, so
    // fma(M0, x, M3) with both in scalar registers costs a move per texel.
    float mc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) asm("v_mov_b32 %0, %1" : "=v"(mc[k]) : "s"(P.M[4 * k + 3]));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        xn[k] = 0.0f;
        yn[k] = 0.0f;
        cand[k] = lasso_front(P, mc, xs[k], ys[k], zs[k], xn[k], yn[k], cz[k], cw[k]);
        inside[k] = false;
        if (cand[k]) {
            const unsigned s = (unsigned)lasso_slab(P, yn[k]);
            smin = min(smin, s);
            smax = max(smax, s);
            xmin = fminf(xmin, xn[k]);
        }
    }
    const unsigned wmin = all_inside ? 1u : wave_min_u32(smin), wmax = all_inside ? 0u : wave_max_u32(smax);
    if (all_inside) {
#pragma unroll
        for (int k = 0; k < 4; ++k) inside[k] = true;
    } else if (wmin <= wmax) {
        const float wxmin = wave_min_f32(xmin);
        uint64_t m = 0;
        for (unsigned s = wmin; s <= wmax; ++s) m |= P.slab_edges[s];
        // crossing parities as wave-wide lane masks (one bit per lane per
        // texel slot), toggled with scalar XORs of the per-edge ballots
        uint64_t par[4] = {0, 0, 0, 0};
        while (m) {
            const int e = __builtin_ctzll(m);
            m &= m - 1;
            const float ex0 = P.edge[e].x0, ey0 = P.edge[e].y0, ey1 = P.edge[e].y1;
            const float esdx = P.edge[e].sdx, esdy = P.edge[e].sdy, exmax = P.edge[e].xmax;
            if (exmax < wxmin) continue;
#pragma unroll
            for (int k = 0; k < 4; ++k) par[k] ^= lasso_crosses_mask(ex0, ey0, ey1, esdx, esdy, xn[k], yn[k]);
        }
        const int lane = __lane_id();
#pragma unroll
        for (int k = 0; k < 4; ++k) inside[k] = (par[k] >> lane) & 1;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        pix[k] = -1;
        d[k] = 0.0f;
        if (cand[k] && inside[k] && !lasso_depth_index(P, xn[k], yn[k], cz[k], cw[k], pix[k], d[k])) pix[k] = -1;
    }
}

// The whole lasso predicate for 4 texels per lane (all 64 lanes).
template <class PT>
__device__ __forceinline__ void lasso_quad(const PT &P, const float *__restrict__ depth, const float4 &X,
                                           const float4 &Y, const float4 &Z, bool sel[4], bool all_inside = false) {
    int pix[4];
    float d[4];
    lasso_quad_index(P, X, Y, Z, pix, d, all_inside);
#pragma unroll
    for (int k = 0; k < 4; ++k) sel[k] = pix[k] >= 0 && lasso_depth_pass(P, d[k], depth[pix[k]]);
}

// ---------------------------------------------------------------------------
// Conservative tile tests.  box = {min x, min y, min z, max x, max y, max z}
// of the covered positions of a tile (min > max: no covered texel).  A tile
// is reported culled only if no texel of it can be selected by the fp32
// predicate above, so skipping culled tiles leaves every result unchanged.

// Brush: the fp32 squared distance of the box to the centre, D2, is within
// 6 ulps of the exact one, and a texel's fp32 d2 within 6 ulps of its exact
// squared distance, which is >= the box's; D2 > r2 (1 + 1e-5) + 1e-30 then
// forces d2 > r2 (the 1e-30 covers underflow).
__device__ __forceinline__ bool brush_culls(const BrushParams &B, const float box[6]) {
    if (!(box[0] <= box[3])) return true;
    const float dx = fmaxf(fmaxf(box[0] - B.cx, B.cx - box[3]), 0.0f);
    const float dy = fmaxf(fmaxf(box[1] - B.cy, B.cy - box[4]), 0.0f);
    const float dz = fmaxf(fmaxf(box[2] - B.cz, B.cz - box[5]), 0.0f);
    const float d2 = dx * dx + dy * dy + dz * dz;
    return d2 > B.r2 * 1.00001f + 1e-30f;
}

// Lasso: a texel can only be selected if its fp32 NDC position lies in R
// (outside R it fails the frustum test, the exact y / right-side rejections,
// or -- left of every vertex by more than 1e-3 -- the crossing test counts
// every straddling edge and leaves it outside).  The exact NDC position of a
// point in front of the camera is beyond the widened side k iff L_k(p) < 0,
// and L_k is linear, so max over the box of L_k < 0 (in fp64) puts every
// texel of the tile beyond that side; its fp32 NDC position is within 4e-4 of
// the exact one while clip w >= 1e-3 of the rows' |M| sums over the box
// (checked first; otherwise nothing is culled), inside the 2e-3 widening.
__device__ __forceinline__ double box_max(const double a[4], const float box[6]) {
    double v = a[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) v += a[j] >= 0.0 ? a[j] * (double)box[3 + j] : a[j] * (double)box[j];
    return v;
}

__device__ __forceinline__ double box_abs_max(const double a[4], const float box[6]) {
    double v = a[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) v += a[j] * fmax(fabs((double)box[j]), fabs((double)box[3 + j]));
    return v;
}

template <class PT>
__device__ __forceinline__ double row_abs_max(const PT &row, const float box[6]) {
    double a[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = row[j];
    return box_abs_max(a, box);
}

// Further lasso tests, reached with the conditioning satisfied and every
// corner in front of the camera (wmin > 0).  The box then projects into the
// bounding box of its corners' NDC images (fp64 here, so within 1e-12), and
// every texel's fp32 NDC position lies within eps = 5e-4 of that box.
//
// Slabs: a texel whose fp32 y falls in slab s and whose fp32 x exceeds
// slab_x1[s] is right of every edge that can straddle it (outside exactly),
// and one with x below slab_x0[s] - 1e-3 is left of all of them by the margin
// (outside).  The texel slab index is floor((y - ylo) inv_h) of an fp32 y;
// the slab range of the tile's y-range is taken one slab wider on each side.
// If every slab in that range misses the tile's x-range, the tile is culled.
//
// Depth (when a depth map is given): z/w over the box is a linear-fractional
// function with a positive denominator, so its minimum is the corners'
// minimum zmin.  A texel's fp32 NDC z differs from its exact z/w by at most
// (|dc_z| + 2 |dc_w|) / w_hat + u (its fp32 z being in [-1, 1] when it gets
// that far, so its exact z/w is within 2), where |dc| <= 3.01 u (row |M|
// sum over the box) bounds the fma chains and u = 2^-24; its window depth
// adds u.  Its depth-map pixel lies in the rectangle of the NDC box widened
// by eps, one pixel more on each side.  If the smallest window depth a texel
// can have exceeds the largest fl(D + bias) over that rectangle, every texel
// fails the depth test.  The rectangle is read directly when it has at most
// kDepthCullPixels pixels.
constexpr int kDepthCullPixels = 1024;

// Results of the lasso tile tests.
enum LassoTile { kTileCulled = 0, kTileLive = 1, kTileInside = 2 };

// Rectangle R = [rx0, rx1] x [ry0, ry1] that holds the fp32 NDC position of
// every texel of a tile, against the polygon.  The fp32 crossing test of
// edge e at a point q uses the line through (x0, y0) with the stored
// direction (sdx, sdy), over the half-open y-range of the edge; its side test
// is exact when q is at horizontal distance >= m from that line, m > 4.02 u
// (1 + X) with X the largest |x| of a vertex (the two rounded products
// differ from the exact ones by 2.01 u of their sizes, and |xn| <= 1).  If
// no edge's piece over R's y-range comes within m of R (fp64 here, error
// far below m), no edge crosses R and the vertices lie outside it, so the
// even-odd parity is the same at every point of R, and every texel's fp32
// test gives that parity: the parity of R's centre (fp64).  Horizontal
// edges never count, but the parity changes across them (the straddle
// ranges of their neighbours end there), so they take part in the "near R"
// test as the segment between their vertices.  Returns kTileCulled (all
// outside), kTileInside (all inside) or kTileLive.
template <class PT>
__device__ __forceinline__ int lasso_rect_class(const PT &P, double rx0, double rx1, double ry0, double ry1) {
    const double m = 1e-5 * (2.0 + (double)P.cull.xabs);
    const double a0 = rx0 - m, a1 = rx1 + m, b0 = ry0 - m, b1 = ry1 + m;
    const double cx = 0.5 * (rx0 + rx1), cy = 0.5 * (ry0 + ry1);
    bool odd = false;
    for (int k = 0; k < P.n; ++k) {
        const double ex0 = P.edge[k].x0, ey0 = P.edge[k].y0, ey1 = P.edge[k].y1;
        if (ey0 == ey1) {
            // horizontal: never straddles, but bounds the inside
            const double ex1 = P.edge[k].x1;
            if (ey0 >= b0 && ey0 <= b1 && fmin(ex0, ex1) <= a1 && fmax(ex0, ex1) >= a0) return kTileLive;
            continue;
        }
        const double slope = P.cull.slope[k];
        const double ya = fmax(fmin(ey0, ey1), b0), yb = fmin(fmax(ey0, ey1), b1);
        if (ya <= yb) {
            const double xa = ex0 + slope * (ya - ey0), xb = ex0 + slope * (yb - ey0);
            if (fmin(xa, xb) <= a1 && fmax(xa, xb) >= a0) return kTileLive;   // the edge comes near R
        }
        const double sdx = P.edge[k].sdx, sdy = P.edge[k].sdy;
        if (((ey0 > cy) != (ey1 > cy)) && ((cx - ex0) * sdy < sdx * (cy - ey0))) odd = !odd;
    }
    return odd ? kTileInside : kTileCulled;
}

template <class PT>
__device__ __forceinline__ int lasso_culls_more(const PT &P, const float box[6], const float *depth, double wmin) {
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY, zmin = INFINITY;
#pragma unroll 1
    for (int k = 0; k < 8; ++k) {
        const double x = (k & 1) ? box[3] : box[0];
        const double y = (k & 2) ? box[4] : box[1];
        const double z = (k & 4) ? box[5] : box[2];
        double c[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            c[r] = (double)P.M[4 * r] * x + (double)P.M[4 * r + 1] * y + (double)P.M[4 * r + 2] * z + (double)P.M[4 * r + 3];
        if (!(c[3] > 0.0)) return kTileLive;
        const double xn = c[0] / c[3], yn = c[1] / c[3], zn = c[2] / c[3];
        x0 = fmin(x0, xn);
        x1 = fmax(x1, xn);
        y0 = fmin(y0, yn);
        y1 = fmax(y1, yn);
        zmin = fmin(zmin, zn);
    }
    const double eps = 5e-4;
    if (P.inv_h > 0.0f) {
        const double h = 1.0 / (double)P.inv_h;
        int s0 = (int)floor((y0 - eps - (double)P.ylo) / h) - 1;
        int s1 = (int)floor((y1 + eps - (double)P.ylo) / h) + 1;
        s0 = s0 < 0 ? 0 : s0;
        s1 = s1 > kSlabs - 1 ? kSlabs - 1 : s1;
        bool hit = false;
        for (int s = s0; s <= s1 && !hit; ++s) {
            const double a = (double)P.cull.slab_x0[s] - 1e-3, b = (double)P.cull.slab_x1[s];
            hit = a <= x1 + eps && b >= x0 - eps;
        }
        if (!hit) return kTileCulled;
    }
    const int cls = lasso_rect_class(P, x0 - eps, x1 + eps, y0 - eps, y1 + eps);
    if (cls == kTileCulled) return kTileCulled;
    if (!depth) return cls;
    const double u = 0x1p-24;
    const double az = row_abs_max(P.cull.az, box), aw = row_abs_max(P.cull.aw, box);
    const double dcz = 3.01 * u * az, dcw = 3.01 * u * aw;
    if (!(dcw < 0.5 * wmin)) return cls;
    const double err_z = (dcz + 2.0 * dcw) / (wmin - dcw) + 2.0 * u + 1e-12;
    const double dlo = 0.5 * (zmin - err_z) + 0.5 - 2.0 * u;   // smallest fp32 window depth of a texel
    const int dw = P.dw, dh = P.dh;
    int ix0 = (int)floor(((x0 - eps) * 0.5 + 0.5) * dw) - 1, ix1 = (int)floor(((x1 + eps) * 0.5 + 0.5) * dw) + 1;
    int iy0 = (int)floor(((y0 - eps) * 0.5 + 0.5) * dh) - 1, iy1 = (int)floor(((y1 + eps) * 0.5 + 0.5) * dh) + 1;
    ix0 = ix0 < 0 ? 0 : ix0;
    iy0 = iy0 < 0 ? 0 : iy0;
    ix1 = ix1 > dw - 1 ? dw - 1 : ix1;
    iy1 = iy1 > dh - 1 ? dh - 1 : iy1;
    if (ix0 > ix1 || iy0 > iy1) return cls;
    if ((int64_t)(ix1 - ix0 + 1) * (iy1 - iy0 + 1) > kDepthCullPixels) return cls;
    // fl(D + bias) <= (D + bias) + u |D + bias|; culled iff dlo exceeds that
    // for every pixel of the rectangle.  The pixels are read 16 at a time
    // (independent loads in flight together), each batch tested on its max.
    const double bias = P.bias;
    const int rw = ix1 - ix0 + 1, npix = rw * (iy1 - iy0 + 1);
    const float inv_rw = 1.0f / (float)rw;   // (p + 0.5) / rw is >= 0.5 / rw from an integer: exact floor
    for (int p0 = 0; p0 < npix; p0 += 16) {
        float dmax = -INFINITY;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int p = p0 + i < npix ? p0 + i : npix - 1;
            const int r = (int)(((float)p + 0.5f) * inv_rw);
            const float v = depth[(int64_t)(iy0 + r) * dw + ix0 + (p - r * rw)];
            dmax = fmaxf(dmax, v);
        }
        const double v = (double)dmax + bias;
        if (!(dlo > v + u * fabs(v) + 1e-12)) return cls;
    }
    return kTileCulled;
}

// Lasso tile test: kTileCulled if no texel of the box can be selected,
// kTileInside if every texel that passes the projective tests is inside the
// polygon, kTileLive otherwise.
template <class PT>
__device__ __forceinline__ int lasso_tile(const PT &P, const float box[6], const float *depth = nullptr) {
    const auto &C = P.cull;
    if (!(box[0] <= box[3] && box[1] <= box[4] && box[2] <= box[5])) return kTileCulled;
    double wneg[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) wneg[j] = -C.wrow[j];
    const double wmin = -box_max(wneg, box);
    const double smax = fmax(row_abs_max(C.ax, box), row_abs_max(C.ay, box)) + row_abs_max(C.aw, box);
    if (!(wmin >= 1e-3 * smax) || !(wmin > 0.0)) return kTileLive;
#pragma unroll 1
    for (int k = 0; k < 4; ++k) {
        double a[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) a[j] = C.plane[k][j];
        if (box_max(a, box) < 0.0) return kTileCulled;
    }
    return lasso_culls_more(P, box, depth, wmin);
}

}  // namespace uvl
