/*
 * uvl_oracle.c - plain, slow CPU oracle for the texture-layer method.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code with the GPU library.
 *
 * Paper: "An Efficient GPU Approach for Designing 3D Cultural Heritage
 * Information Systems" (arXiv 2501.14807).  Each function cites the passage
 * it follows.  Where the paper is silent, the reading used is the one written
 * next to the code; the same readings bind the GPU path.
 *
 * Numerics: geometry in fp64; selection predicates in fp32 with every
 * operation rounded once (build with -ffp-contract=off; fmaf() is the
 * correctly rounded C99 fused multiply-add; '/' is IEEE division).
 * Pinned by tests against closed forms, invariants and brute force; see the
 * header comment of each function for its pins.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_U8 1
#define ORC_U16 2
#define ORC_AND 0
#define ORC_OR 1
#define ORC_XOR 2
#define ORC_REMAP 3

/* ------------------------------------------------------------------------
 * Shared 2D raster rule (used by the texture-space raster of §4.3.1, where
 * the mesh is drawn with its texture coordinates in place of its positions,
 * and by the depth texture of the same section).  The paper relies on the GPU
 * rasteriser and states no sample or tie rule, so the reading is:
 *   - coordinates are snapped to fixed point with 8 fractional bits,
 *     X = round-half-even(x * 256) in fp64;
 *   - sample point of cell (i, j) is its centre (256 i + 128, 256 j + 128);
 *   - a sample is inside a triangle when, for the counter-clockwise order,
 *     every edge function is > 0, or == 0 on an edge that owns its boundary:
 *     edge s->t owns it iff (t.y - s.y) < 0, or == 0 and (t.x - s.x) > 0;
 *   - zero-area triangles cover nothing; clockwise ones are tested with two
 *     vertices swapped, barycentrics reported in the original order.
 * ------------------------------------------------------------------------ */

static int64_t snap256(double x) { return (int64_t)nearbyint(x * 256.0); }

static int edge_owns(int64_t sx, int64_t sy, int64_t tx, int64_t ty)
{
    int64_t dx = tx - sx, dy = ty - sy;
    return dy < 0 || (dy == 0 && dx > 0);
}

static int64_t edge_fn(int64_t sx, int64_t sy, int64_t tx, int64_t ty, int64_t px, int64_t py)
{
    return (tx - sx) * (py - sy) - (ty - sy) * (px - sx);
}

/* Inside test of sample (px,py) against triangle (X[k],Y[k]).  On success
 * e[k] holds the edge function opposite vertex k (original order) and *area2
 * the absolute doubled area, so that barycentric k = e[k] / *area2. */
static int tri_sample(const int64_t X[3], const int64_t Y[3], int64_t px, int64_t py,
                      int64_t e[3], int64_t *area2)
{
    int64_t E = edge_fn(X[0], Y[0], X[1], Y[1], X[2], Y[2]);
    if (E == 0) return 0;
    int a = 0, b = 1, c = 2;
    if (E < 0) { b = 2; c = 1; E = -E; }
    /* edges of the counter-clockwise order a->b->c->a; e_k is opposite k */
    int64_t ea = edge_fn(X[b], Y[b], X[c], Y[c], px, py);
    int64_t eb = edge_fn(X[c], Y[c], X[a], Y[a], px, py);
    int64_t ec = edge_fn(X[a], Y[a], X[b], Y[b], px, py);
    int in_a = ea > 0 || (ea == 0 && edge_owns(X[b], Y[b], X[c], Y[c]));
    int in_b = eb > 0 || (eb == 0 && edge_owns(X[c], Y[c], X[a], Y[a]));
    int in_c = ec > 0 || (ec == 0 && edge_owns(X[a], Y[a], X[b], Y[b]));
    if (!(in_a && in_b && in_c)) return 0;
    e[a] = ea; e[b] = eb; e[c] = ec;
    *area2 = E;
    return 1;
}

/* Range of cells [lo, hi] whose centre 256 k + 128 lies in [mn, mx]. */
static void cell_range(int64_t mn, int64_t mx, int n, int *lo, int *hi)
{
    /* smallest k with 256k+128 >= mn, largest with 256k+128 <= mx */
    int64_t a = mn - 128, b = mx - 128;
    int64_t klo = a >= 0 ? (a + 255) / 256 : -((-a) / 256);
    int64_t khi = b >= 0 ? b / 256 : -((-b + 255) / 256);
    if (klo < 0) klo = 0;
    if (khi > n - 1) khi = n - 1;
    *lo = (int)klo;
    *hi = (int)khi;
}

static void snap_uv(const float *uv, int64_t v, int W, int H, int64_t *X, int64_t *Y)
{
    *X = snap256((double)uv[2 * v] * (double)W);
    *Y = snap256((double)uv[2 * v + 1] * (double)H);
}

/* ------------------------------------------------------------------------
 * Geometry image (§4.3.1: the mesh is rendered into texture space with its
 * texture coordinates as positions; §4.1: texture coordinates index the data).
 *
 * For texel rows [j0, j1) of a W x H atlas: owner triangle (lowest index
 * among those whose raster covers the centre; -1 if none), barycentrics of
 * vertices 1 and 2, position and unit normal interpolated in fp64, and the
 * texel's surface-area weight w = 131072 * A3 / |E| (A3 the triangle's 3D
 * area, |E| its doubled fixed-point UV area: the surface area one texel of
 * UV area 1/(W H) maps to, since A_uv = |E| / (2 * 256^2 * W * H)).
 * pos = b0*P0 + b1*P1 + b2*P2 with b_k = e_k / |E|, summed left to right.
 * nrm = normalise(b0*N0 + b1*N1 + b2*N2), or the face normal if nrm == NULL.
 * Uncovered texels: tri -1, pos NaN, nrm 0, bary 0, w 0.
 * Outputs are planes of (j1-j0)*W values; any output pointer may be NULL.
 * cover_count (optional, int32) counts all covering triangles per texel.
 * ------------------------------------------------------------------------ */
int orc_geometry_image(const float *pos, const float *nrm, const float *uv, const int32_t *tri,
                       int64_t nv, int64_t nt, int W, int H, int j0, int j1,
                       int32_t *tri_id, double *bary, double *pos_out, double *nrm_out,
                       double *w_out, int32_t *cover_count)
{
    if (W <= 0 || H <= 0 || j0 < 0 || j1 > H || j0 > j1) return -1;
    const int64_t n = (int64_t)(j1 - j0) * W;
    int32_t *own = tri_id ? tri_id : (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int64_t k = 0; k < n; ++k) own[k] = -1;
    if (cover_count) memset(cover_count, 0, sizeof(int32_t) * (size_t)n);

    for (int64_t t = 0; t < nt; ++t) {
        int64_t X[3], Y[3];
        for (int k = 0; k < 3; ++k) {
            int64_t v = tri[3 * t + k];
            if (v < 0 || v >= nv) return -2;
            snap_uv(uv, v, W, H, &X[k], &Y[k]);
        }
        int64_t mnx = X[0], mxx = X[0], mny = Y[0], mxy = Y[0];
        for (int k = 1; k < 3; ++k) {
            if (X[k] < mnx) mnx = X[k];
            if (X[k] > mxx) mxx = X[k];
            if (Y[k] < mny) mny = Y[k];
            if (Y[k] > mxy) mxy = Y[k];
        }
        int i_lo, i_hi, r_lo, r_hi;
        cell_range(mnx, mxx, W, &i_lo, &i_hi);
        cell_range(mny, mxy, H, &r_lo, &r_hi);
        if (r_lo < j0) r_lo = j0;
        if (r_hi > j1 - 1) r_hi = j1 - 1;
        for (int j = r_lo; j <= r_hi; ++j)
            for (int i = i_lo; i <= i_hi; ++i) {
                int64_t e[3], E;
                if (!tri_sample(X, Y, 256 * (int64_t)i + 128, 256 * (int64_t)j + 128, e, &E))
                    continue;
                int64_t idx = (int64_t)(j - j0) * W + i;
                if (own[idx] < 0) own[idx] = (int32_t)t;
                if (cover_count) cover_count[idx] += 1;
            }
    }

    for (int j = j0; j < j1; ++j)
        for (int i = 0; i < W; ++i) {
            int64_t idx = (int64_t)(j - j0) * W + i;
            int32_t t = own[idx];
            if (t < 0) {
                if (bary) { bary[idx] = 0.0; bary[n + idx] = 0.0; }
                if (pos_out) { pos_out[idx] = NAN; pos_out[n + idx] = NAN; pos_out[2 * n + idx] = NAN; }
                if (nrm_out) { nrm_out[idx] = 0.0; nrm_out[n + idx] = 0.0; nrm_out[2 * n + idx] = 0.0; }
                if (w_out) w_out[idx] = 0.0;
                continue;
            }
            int64_t X[3], Y[3], e[3], E;
            int64_t v[3];
            for (int k = 0; k < 3; ++k) {
                v[k] = tri[3 * (int64_t)t + k];
                snap_uv(uv, v[k], W, H, &X[k], &Y[k]);
            }
            tri_sample(X, Y, 256 * (int64_t)i + 128, 256 * (int64_t)j + 128, e, &E);
            double b[3];
            for (int k = 0; k < 3; ++k) b[k] = (double)e[k] / (double)E;
            if (bary) { bary[idx] = b[1]; bary[n + idx] = b[2]; }
            double P[3][3];
            for (int k = 0; k < 3; ++k)
                for (int c = 0; c < 3; ++c) P[k][c] = (double)pos[3 * v[k] + c];
            if (pos_out)
                for (int c = 0; c < 3; ++c)
                    pos_out[c * n + idx] = b[0] * P[0][c] + b[1] * P[1][c] + b[2] * P[2][c];
            double u1[3], u2[3], f[3];
            for (int c = 0; c < 3; ++c) { u1[c] = P[1][c] - P[0][c]; u2[c] = P[2][c] - P[0][c]; }
            f[0] = u1[1] * u2[2] - u1[2] * u2[1];
            f[1] = u1[2] * u2[0] - u1[0] * u2[2];
            f[2] = u1[0] * u2[1] - u1[1] * u2[0];
            double flen = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
            if (nrm_out) {
                double m[3];
                if (nrm) {
                    for (int c = 0; c < 3; ++c)
                        m[c] = b[0] * (double)nrm[3 * v[0] + c] + b[1] * (double)nrm[3 * v[1] + c] +
                               b[2] * (double)nrm[3 * v[2] + c];
                } else {
                    for (int c = 0; c < 3; ++c) m[c] = f[c];
                }
                double len = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
                for (int c = 0; c < 3; ++c) nrm_out[c * n + idx] = len > 0.0 ? m[c] / len : 0.0;
            }
            if (w_out) w_out[idx] = 131072.0 * (0.5 * flen) / (double)E;
        }
    if (!tri_id) free(own);
    return 0;
}

/* ------------------------------------------------------------------------
 * Canonical fp32 projection of a point by the row-major camera matrix M
 * (clip = M [x y z 1]^T), §4.3.1 (projective texture mapping from the camera
 * position; homogeneous coordinates divided by w).  Returns 0 when clip w is
 * not > 0 (behind the camera, or NaN input).
 * ------------------------------------------------------------------------ */
static int project(const float M[16], float x, float y, float z, float *xn, float *yn, float *zn)
{
    float c[4];
    for (int k = 0; k < 4; ++k)
        c[k] = fmaf(M[4 * k + 2], z, fmaf(M[4 * k + 1], y, fmaf(M[4 * k + 0], x, M[4 * k + 3])));
    if (!(c[3] > 0.0f)) return 0;
    *xn = c[0] / c[3];
    *yn = c[1] / c[3];
    *zn = c[2] / c[3];
    return 1;
}

/* ------------------------------------------------------------------------
 * Depth texture (§4.3.1: the depth of the scene seen from the editing
 * camera, against which occluded fragments are discarded).  Rows [r0, r1) of
 * a Wd x Hd map, initialised to 1.0 (far).  Reading: GL window depth
 * d = 0.5 z_ndc + 0.5; pixel (ix, iy) samples its centre, row 0 at NDC
 * y = -1.  A triangle whose three vertices lie in front of the near plane
 * (z_clip + w_clip >= 0, w_clip > 0) and inside the guard band
 * |x_clip|, |y_clip| <= 16 w_clip is drawn as it is; one with a vertex
 * beyond any of these five planes is clipped against them (as the fixed-
 * function pipeline clips primitives) and the remaining polygon drawn as a
 * fan from its first vertex.  Clipping is in fp64 on the fp32 clip
 * coordinates, one plane after the other; a cut edge is split at
 * s + t (o - s), t = f(s) / (f(s) - f(o)), from its inside end s to its
 * outside end o (f the plane's signed distance), so that the two triangles
 * sharing an edge cut it at the same point.  A vertex of the triangle keeps
 * its fp32 projection (x_clip / w_clip in fp32); a cut point's NDC is its
 * fp64 quotient rounded to fp32, x and y clamped to [-16, 16].  Screen
 * position s = fmaf(ndc, .5, .5) * size in fp32, then the shared fixed-point
 * raster rule; depth is interpolated with the screen-space barycentrics in
 * fp64 (window depth is affine on screen), samples outside [0, 1] are
 * dropped, the nearest is kept, stored as fp32.
 * ------------------------------------------------------------------------ */
static void depth_raster(const float xn[3], const float yn[3], const float zn[3], int Wd, int Hd, int r0, int r1,
                         float *depth)
{
    int64_t X[3], Y[3];
    double d[3];
    for (int k = 0; k < 3; ++k) {
        float sx = fmaf(xn[k], 0.5f, 0.5f) * (float)Wd;
        float sy = fmaf(yn[k], 0.5f, 0.5f) * (float)Hd;
        X[k] = snap256((double)sx);
        Y[k] = snap256((double)sy);
        d[k] = (double)fmaf(zn[k], 0.5f, 0.5f);
    }
    int64_t mnx = X[0], mxx = X[0], mny = Y[0], mxy = Y[0];
    for (int k = 1; k < 3; ++k) {
        if (X[k] < mnx) mnx = X[k];
        if (X[k] > mxx) mxx = X[k];
        if (Y[k] < mny) mny = Y[k];
        if (Y[k] > mxy) mxy = Y[k];
    }
    int i_lo, i_hi, q_lo, q_hi;
    cell_range(mnx, mxx, Wd, &i_lo, &i_hi);
    cell_range(mny, mxy, Hd, &q_lo, &q_hi);
    if (q_lo < r0) q_lo = r0;
    if (q_hi > r1 - 1) q_hi = r1 - 1;
    for (int iy = q_lo; iy <= q_hi; ++iy)
        for (int ix = i_lo; ix <= i_hi; ++ix) {
            int64_t e[3], E;
            if (!tri_sample(X, Y, 256 * (int64_t)ix + 128, 256 * (int64_t)iy + 128, e, &E)) continue;
            double z = ((double)e[0] / (double)E) * d[0] + ((double)e[1] / (double)E) * d[1] +
                       ((double)e[2] / (double)E) * d[2];
            if (!(z >= 0.0 && z <= 1.0)) continue;
            float zf = (float)z;
            int64_t idx = (int64_t)(iy - r0) * Wd + ix;
            if (zf < depth[idx]) depth[idx] = zf;
        }
}

/* signed distance to clipping plane p (>= 0 inside): the near plane, then
 * the guard band's right, left, top and bottom sides */
static double clip_dist(int p, const double c[4])
{
    switch (p) {
    case 0: return c[2] + c[3];
    case 1: return 16.0 * c[3] - c[0];
    case 2: return 16.0 * c[3] + c[0];
    case 3: return 16.0 * c[3] - c[1];
    default: return 16.0 * c[3] + c[1];
    }
}

typedef struct {
    double c[4];
    int orig;           /* the triangle's vertex it is, or -1 for a cut point */
} clip_vert;

/* Sutherland-Hodgman step: the part of polygon in[0..n) inside plane p */
static int clip_plane(const clip_vert *in, int n, int p, clip_vert *out)
{
    int m = 0;
    for (int i = 0; i < n; ++i) {
        const clip_vert *a = &in[i], *b = &in[(i + 1) % n];
        double fa = clip_dist(p, a->c), fb = clip_dist(p, b->c);
        int ina = fa >= 0.0, inb = fb >= 0.0;
        if (ina) out[m++] = *a;
        if (ina != inb) {
            const clip_vert *sv = ina ? a : b, *ov = ina ? b : a;
            double fs = ina ? fa : fb, fo = ina ? fb : fa;
            double t = fs / (fs - fo);
            clip_vert q;
            q.orig = -1;
            for (int k = 0; k < 4; ++k) q.c[k] = sv->c[k] + t * (ov->c[k] - sv->c[k]);
            out[m++] = q;
        }
    }
    return m;
}

static float clamp16(float x) { return x < -16.0f ? -16.0f : (x > 16.0f ? 16.0f : x); }

int orc_depth_map(const float *pos, const int32_t *tri, int64_t nv, int64_t nt, const float M[16],
                  int Wd, int Hd, int r0, int r1, float *depth)
{
    if (Wd <= 0 || Hd <= 0 || r0 < 0 || r1 > Hd || r0 > r1) return -1;
    const int64_t n = (int64_t)(r1 - r0) * Wd;
    for (int64_t k = 0; k < n; ++k) depth[k] = 1.0f;
    for (int64_t t = 0; t < nt; ++t) {
        float cf[3][4];
        int finite = 1, inside = 1;
        for (int k = 0; k < 3; ++k) {
            int64_t v = tri[3 * t + k];
            if (v < 0 || v >= nv) return -2;
            float x = pos[3 * v], y = pos[3 * v + 1], z = pos[3 * v + 2];
            for (int q = 0; q < 4; ++q) {
                cf[k][q] = fmaf(M[4 * q + 2], z, fmaf(M[4 * q + 1], y, fmaf(M[4 * q + 0], x, M[4 * q + 3])));
                if (!isfinite(cf[k][q])) finite = 0;
            }
            double c[4] = {cf[k][0], cf[k][1], cf[k][2], cf[k][3]};
            if (!(cf[k][3] > 0.0f)) inside = 0;
            for (int p = 0; p < 5; ++p)
                if (!(clip_dist(p, c) >= 0.0)) inside = 0;
        }
        if (!finite) continue;
        float xn[3], yn[3], zn[3];
        if (inside) {
            for (int k = 0; k < 3; ++k) {
                xn[k] = cf[k][0] / cf[k][3];
                yn[k] = cf[k][1] / cf[k][3];
                zn[k] = cf[k][2] / cf[k][3];
            }
            depth_raster(xn, yn, zn, Wd, Hd, r0, r1, depth);
            continue;
        }
        clip_vert poly[2][9];
        int m = 3;
        for (int k = 0; k < 3; ++k) {
            for (int q = 0; q < 4; ++q) poly[0][k].c[q] = (double)cf[k][q];
            poly[0][k].orig = k;
        }
        int cur = 0;
        for (int p = 0; p < 5 && m >= 3; ++p) {
            m = clip_plane(poly[cur], m, p, poly[1 - cur]);
            cur = 1 - cur;
        }
        if (m < 3) continue;
        float px[9], py[9], pz[9];
        int ok = 1;
        for (int k = 0; k < m; ++k) {
            const clip_vert *v = &poly[cur][k];
            if (!(v->c[3] > 0.0)) { ok = 0; break; }
            if (v->orig >= 0) {
                const float *c = cf[v->orig];
                px[k] = c[0] / c[3];
                py[k] = c[1] / c[3];
                pz[k] = c[2] / c[3];
            } else {
                px[k] = clamp16((float)(v->c[0] / v->c[3]));
                py[k] = clamp16((float)(v->c[1] / v->c[3]));
                pz[k] = (float)(v->c[2] / v->c[3]);
            }
        }
        if (!ok) continue;
        for (int k = 1; k + 1 < m; ++k) {
            xn[0] = px[0]; yn[0] = py[0]; zn[0] = pz[0];
            xn[1] = px[k]; yn[1] = py[k]; zn[1] = pz[k];
            xn[2] = px[k + 1]; yn[2] = py[k + 1]; zn[2] = pz[k + 1];
            depth_raster(xn, yn, zn, Wd, Hd, r0, r1, depth);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Layer write (§4.3.1: the edit writes its value into the layer's data
 * texture wherever the tool selects).  Reading: overwrite; label 0 erases; u8 or u16 planes.
 * ------------------------------------------------------------------------ */
static void put(void *layer, int dtype, int64_t t, uint32_t label)
{
    if (dtype == ORC_U8) ((uint8_t *)layer)[t] = (uint8_t)label;
    else ((uint16_t *)layer)[t] = (uint16_t)label;
}

static uint32_t get(const void *layer, int dtype, int64_t t)
{
    return dtype == ORC_U8 ? ((const uint8_t *)layer)[t] : ((const uint16_t *)layer)[t];
}

/* ------------------------------------------------------------------------
 * Brush edit.  The paper's tool selects a region of the surface and writes
 * the chosen value there (§4.3.1); this surface brush selects the texels whose
 * surface point lies in the closed ball |p - c| <= r, with no visibility test:
 *   d2 = fmaf(dz, dz, fmaf(dy, dy, dx*dx)),  selected iff d2 <= r*r   (fp32)
 * Uncovered texels carry NaN positions and are never selected.
 * ------------------------------------------------------------------------ */
int64_t orc_brush(const float *px, const float *py, const float *pz, int64_t n,
                  const float c[3], float r, uint32_t label, void *layer, int dtype)
{
    int64_t count = 0;
    float r2 = r * r;
    for (int64_t t = 0; t < n; ++t) {
        float dx = px[t] - c[0], dy = py[t] - c[1], dz = pz[t] - c[2];
        float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        if (d2 <= r2) { put(layer, dtype, t, label); ++count; }
    }
    return count;
}

/* ------------------------------------------------------------------------
 * Point in polygon by the even-odd crossing number of a ray towards +x,
 * half-open in y (an edge counts when exactly one end is above yn).
 * The paper masks the projected tool square with a shape texture (§4.3.1,
 * shape masking); a lasso polygon in NDC replaces the bitmap shape.
 * ------------------------------------------------------------------------ */
int orc_point_in_polygon(float xn, float yn, const float *poly, int n)
{
    int inside = 0;
    for (int k = 0; k < n; ++k) {
        float x0 = poly[2 * k], y0 = poly[2 * k + 1];
        float x1 = poly[2 * ((k + 1) % n)], y1 = poly[2 * ((k + 1) % n) + 1];
        if ((y0 > yn) != (y1 > yn)) {
            float lhs = (xn - x0) * (y1 - y0);
            float rhs = (x1 - x0) * (yn - y0);
            if (y1 > y0 ? lhs < rhs : lhs > rhs) inside = !inside;
        }
    }
    return inside;
}

/* ------------------------------------------------------------------------
 * Lasso edit (§4.3.1: depth test against the depth texture with a small bias,
 * projective mapping through the camera, discard outside [0,1], shape mask,
 * write).  Per texel, canonical fp32:
 *   project with M; reject unless w > 0 and x, y, z_ndc all in [-1, 1];
 *   ix = min(floor(fmaf(xn,.5,.5) * Wd), Wd-1), iy likewise;
 *   visible iff fmaf(zn,.5,.5) <= D[iy*Wd + ix] + bias;
 *   inside iff orc_point_in_polygon(xn, yn).
 * ------------------------------------------------------------------------ */
int64_t orc_lasso(const float *px, const float *py, const float *pz, int64_t n, const float M[16],
                  const float *poly, int npoly, const float *depth, int Wd, int Hd, float bias,
                  uint32_t label, void *layer, int dtype)
{
    int64_t count = 0;
    for (int64_t t = 0; t < n; ++t) {
        float xn, yn, zn;
        if (!project(M, px[t], py[t], pz[t], &xn, &yn, &zn)) continue;
        if (!(xn >= -1.0f && xn <= 1.0f && yn >= -1.0f && yn <= 1.0f && zn >= -1.0f && zn <= 1.0f))
            continue;
        int ix = (int)floorf(fmaf(xn, 0.5f, 0.5f) * (float)Wd);
        int iy = (int)floorf(fmaf(yn, 0.5f, 0.5f) * (float)Hd);
        if (ix > Wd - 1) ix = Wd - 1;
        if (iy > Hd - 1) iy = Hd - 1;
        float d = fmaf(zn, 0.5f, 0.5f);
        if (!(d <= depth[(int64_t)iy * Wd + ix] + bias)) continue;
        if (!orc_point_in_polygon(xn, yn, poly, npoly)) continue;
        put(layer, dtype, t, label);
        ++count;
    }
    return count;
}

/* ------------------------------------------------------------------------
 * Layer algebra (§3.4.2: layer systems combine layers with logic operations;
 * §4.2: database layers hold unsigned keys).  Reading: each operand gives a
 * predicate P_X = (sel_X == 0 ? X != 0 : X == sel_X); AND / OR / XOR write
 * out_label where the combined predicate holds and 0 elsewhere; REMAP writes
 * lut[a] (lut[0] must be 0).  dst may alias a or b.
 * ------------------------------------------------------------------------ */
int orc_layer_op(int op, void *dst, int dt_dst, const void *a, int dt_a, const void *b, int dt_b,
                 int64_t n, uint32_t sel_a, uint32_t sel_b, uint32_t out_label, const uint16_t *lut)
{
    for (int64_t t = 0; t < n; ++t) {
        uint32_t va = get(a, dt_a, t);
        uint32_t res;
        if (op == ORC_REMAP) {
            res = lut[va];
        } else {
            uint32_t vb = get(b, dt_b, t);
            int pa = sel_a == 0 ? va != 0 : va == sel_a;
            int pb = sel_b == 0 ? vb != 0 : vb == sel_b;
            int p = op == ORC_AND ? (pa && pb) : op == ORC_OR ? (pa || pb) : (pa != pb);
            res = p ? out_label : 0;
        }
        put(dst, dt_dst, t, res);
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Per-label surface area.  Table 1 reports the surface area one texel
 * stands for; summing those texel areas over the texels holding a label
 * gives the labelled area.  area[l] = sum over covered texels with L = l of
 * w, in fp64 with Neumaier compensation; all nbins bins, including label 0.
 * ------------------------------------------------------------------------ */
int orc_area(const double *w, const int32_t *tri_id, const void *layer, int dtype, int64_t n,
             double *area, int nbins)
{
    double *comp = (double *)calloc((size_t)nbins, sizeof(double));
    for (int l = 0; l < nbins; ++l) area[l] = 0.0;
    for (int64_t t = 0; t < n; ++t) {
        if (tri_id[t] < 0) continue;
        uint32_t l = get(layer, dtype, t);
        if ((int)l >= nbins) { free(comp); return -1; }
        double s = area[l], x = w[t], u = s + x;
        if (fabs(s) >= fabs(x)) comp[l] += (s - u) + x;
        else comp[l] += (x - u) + s;
        area[l] = u;
    }
    for (int l = 0; l < nbins; ++l) area[l] += comp[l];
    free(comp);
    return 0;
}

/* ------------------------------------------------------------------------
 * Texture padding (§4.3.2, TPA).  The outline mask holds the texels around
 * the texture islands: texels no triangle covers whose distance to a
 * covered texel is at most k.  After an edit, every outline texel whose
 * distance to the edited area (the texels that edit selected) is at most k
 * takes the edit's label.  Reading: distance between texels is the
 * Chebyshev distance of their indices (the paper's square kernel of radius
 * k, a (2k+1) x (2k+1) window), windows clipped at the atlas border; the
 * paper pads one texel, k = 1, for both masks.
 * ------------------------------------------------------------------------ */
int64_t orc_outline(const int32_t *tri_id, int W, int H, int k, uint8_t *outline)
{
    int64_t count = 0;
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            int64_t t = (int64_t)j * W + i;
            outline[t] = 0;
            if (tri_id[t] >= 0) continue;
            for (int v = j - k; v <= j + k && !outline[t]; ++v)
                for (int u = i - k; u <= i + k; ++u) {
                    if (u < 0 || v < 0 || u >= W || v >= H) continue;
                    if (tri_id[(int64_t)v * W + u] >= 0) { outline[t] = 1; break; }
                }
            count += outline[t];
        }
    return count;
}

int64_t orc_pad(const uint8_t *outline, const uint8_t *edited, int W, int H, int k, uint32_t label,
                void *layer, int dtype)
{
    int64_t count = 0;
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            int64_t t = (int64_t)j * W + i;
            if (!outline[t]) continue;
            int hit = 0;
            for (int v = j - k; v <= j + k && !hit; ++v)
                for (int u = i - k; u <= i + k; ++u) {
                    if (u < 0 || v < 0 || u >= W || v >= H) continue;
                    if (edited[(int64_t)v * W + u]) { hit = 1; break; }
                }
            if (hit) { put(layer, dtype, t, label); ++count; }
        }
    return count;
}

/* ------------------------------------------------------------------------
 * Screen-space tool (§4.3.1, the paper's own TEA selection): the camera
 * doubles as a slide projector whose frustum is narrowed, by the tool
 * transform of §4.3.1, to the tool's square on the window; a fragment's
 * projective texture coordinates outside [0,1] are discarded, the rest
 * index the tool's shape texture, and the depth test applies.
 * Reading (the printed translate factor has the sign that does not centre
 * the tool on its position): with window size (Ww, Wh), tool position
 * (Tpx, Tpy) in window pixels from the lower-left corner and tool size
 * (Tw, Th) pixels, a point with NDC (xn, yn) gets
 *   s = xn Ww/(2 Tw) - (Tpx - Ww/2)/Tw + 1/2,   t likewise with Wh, Tpy, Th,
 * i.e. s = (wx - Tpx)/Tw + 1/2 for its window position wx = (xn + 1) Ww/2:
 * the Tw x Th square centred on the tool maps onto [0,1]^2.  In fp32,
 * s = fmaf(xn, a, b) with a = Ww/(2 Tw) and b = 1/2 - (Tpx - Ww/2)/Tw each
 * computed in fp64 and rounded once (orc_tool_coeffs).  Selected iff the
 * lasso's projective and depth tests pass (clip w > 0; x, y, z_ndc in
 * [-1, 1]; d <= D + bias), s and t lie in [0, 1], and the shape texel
 * (min(floor(s sw), sw - 1), min(floor(t sh), sh - 1)) of the sw x sh u8
 * shape texture (row 0 at t = 0) is not 0.
 * ------------------------------------------------------------------------ */
void orc_tool_coeffs(const double tool[6], float ab[4])
{
    /* tool = {Ww, Wh, Tpx, Tpy, Tw, Th} */
    ab[0] = (float)(tool[0] / (2.0 * tool[4]));
    ab[1] = (float)(0.5 - (tool[2] - 0.5 * tool[0]) / tool[4]);
    ab[2] = (float)(tool[1] / (2.0 * tool[5]));
    ab[3] = (float)(0.5 - (tool[3] - 0.5 * tool[1]) / tool[5]);
}

int64_t orc_tool(const float *px, const float *py, const float *pz, int64_t n, const float M[16],
                 const double tool[6], const uint8_t *shape, int sw, int sh, const float *depth, int Wd,
                 int Hd, float bias, uint32_t label, void *layer, int dtype)
{
    float ab[4];
    orc_tool_coeffs(tool, ab);
    int64_t count = 0;
    for (int64_t t = 0; t < n; ++t) {
        float xn, yn, zn;
        if (!project(M, px[t], py[t], pz[t], &xn, &yn, &zn)) continue;
        if (!(xn >= -1.0f && xn <= 1.0f && yn >= -1.0f && yn <= 1.0f && zn >= -1.0f && zn <= 1.0f))
            continue;
        int ix = (int)floorf(fmaf(xn, 0.5f, 0.5f) * (float)Wd);
        int iy = (int)floorf(fmaf(yn, 0.5f, 0.5f) * (float)Hd);
        if (ix > Wd - 1) ix = Wd - 1;
        if (iy > Hd - 1) iy = Hd - 1;
        float d = fmaf(zn, 0.5f, 0.5f);
        if (!(d <= depth[(int64_t)iy * Wd + ix] + bias)) continue;
        float s = fmaf(xn, ab[0], ab[1]), u = fmaf(yn, ab[2], ab[3]);
        if (!(s >= 0.0f && s <= 1.0f && u >= 0.0f && u <= 1.0f)) continue;
        int sx = (int)floorf(s * (float)sw), sy = (int)floorf(u * (float)sh);
        if (sx > sw - 1) sx = sw - 1;
        if (sy > sh - 1) sy = sh - 1;
        if (!shape[(int64_t)sy * sw + sx]) continue;
        put(layer, dtype, t, label);
        ++count;
    }
    return count;
}
