/*
 * uvl.h - C ABI of libuvl.so: thematic layers stored as 2D texture atlases
 * indexed by a mesh's texture coordinates, edited and queried on an AMD
 * Instinct MI355X (gfx950).
 *
 * Method: "An Efficient GPU Approach for Designing 3D Cultural Heritage
 * Information Systems" (arXiv 2501.14807).  The paper keeps every layer as a
 * data texture on the GPU (§4.2), indexes it with the mesh's texture
 * coordinates (§4.1), and edits it with the Texture Editing Algorithm
 * (§4.3.1): depth test against a depth texture, projective mapping of the
 * tool through the camera, shape masking, and a write of the chosen value.
 *
 * Conventions shared by every call:
 *  - Every call returns a uvl_status.  Arguments are validated on the host
 *    before anything is enqueued; on error nothing is enqueued.  A failing
 *    HIP launch returns UVL_E_DEVICE.  Nothing aborts the process.
 *  - Device pointers are borrowed: the caller allocates and frees all device
 *    memory and keeps it alive until the work on `stream` has completed.
 *    The library allocates no device memory, except the layer pool
 *    (uvl_pool_*), whose purpose that is.
 *  - Host arrays (centre, matrix, polygon) are read during the call and may
 *    be freed on return.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous on it unless stated otherwise.
 *  - Texel (i, j) of a W x H atlas is element j*W + i; row j holds texture
 *    coordinate v in [j/H, (j+1)/H) and its sample is the texel centre.
 *  - Two calls on different streams that write the same layer race; the
 *    caller orders them.
 */
#ifndef UVL_H
#define UVL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    UVL_OK = 0,
    UVL_E_INVAL = -1,        /* null pointer, bad size, value out of range    */
    UVL_E_SHAPE = -2,        /* layer / geometry image sizes do not match     */
    UVL_E_DTYPE = -3,        /* unknown layer dtype or label does not fit     */
    UVL_E_NOMEM = -4,        /* workspace too small                           */
    UVL_E_DEVICE = -5,       /* a HIP call or kernel launch failed            */
    UVL_E_UNSUPPORTED = -6,  /* the current device is not gfx950              */
    UVL_E_RANGE = -7         /* texel areas span too wide a range for one
                                uint32 word per texel: give area_w_hi         */
} uvl_status;

/* Layer data types (§4.2: the data texture holds 8/16/32-bit integers or
 * 16/32-bit floats; database layers hold unsigned primary keys).  Label
 * (database) layers, uvl_layer, are UVL_U8 or UVL_U16; their value 0 is the
 * null key ("no data"), standing in for the layer's mask texture.  Numeric
 * layers, uvl_numeric, take any of the five and carry a mask plane.
 * UVL_I32 is signed; UVL_F16 and UVL_F32 are IEEE binary16 and binary32. */
typedef enum { UVL_U8 = 1, UVL_U16 = 2, UVL_I32 = 3, UVL_F16 = 4, UVL_F32 = 5 } uvl_dtype;

/* Layer operations (§3.4.2: layer systems combine layers with logic
 * operations).  See uvl_layer_op. */
typedef enum { UVL_AND = 0, UVL_OR = 1, UVL_XOR = 2, UVL_REMAP = 3 } uvl_op;

/* A triangle mesh in device memory (§4.3.1 lists vertices, normals and
 * texture coordinates as inputs of the editing algorithm).
 *   pos [nv][3] fp32, nrm [nv][3] fp32 (NULL: face normals are used),
 *   uv  [nv][2] fp32 with every coordinate in [-4, 4],
 *   tri [nt][3] int32 vertex indices in [0, nv). */
typedef struct {
    const float *pos;
    const float *nrm;
    const float *uv;
    const int32_t *tri;
    int64_t nv;
    int64_t nt;
} uvl_mesh;

/* Geometry image: the mesh rendered into texture space once per model and
 * atlas size, so that each edit reads per-texel surface data instead of
 * re-rasterising the mesh (§4.3.1 renders the mesh with its texture
 * coordinates as vertex positions on every edit).  Structure of arrays, one
 * plane of N = width*height elements each, every plane pointer 16-byte
 * aligned, all in device memory and owned by the caller:
 *   tri_id        owning triangle, -1 where no triangle covers the centre
 *   pos_x/y/z     surface position (fp32 of an fp64 interpolation), NaN
 *                 where uncovered
 *   nrm_x/y/z     unit normal, 0 where uncovered (all three NULL: skipped)
 *   bary1/2       barycentrics of vertices 1 and 2 (both NULL: skipped)
 *   area_w        surface area of the texel in units of area_scale, 0 where
 *                 uncovered (uint32 fixed point; the low word when
 *                 area_w_hi is given)
 *   area_w_hi     optional (NULL: one word per texel): the high words, the
 *                 texel's area then being (area_w_hi * 2^32 + area_w) *
 *                 area_scale
 * area_scale and area_abs_err are written by uvl_build_geometry_image: a
 * texel's area is area_w * area_scale (or the two-word form), off from the
 * exact fp64 weight by at most area_abs_err = area_scale / 2, so a label's
 * area over k texels is within k * area_abs_err.  The scale is a power of
 * two chosen from the largest texel area w_max (area_abs_err <= 2^-31 w_max
 * with one word, 2^-63 w_max with two), so a texel of area at least 2^-11
 * w_max (one word) or 2^-43 w_max (two words) is within 2^-20 (< 1e-6)
 * relative.  The one-word build fails with UVL_E_RANGE when some texel's
 * area lies in [2^-43, 2^-11) w_max (two words would hold it to 2^-20);
 * texels lighter than 2^-43 w_max (triangles of numerically zero 3D area)
 * keep the absolute bound only.
 *   tile_box      optional (NULL: skipped): for each tile of UVL_TILE_SIDE x
 *                 UVL_TILE_SIDE texels (tile (tx, ty) holds texels i in
 *                 [32 tx, 32 tx + 32), j in [32 ty, 32 ty + 32); tiles are
 *                 stored row-major, ceil(W/32) per row), the bounds of its
 *                 covered positions as {min x, min y, min z, max x, max y,
 *                 max z}; a tile without covered texels holds min = +inf,
 *                 max = -inf: ntiles = ceil(W/32) * ceil(H/32) boxes of 6
 *                 floats, followed by the boxes of the blocks of
 *                 UVL_TILE_BLOCK x UVL_TILE_BLOCK tiles (block (bx, by) holds
 *                 tiles tx in [8 bx, 8 bx + 8), ty in [8 by, 8 by + 8);
 *                 row-major, ceil(ceil(W/32) / 8) per row), each the union
 *                 of its tiles' boxes.  Batched waves use them to skip tiles
 *                 (and whole blocks) an edit provably cannot select. */
#define UVL_TILE_SIDE 32
#define UVL_TILE_BLOCK 8
/*   area_blk      optional (NULL: skipped), one-word weights only (ignored
 *                 when area_w_hi is given): for each block of
 *                 UVL_AREA_BLK_ROWS x UVL_AREA_BLK_COLS texels (block (bx,
 *                 by) holds texels i in [8 bx, 8 bx + 8), j in [4 by,
 *                 4 by + 4); row-major, ceil(W/8) per row), the exact sum of
 *                 its area_w words: ceil(W/8) * ceil(H/4) uint64, 8-byte
 *                 aligned, written by uvl_build_geometry_image (a caller
 *                 that sets it afterwards must fill it the same way or
 *                 leave it NULL).  uvl_area_query, for one or two layers,
 *                 adds a block's sum for a layer whose labels are equal over
 *                 it instead of reading its 32 weights. */
#define UVL_AREA_BLK_ROWS 4
#define UVL_AREA_BLK_COLS 8
typedef struct {
    int32_t width, height;
    int32_t *tri_id;
    float *pos_x, *pos_y, *pos_z;
    float *nrm_x, *nrm_y, *nrm_z;
    float *bary1, *bary2;
    uint32_t *area_w;
    double area_scale;      /* out: texel area = area_w * area_scale            */
    double area_abs_err;    /* out: bound on the rounding of one texel's area   */
    float *tile_box;        /* optional per-tile position bounds (see above)    */
    uint32_t *area_w_hi;    /* optional high words of the texel areas           */
    uint64_t *area_blk;     /* optional per-block sums of area_w (see above)    */
} uvl_geom;

/* A layer's data texture: width*height values of `dtype`, device memory,
 * 16-byte aligned, row-major as above (§4.2 "data texture"). */
typedef struct {
    void *data;
    int32_t width, height;
    int32_t dtype;          /* uvl_dtype */
} uvl_layer;

/* Planes of a geometry image, for uvl_geom_bytes: tri_id, pos_x/y/z and
 * area_w always, these besides. */
#define UVL_GEOM_NRM      1u   /* nrm_x, nrm_y, nrm_z */
#define UVL_GEOM_BARY     2u   /* bary1, bary2 */
#define UVL_GEOM_TILE_BOX 4u   /* tile_box */
#define UVL_GEOM_AREA_HI  8u   /* area_w_hi */
#define UVL_GEOM_AREA_BLK 16u  /* area_blk */

/* Device bytes of the planes of a width x height geometry image: each plane
 * of N = width*height elements rounded up to a multiple of 256 bytes (so
 * that planes cut from one buffer stay aligned), plus the planes named by
 * plane_flags.  0 for a size outside [1, 32768] or an unknown flag. */
size_t uvl_geom_bytes(int32_t width, int32_t height, uint32_t plane_flags);

/* Text for a status code (static storage). */
const char *uvl_status_str(int32_t status);

/* Returns UVL_OK if the current HIP device is a gfx950, else
 * UVL_E_UNSUPPORTED (or UVL_E_DEVICE if HIP fails). */
int32_t uvl_device_check(void);

/* Workspace bytes uvl_build_geometry_image needs for a mesh of nt
 * triangles and a width x height atlas (0 for sizes out of range). */
size_t uvl_build_workspace_bytes(int64_t nt, int32_t width, int32_t height);

/* Render the mesh into texture space (§4.3.1, the texture-space render with
 * texture coordinates as positions; §4.1, texture coordinates index the
 * layer).  For each texel centre: the covering triangle (coordinates snapped
 * to 1/256 texel, round half to even; a centre on an edge belongs to the
 * triangle whose counter-clockwise edge s->t has t.y < s.y, or t.y == s.y and
 * t.x > s.x; the lowest triangle index wins where triangles overlap;
 * zero-area triangles cover nothing), its barycentrics b_k = e_k/|E| from the
 * exact integer edge functions, position b0 P0 + b1 P1 + b2 P2 summed left to
 * right in fp64 and rounded to fp32, unit normal, and area weight
 * 131072 * A3 / |E| (A3 the triangle's 3D area) quantised to one uint32
 * word (area_w_hi NULL) or two (low and high words) with a power-of-two
 * scale.
 * ws: device workspace of uvl_build_workspace_bytes(nt, width, height) bytes.
 * SYNCHRONOUS: waits for `stream` to read back area_scale.
 * mesh->tri may be NULL when nt == 0 (every texel is then uncovered).
 * Errors: UVL_E_INVAL for null planes, width/height outside [1, 32768],
 * a texture coordinate outside [-4, 4] or a vertex index outside [0, nv)
 * (the planes are then undefined); UVL_E_NOMEM if ws_bytes is too small;
 * UVL_E_RANGE (one word only) if some texel's area lies in [2^-43, 2^-11)
 * of the largest: every plane is written, but such texels may be off by
 * more than 2^-20 relative (build again with area_w_hi). */
int32_t uvl_build_geometry_image(const uvl_mesh *mesh, uvl_geom *geom, void *ws, size_t ws_bytes,
                                 void *stream);

/* Validate a layer descriptor and fill its data with 0 (the null key). */
int32_t uvl_create_layer(const uvl_layer *layer, void *stream);

/* Workspace bytes uvl_render_depth needs for a mesh of nt triangles. */
size_t uvl_depth_workspace_bytes(int64_t nt);

/* Depth texture of the scene from a camera (§4.3.1: scene depth from the
 * current viewpoint, rebuilt when the viewpoint changes).  view_proj: host
 * fp32 row-major 4x4 with clip = M [x y z 1]^T.  depth: device fp32 [dh][dw],
 * row 0 at NDC y = -1, window depth 0.5 z_ndc + 0.5, cleared to 1.0; each
 * pixel keeps the nearest sample of the mesh, rasterised with the rule of
 * uvl_build_geometry_image on screen positions fmaf(ndc, .5, .5) * size and
 * interpolated in fp64; samples outside [0, 1] are dropped.  A triangle
 * whose vertices all have clip w > 0 and lie in front of the near plane
 * (z + w >= 0) and inside the guard band |x|, |y| <= 16 w is drawn as it
 * is; any other is clipped against those five planes (fp64 Sutherland-
 * Hodgman on the fp32 clip coordinates, each cut edge split from its inside
 * end) and the polygon drawn as a fan from its first vertex, so that
 * occluders close to the camera stay in the depth texture.
 * Errors: UVL_E_INVAL for null pointers or dw/dh outside [1, 16384];
 * UVL_E_NOMEM if ws_bytes is too small. */
int32_t uvl_render_depth(const uvl_mesh *mesh, const float view_proj[16], float *depth, int32_t dw,
                         int32_t dh, void *ws, size_t ws_bytes, void *stream);

/* Allocation-free variant of uvl_render_depth, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, result and
 * errors without ws/ws_bytes: the workspace is a static device array of
 * 256 + 4 * UVL_DEPTH_NOALLOC_MAX_TRIS bytes (16 MiB) per device, held
 * until the process ends, so meshes of more than UVL_DEPTH_NOALLOC_MAX_TRIS
 * triangles are refused with UVL_E_NOMEM.  Every call on one device shares
 * that array: calls that overlap on one device (different streams, or
 * different host threads) race and must be ordered by the caller.  The
 * call allocates nothing itself. */
#define UVL_DEPTH_NOALLOC_MAX_TRIS 4194304
int32_t uvl_render_depth_noalloc(const uvl_mesh *mesh, const float view_proj[16], float *depth, int32_t dw,
                                 int32_t dh, void *stream);

/* Surface brush (§4.3.1 selects part of the surface and stores the chosen
 * value in the selected texels; here the tool is a 3D ball).  Every texel
 * whose position p satisfies, in fp32,
 *   fmaf(dz, dz, fmaf(dy, dy, dx*dx)) <= r*r,   d = p - centre,
 * gets `label` (uncovered texels hold NaN and never match).  center: host
 * float[3].  Errors: UVL_E_INVAL (null, radius negative or not finite),
 * UVL_E_SHAPE (layer size != geometry size), UVL_E_DTYPE (label too wide). */
int32_t uvl_edit_brush(const uvl_geom *geom, const uvl_layer *layer, const float center[3],
                       float radius, uint32_t label, void *stream);

/* Lasso (§4.3.1: depth test with a small bias, projective mapping through
 * the camera with coordinates outside the unit range discarded, then the
 * tool shape mask).  Per texel, in fp32 with fmaf and IEEE division:
 *   clip = M p (fmaf chains); require clip.w > 0 and x, y, z_ndc in [-1, 1];
 *   ix = min(floor(fmaf(x_ndc, .5, .5) * dw), dw-1), iy likewise;
 *   require fmaf(z_ndc, .5, .5) <= depth[iy*dw + ix] + bias;
 *   require (x_ndc, y_ndc) inside the polygon by the even-odd crossing rule
 *   (an edge counts when exactly one end is above y_ndc and the crossing lies
 *   to the right of x_ndc);
 * then writes `label`.  poly_xy: host float[n][2] in NDC, 3 <= n <= 64.
 * depth: device map from uvl_render_depth with the same matrix.
 * Errors: UVL_E_INVAL (null, n out of range, bias not finite, dw/dh < 1),
 * UVL_E_SHAPE, UVL_E_DTYPE as for uvl_edit_brush. */
int32_t uvl_edit_lasso(const uvl_geom *geom, const uvl_layer *layer, const float view_proj[16],
                       const float *poly_xy, int32_t n, const float *depth, int32_t dw, int32_t dh,
                       float bias, uint32_t label, void *stream);

/* Layer algebra (§3.4.2: logic operations between layers; §4.2: database
 * layers hold unsigned keys).  Operand predicate P_X = (sel_X == 0 ?
 * X != 0 : X == sel_X).  AND / OR / XOR: dst = (P_a op P_b) ? out_label : 0.
 * REMAP: dst = lut[a], lut a HOST array of 256 (a is u8) or 65536 (a is
 * u16) uint16 entries with lut[0] == 0 (the null key stays null) and every
 * entry within dst's dtype; it is read during the call and may be freed on
 * return (a 65536-entry table is staged through a ring of 16 library-owned
 * slots; a call that finds its slot still in use by an earlier REMAP waits
 * for that REMAP to finish).  b, sel_a, sel_b, out_label are ignored by
 * REMAP.  dst may alias a or b; all three must have the same size; their
 * dtypes may differ.  Errors: UVL_E_INVAL (null pointers, lut[0] != 0),
 * UVL_E_SHAPE, UVL_E_DTYPE (out_label or a table entry does not fit dst). */
int32_t uvl_layer_op(int32_t op, const uvl_layer *dst, const uvl_layer *a, const uvl_layer *b,
                     uint32_t sel_a, uint32_t sel_b, uint32_t out_label, const uint16_t *lut,
                     void *stream);

/* Per-label surface area (Table 1 reports the surface area one texel
 * represents; summed over the texels holding a label it gives the labelled
 * area).  For each of nlayers layers (1..32, same size as geom): bins[l] =
 * sum of area_w over covered texels with value l, exact uint64; layer k's
 * 256 (u8) or 65536 (u16) bins follow layer k-1's in bins_dev (device,
 * 8-byte aligned).  With two-word weights (geom->area_w_hi non-NULL) the
 * sums of the low words come first, then as many sums of the high words in
 * the same layout, and a bin's area is (high * 2^32 + low) * area_scale;
 * uvl_area_bin_count gives the number of uint64 either way.  One pass reads
 * each weight once for all the layers (two-word weights: once per 16 u8
 * layers).  If areas_host is non-NULL the call is SYNCHRONOUS and writes
 * the fp64 area of each bin there (one double per bin, the layers' bins in
 * order); otherwise it is asynchronous and the bins stay on the device.
 * Errors: UVL_E_INVAL, UVL_E_SHAPE, UVL_E_DTYPE. */
int32_t uvl_area_query(const uvl_geom *geom, const uvl_layer *layers, int32_t nlayers,
                       uint64_t *bins_dev, double *areas_host, void *stream);

/* Number of uint64 bins_dev must hold for uvl_area_query on these layers:
 * the layers' bins (256 per u8 layer, 65536 per u16 layer), twice that with
 * two-word weights.  0 for null pointers, nlayers outside 1..32 or a dtype
 * that is not u8/u16. */
int64_t uvl_area_bin_count(const uvl_geom *geom, const uvl_layer *layers, int32_t nlayers);

/* The paper's screen-space editing tool (§4.3.1): projective texture
 * mapping of the tool's shape texture through the camera, narrowed to the
 * tool's square on the window.  tool (host double[6]) = {Ww, Wh, Tpx, Tpy,
 * Tw, Th}: window size, tool position (window pixels from the lower-left
 * corner) and tool size (pixels), all finite, sizes > 0.  A texel is
 * selected iff, with xn, yn, z_ndc and the depth test exactly as for
 * uvl_edit_lasso (view_proj, depth [dh][dw], bias), its tool coordinates
 *   s = fmaf(xn, ax, bx), t = fmaf(yn, ay, by),
 *   ax = Ww / (2 Tw), bx = 1/2 - (Tpx - Ww/2) / Tw (fp64, rounded once to
 *   fp32; ay, by likewise with Wh, Tpy, Th)
 * lie in [0, 1] and the shape texel (min(floor(s sw), sw-1),
 * min(floor(t sh), sh-1)) of shape (device u8 [sh][sw], row 0 at t = 0,
 * 1 <= sw, sh <= 4096) is not 0.  The Tw x Th square centred on the tool
 * maps onto [0, 1]^2.
 * Errors: UVL_E_INVAL (pointers, tool, shape or depth sizes, bias),
 * UVL_E_SHAPE, UVL_E_DTYPE. */
int32_t uvl_edit_tool(const uvl_geom *geom, const uvl_layer *layer, const float view_proj[16], const double tool[6],
                      const uint8_t *shape, int32_t sw, int32_t sh, const float *depth, int32_t dw, int32_t dh,
                      float bias, uint32_t label, void *stream);

/* ------------------------------------------------------------------------
 * Texture padding (§4.3.2).  Around every texture island (the texels
 * triangles cover) the outline is the band of uncovered texels within
 * Chebyshev distance k of a covered texel (the paper's square kernel; it
 * pads one texel, k = 1).  After an edit, padding writes the edit's label
 * into every outline texel within distance k of a texel the edit selected,
 * so that sampling across an island's border reads the edited value.
 * Padding writes uncovered texels only (areas never change) and edits write
 * covered texels only, so a padding call may follow its edit at any time.
 * ------------------------------------------------------------------------ */

/* Device workspace bytes uvl_build_outline needs for a width x height
 * atlas (0 if the size is invalid). */
size_t uvl_outline_workspace_bytes(int32_t width, int32_t height);

/* Outline texels of geom for radius k (0..8): their indices j*W+i, in
 * ascending order, into outline (device int32, capacity entries); *count
 * (host) receives their number.  SYNCHRONOUS.
 * Errors: UVL_E_INVAL, UVL_E_NOMEM (ws too small, or more than capacity
 * outline texels: *count is still set and the first capacity are written),
 * UVL_E_DEVICE. */
int32_t uvl_build_outline(const uvl_geom *geom, int32_t k, int32_t *outline, int64_t capacity, int64_t *count,
                          void *ws, size_t ws_bytes, void *stream);

/* Padding after a brush edit (same center, radius, label as the edit):
 * outline[0..n) from uvl_build_outline on this geometry image (entries that
 * are not texel indices are ignored), k the padding radius (0..8).  Each
 * outline texel tests the brush predicate of uvl_edit_brush on the covered
 * texels of its (2k+1)^2 window.  Errors as uvl_edit_brush, plus UVL_E_INVAL
 * for k out of range and UVL_E_SHAPE for n > width*height. */
int32_t uvl_pad_brush(const uvl_geom *geom, const uvl_layer *layer, const int32_t *outline, int64_t n, int32_t k,
                      const float center[3], float radius, uint32_t label, void *stream);

/* Padding after a lasso edit (same arguments as the edit's). */
int32_t uvl_pad_lasso(const uvl_geom *geom, const uvl_layer *layer, const int32_t *outline, int64_t n, int32_t k,
                      const float view_proj[16], const float *poly_xy, int32_t npoly, const float *depth, int32_t dw,
                      int32_t dh, float bias, uint32_t label, void *stream);

/* ------------------------------------------------------------------------
 * Numeric layers (§4.2: numeric layers hold integer or real properties such
 * as curvature or age; an information layer is a data texture plus a mask
 * texture saying which texels hold valid data).  Edits select texels with
 * the same predicates as the label edits above and SET them (store the
 * value, set the mask bit) or ERASE them (clear the mask bit, keep the
 * data).  The value arrives as a double and is converted once on the host:
 * integer dtypes need an integral value in range (else UVL_E_DTYPE); floats
 * round to nearest, ties to even, and must stay finite (else UVL_E_DTYPE);
 * NaN is UVL_E_INVAL.
 * ------------------------------------------------------------------------ */
typedef enum { UVL_SET = 0, UVL_ERASE = 1 } uvl_value_mode;

/* A numeric layer: data as uvl_layer (width*height values of dtype, device,
 * 16-byte aligned, row-major) and mask, device uint32[ceil(width*height/32)]
 * 16-byte aligned, texel t = j*W + i valid iff bit t % 32 of mask[t / 32]
 * is set.  Bits beyond the last texel are never written. */
typedef struct {
    void *data;
    uint32_t *mask;
    int32_t width, height;
    int32_t dtype;          /* uvl_dtype, any of the five */
} uvl_numeric;

/* Zero the data and the mask (no texel valid).  Asynchronous. */
int32_t uvl_numeric_create(const uvl_numeric *layer, void *stream);

/* Numeric brush, lasso and screen-space tool: the selection of
 * uvl_edit_brush, uvl_edit_lasso and uvl_edit_tool (same arguments and
 * errors), then `mode` (uvl_value_mode) with `value` (ignored by ERASE). */
int32_t uvl_numeric_brush(const uvl_geom *geom, const uvl_numeric *layer, const float center[3], float radius,
                          int32_t mode, double value, void *stream);
int32_t uvl_numeric_lasso(const uvl_geom *geom, const uvl_numeric *layer, const float view_proj[16],
                          const float *poly_xy, int32_t n, const float *depth, int32_t dw, int32_t dh, float bias,
                          int32_t mode, double value, void *stream);
int32_t uvl_numeric_tool(const uvl_geom *geom, const uvl_numeric *layer, const float view_proj[16],
                         const double tool[6], const uint8_t *shape, int32_t sw, int32_t sh, const float *depth,
                         int32_t dw, int32_t dh, float bias, int32_t mode, double value, void *stream);

/* Range selection, turning quantitative data into a label: every texel of
 * src whose mask bit is set and whose value v (exact in fp64) satisfies
 * lo <= v <= hi gets `label` in the label layer dst (same size); other
 * texels of dst are untouched.  lo > hi selects nothing.
 * Errors: UVL_E_INVAL (pointers, NaN bounds), UVL_E_SHAPE, UVL_E_DTYPE
 * (dst not u8/u16 or label too wide). */
int32_t uvl_numeric_select(const uvl_numeric *src, double lo, double hi, const uvl_layer *dst, uint32_t label,
                           void *stream);

/* Operations between numeric layers (§4.2: numeric layers are for
 * annotating and operating with quantitative information).  Per texel, a
 * result validity r from the operands' mask bits va, vb:
 *   UVL_NUM_AND: va && vb    UVL_NUM_OR: va || vb    UVL_NUM_XOR: va != vb
 *   UVL_NUM_MIN, UVL_NUM_MAX, UVL_NUM_ADD: va && vb;
 * where r holds dst's data become (AND / OR / XOR) a's value if va, else
 * b's; (MIN) a if a <= b, else b; (MAX) a if a >= b, else b; (ADD) a + b
 * rounded once to the dtype (integers exactly, binary32 by its own
 * addition, binary16 from the exact sum), results beyond the dtype's range
 * taking its extreme finite value; where r does not hold dst's data stay
 * and its bit is cleared.  dst's mask bit = r.  All three layers have one
 * dtype and one size; dst may be a or b (the same data and mask planes) or
 * share no plane with them.  A NaN operand (edits never store one) leaves
 * that texel's data unspecified.
 * Errors: UVL_E_INVAL (op, pointers, partial aliasing), UVL_E_DTYPE
 * (dtypes differ), UVL_E_SHAPE (sizes differ). */
typedef enum { UVL_NUM_AND = 0, UVL_NUM_OR = 1, UVL_NUM_XOR = 2, UVL_NUM_MIN = 3, UVL_NUM_MAX = 4,
               UVL_NUM_ADD = 5 } uvl_numeric_opcode;
int32_t uvl_numeric_op(int32_t op, const uvl_numeric *dst, const uvl_numeric *a, const uvl_numeric *b,
                       void *stream);

/* One group of zonal statistics. */
typedef struct {
    uint64_t count;     /* texels counted                                     */
    uint64_t area_w;    /* sum of their area_w (exact); area = area_w * area_scale */
    double wsum;        /* sum of area_w * value in fp64, in an unspecified order */
    double vmin, vmax;  /* extremes of the value (+inf / -inf when count is 0) */
    uint64_t area_w_hi; /* two-word weights: sum of the high words (exact), the
                           area being (area_w_hi * 2^32 + area_w) * area_scale
                           and wsum summing (high * 2^32 + low) * value; else 0 */
} uvl_numstat;

/* Texture padding of a numeric layer after a numeric brush or lasso edit
 * (same arguments as uvl_pad_brush / uvl_pad_lasso, with the edit's mode
 * and value in place of the label): the outline texels the label padding
 * would label are SET or ERASEd instead.  Errors as those calls and the
 * numeric edits. */
int32_t uvl_numeric_pad_brush(const uvl_geom *geom, const uvl_numeric *layer, const int32_t *outline, int64_t n,
                              int32_t k, const float center[3], float radius, int32_t mode, double value,
                              void *stream);
int32_t uvl_numeric_pad_lasso(const uvl_geom *geom, const uvl_numeric *layer, const int32_t *outline, int64_t n,
                              int32_t k, const float view_proj[16], const float *poly_xy, int32_t npoly,
                              const float *depth, int32_t dw, int32_t dh, float bias, int32_t mode, double value,
                              void *stream);

/* Zonal statistics of a numeric layer (Table 1 gives the surface area one
 * texel stands for; weighting values by it gives the area-weighted mean
 * wsum / area_w of a group).  Counted texels: covered (tri_id >= 0) with
 * the mask bit set.  They are grouped by the value of the label layer `region` (u8: 256
 * groups, u16: 65536), or form one group when region is NULL.  bins_dev:
 * device uvl_numstat[groups], 8-byte aligned, overwritten.  If bins_host is
 * non-NULL the call is SYNCHRONOUS and copies the groups there; otherwise
 * it is asynchronous.  wsum is within (count + 1) * 2^-53 * sum |area_w v|
 * of the exact sum.  A NaN value (edits never store one; the caller's own
 * writes can) leaves its group's wsum, vmin and vmax unspecified.
 * Errors: UVL_E_INVAL (pointers, alignment), UVL_E_SHAPE, UVL_E_DTYPE. */
int32_t uvl_numeric_stats(const uvl_geom *geom, const uvl_numeric *layer, const uvl_layer *region,
                          uvl_numstat *bins_dev, uvl_numstat *bins_host, void *stream);

/* ------------------------------------------------------------------------
 * Layer pool (§4.2: the Texture Manager sorts textures into texture arrays
 * by a key joining width, height and data type; sparse textures separate
 * reserving address space from committing memory).  Per key (width,
 * height, dtype) a pool reserves one virtual address range of
 * `slots_per_key` slots, each the layer's size rounded up to the device's
 * allocation granularity: slot k lives at base + k * stride, the key's
 * array.  Allocating a layer commits device memory to the lowest free slot;
 * freeing it unmaps and releases that memory.  Reserved address space costs
 * no memory.  The pool is the one part of the library that allocates device
 * memory; its layers are ordinary device memory for every other call (a
 * numeric layer's mask plane comes from the caller).  Calls on one pool are
 * serialised by a lock; a pool belongs to the device current at creation.
 * ------------------------------------------------------------------------ */
typedef struct uvl_pool uvl_pool;

/* New pool on the current device.  slots_per_key in 1..65536.
 * Errors: UVL_E_INVAL, UVL_E_UNSUPPORTED (not gfx950, or no virtual memory
 * management), UVL_E_DEVICE. */
int32_t uvl_pool_create(int32_t slots_per_key, uvl_pool **out);

/* Commit a layer of width x height values of dtype (uvl_dtype): *data
 * receives its device address (16-byte aligned; contents undefined, clear
 * it with uvl_create_layer or uvl_numeric_create), *slot (may be NULL) its
 * slot in the key's array.  SYNCHRONOUS: the memory is mapped on return.
 * Errors: UVL_E_INVAL, UVL_E_DTYPE, UVL_E_NOMEM (every slot of the key in
 * use, address space or device memory exhausted), UVL_E_DEVICE (also when
 * called with another device current). */
int32_t uvl_pool_alloc(uvl_pool *pool, int32_t width, int32_t height, int32_t dtype, void **data, int32_t *slot);

/* Release a layer from uvl_pool_alloc.  SYNCHRONOUS: waits for all work
 * queued on the pool's device (every stream) before the memory is unmapped,
 * so no queued kernel can still touch it.  Errors: UVL_E_INVAL (not a
 * committed layer of this pool), UVL_E_DEVICE (another device current, or
 * HIP fails; if the unmap itself fails the layer stays committed). */
int32_t uvl_pool_free(uvl_pool *pool, void *data);

/* The array of a key: base address, slot stride in bytes, slot count.
 * Errors: UVL_E_INVAL (null, or the key was never allocated). */
int32_t uvl_pool_array(const uvl_pool *pool, int32_t width, int32_t height, int32_t dtype, void **base,
                       size_t *stride, int32_t *slots);

/* Bytes of address space reserved, bytes of device memory committed, and
 * the number of keys. */
int32_t uvl_pool_stats(const uvl_pool *pool, uint64_t *reserved, uint64_t *committed, int32_t *keys);

/* Release every layer and reservation of the pool, then the pool (waits for
 * the pool's device first, as uvl_pool_free; call it with that device
 * current). */
int32_t uvl_pool_destroy(uvl_pool *pool);

/* ------------------------------------------------------------------------
 * Batched edit waves.  The paper applies one edit per rendering pass
 * (§4.3.1); a wave applies many pending edits -- of many models and layers --
 * with one persistent-kernel launch.  Each edit's selection depends only on
 * the texel's stored position, so the result of a wave is bit-identical to
 * calling uvl_edit_brush / uvl_edit_lasso once per edit in array order.
 * ------------------------------------------------------------------------ */
typedef enum { UVL_EDIT_BRUSH = 0, UVL_EDIT_LASSO = 1, UVL_EDIT_TOOL = 2 } uvl_edit_kind;

/* One edit of a wave.  geom and layer are host pointers to descriptors of
 * device data (as for the single-edit calls); all edits of one layer must
 * name the same geometry image.  Brush: center, radius.  Lasso: view_proj
 * (host float[16]), poly_xy (host float[npoly][2], 3 <= npoly <= 64), depth
 * (device [dh][dw] map rendered with that matrix), bias.  Tool (the paper's
screen-space tool, as uvl_edit_tool): view_proj, depth, dw, dh, bias as for
a lasso, tool (host double[6]), shape (device u8 [sh][sw]); tools count
towards the wave's lasso capacity.  With numeric
 * non-NULL (and layer NULL) the edit SETs or ERASEs that numeric layer
 * (mode, value as for uvl_numeric_brush / uvl_numeric_lasso; label ignored):
 * the result is that of the numeric single-edit calls in array order.
 * Records without numeric edits leave numeric NULL and the rest 0.
 * bins (label edits only; every edit of a layer names the same bins or
 * none): device uint64, 8-byte aligned, the layer's bins in the layout
 * uvl_area_query writes for this one layer (uvl_area_bin_count words).  The
 * wave moves the area of every covered texel whose label it changes from the
 * old label's bin to the new one's, so bins that held the layer's areas
 * before the wave hold them after it (exact integers; bins are unsigned and
 * a decrease wraps, the totals coming out exact).  Texture padding writes
 * uncovered texels only and changes no bin. */
typedef struct {
    const uvl_geom *geom;
    const uvl_layer *layer;
    int32_t kind;           /* uvl_edit_kind */
    uint32_t label;
    float center[3];
    float radius;
    const float *view_proj;
    const float *poly_xy;
    int32_t npoly;
    int32_t dw, dh;
    float bias;
    const float *depth;
    const uvl_numeric *numeric;
    int32_t mode;           /* uvl_value_mode */
    int32_t reserved;       /* 0 */
    double value;
    const double *tool;     /* tool edits: {Ww, Wh, Tpx, Tpy, Tw, Th} */
    const uint8_t *shape;
    int32_t sw, sh;
    uint64_t *bins;         /* label edits, optional (NULL: none): the layer's
                               area bins, see below */
} uvl_edit;

typedef struct uvl_wave uvl_wave;   /* opaque handle */

/* Device workspace bytes for waves of up to max_edits edits, of which up to
 * max_lassos are lassos, with room for max_cull_words tile-culling words (a
 * layer whose geometry image has tile bounds needs ceil(edits / 64) words
 * per 32 x 32 tile of its atlas; layers whose words do not fit run without
 * culling, with identical results).  Each word takes 20 bytes (the live
 * mask, the inside mask and a live-list entry). */
size_t uvl_wave_workspace_bytes(int32_t max_edits, int32_t max_lassos, int64_t max_cull_words);

/* Create a wave handle over a caller-owned device workspace (256-byte
 * aligned, uvl_wave_workspace_bytes bytes, kept alive until destroy).  The
 * handle owns a pinned host staging buffer, a capture stream and the HIP
 * graph of the launch; it allocates no device memory itself.
 * Errors: UVL_E_INVAL, UVL_E_NOMEM (workspace too small), UVL_E_DEVICE. */
int32_t uvl_wave_create(int32_t max_edits, int32_t max_lassos, int64_t max_cull_words, void *ws, size_t ws_bytes,
                        uvl_wave **out);

/* Apply edits[0..n) on `stream`: the descriptor is copied host->device into
 * the workspace, then the captured graph (counter reset, tile culling into
 * per-layer lists of live tiles, item planning, persistent kernel) is
 * replayed.  A tile is skipped when its position bounds prove that no edit
 * selects a texel there: brushes by distance, lassos by the polygon's screen
 * extent and, when the tile's depth-map footprint is at most 1024 pixels,
 * by the depth test (every texel behind the stored depth plus bias).  tile_chunks in 1..8 forces tiles of tile_chunks*1024 texels;
 * 0 uses the tuned size of each layer's atlas size (4 if not tuned).  Edits
 * of different layers are independent; edits of one layer apply in order.
 * The edits array may be freed on return.  Submits on one handle are
 * serialised and must go to one stream (the device descriptor is reused in
 * stream order); up to 4 submits may be in flight before a submit waits for
 * the oldest one's descriptor copy.
 * Errors: as the single-edit calls, plus UVL_E_NOMEM if n exceeds the
 * handle's capacity. */
int32_t uvl_wave_submit(uvl_wave *w, const uvl_edit *edits, int32_t n, int32_t tile_chunks, void *stream);

/* Texture padding in a wave (§4.3.2).  One entry per geometry image to pad
 * around: its outline list from uvl_build_outline (n texel indices) and the
 * padding radius k (0..8). */
typedef struct {
    const uvl_geom *geom;
    const int32_t *outline;
    int64_t n;
    int32_t k;
    int32_t reserved;       /* 0 */
} uvl_wave_outline;

/* uvl_wave_submit, then padding: every layer whose edits read a geometry
 * image listed in outlines[0..noutlines) is padded after its edits, with the
 * result of padding after each edit in order (uvl_pad_brush / uvl_pad_lasso
 * and their numeric forms; a tool edit pads by the same rule with the tool's
 * predicate).  Padding writes uncovered texels only and edits covered ones,
 * so the padding of all of a layer's edits can follow them: an outline
 * texel takes the label (or the numeric decisions) of the last edit that
 * selects a covered texel of its (2k+1)^2 window.  Edits a tile test has
 * culled around the window are skipped.
 * Errors: as uvl_wave_submit, plus UVL_E_INVAL for a bad outline entry. */
int32_t uvl_wave_submit_padded(uvl_wave *w, const uvl_edit *edits, int32_t n, int32_t tile_chunks,
                               const uvl_wave_outline *outlines, int32_t noutlines, void *stream);

/* Autotune the tile size per atlas size class (power of two of the texel
 * count) present in edits: each of 1, 2, 4, 8 chunks is timed on the class's
 * edits (applying a wave again leaves the layers unchanged, so the layers
 * end as after one submit).  SYNCHRONOUS. */
int32_t uvl_wave_tune(uvl_wave *w, const uvl_edit *edits, int32_t n, void *stream);

/* The tuned tile size (chunks of 1024 texels) for an atlas of `texels`
 * texels, 0 if that size class is not tuned. */
int32_t uvl_wave_tuned_chunks(const uvl_wave *w, int64_t texels);

/* Tiles the last submit on this handle visited (the live tiles of layers
 * with culling plus every tile of layers without), written to *tiles.
 * SYNCHRONOUS on `stream`, which must be the stream of that submit.
 * Errors: UVL_E_INVAL, UVL_E_DEVICE. */
int32_t uvl_wave_visited_tiles(uvl_wave *w, int64_t *tiles, void *stream);

/* Release the handle (waits for its last descriptor copy). */
int32_t uvl_wave_destroy(uvl_wave *w);

#ifdef __cplusplus
}
#endif

#endif /* UVL_H */
