// The texture-space geometry image (§4.3.1 renders the mesh with its
// texture coordinates as vertex positions; §4.1, texture coordinates index
// the layers): per texel centre the owning triangle (raster_rule.h; the
// lowest triangle index wins where triangles overlap), barycentrics,
// position, normal and the surface area the texel stands for (Table 1),
// built once per model so that edits read per-texel surface data.
//
// Tile-binned on gfx950, so that every plane is written once, coalesced:
//   1. k_setup, a thread per triangle: snapped coordinates, exact edge
//      functions in the original vertex order, doubled area |E| and texel
//      weight 131072 A3 / |E| into a 64-byte record; the cell bounding box;
//      a triangle whose box spans at most 4 tiles of 32 x 32 texels takes a
//      slot in each of their lists (one atomic add per tile), a larger one
//      goes to a queue;
//   2. an exclusive scan of the per-tile counts (three small kernels), then
//      k_bin writes every triangle index into its tiles' lists (no atomics:
//      the slots came from step 1);
//   3. queued (large) triangles: their tiles are marked and their texels set
//      to "no owner" in the tri_id plane, then a workgroup per triangle
//      rasterises it with atomicMin into that plane;
//   4. k_tile, a 256-thread workgroup per tile: its triangles' records,
//      vertex positions and normals staged in LDS (a small hash maps a
//      triangle index to its record), ownership resolved with LDS
//      atomicMin, starting from the plane for marked tiles; then every
//      texel's attributes from its owner's record (fp64, in the order the
//      definition gives), the area weight quantised, and the tile's
//      position bounds, all written once.
// The area scale comes from the largest weight among the triangles whose
// box holds a texel centre (found in step 1), so the tile pass can quantise
// at once; it also finds the smallest owner weight for the range check.
#include <math.h>

#include "raster_rule.h"
#include "uvl_internal.h"

namespace uvl {
namespace {

constexpr int kTile = UVL_TILE_SIDE;            // 32
constexpr int kTileTexels = kTile * kTile;      // 1024
constexpr int kTileThreads = 256;               // 4 texels per thread
constexpr int kTileRecs = 128;                  // records staged in LDS per tile
constexpr int kCoopCells = 96;                  // more cells in a tile: rasterised by the whole workgroup
constexpr int kMaxCoop = 64;
constexpr int kMaxSpan = 4;                     // tiles a binned triangle may span
constexpr int kBigGrid = 2048;
constexpr int kScanThreads = 1024, kScanPer = 8, kScanSpan = kScanThreads * kScanPer;
constexpr int32_t kNoOwner = 0x7fffffff;
constexpr int kHashBits = 8, kHashSlots = 1 << kHashBits;   // staged records by triangle index

// Largest ratio of texel weights for which one rounding onto the scale's
// grid stays within 2^-20 relative: one word (largest weight in [2^30,
// 2^31)) and two words (in [2^62, 2^63)).
constexpr int kNarrowRatioLog2 = 11, kWideRatioLog2 = 43;

struct GCounters {
    unsigned int big_len;            // queued large triangles
    unsigned int flags;              // bit 0: vertex index out of range, bit 1: uv out of range
    unsigned int pad0, pad1;
    unsigned long long max_w_bits;   // largest weight of a triangle whose box holds a texel centre
    unsigned long long min_w_bits;   // smallest owner weight two words hold to 2^-20
};

constexpr unsigned kFlagIndex = 1u, kFlagUV = 2u;

// A triangle's set-up: edge v (opposite original vertex v) is
// e_v = A[v] px + B[v] py + C[v] in 1/256-texel units.  E = 0: covers nothing.
struct alignas(16) TriRec {
    long long C[3];
    long long E;
    double w;
    int A[3], B[3];
};
static_assert(sizeof(TriRec) == 64, "one 64-byte record per triangle");

// The staged records of a tile, one array per field: lanes reading
// consecutive records touch consecutive banks (an array of 160-byte records
// put every 4th lane on one bank).
struct TileRecs {
    long long C[3][kTileRecs];
    long long E[kTileRecs];
    double w[kTileRecs];                // texel weight
    double rE[kTileRecs];               // 1 / |E|, correctly rounded
    unsigned long long q[kTileRecs];    // the quantised texel weight (one or two words)
    int A[3][kTileRecs], B[3][kTileRecs];
    float P[9][kTileRecs];              // vertex positions, original order
    float N[9][kTileRecs];              // vertex normals (when the mesh has them)

    __device__ __forceinline__ TriRec rec(int k) const {
        TriRec R;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            R.C[v] = C[v][k];
            R.A[v] = A[v][k];
            R.B[v] = B[v][k];
        }
        R.E = E[k];
        R.w = w[k];
        return R;
    }
};

// The quantised texel weight of a triangle: the largest weight of the
// image maps into [2^30, 2^31) (one word) or [2^62, 2^63) (two words).
__device__ __forceinline__ unsigned long long quantise(double w, int ex, bool wide) {
    return wide ? (unsigned long long)rint(ldexp(w, 63 - ex)) : (unsigned long long)rint(ldexp(w, 31 - ex));
}

// b = e / E correctly rounded from r = RN(1 / E): q0 = RN(e r) is within an
// ulp of e / E, the remainder e - E q0 is exact (one fma), and q0 + rem r
// rounded once is the correctly rounded quotient (Markstein's theorem; e
// and E are integers below 2^53, far from overflow and underflow).
__device__ __forceinline__ double div_by(double e, double E, double r) {
    const double q0 = e * r;
    const double rem = fma(-q0, E, e);
    return fma(rem, r, q0);
}

struct GeomArgs {
    const float *uv, *pos, *nrm;
    const int32_t *tri;
    int64_t nv, nt;
    int W, H, tiles_x, tiles_y;
    TriRec *recs;
    int4 *boxes;         // {i0, i1, j0, j1}; empty when i1 < i0
    int4 *slots;         // a binned triangle's slot in each of its tiles' lists
    int32_t *list;
    unsigned *big;
    unsigned *tcount, *toff, *tflag, *blk;
    GCounters *ctr;
};

struct GeomOut {
    int32_t *tri_id;
    float *px, *py, *pz, *nx, *ny, *nz, *b1, *b2;
    uint32_t *aw, *aw_hi;
    float *box;
    unsigned long long *blk;   // per 4 x 8 block area sums (one-word weights), or null
};

__device__ __forceinline__ bool geom_tri(const GeomArgs &a, int64_t t, Tri2 &T, int v[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[k] = a.tri[3 * t + k];
        if (v[k] < 0 || v[k] >= a.nv) {
            atomicOr(&a.ctr->flags, kFlagIndex);
            return false;
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float u = a.uv[2 * (int64_t)v[k]], w = a.uv[2 * (int64_t)v[k] + 1];
        if (!(fabsf(u) <= 4.0f) || !(fabsf(w) <= 4.0f)) {
            atomicOr(&a.ctr->flags, kFlagUV);
            return false;
        }
        T.X[k] = snap256((double)u * (double)a.W);
        T.Y[k] = snap256((double)w * (double)a.H);
    }
    return tri_setup(T);
}

// Slots in the tiles' lists for one entry per lane (tile < 0: none): the
// lanes asking for one tile get consecutive slots from a single atomic add
// by the first of them, since neighbouring triangles share tiles and one
// counter hit by a whole wave would serialise.  All lanes take part.
__device__ __forceinline__ int wave_slot(unsigned *__restrict__ count, int tile) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    bool pend = tile >= 0;
    int slot = -1;
    for (;;) {
        const unsigned long long m = __builtin_amdgcn_ballot_w64(pend);
        if (m == 0) break;
        const int leader = __builtin_ctzll(m);
        const int lt = __shfl(tile, leader);
        const bool same = pend && tile == lt;
        const unsigned long long group = __builtin_amdgcn_ballot_w64(same);
        unsigned base = 0;
        if (lane == leader) base = atomicAdd(count + lt, (unsigned)__builtin_popcountll(group));
        base = __shfl(base, leader);
        if (same) {
            slot = (int)(base + (unsigned)__builtin_popcountll(group & below));
            pend = false;
        }
    }
    return slot;
}

// 1. set-up, binning counts, queue of large triangles, largest weight
__global__ __launch_bounds__(kBlock) void k_setup(GeomArgs a) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double wmax = 0.0;
    int tiles[kMaxSpan] = {-1, -1, -1, -1};
    if (t < a.nt) {
        Tri2 T;
        int v[3];
        TriRec R{};
        int4 box = make_int4(0, -1, 0, -1);
        if (geom_tri(a, t, T, v)) {
            // texel area weight 131072 A3 / |E| (surface area per 1/(W H) of UV area)
            double P[3][3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) P[k][c] = (double)a.pos[3 * (int64_t)v[k] + c];
            double u1[3], u2[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) { u1[c] = P[1][c] - P[0][c]; u2[c] = P[2][c] - P[0][c]; }
            const double f0 = u1[1] * u2[2] - u1[2] * u2[1];
            const double f1 = u1[2] * u2[0] - u1[0] * u2[2];
            const double f2 = u1[0] * u2[1] - u1[1] * u2[0];
            const double flen = sqrt(f0 * f0 + f1 * f1 + f2 * f2);
            R.w = 131072.0 * (0.5 * flen) / (double)T.E;
            R.E = T.E;
            // edge k of the counter-clockwise order is opposite vertex
            // ord[k]: ord = (0, 1, 2) when E > 0, else (0, 2, 1)
            const bool ccw = T.ord[1] == 1;
            R.A[0] = (int)T.A[0];
            R.B[0] = (int)T.B[0];
            R.C[0] = T.C[0];
            R.A[1] = (int)(ccw ? T.A[1] : T.A[2]);
            R.B[1] = (int)(ccw ? T.B[1] : T.B[2]);
            R.C[1] = ccw ? T.C[1] : T.C[2];
            R.A[2] = (int)(ccw ? T.A[2] : T.A[1]);
            R.B[2] = (int)(ccw ? T.B[2] : T.B[1]);
            R.C[2] = ccw ? T.C[2] : T.C[1];
            int i0, i1, j0, j1;
            bbox(T, a.W, a.H, i0, i1, j0, j1);
            if (i0 <= i1 && j0 <= j1) {
                box = make_int4(i0, i1, j0, j1);
                wmax = R.w;
                const int tx0 = i0 / kTile, ty0 = j0 / kTile;
                const int wx = i1 / kTile - tx0 + 1, span = wx * (j1 / kTile - ty0 + 1);
                if (span <= kMaxSpan) {
#pragma unroll
                    for (int k = 0; k < kMaxSpan; ++k)
                        if (k < span) tiles[k] = (ty0 + k / wx) * a.tiles_x + tx0 + k % wx;
                } else {
                    a.big[atomicAdd(&a.ctr->big_len, 1u)] = (unsigned)t;
                }
            }
        }
        a.recs[t] = R;
        a.boxes[t] = box;
    }
    int s[kMaxSpan];
#pragma unroll
    for (int k = 0; k < kMaxSpan; ++k) s[k] = wave_slot(a.tcount, tiles[k]);
    if (t < a.nt) a.slots[t] = make_int4(s[0], s[1], s[2], s[3]);
    // one atomic per workgroup at most: the counter only grows, so a value
    // read is a lower bound of the final one
    __shared__ double s_w[kBlock / 64];
    wmax = wave_max(wmax);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = wmax;
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 1; k < kBlock / 64; ++k) wmax = fmax(wmax, s_w[k]);
        const unsigned long long b = (unsigned long long)__double_as_longlong(wmax);
        if (wmax > 0.0 && b > __atomic_load_n(&a.ctr->max_w_bits, __ATOMIC_RELAXED)) atomicMax(&a.ctr->max_w_bits, b);
    }
}

// Exclusive prefix of x over a workgroup of kScanThreads; *total = the sum.
__device__ __forceinline__ unsigned block_exscan(unsigned x, unsigned *s_wave, unsigned &total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int kWaves = kScanThreads / 64;
    unsigned inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_wave[wv] = inc;
    __syncthreads();
    if (wv == 0) {
        const unsigned v = lane < kWaves ? s_wave[lane] : 0u;
        unsigned vi = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned y = __shfl_up(vi, o);
            if (lane >= o) vi += y;
        }
        if (lane < kWaves) s_wave[lane] = vi - v;
        if (lane == kWaves - 1) s_wave[kWaves] = vi;
    }
    __syncthreads();
    total = s_wave[kWaves];
    const unsigned r = inc - x + s_wave[wv];
    __syncthreads();
    return r;
}

// 2a. per scan block: the sum of its kScanSpan counts
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const unsigned *__restrict__ cnt, int64_t n,
                                                              unsigned *__restrict__ blk) {
    __shared__ unsigned s_wave[kScanThreads / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanSpan + (int64_t)threadIdx.x * kScanPer;
    unsigned x = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < n) x += cnt[base + k];
    unsigned total;
    block_exscan(x, s_wave, total);
    if (threadIdx.x == 0) blk[blockIdx.x] = total;
}

// 2b. exclusive prefix of the block sums (at most kScanThreads blocks)
__global__ __launch_bounds__(kScanThreads) void k_scan_top(unsigned *__restrict__ blk, int nblk) {
    __shared__ unsigned s_wave[kScanThreads / 64 + 1];
    const unsigned x = (int)threadIdx.x < nblk ? blk[threadIdx.x] : 0u;
    unsigned total;
    const unsigned r = block_exscan(x, s_wave, total);
    if ((int)threadIdx.x < nblk) blk[threadIdx.x] = r;
}

// 2c. every tile's list offset
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const unsigned *__restrict__ cnt, int64_t n,
                                                            const unsigned *__restrict__ blk,
                                                            unsigned *__restrict__ off) {
    __shared__ unsigned s_wave[kScanThreads / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanSpan + (int64_t)threadIdx.x * kScanPer;
    unsigned c[kScanPer], x = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        c[k] = base + k < n ? cnt[base + k] : 0u;
        x += c[k];
    }
    unsigned total;
    unsigned run = block_exscan(x, s_wave, total) + blk[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) off[base + k] = run;
        run += c[k];
    }
}

// 2d. list entries at the slots taken in k_setup
__global__ __launch_bounds__(kBlock) void k_bin(GeomArgs a) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= a.nt) return;
    const int4 sl = a.slots[t];
    if (sl.x < 0) return;
    const int4 b = a.boxes[t];
    const int s[kMaxSpan] = {sl.x, sl.y, sl.z, sl.w};
    const int tx0 = b.x / kTile, ty0 = b.z / kTile, wx = b.y / kTile - tx0 + 1;
#pragma unroll
    for (int k = 0; k < kMaxSpan; ++k)
        if (s[k] >= 0) a.list[a.toff[(int64_t)(ty0 + k / wx) * a.tiles_x + tx0 + k % wx] + s[k]] = (int32_t)t;
}

// 3a. large triangles: mark their tiles and clear those tiles' owners
__global__ __launch_bounds__(kBlock) void k_big_fill(GeomArgs a, int32_t *__restrict__ owner) {
    const unsigned n = a.ctr->big_len;
    for (unsigned q = blockIdx.x; q < n; q += gridDim.x) {
        const int4 b = a.boxes[a.big[q]];
        for (int ty = b.z / kTile; ty <= b.w / kTile; ++ty)
            for (int tx = b.x / kTile; tx <= b.y / kTile; ++tx) {
                if (threadIdx.x == 0) a.tflag[(int64_t)ty * a.tiles_x + tx] = 1u;
                for (int c = threadIdx.x; c < kTileTexels; c += kBlock) {
                    const int i = tx * kTile + (c % kTile), j = ty * kTile + (c / kTile);
                    if (i < a.W && j < a.H) owner[(int64_t)j * a.W + i] = kNoOwner;
                }
            }
    }
}

__device__ __forceinline__ bool inside(const TriRec &R, long long px, long long py) {
    bool in = true;
#pragma unroll
    for (int v = 0; v < 3; ++v)
        in &= (long long)R.A[v] * px + (long long)R.B[v] * py + R.C[v] >= edge_bias(R.A[v], R.B[v]);
    return in;
}

// 3b. large triangles: a workgroup per triangle, atomicMin into the plane
__global__ __launch_bounds__(kBlock) void k_big_raster(GeomArgs a, int32_t *__restrict__ owner) {
    const unsigned n = a.ctr->big_len;
    for (unsigned q = blockIdx.x; q < n; q += gridDim.x) {
        const unsigned t = a.big[q];
        const TriRec R = a.recs[t];
        const int4 b = a.boxes[t];
        const unsigned bw = (unsigned)(b.y - b.x + 1);
        const unsigned cells = bw * (unsigned)(b.w - b.z + 1);
        for (unsigned c = threadIdx.x; c < cells; c += kBlock) {
            const int i = b.x + (int)(c % bw), j = b.z + (int)(c / bw);
            if (inside(R, 256LL * i + 128, 256LL * j + 128)) atomicMin(owner + (int64_t)j * a.W + i, (int32_t)t);
        }
    }
}

// Owner candidates of one triangle over cells [bi0, bi1] x [bj0, bj1] of
// the tile at (ti0, tj0), by one thread: incremental edge functions.
__device__ __forceinline__ void raster_cells(const TriRec &R, int bi0, int bi1, int bj0, int bj1, int ti0, int tj0,
                                             int32_t key, int32_t *own) {
    const long long px0 = 256LL * bi0 + 128;
    long long s[3], bs[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        s[v] = 256LL * R.A[v];
        bs[v] = edge_bias(R.A[v], R.B[v]);
    }
    for (int j = bj0; j <= bj1; ++j) {
        const long long py = 256LL * j + 128;
        long long e[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) e[v] = (long long)R.A[v] * px0 + (long long)R.B[v] * py + R.C[v] - bs[v];
        int32_t *row = own + (j - tj0) * kTile - ti0;
        for (int i = bi0; i <= bi1; ++i) {
            if ((e[0] | e[1] | e[2]) >= 0) atomicMin(row + i, key);
#pragma unroll
            for (int v = 0; v < 3; ++v) e[v] += s[v];
        }
    }
}

__device__ __forceinline__ float wave_minf(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fminf(x, __shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ float wave_maxf(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o));
    return x;
}

// 4. a workgroup per tile: ownership in LDS, then attributes written once
__global__ __launch_bounds__(kTileThreads) void k_tile(GeomArgs a, GeomOut g) {
    __shared__ int32_t s_own[kTileTexels];
    __shared__ TileRecs s_rec;
    __shared__ int32_t s_hkey[kHashSlots];
    __shared__ int32_t s_hval[kHashSlots];
    __shared__ int s_coop[kMaxCoop];
    __shared__ int s_ncoop;
    __shared__ float s_red[7][kTileThreads / 64];
    // area sums of the tile's 8 x 4 blocks of 4 rows x 8 columns (one-word weights)
    constexpr int kBlkRows = kTile / UVL_AREA_BLK_ROWS, kBlkCols = kTile / UVL_AREA_BLK_COLS;
    __shared__ unsigned long long s_blk[kBlkRows * kBlkCols];
    const int64_t tile = blockIdx.x;
    const int tx = (int)(tile % a.tiles_x), ty = (int)(tile / a.tiles_x);
    const int ti0 = tx * kTile, tj0 = ty * kTile;
    const int W = a.W, H = a.H;
    const unsigned cnt = a.tcount[tile], off = a.toff[tile];
    const bool marked = a.tflag[tile] != 0u;
    for (int c = threadIdx.x; c < kTileTexels; c += kTileThreads) {
        const int i = ti0 + (c % kTile), j = tj0 + (c / kTile);
        s_own[c] = marked && i < W && j < H ? g.tri_id[(int64_t)j * W + i] : kNoOwner;
    }
    for (int h = threadIdx.x; h < kHashSlots; h += kTileThreads) s_hkey[h] = -1;
    if (threadIdx.x < kBlkRows * kBlkCols) s_blk[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) s_ncoop = 0;
    __syncthreads();
    int ex;
    const double mx = __longlong_as_double((long long)a.ctr->max_w_bits);
    frexp(mx, &ex);
    const bool wide = g.aw_hi != nullptr;
    const int nstage = cnt < (unsigned)kTileRecs ? (int)cnt : kTileRecs;
    for (int k = threadIdx.x; k < nstage; k += kTileThreads) {
        const int32_t t = a.list[off + k];
        const TriRec R = a.recs[t];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            s_rec.C[v][k] = R.C[v];
            s_rec.A[v][k] = R.A[v];
            s_rec.B[v][k] = R.B[v];
        }
        s_rec.E[k] = R.E;
        s_rec.w[k] = R.w;
        s_rec.rE[k] = 1.0 / (double)R.E;
        s_rec.q[k] = quantise(R.w, ex, wide);
        // triangle index -> LDS slot (open addressing; a triangle is listed once)
        for (uint32_t h = ((uint32_t)t * 2654435761u) >> (32 - kHashBits);; h = (h + 1) & (kHashSlots - 1))
            if (atomicCAS(&s_hkey[h], -1, t) == -1) {
                s_hval[h] = k;
                break;
            }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int64_t v = a.tri[3 * (int64_t)t + q];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                s_rec.P[3 * q + c][k] = a.pos[3 * v + c];
                s_rec.N[3 * q + c][k] = a.nrm ? a.nrm[3 * v + c] : 0.0f;
            }
        }
    }
    __syncthreads();
    // ownership: a thread per triangle; triangles with many cells in this
    // tile are left to the whole workgroup
    for (int k = threadIdx.x; k < (int)cnt; k += kTileThreads) {
        const int32_t t = a.list[off + k];
        const TriRec R = k < kTileRecs ? s_rec.rec(k) : a.recs[t];
        const int4 b = a.boxes[t];
        const int bi0 = max(b.x, ti0), bi1 = min(b.y, ti0 + kTile - 1);
        const int bj0 = max(b.z, tj0), bj1 = min(b.w, tj0 + kTile - 1);
        if (bi0 > bi1 || bj0 > bj1) continue;
        if ((bi1 - bi0 + 1) * (bj1 - bj0 + 1) > kCoopCells) {
            const int s = atomicAdd(&s_ncoop, 1);
            if (s < kMaxCoop) {
                s_coop[s] = k;
                continue;
            }
        }
        raster_cells(R, bi0, bi1, bj0, bj1, ti0, tj0, t, s_own);
    }
    __syncthreads();
    const int ncoop = s_ncoop < kMaxCoop ? s_ncoop : kMaxCoop;
    for (int q = 0; q < ncoop; ++q) {
        const int k = s_coop[q];
        const int32_t t = a.list[off + k];
        const TriRec R = k < kTileRecs ? s_rec.rec(k) : a.recs[t];
        const int4 b = a.boxes[t];
        const int bi0 = max(b.x, ti0), bi1 = min(b.y, ti0 + kTile - 1);
        const int bj0 = max(b.z, tj0), bj1 = min(b.w, tj0 + kTile - 1);
        const int bw = bi1 - bi0 + 1, cells = bw * (bj1 - bj0 + 1);
        for (int c = threadIdx.x; c < cells; c += kTileThreads) {
            const int i = bi0 + c % bw, j = bj0 + c / bw;
            if (inside(R, 256LL * i + 128, 256LL * j + 128)) atomicMin(&s_own[(j - tj0) * kTile + (i - ti0)], t);
        }
    }
    __syncthreads();
    // attributes, every plane written once per texel
    const double wfloor = ldexp(mx, -kWideRatioLog2);
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mxp[3] = {-INFINITY, -INFINITY, -INFINITY};
    double wmin = INFINITY;
    const float nan = __builtin_nanf("");
    for (int c = threadIdx.x; c < kTileTexels; c += kTileThreads) {
        const int i = ti0 + (c % kTile), j = tj0 + (c / kTile);
        if (i >= W || j >= H) continue;
        const int64_t idx = (int64_t)j * W + i;
        const int32_t t = s_own[c];
        if (t == kNoOwner) {
            g.tri_id[idx] = -1;
            g.px[idx] = g.py[idx] = g.pz[idx] = nan;
            if (g.nx) g.nx[idx] = g.ny[idx] = g.nz[idx] = 0.0f;
            if (g.b1) g.b1[idx] = g.b2[idx] = 0.0f;
            g.aw[idx] = 0u;
            if (g.aw_hi) g.aw_hi[idx] = 0u;
            continue;
        }
        unsigned slot = 0xffffffffu;          // the owner's LDS record, if staged
        for (uint32_t h = ((uint32_t)t * 2654435761u) >> (32 - kHashBits);; h = (h + 1) & (kHashSlots - 1)) {
            const int32_t key = s_hkey[h];
            if (key == t) {
                slot = (unsigned)s_hval[h];
                break;
            }
            if (key == -1) break;
        }
        TriRec R;
        float P[9], N[9];
        double rE;
        unsigned long long qw;
        if (slot < (unsigned)kTileRecs) {
            R = s_rec.rec(slot);
            rE = s_rec.rE[slot];
            qw = s_rec.q[slot];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                P[q] = s_rec.P[q][slot];
                N[q] = s_rec.N[q][slot];
            }
        } else {
            R = a.recs[t];
            rE = 1.0 / (double)R.E;
            qw = quantise(R.w, ex, wide);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int64_t v = a.tri[3 * (int64_t)t + q];
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    P[3 * q + cc] = a.pos[3 * v + cc];
                    N[3 * q + cc] = a.nrm ? a.nrm[3 * v + cc] : 0.0f;
                }
            }
        }
        const long long px = 256LL * i + 128, py = 256LL * j + 128;
        const double E = (double)R.E;
        double b[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) b[v] = div_by((double)((long long)R.A[v] * px + (long long)R.B[v] * py + R.C[v]), E, rE);
        g.tri_id[idx] = t;
        if (g.b1) {
            g.b1[idx] = (float)b[1];
            g.b2[idx] = (float)b[2];
        }
        float pf[3];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
            pf[cc] = (float)(b[0] * (double)P[cc] + b[1] * (double)P[3 + cc] + b[2] * (double)P[6 + cc]);
        g.px[idx] = pf[0];
        g.py[idx] = pf[1];
        g.pz[idx] = pf[2];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            mn[cc] = fminf(mn[cc], pf[cc]);
            mxp[cc] = fmaxf(mxp[cc], pf[cc]);
        }
        if (g.nx) {
            double m[3];
            if (a.nrm) {
#pragma unroll
                for (int cc = 0; cc < 3; ++cc)
                    m[cc] = b[0] * (double)N[cc] + b[1] * (double)N[3 + cc] + b[2] * (double)N[6 + cc];
            } else {
                double u1[3], u2[3];
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    u1[cc] = (double)P[3 + cc] - (double)P[cc];
                    u2[cc] = (double)P[6 + cc] - (double)P[cc];
                }
                m[0] = u1[1] * u2[2] - u1[2] * u2[1];
                m[1] = u1[2] * u2[0] - u1[0] * u2[2];
                m[2] = u1[0] * u2[1] - u1[1] * u2[0];
            }
            const double len2 = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
            double inv;
            if (len2 >= 1e-30 && len2 <= 1e30) {
                // 1 / sqrt(len2): the hardware fp32 estimate (about 1 ulp)
                // and one Newton step in fp64 (relative error ~1e-14; the
                // normal is not part of the bit-exact contract)
                const double y = (double)__builtin_amdgcn_rsqf((float)len2);
                inv = y * (1.5 - 0.5 * len2 * y * y);
            } else {
                const double len = sqrt(len2);
                inv = len > 0.0 ? 1.0 / len : 0.0;
            }
            g.nx[idx] = (float)(m[0] * inv);
            g.ny[idx] = (float)(m[1] * inv);
            g.nz[idx] = (float)(m[2] * inv);
        }
        g.aw[idx] = (uint32_t)qw;
        if (wide) g.aw_hi[idx] = (uint32_t)(qw >> 32);
        if (g.blk && qw)
            atomicAdd(&s_blk[((c / kTile) / UVL_AREA_BLK_ROWS) * kBlkCols + (c % kTile) / UVL_AREA_BLK_COLS],
                      (unsigned long long)(uint32_t)qw);
        if (R.w >= wfloor) wmin = fmin(wmin, R.w);
    }
    // the tile's position bounds and the smallest owner weight
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
        mn[cc] = wave_minf(mn[cc]);
        mxp[cc] = wave_maxf(mxp[cc]);
    }
    wmin = wave_min(wmin);
    __shared__ double s_wmin[kTileThreads / 64];
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            s_red[cc][wv] = mn[cc];
            s_red[3 + cc][wv] = mxp[cc];
        }
        s_wmin[wv] = wmin;
    }
    __syncthreads();
    if (g.blk && threadIdx.x < kBlkRows * kBlkCols) {
        const int bi = ti0 / UVL_AREA_BLK_COLS + (int)threadIdx.x % kBlkCols;
        const int bj = tj0 / UVL_AREA_BLK_ROWS + (int)threadIdx.x / kBlkCols;
        const int bw = (W + UVL_AREA_BLK_COLS - 1) / UVL_AREA_BLK_COLS, bh = (H + UVL_AREA_BLK_ROWS - 1) / UVL_AREA_BLK_ROWS;
        if (bi < bw && bj < bh) g.blk[(int64_t)bj * bw + bi] = s_blk[threadIdx.x];
    }
    if (threadIdx.x < 6 && g.box) {
        const int cc = threadIdx.x;
        float r = s_red[cc][0];
        for (int w = 1; w < kTileThreads / 64; ++w) r = cc < 3 ? fminf(r, s_red[cc][w]) : fmaxf(r, s_red[cc][w]);
        g.box[6 * tile + cc] = r;
    }
    if (threadIdx.x == 0) {
        double m = s_wmin[0];
        for (int w = 1; w < kTileThreads / 64; ++w) m = fmin(m, s_wmin[w]);
        const unsigned long long bits = (unsigned long long)__double_as_longlong(m);
        if (m < INFINITY && bits < __atomic_load_n(&a.ctr->min_w_bits, __ATOMIC_RELAXED))
            atomicMin(&a.ctr->min_w_bits, bits);
    }
}

// 5. the bounds of each block of 8 x 8 tiles (the union of its tiles'),
// after the tile bounds: one wave per block.
__global__ __launch_bounds__(kBlock) void k_block_box(float *__restrict__ box, int tiles_x, int tiles_y) {
    const int nbx = (tiles_x + UVL_TILE_BLOCK - 1) / UVL_TILE_BLOCK;
    const int nby = (tiles_y + UVL_TILE_BLOCK - 1) / UVL_TILE_BLOCK;
    const int64_t nb = (int64_t)nbx * nby, ntiles = (int64_t)tiles_x * tiles_y;
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (b >= nb) return;   // whole waves
    const int tx = (int)(b % nbx) * UVL_TILE_BLOCK + (lane % UVL_TILE_BLOCK);
    const int ty = (int)(b / nbx) * UVL_TILE_BLOCK + (lane / UVL_TILE_BLOCK);
    const bool in = tx < tiles_x && ty < tiles_y;
    float v[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) v[q] = in ? box[6 * ((int64_t)ty * tiles_x + tx) + q] : (q < 3 ? INFINITY : -INFINITY);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        v[q] = wave_minf(v[q]);
        v[q + 3] = wave_maxf(v[q + 3]);
    }
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (lane == q) box[6 * (ntiles + b) + q] = v[q];
}

__global__ void k_geom_counters(GCounters *ctr) {
    if (threadIdx.x == 0) {
        ctr->big_len = 0;
        ctr->flags = 0;
        ctr->pad0 = ctr->pad1 = 0;
        ctr->max_w_bits = 0;
        ctr->min_w_bits = ~0ull;
    }
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace regions for nt triangles and ntiles tiles.
struct GeomLayout {
    size_t recs, boxes, slots, list, big, tcount, toff, tflag, blk, total;
};

GeomLayout geom_layout(int64_t nt, int64_t ntiles) {
    GeomLayout L;
    const size_t n = (size_t)(nt > 0 ? nt : 0), nb = (size_t)ceil_div(ntiles, kScanSpan);
    L.recs = 256;
    L.boxes = L.recs + a256(n * sizeof(TriRec));
    L.slots = L.boxes + a256(n * sizeof(int4));
    L.list = L.slots + a256(n * sizeof(int4));
    L.big = L.list + a256(n * kMaxSpan * sizeof(int32_t));
    L.tcount = L.big + a256(n * sizeof(unsigned));
    L.toff = L.tcount + a256((size_t)ntiles * sizeof(unsigned));
    L.tflag = L.toff + a256((size_t)ntiles * sizeof(unsigned));
    L.blk = L.tflag + a256((size_t)ntiles * sizeof(unsigned));
    L.total = L.blk + a256((nb + 1) * sizeof(unsigned));
    return L;
}

}  // namespace
}  // namespace uvl

using namespace uvl;

extern "C" size_t uvl_geom_bytes(int32_t width, int32_t height, uint32_t flags) {
    if (width < 1 || height < 1 || width > kMaxSide || height > kMaxSide) return 0;
    if (flags & ~(uint32_t)(UVL_GEOM_NRM | UVL_GEOM_BARY | UVL_GEOM_TILE_BOX | UVL_GEOM_AREA_HI | UVL_GEOM_AREA_BLK))
        return 0;
    const size_t n = (size_t)width * height;
    const size_t plane = a256(n * 4);        // every plane holds 4-byte elements
    size_t planes = 5;                        // tri_id, pos x/y/z, area_w
    if (flags & UVL_GEOM_NRM) planes += 3;
    if (flags & UVL_GEOM_BARY) planes += 2;
    if (flags & UVL_GEOM_AREA_HI) planes += 1;
    size_t bytes = planes * plane;
    if (flags & UVL_GEOM_TILE_BOX) {
        const int64_t tx = ceil_div(width, UVL_TILE_SIDE), ty = ceil_div(height, UVL_TILE_SIDE);
        const int64_t nb = ceil_div(tx, UVL_TILE_BLOCK) * ceil_div(ty, UVL_TILE_BLOCK);
        bytes += a256((size_t)(tx * ty + nb) * 6 * sizeof(float));
    }
    if (flags & UVL_GEOM_AREA_BLK)
        bytes += a256((size_t)ceil_div(width, UVL_AREA_BLK_COLS) * ceil_div(height, UVL_AREA_BLK_ROWS) * 8);
    return bytes;
}

extern "C" size_t uvl_build_workspace_bytes(int64_t nt, int32_t width, int32_t height) {
    if (nt < 0 || width < 1 || height < 1 || width > kMaxSide || height > kMaxSide) return 0;
    const int64_t ntiles = ceil_div(width, kTile) * ceil_div(height, kTile);
    return geom_layout(nt, ntiles).total;
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
    if (reinterpret_cast<uintptr_t>(g->area_blk) & 7) return UVL_E_INVAL;
    if (ws_bytes < uvl_build_workspace_bytes(mesh->nt, g->width, g->height)) return UVL_E_NOMEM;
    if (int32_t s = device_ok()) return s;

    hipStream_t s = as_stream(stream);
    GeomArgs a{};
    a.uv = mesh->uv;
    a.pos = mesh->pos;
    a.nrm = mesh->nrm;
    a.tri = mesh->tri;
    a.nv = mesh->nv;
    a.nt = mesh->nt;
    a.W = g->width;
    a.H = g->height;
    a.tiles_x = (int)ceil_div(a.W, kTile);
    a.tiles_y = (int)ceil_div(a.H, kTile);
    const int64_t ntiles = (int64_t)a.tiles_x * a.tiles_y;
    const GeomLayout L = geom_layout(a.nt, ntiles);
    char *w = static_cast<char *>(ws);
    a.ctr = reinterpret_cast<GCounters *>(w);
    a.recs = reinterpret_cast<TriRec *>(w + L.recs);
    a.boxes = reinterpret_cast<int4 *>(w + L.boxes);
    a.slots = reinterpret_cast<int4 *>(w + L.slots);
    a.list = reinterpret_cast<int32_t *>(w + L.list);
    a.big = reinterpret_cast<unsigned *>(w + L.big);
    a.tcount = reinterpret_cast<unsigned *>(w + L.tcount);
    a.toff = reinterpret_cast<unsigned *>(w + L.toff);
    a.tflag = reinterpret_cast<unsigned *>(w + L.tflag);
    a.blk = reinterpret_cast<unsigned *>(w + L.blk);
    GeomOut o{g->tri_id, g->pos_x, g->pos_y, g->pos_z, has_n ? g->nrm_x : nullptr, g->nrm_y, g->nrm_z,
              has_b ? g->bary1 : nullptr, g->bary2, g->area_w, g->area_w_hi, g->tile_box,
              g->area_w_hi ? nullptr : reinterpret_cast<unsigned long long *>(g->area_blk)};

    hipLaunchKernelGGL(k_geom_counters, dim3(1), dim3(64), 0, s, a.ctr);
    fill_bytes(a.tcount, ntiles * 4, s);
    fill_bytes(a.tflag, ntiles * 4, s);
    if (a.nt > 0) {
        const unsigned tg = (unsigned)ceil_div(a.nt, kBlock);
        hipLaunchKernelGGL(k_setup, dim3(tg), dim3(kBlock), 0, s, a);
        const int nblk = (int)ceil_div(ntiles, kScanSpan);
        hipLaunchKernelGGL(k_scan_reduce, dim3(nblk), dim3(kScanThreads), 0, s, a.tcount, ntiles, a.blk);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, a.blk, nblk);
        hipLaunchKernelGGL(k_scan_down, dim3(nblk), dim3(kScanThreads), 0, s, a.tcount, ntiles, a.blk, a.toff);
        hipLaunchKernelGGL(k_bin, dim3(tg), dim3(kBlock), 0, s, a);
        hipLaunchKernelGGL(k_big_fill, dim3(kBigGrid), dim3(kBlock), 0, s, a, g->tri_id);
        hipLaunchKernelGGL(k_big_raster, dim3(kBigGrid), dim3(kBlock), 0, s, a, g->tri_id);
    } else {
        fill_bytes(a.toff, ntiles * 4, s);
    }
    hipLaunchKernelGGL(k_tile, dim3((unsigned)ntiles), dim3(kTileThreads), 0, s, a, o);
    if (g->tile_box) {
        const int64_t nb = ceil_div(a.tiles_x, UVL_TILE_BLOCK) * ceil_div(a.tiles_y, UVL_TILE_BLOCK);
        hipLaunchKernelGGL(k_block_box, dim3((unsigned)ceil_div(nb, kBlock / 64)), dim3(kBlock), 0, s, g->tile_box,
                           a.tiles_x, a.tiles_y);
    }
    if (launch_status() != UVL_OK) return UVL_E_DEVICE;
    GCounters host{};
    if (hipMemcpyAsync(&host, a.ctr, sizeof(GCounters), hipMemcpyDeviceToHost, s) != hipSuccess) return UVL_E_DEVICE;
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
