// Device-side render-layout conversion (shared with the batched persistent
// kernel).  Render layout of a volume level: 4 x 4 x 4-voxel bricks (a 128-byte line
// for u16) and an occupancy grid that tells the ray caster where every tap of
// a trilinear fetch is zero (or, for u16 with a marking level V > 0, at most V).
//
// Brick (bx, by, bz) starts at element ((bz * nby + by) * nbx + bx) * 64 and
// voxel (x, y, z) sits at ((z & 3) * 16 + (y & 3) * 4 + (x & 3)) inside it.
// occupancy[b] != 0 iff some marking voxel (non-zero; above V) is one of the eight taps of a
// trilinear fetch whose base tap (the floor corner, clamped to the volume)
// lies in brick b; a voxel at (x, y, z) is a tap for base taps
// (x - {0,1}, y - {0,1}, z - {0,1}), so it marks up to eight bricks.  A second
// grid follows the first: one byte per 4 x 4 x 4 bricks (16^3 voxels), set
// when any of its bricks is marked.  Then one byte per brick: the Chebyshev
// distance, in bricks, to the nearest marked brick, capped at kDistCap (0 for
// a marked brick): every brick within distance r - 1 of a brick whose byte is
// r is empty, so a ray can leave that whole cube of bricks in one step.  A
// last byte per brick is working storage of the distance passes.
//
// Pair variant: the same brick order, but element (x, y, z) holds the two x
// taps (voxel x and voxel min(x + 1, nx - 1)), so a trilinear fetch reads
// four elements instead of eight voxels.  Elements past the volume's end are 0.
#pragma once

#include <type_traits>

#include "common.h"

namespace vr {
namespace bk {

constexpr int kThreads = 256;      // threads of one slab group
constexpr int kDistCap = VR_BRICK_DIST_CAP;   // cap of the brick distance grid (bricks)

// Bricks of the apron that follows the last brick of a bricked volume: one
// brick layer, one brick row and one brick.  A trilinear cell on the volume's
// last voxel layer (x, y or z) may then read its far taps one brick, brick row
// or brick layer on without a bounds check: those taps have weight 0, since
// the sample position was clamped to the last voxel centre there.
inline int64_t apron_bricks(int64_t nbx, int64_t nby) { return nbx * nby + nbx + 1; }

// Bricks per axis of a brick layout (host): ceil(n / edge), except along x in
// the overlap layout, where brick bx serves base taps 3 bx .. 3 bx + 2.
inline void brick_grid(int layout, int64_t nx, int64_t ny, int64_t nz, int64_t nb[3])
{
    const int64_t e = layout == VR_LAYOUT_BRICK8 ? 8 : 4;
    nb[0] = layout == VR_LAYOUT_BRICK4_OVERLAP ? (nx - 1) / 3 + 1 : (nx + e - 1) / e;
    nb[1] = (ny + e - 1) / e;
    nb[2] = (nz + e - 1) / e;
}

// Brick x of base tap x in the overlap layout: x / 3 (exact for 32-bit x).
__device__ __forceinline__ uint32_t ovl_bx(uint32_t x) { return __umulhi(x, 0xAAAAAAABu) >> 1; }

// Whether a voxel marks its bricks: a u16 voxel above `above` (0: any non-zero
// voxel), an f32 voxel that is non-zero (`above` is 0 for f32).
__device__ __forceinline__ bool marks(uint16_t v, uint32_t above) { return (uint32_t)v > above; }
__device__ __forceinline__ bool marks(float v, uint32_t) { return v != 0.0f; }

// Element of the pair layout: (voxel x, voxel x + 1) in one load.
template <typename T> struct PairOf;
template <> struct PairOf<uint16_t> { typedef uint32_t type; };
template <> struct PairOf<float> { typedef float2 type; };

__device__ __forceinline__ uint32_t make_pair(uint16_t lo, uint16_t hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }
__device__ __forceinline__ float2 make_pair(float lo, float hi) { return make_float2(lo, hi); }

// Element type of a layout: the voxel, or its x pair.
template <typename T, bool PAIRS> struct ElemOf { typedef T type; };
template <typename T> struct ElemOf<T, true> { typedef typename PairOf<T>::type type; };

// Four consecutive voxels from one vector load.
__device__ __forceinline__ void unpack4(uint2 w, uint16_t (&v)[4])
{
    v[0] = (uint16_t)(w.x & 0xFFFFu);
    v[1] = (uint16_t)(w.x >> 16);
    v[2] = (uint16_t)(w.y & 0xFFFFu);
    v[3] = (uint16_t)(w.y >> 16);
}
__device__ __forceinline__ void unpack4(float4 w, float (&v)[4])
{
    v[0] = w.x;
    v[1] = w.y;
    v[2] = w.z;
    v[3] = w.w;
}

// LDS of one slab group.
template <typename T, bool PAIRS = false>
struct SlabLds {
    __align__(16) typename ElemOf<T, PAIRS>::type slab[16 * 64];
    uint32_t marks[17 * 2 * 2];      // (bx - 1 .. bx + 15) x (by - 1, by) x (bz - 1, bz)
};

// A group of kThreads threads (thread `t` of the group) converts a 64 x 4 x 4
// voxel slab (16 bricks along x) at brick row (by, bz): thread t reads 4
// voxels of volume row (t / 16) at x offset 4 (t % 16), which is row t / 16
// of brick t % 16.  The slab goes through LDS in brick order so that stores
// are 16-byte pieces of whole bricks.  The occupancy marks of the slab (its 16
// bricks and the neighbours at -1 in x, y and z) are gathered in LDS and
// written once per slab, to the brick grid and to the 16^3 group grid.
// Inactive groups take the same barriers.  VEC: nx is a multiple of 4 and
// src is aligned to four voxels, so each thread's four voxels are one load.
template <typename T, bool PAIRS = false, bool VEC = false>
__device__ inline void slab_body(const T* __restrict__ src, int nx, int ny, int nz, int nbx, int nby,
                                 typename ElemOf<T, PAIRS>::type* __restrict__ dst, uint8_t* __restrict__ occ,
                                 uint8_t* __restrict__ macro, int nmx, int nmy, uint32_t above, int bx0, int by,
                                 int bz, bool active, int t, SlabLds<T, PAIRS>& G)
{
    typedef typename ElemOf<T, PAIRS>::type P;
    if (t < 17 * 4) G.marks[t] = 0;
    __syncthreads();
    const int r = t >> 4, lb = t & 15;          // row inside the brick, brick within the slab
    if (active) {
        const int y = by * 4 + (r & 3), z = bz * 4 + (r >> 2), x0 = (bx0 + lb) * 4;
        T v[4];
        const bool rowok = y < ny && z < nz;
        const T* row = src + ((int64_t)z * ny + y) * nx;
        if constexpr (VEC) {
            using V4 = typename std::conditional<sizeof(T) == 2, uint2, float4>::type;
            if (rowok && x0 < nx) {
                unpack4(*reinterpret_cast<const V4*>(row + x0), v);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = (T)0;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = (rowok && x0 + e < nx) ? row[x0 + e] : (T)0;
        }
        if constexpr (PAIRS) {
            // the voxel after the four (clamped to the row's last voxel)
            const T nxt = (rowok && x0 + 4 < nx) ? row[x0 + 4] : v[3];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const T hi = (x0 + e + 1 < nx) ? (e < 3 ? v[e + 1] : nxt) : v[e];
                G.slab[lb * 64 + r * 4 + e] = make_pair(v[e], hi);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) G.slab[lb * 64 + r * 4 + e] = v[e];
        }
        if (occ != nullptr) {
            bool any = false;
#pragma unroll
            for (int e = 0; e < 4; ++e) any |= marks(v[e], above);
            if (any) {
                // a voxel at x marks the base-tap bricks of x and x - 1 (and likewise in y, z)
                const int xs[2] = {lb + 1, marks(v[0], above) ? lb : -1};          // index into -1..15 (+1)
                const int ys[2] = {1, (r & 3) == 0 ? 0 : -1};
                const int zs[2] = {1, (r >> 2) == 0 ? 0 : -1};
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int c = 0; c < 2; ++c)
                            if (xs[a] >= 0 && ys[b] >= 0 && zs[c] >= 0)
                                G.marks[(zs[c] * 2 + ys[b]) * 17 + xs[a]] = 1u;
            }
        }
    }
    __syncthreads();
    if (!active) return;
    // whole bricks out: 16 bricks x 64 elements, 16 bytes per store
    constexpr int kPer = 16 / sizeof(P);
    const int nb_here = min(16, nbx - bx0);
    for (int q = t; q < 16 * 64 / kPer; q += kThreads) {
        const int e = q * kPer;
        if (e / 64 < nb_here) {
            const int64_t brick = ((int64_t)bz * nby + by) * nbx + bx0 + e / 64;
            *reinterpret_cast<uint4*>(dst + (brick << 6) + (e & 63)) =
                *reinterpret_cast<const uint4*>(G.slab + e);
        }
    }
    if (occ != nullptr && t < 17 * 4) {
        const int xi = t % 17, yi = (t / 17) & 1, zi = t / 34;
        const int bx = bx0 + xi - 1, byy = by + yi - 1, bzz = bz + zi - 1;
        if (G.marks[t] && bx >= 0 && bx < nbx && byy >= 0 && bzz >= 0) {
            occ[((int64_t)bzz * nby + byy) * nbx + bx] = 1;
            macro[((int64_t)(bzz >> 2) * nmy + (byy >> 2)) * nmx + (bx >> 2)] = 1;
        }
    }
}

// 8^3 bricks: row piece r = ((z * 8 nby) + y) * nbx + bx holds the 8 voxels
// [8 bx, 8 bx + 8) of row (y, z) of the volume padded to whole bricks (0 past
// its end), one brick row, stored with 16-byte vectors at element
// ((z & 7) * 8 + (y & 7)) * 8 of brick (bx, y >> 3, z >> 3); the pieces
// r < nbx * 8 nby * 8 nbz cover every brick.  Marks (bytes of 1, written by every piece that sees
// a non-zero voxel, so overlapping writes agree): the piece's own brick, and
// the brick below in x, y or z when the piece's first voxel, first row of a
// brick or first slice of a brick reaches back into it, with the group marks
// of each (4^3 bricks).
template <typename T>
__device__ inline void row8_body(const T* __restrict__ src, int nx, int ny, int nz, int nbx, int nby,
                                 T* __restrict__ dst, uint8_t* __restrict__ occ, uint8_t* __restrict__ macro,
                                 int nmx, int nmy, uint32_t above, int64_t r)
{
    const int bx = (int)(r % nbx);
    const int64_t yz = r / nbx;
    const int py = nby * 8;
    const int y = (int)(yz % py), z = (int)(yz / py);
    const bool rowok = y < ny && z < nz;
    const T* row = src + ((int64_t)(rowok ? z : 0) * ny + (rowok ? y : 0)) * nx;
    const int x0 = bx * 8;
    T v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (rowok && x0 + e < nx) ? row[x0 + e] : (T)0;
    const int64_t brick = ((int64_t)(z >> 3) * nby + (y >> 3)) * nbx + bx;
    T* out = dst + (brick << 9) + (((z & 7) << 6) | ((y & 7) << 3));
    using V = typename std::conditional<sizeof(T) == 2, uint4, float4>::type;
    constexpr int kPerVec = 16 / (int)sizeof(T);
#pragma unroll
    for (int q = 0; q < 8 / kPerVec; ++q) {
        V w;
        T* wt = reinterpret_cast<T*>(&w);
#pragma unroll
        for (int e = 0; e < kPerVec; ++e) wt[e] = v[q * kPerVec + e];
        *reinterpret_cast<V*>(out + q * kPerVec) = w;
    }
    if (occ == nullptr) return;
    bool any = false;
#pragma unroll
    for (int e = 0; e < 8; ++e) any |= marks(v[e], above);
    if (!any) return;
    const int by = y >> 3, bz = z >> 3;
    const int xs[2] = {bx, (marks(v[0], above) && bx > 0) ? bx - 1 : -1};
    const int ys[2] = {by, ((y & 7) == 0 && by > 0) ? by - 1 : -1};
    const int zs[2] = {bz, ((z & 7) == 0 && bz > 0) ? bz - 1 : -1};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c)
                if (xs[a] >= 0 && ys[b] >= 0 && zs[c] >= 0) {
                    occ[((int64_t)zs[c] * nby + ys[b]) * nbx + xs[a]] = 1;
                    macro[((int64_t)(zs[c] >> 2) * nmy + (ys[b] >> 2)) * nmx + (xs[a] >> 2)] = 1;
                }
}

// Overlap layout: a group of kThreads threads (thread t) converts the
// kOvlBricks bricks bx0 .. bx0 + kOvlBricks - 1 of brick row (by, bz): their 16
// voxel rows (4 y x 4 z) hold voxels 3 bx0 .. 3 bx0 + 3 kOvlBricks (0 past the
// volume's end).  With 64 bricks a row's 192 + 1 voxels start on a 384-byte
// boundary (bx0 is a multiple of 64), so the row reads fill whole cache lines.
// The rows go through LDS in order, four voxels per load (each thread's loads
// all issued before its LDS stores); brick bi's row r is
// then voxels 3 bi .. 3 bi + 3 of LDS row r, and the bricks leave as 16-byte
// stores (two rows of one brick each).  Marks: the four voxels of a brick row
// are the x taps of every cell the brick serves in that row, so a marking
// voxel marks the row's brick, and the brick below in y or z when the row is
// the first of its brick there (its cells at y - 1 or z - 1 take the row as
// their far tap); the group marks of each follow.  VEC: nx is a multiple of 4
// and src is aligned to four voxels, so each four voxels are one load.
constexpr int kOvlBricks = 64;
constexpr int kOvlRow = 3 * kOvlBricks + 4;      // voxels of an LDS row (one load past the last brick)
struct OvlLds {
    __align__(16) uint16_t rows[16][kOvlRow];
    uint32_t marks[kOvlBricks][4];   // brick bi: own, below in y, below in z, below in both
};

template <bool VEC>
__device__ inline void slab_ovl_body(const uint16_t* __restrict__ src, int nx, int ny, int nz, int nbx, int nby,
                                     uint16_t* __restrict__ dst, uint8_t* __restrict__ occ,
                                     uint8_t* __restrict__ macro, int nmx, int nmy, uint32_t above, int bx0, int by,
                                     int bz, int t, OvlLds& G)
{
    constexpr int kQuads = kOvlRow / 4;             // four-voxel loads per row
    constexpr int kLoads = (16 * kQuads + kThreads - 1) / kThreads;   // per thread
    for (int q = t; q < kOvlBricks * 4; q += kThreads) G.marks[q >> 2][q & 3] = 0u;
    // All of a thread's loads are issued before the first LDS store, so that
    // they are in flight together.
    uint2 w[kLoads];
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {
        const int q = t + k * kThreads;
        w[k] = make_uint2(0u, 0u);
        if (q < 16 * kQuads) {
            const int r = q / kQuads, c = q % kQuads;
            const int y = by * 4 + (r & 3), z = bz * 4 + (r >> 2);
            const int x = bx0 * 3 + c * 4;
            const bool rowok = y < ny && z < nz;
            const uint16_t* row = src + ((int64_t)(rowok ? z : 0) * ny + (rowok ? y : 0)) * nx;
            if (VEC && rowok && x + 3 < nx) {
                w[k] = *reinterpret_cast<const uint2*>(row + x);
            } else {
                uint32_t v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = (rowok && x + e < nx) ? (uint32_t)row[x + e] : 0u;
                w[k] = make_uint2(v[0] | (v[1] << 16), v[2] | (v[3] << 16));
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {   // voxels 4 c .. 4 c + 3 of row r: one 8-byte store
        const int q = t + k * kThreads;
        if (q < 16 * kQuads) *reinterpret_cast<uint2*>(&G.rows[q / kQuads][(q % kQuads) * 4]) = w[k];
    }
    __syncthreads();
    const int nb_here = min(kOvlBricks, nbx - bx0);
    for (int q = t; q < kOvlBricks * 16; q += kThreads) {   // marks: row q % 16 of brick q / 16
        const int bi = q >> 4, r = q & 15;
        bool any = false;
#pragma unroll
        for (int e = 0; e < 4; ++e) any |= marks(G.rows[r][bi * 3 + e], above);
        if (any && bi < nb_here) {
            G.marks[bi][0] = 1u;
            const bool y0 = (r & 3) == 0 && by > 0, z0 = (r >> 2) == 0 && bz > 0;
            if (y0) G.marks[bi][1] = 1u;
            if (z0) G.marks[bi][2] = 1u;
            if (y0 && z0) G.marks[bi][3] = 1u;
        }
    }
    for (int q = t; q < kOvlBricks * 8; q += kThreads) {    // brick q / 8, rows 2 (q % 8) and 2 (q % 8) + 1
        const int bi = q >> 3, r = (q & 7) * 2;
        if (bi < nb_here) {
            uint4 w;
            w.x = (uint32_t)G.rows[r][bi * 3] | ((uint32_t)G.rows[r][bi * 3 + 1] << 16);
            w.y = (uint32_t)G.rows[r][bi * 3 + 2] | ((uint32_t)G.rows[r][bi * 3 + 3] << 16);
            w.z = (uint32_t)G.rows[r + 1][bi * 3] | ((uint32_t)G.rows[r + 1][bi * 3 + 1] << 16);
            w.w = (uint32_t)G.rows[r + 1][bi * 3 + 2] | ((uint32_t)G.rows[r + 1][bi * 3 + 3] << 16);
            const int64_t brick = ((int64_t)bz * nby + by) * nbx + bx0 + bi;
            *reinterpret_cast<uint4*>(dst + (brick << 6) + r * 4) = w;
        }
    }
    __syncthreads();
    if (occ == nullptr) return;
    for (int q = t; q < kOvlBricks * 4; q += kThreads) {
        const int bi = q >> 2, k = q & 3;
        if (bi < nb_here && G.marks[bi][k]) {
            const int bx = bx0 + bi, byy = by - (k & 1), bzz = bz - (k >> 1);
            occ[((int64_t)bzz * nby + byy) * nbx + bx] = 1;
            macro[((int64_t)(bzz >> 2) * nmy + (byy >> 2)) * nmx + (bx >> 2)] = 1;
        }
    }
}

}  // namespace bk
}  // namespace vr
