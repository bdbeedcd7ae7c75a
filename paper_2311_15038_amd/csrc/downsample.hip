// Thresholding fused with the multi-resolution pyramid (Sections II, III-A,
// III-D): one streaming pass over the u16 volume writes up to four box-mean
// levels, each rounded from its own exact integer sum.
//
// A workgroup (512 threads) walks 256 x 16 x 16-voxel tiles, two steps of
// loads ahead of its sums.  Each lane owns
// an 8-voxel x-run of a 2 x 2 (y, z) pair of rows: it loads 4 x 16 bytes
// (the 32 lanes of a half-wave read a 512-byte piece of each row), looks every
// voxel up in the keep mask held in LDS, and forms four level-1 sums.
// Level-k sums for k > 1 are reduced from the level-1 sums in LDS.  When the
// keep mask is one interval [T, 65535] (a plain threshold, or a top-slice
// filter that removed nothing above T) a voxel is kept by a compare instead
// of the LDS lookup; each workgroup detects that once from the mask.
//
// With container removal (Section III-B) a voxel outside the kept disc of
// its slice counts as removed: each workgroup tabulates the kept column run
// of every image row in LDS once, loads only the 16-byte pieces that touch
// the disc and zeroes the voxels of a piece that fall outside it.
#include <type_traits>

#include "disc_dev.h"
#include "downsample_dev.h"

namespace {

using namespace vr::ds;

// zero the atlas tiles past the last slice
__global__ void __launch_bounds__(kThreads)
zero_tiles(void* atlas, int bits, int64_t W, int tiles_x, int nxk, int nyk, int first_tile, int n_tiles)
{
    const int64_t per = (int64_t)nxk * nyk;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < per * n_tiles;
         q += (int64_t)gridDim.x * kThreads) {
        const int t = first_tile + (int)(q / per);
        const int64_t r = q % per;
        const int y = (int)(r / nxk), x = (int)(r % nxk);
        const int64_t a = ((int64_t)(t / tiles_x) * nyk + y) * W + (int64_t)(t % tiles_x) * nxk + x;
        if (bits == 16) static_cast<uint16_t*>(atlas)[a] = 0;
        else static_cast<uint8_t*>(atlas)[a] = 0;
    }
}

// Wide tiles of the standalone pass: 256 x 16 x 16 voxels per four steps of
// a 512-thread workgroup.  Half-wave h (32 lanes) streams 512-byte pieces of
// rows, eight voxels per lane: at step it = 0..3 of a tile it reads the rows
// of (y, z) pair (2 (h & 3) + (it & 1), 2 (h >> 2) + (it >> 1)), so over the
// four steps a lane covers whole level-2 boxes and keeps their sums in
// registers.  Levels 3 and 4 are reduced from the level-2 sums in LDS.
constexpr int WX = 256, WT = 512;

// How a voxel is kept: looked up in the mask, by the interval [T, 65535]
// (T >= 1), or every voxel (T = 0).
enum { KEEP_LOOKUP = 0, KEEP_INTERVAL = 1, KEEP_ALL = 2 };

struct WideLds {
    uint32_t s2[TZ / 4][TY / 4][WX / 4];
    uint32_t s3[TZ / 8][TY / 8][WX / 8];
};

struct WideTile {
    int X0, Y0, Z0;
    bool interior;
};

__device__ __forceinline__ WideTile wide_tile(int tile, int tiles_x, int tiles_y, int nx, int ny, int nz, int aligned)
{
    WideTile t;
    t.X0 = (tile % tiles_x) * WX;
    t.Y0 = ((tile / tiles_x) % tiles_y) * TY;
    t.Z0 = (tile / (tiles_x * tiles_y)) * TZ;
    t.interior = aligned && t.X0 + WX <= nx && t.Y0 + TY <= ny && t.Z0 + TZ <= nz;
    return t;
}

// (y, z) row pair of half-wave h at step it of a tile
__device__ __forceinline__ int pair_y(int h, int it) { return 2 * (h & 3) + (it & 1); }
__device__ __forceinline__ int pair_z(int h, int it) { return 2 * (h >> 2) + (it >> 1); }

constexpr int kMaxDiscSide = 8192;          // rows tabulated by the disc variant

// Bits e (0..7) of the voxels x + e of a row inside its kept run, from the
// packed run x0 | x1 << 16 (an empty run has x0 > x1).
__device__ __forceinline__ uint32_t run_bits(uint32_t sp, int x)
{
    const int lo = max((int)(sp & 0xFFFFu) - x, 0), hi = min((int)(sp >> 16) - x, 7);
    return lo > hi ? 0u : (0xFFu >> (7 - hi)) & (0xFFu << lo);
}

// Zero the voxels of an 8-voxel piece whose bit in k is clear.
__device__ __forceinline__ uint4 mask_piece(uint4 q, uint32_t k)
{
    auto m = [k](int i) {
        return (((k >> (2 * i)) & 1u) ? 0x0000FFFFu : 0u) | (((k >> (2 * i + 1)) & 1u) ? 0xFFFF0000u : 0u);
    };
    return make_uint4(q.x & m(0), q.y & m(1), q.z & m(2), q.w & m(3));
}

// The four rows (y pair yp, z pair zp) of the lane's 8-voxel x-run, zero past
// the volume's end (and, with DISC, outside the kept disc of the rows).
template <bool DISC>
__device__ __forceinline__ void load_rows(const uint16_t* __restrict__ vol, int nx, int ny, int nz,
                                          const WideTile& t, int yp, int zp, int l, const uint32_t* spans,
                                          uint4 (&q)[4])
{
    const int x = t.X0 + 8 * l, y = t.Y0 + 2 * yp, z = t.Z0 + 2 * zp;
    const int64_t nxy = (int64_t)nx * ny;
    const uint16_t* p = vol + ((int64_t)z * ny + y) * nx + x;
    uint32_t kb[2] = {0xFFu, 0xFFu};
    if (DISC) {
        kb[0] = y < ny ? run_bits(spans[y], x) : 0u;
        kb[1] = y + 1 < ny ? run_bits(spans[y + 1], x) : 0u;
    }
    if (t.interior) {
        const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
        q[0] = !DISC || kb[0] ? load_stream(p) : zero;
        q[1] = !DISC || kb[1] ? load_stream(p + nx) : zero;
        q[2] = !DISC || kb[0] ? load_stream(p + nxy) : zero;
        q[3] = !DISC || kb[1] ? load_stream(p + nxy + nx) : zero;
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool rowok = y + (r & 1) < ny && z + (r >> 1) < nz && (!DISC || kb[r & 1]);
            const uint16_t* row = p + (r & 1) * (int64_t)nx + (r >> 1) * nxy;
            uint32_t w[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t lo = (rowok && x + 2 * e < nx) ? (uint32_t)row[2 * e] : 0u;
                const uint32_t hi = (rowok && x + 2 * e + 1 < nx) ? (uint32_t)row[2 * e + 1] : 0u;
                w[e] = lo | (hi << 16);
            }
            q[r] = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
    if (DISC) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (kb[r & 1] != 0xFFu) q[r] = mask_piece(q[r], kb[r & 1]);
    }
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// 1 in each 16-bit half of w whose voxel is >= T, else 0; t2 = (T - 1) in both
// halves: a saturating packed subtract leaves a non-zero half exactly for the
// kept voxels, and a packed minimum with 1 turns it into the flag.
__device__ __forceinline__ uint32_t kept_flags(uint32_t w, uint32_t t2)
{
    uint32_t d, m;
    asm("v_pk_sub_u16 %0, %1, %2 clamp" : "=v"(d) : "v"(w), "v"(t2));
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(m) : "v"(d), "v"(0x00010001u));
    return m;
}

// acc + the kept voxels of the two halves of w: one packed dot product with
// their 0/1 flags.
template <int MODE>
__device__ __forceinline__ uint32_t add_kept(uint32_t acc, uint32_t w, const uint32_t* bits, uint32_t T, uint32_t t2)
{
    if (MODE == KEEP_LOOKUP)
        return acc + keepv<false>(bits, w & 0xFFFFu, T) + keepv<false>(bits, w >> 16, T);
    const uint32_t m = MODE == KEEP_ALL ? 0x00010001u : kept_flags(w, t2);
    return __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, w), __builtin_bit_cast(u16x2, m), acc, false);
}

template <int MODE>
__device__ __forceinline__ uint32_t sum_column(uint32_t a, uint32_t b, uint32_t c, uint32_t d, const uint32_t* bits,
                                               uint32_t T, uint32_t t2)
{
    return add_kept<MODE>(add_kept<MODE>(add_kept<MODE>(add_kept<MODE>(0u, a, bits, T, t2), b, bits, T, t2), c, bits,
                                         T, t2), d, bits, T, t2);
}

// Store of level k at (x, y, z) of the level, with the atlas copy when k is
// the atlas level and, with SUMS, the exact sum when that level's sums are
// asked for; arow is the atlas offset of the tile holding slice z.
template <bool SUMS>
__device__ __forceinline__ void store_at(const LevelOut& L, int k, int x, int y, int z, uint32_t sum, int64_t arow)
{
    const int i = k - 1;
    if (x >= L.nx[i] || y >= L.ny[i] || z >= L.nz[i]) return;
    const uint16_t v = round_level(sum, k);
    const int64_t at = ((int64_t)z * L.ny[i] + y) * L.nx[i] + x;
    L.p[i][at] = v;
    if (SUMS && L.sums[i] != nullptr) L.sums[i][at] = sum;
    if (k == L.atlas_level) {
        const int64_t a = arow + (int64_t)y * ((int64_t)L.atlas_tiles_x * L.nx[i]) + x;
        if (L.atlas_bits == 16) {
            static_cast<uint16_t*>(L.atlas)[a] = v;
        } else {
            const uint32_t b = ((uint32_t)v + 128u) >> 8;
            static_cast<uint8_t*>(L.atlas)[a] = (uint8_t)(b > 255u ? 255u : b);
        }
    }
}

// Atlas offset of the tile (z mod tiles_x, z div tiles_x) of slice z of level k
// (0 unless k is the atlas level).
__device__ __forceinline__ int64_t atlas_row(const LevelOut& L, int k, int z)
{
    if (k != L.atlas_level) return 0;
    const int i = k - 1;
    const uint32_t tx = (uint32_t)z % (uint32_t)L.atlas_tiles_x, ty = (uint32_t)z / (uint32_t)L.atlas_tiles_x;
    return (int64_t)ty * L.ny[i] * ((int64_t)L.atlas_tiles_x * L.nx[i]) + (int64_t)tx * L.nx[i];
}

// Level 1 of one step (four x pairs of the lane's rows) and its addition to
// the lane's two level-2 partial sums.
template <int MODE, bool SUMS>
__device__ __forceinline__ void level1_step(const uint4 (&q)[4], const uint32_t* bits, uint32_t T, uint32_t t2,
                                            const WideTile& t, int yp, int zp, int l, int aligned_out,
                                            const LevelOut& L, uint32_t (&l2)[2])
{
    uint32_t s[4];
    s[0] = sum_column<MODE>(q[0].x, q[1].x, q[2].x, q[3].x, bits, T, t2);
    s[1] = sum_column<MODE>(q[0].y, q[1].y, q[2].y, q[3].y, bits, T, t2);
    s[2] = sum_column<MODE>(q[0].z, q[1].z, q[2].z, q[3].z, bits, T, t2);
    s[3] = sum_column<MODE>(q[0].w, q[1].w, q[2].w, q[3].w, bits, T, t2);
    const int x1 = (t.X0 >> 1) + 4 * l, y1 = (t.Y0 >> 1) + yp, z1 = (t.Z0 >> 1) + zp;
    if (t.interior && aligned_out && !SUMS) {
        uint2 w;
        w.x = (uint32_t)round_level(s[0], 1) | ((uint32_t)round_level(s[1], 1) << 16);
        w.y = (uint32_t)round_level(s[2], 1) | ((uint32_t)round_level(s[3], 1) << 16);
        // streaming store: level 1 is written once and not read again by this pass
        // (measured: 38 us less for the 1024^3 pyramid than a plain store)
        u32x2 wv;
        wv.x = w.x;
        wv.y = w.y;
        __builtin_nontemporal_store(wv, reinterpret_cast<u32x2*>(L.p[0] + ((int64_t)z1 * L.ny[0] + y1) * L.nx[0] + x1));
    } else {
        const int64_t arow = atlas_row(L, 1, z1);
#pragma unroll
        for (int k = 0; k < 4; ++k) store_at<SUMS>(L, 1, x1 + k, y1, z1, s[k], arow);
    }
    l2[0] += s[0] + s[1];
    l2[1] += s[2] + s[3];
}

// Level 2 of a tile from the lane's register sums; levels 3 and 4 from the
// level-2 sums in LDS.
template <bool SUMS>
__device__ __forceinline__ void coarse_levels(const WideTile& t, int n_levels, const LevelOut& L, WideLds& G, int tid,
                                              const uint32_t (&l2)[2])
{
    const int h = tid >> 5, l = tid & 31;
    const int x2 = 2 * l, y2 = h & 3, z2 = h >> 2;
    const int64_t arow = atlas_row(L, 2, (t.Z0 >> 2) + z2);
    const int X2 = (t.X0 >> 2) + x2, Y2 = (t.Y0 >> 2) + y2, Z2 = (t.Z0 >> 2) + z2;
    if (t.interior && L.pair2 && !SUMS) {
        // the lane's two level-2 voxels (an even x and the next) as one 32-bit store,
        // and likewise into the atlas
        const uint32_t w = (uint32_t)round_level(l2[0], 2) | ((uint32_t)round_level(l2[1], 2) << 16);
        *reinterpret_cast<uint32_t*>(L.p[1] + ((int64_t)Z2 * L.ny[1] + Y2) * L.nx[1] + X2) = w;
        if (L.atlas_level == 2)
            *reinterpret_cast<uint32_t*>(static_cast<uint16_t*>(L.atlas) + arow +
                                         (int64_t)Y2 * ((int64_t)L.atlas_tiles_x * L.nx[1]) + X2) = w;
    } else {
        store_at<SUMS>(L, 2, X2, Y2, Z2, l2[0], arow);
        store_at<SUMS>(L, 2, X2 + 1, Y2, Z2, l2[1], arow);
    }
    if (n_levels < 3) return;
    G.s2[z2][y2][x2] = l2[0];
    G.s2[z2][y2][x2 + 1] = l2[1];
    __syncthreads();
    if (tid < (TZ / 8) * (TY / 8) * (WX / 8)) {
        const int x = tid % (WX / 8), y = (tid / (WX / 8)) % (TY / 8), z = tid / ((WX / 8) * (TY / 8));
        uint32_t acc = 0;
#pragma unroll
        for (int d = 0; d < 8; ++d) acc += G.s2[2 * z + (d >> 2)][2 * y + ((d >> 1) & 1)][2 * x + (d & 1)];
        store_at<SUMS>(L, 3, (t.X0 >> 3) + x, (t.Y0 >> 3) + y, (t.Z0 >> 3) + z, acc, atlas_row(L, 3, (t.Z0 >> 3) + z));
        G.s3[z][y][x] = acc;
    }
    if (n_levels > 3) {
        __syncthreads();
        if (tid < WX / 16) {
            uint32_t acc = 0;
#pragma unroll
            for (int d = 0; d < 8; ++d) acc += G.s3[d >> 2][(d >> 1) & 1][2 * tid + (d & 1)];
            store_at<SUMS>(L, 4, (t.X0 >> 4) + tid, t.Y0 >> 4, t.Z0 >> 4, acc, atlas_row(L, 4, t.Z0 >> 4));
        }
    }
    __syncthreads();   // the next tile writes its level-2 sums over these
}

// A workgroup walks its tiles (blockIdx.x, + gridDim.x, ...) as a flat
// sequence of steps (tile, it); the rows of the next two steps are in flight
// while the current step is summed, and the coarse levels of a tile are
// reduced while the first rows of the next tile arrive.
template <int MODE, bool DISC, bool SUMS>
__device__ inline void wide_tiles(const uint16_t* __restrict__ vol, int nx, int ny, int nz, int aligned,
                                  int aligned_out, const uint32_t* bits, uint32_t T, int n_levels,
                                  const LevelOut& L, int tiles_x, int tiles_y, int n_tiles, WideLds& G,
                                  const uint32_t* spans)
{
    const int tid = threadIdx.x, h = tid >> 5, l = tid & 31;
    const int my_tiles = n_tiles > (int)blockIdx.x ? (n_tiles - 1 - (int)blockIdx.x) / (int)gridDim.x + 1 : 0;
    const int steps = 4 * my_tiles;
    const uint32_t tm1 = T > 0u ? T - 1u : 0u, t2 = tm1 | (tm1 << 16);
    auto tile_at = [&](int m) {
        return wide_tile((int)blockIdx.x + m * (int)gridDim.x, tiles_x, tiles_y, nx, ny, nz, aligned);
    };
    // rows of steps k .. k + LA - 1 are in flight; tl is the tile of the last one loaded
    constexpr int LA = 3;
    WideTile t0 = tile_at(0), tl = t0;
    uint4 q[LA][4];
#pragma unroll
    for (int a = 0; a < LA - 1; ++a)
        if (a < steps) load_rows<DISC>(vol, nx, ny, nz, t0, pair_y(h, a), pair_z(h, a), l, spans, q[a]);
    uint32_t l2[2] = {0u, 0u};
    for (int k = 0; k < steps; ++k) {
        if (k + LA - 1 < steps) {
            const int kn = k + LA - 1, itn = kn & 3;
            if (itn == 0) tl = tile_at(kn >> 2);
            load_rows<DISC>(vol, nx, ny, nz, tl, pair_y(h, itn), pair_z(h, itn), l, spans, q[LA - 1]);
        }
        const int it = k & 3;
        level1_step<MODE, SUMS>(q[0], bits, T, t2, t0, pair_y(h, it), pair_z(h, it), l, aligned_out, L, l2);
        if (it == 3) {
            if (n_levels > 1) coarse_levels<SUMS>(t0, n_levels, L, G, tid, l2);
            l2[0] = l2[1] = 0u;
            t0 = tile_at((k + 1) >> 2);
        }
#pragma unroll
        for (int a = 0; a < LA - 1; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) q[a][r] = q[a + 1][r];
    }
}

template <bool DISC, bool SUMS>
__global__ void __launch_bounds__(WT)
downsample_kernel(const uint16_t* __restrict__ vol, int nx, int ny, int nz, int aligned, int aligned_out,
                  const uint32_t* __restrict__ keep_bits, int n_levels, LevelOut L, int tiles_x,
                  int tiles_y, int n_tiles, const int32_t* __restrict__ circle)
{
    __shared__ uint32_t bits[VR_KEEP_WORDS];
    __shared__ WideLds G;
    __shared__ uint32_t s_first, s_bad;
    __shared__ uint32_t spans[DISC ? kMaxDiscSide : 1];
    if (DISC) {
        const vr::disc::Disc d = vr::disc::load_disc(circle);
        for (int y = threadIdx.x; y < ny; y += WT) {
            int64_t x0, x1;
            vr::disc::row_span(d, y, nx, x0, x1);
            spans[y] = x0 > x1 ? 0x0000FFFFu : (uint32_t)x0 | ((uint32_t)x1 << 16);
        }
        __syncthreads();
    }
    const uint32_t T = keep_bits == nullptr ? 0u : load_mask(keep_bits, bits, s_first, s_bad);
    if (T == 0u)
        wide_tiles<KEEP_ALL, DISC, SUMS>(vol, nx, ny, nz, aligned, aligned_out, bits, T, n_levels, L, tiles_x, tiles_y,
                                   n_tiles, G, spans);
    else if (T <= VR_NBINS)
        wide_tiles<KEEP_INTERVAL, DISC, SUMS>(vol, nx, ny, nz, aligned, aligned_out, bits, T, n_levels, L, tiles_x,
                                        tiles_y, n_tiles, G, spans);
    else
        wide_tiles<KEEP_LOOKUP, DISC, SUMS>(vol, nx, ny, nz, aligned, aligned_out, bits, 0u, n_levels, L, tiles_x,
                                      tiles_y, n_tiles, G, spans);
}

template <bool DISC, bool SUMS>
int occupancy()
{
    int n = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, downsample_kernel<DISC, SUMS>, WT, 0) == hipSuccess &&
                   n > 0
               ? n
               : 1;
}

// Levels 5..n from the exact level-4 sums the pass wrote: S_k of a level-k
// voxel is the sum of S_4 over its 2^(k-4) cube of level-4 voxels (those that
// exist: the level-4 grid covers every voxel, and voxels past the volume's
// end are 0 in S_4 already), then L_k = (S_k + 2^(3k-1)) >> 3k.  One
// workgroup per level-k voxel.
constexpr int kCoarseMax = VR_MAX_LEVELS - kFusedLevels;
constexpr int CT = 256;

struct CoarseOut {
    const uint64_t* s4;
    int n4x, n4y, n4z;
    int n_coarse;                          // levels beyond the fourth
    int64_t first[kCoarseMax + 1];         // workgroups of level 5 + i: [first[i], first[i + 1])
    uint16_t* p[kCoarseMax];
    uint64_t* sums[kCoarseMax];
    int nx[kCoarseMax], ny[kCoarseMax], nz[kCoarseMax];
    void* atlas;                           // slicemap of one of these levels, or NULL
    int atlas_level, atlas_tiles_x, atlas_bits;
};

__global__ void __launch_bounds__(CT) coarse_kernel(const CoarseOut C)
{
    __shared__ unsigned long long part[CT / 64];
    const int64_t q = blockIdx.x;
    int i = 0;
    while (i + 1 < C.n_coarse && q >= C.first[i + 1]) ++i;
    const int k = kFusedLevels + 1 + i, e = 1 << (k - kFusedLevels);
    const int64_t r = q - C.first[i];
    const int x = (int)(r % C.nx[i]), y = (int)((r / C.nx[i]) % C.ny[i]), z = (int)(r / ((int64_t)C.nx[i] * C.ny[i]));
    const int x4 = x * e, y4 = y * e, z4 = z * e;
    const int cx = min(e, C.n4x - x4), cy = min(e, C.n4y - y4), cz = min(e, C.n4z - z4);
    unsigned long long acc = 0;
    for (int t = threadIdx.x; t < cx * cy * cz; t += CT) {
        const int a = t % cx, b = (t / cx) % cy, c = t / (cx * cy);
        acc += C.s4[((int64_t)(z4 + c) * C.n4y + (y4 + b)) * C.n4x + (x4 + a)];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long S = 0;
#pragma unroll
        for (int w = 0; w < CT / 64; ++w) S += part[w];
        const uint16_t v = (uint16_t)((S + (1ull << (3 * k - 1))) >> (3 * k));
        const int64_t at = ((int64_t)z * C.ny[i] + y) * C.nx[i] + x;
        C.p[i][at] = v;
        if (C.sums[i] != nullptr) C.sums[i][at] = S;
        if (k == C.atlas_level) {
            const int tx = z % C.atlas_tiles_x, ty = z / C.atlas_tiles_x;
            const int64_t W = (int64_t)C.atlas_tiles_x * C.nx[i];
            const int64_t a = ((int64_t)ty * C.ny[i] + y) * W + (int64_t)tx * C.nx[i] + x;
            if (C.atlas_bits == 16) {
                static_cast<uint16_t*>(C.atlas)[a] = v;
            } else {
                const uint32_t b8 = ((uint32_t)v + 128u) >> 8;
                static_cast<uint8_t*>(C.atlas)[a] = (uint8_t)(b8 > 255u ? 255u : b8);
            }
        }
    }
}

}  // namespace

namespace {

int downsample(const uint16_t* d_vol, int64_t nx, int64_t ny, int64_t nz, const uint32_t* d_keep_bits,
               const int32_t* d_circle, int n_levels, uint16_t* const* h_levels, uint64_t* const* h_level_sums,
               const vr_atlas_spec* atlas, void* stream)
{
    VR_REQUIRE(d_vol && h_levels, VR_ERR_NULL, "vr_threshold_downsample: NULL pointer");
    VR_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1 && nx < (1 << 30) && ny < (1 << 30) && nz < (1 << 30),
               VR_ERR_DIMS, "vr_threshold_downsample: dims %lld x %lld x %lld", (long long)nx,
               (long long)ny, (long long)nz);
    VR_REQUIRE(n_levels >= 1 && n_levels <= VR_MAX_LEVELS, VR_ERR_RANGE,
               "vr_threshold_downsample: n_levels %d outside [1, %d]", n_levels, VR_MAX_LEVELS);
    // dims of every level
    int dims[VR_MAX_LEVELS][3];
    for (int k = 1; k <= VR_MAX_LEVELS; ++k) {
        const int64_t d = int64_t(1) << k;
        dims[k - 1][0] = (int)((nx + d - 1) / d);
        dims[k - 1][1] = (int)((ny + d - 1) / d);
        dims[k - 1][2] = (int)((nz + d - 1) / d);
    }
    for (int k = 1; k <= n_levels; ++k)
        VR_REQUIRE(h_levels[k - 1] != nullptr, VR_ERR_NULL, "vr_threshold_downsample: level %d pointer is NULL", k);
    // levels past the fourth are summed from the exact level-4 sums, which go to h_level_sums[3]
    VR_REQUIRE(n_levels <= kFusedLevels || (h_level_sums != nullptr && h_level_sums[kFusedLevels - 1] != nullptr),
               VR_ERR_NULL, "vr_threshold_downsample: %d levels need the level-4 sums buffer h_level_sums[3]",
               n_levels);
    const int fused = std::min(n_levels, kFusedLevels);
    LevelOut L{};
    bool sums = false;
    for (int k = 1; k <= kFusedLevels; ++k) {
        L.nx[k - 1] = dims[k - 1][0];
        L.ny[k - 1] = dims[k - 1][1];
        L.nz[k - 1] = dims[k - 1][2];
        L.p[k - 1] = k <= fused ? h_levels[k - 1] : nullptr;
        L.sums[k - 1] = (k <= fused && h_level_sums) ? h_level_sums[k - 1] : nullptr;
        sums = sums || L.sums[k - 1] != nullptr;
    }
    L.atlas = nullptr;
    L.atlas_level = 0;
    hipStream_t s = vr::as_stream(stream);
    if (atlas != nullptr) {
        VR_REQUIRE(atlas->data != nullptr, VR_ERR_NULL, "vr_threshold_downsample: atlas data is NULL");
        VR_REQUIRE(atlas->level >= 1 && atlas->level <= n_levels, VR_ERR_RANGE,
                   "vr_threshold_downsample: atlas level %d not among levels 1..%d", atlas->level, n_levels);
        VR_REQUIRE(atlas->out_bits == 8 || atlas->out_bits == 16, VR_ERR_RANGE,
                   "vr_threshold_downsample: atlas out_bits %d", atlas->out_bits);
        const int i = atlas->level - 1;
        VR_REQUIRE(atlas->tiles_x >= 1 && atlas->tiles_y >= 1 &&
                       (int64_t)atlas->tiles_x * atlas->tiles_y >= dims[i][2],
                   VR_ERR_RANGE, "vr_threshold_downsample: %d x %d atlas tiles cannot hold %d slices",
                   atlas->tiles_x, atlas->tiles_y, dims[i][2]);
        if (atlas->level <= kFusedLevels) {
            L.atlas = atlas->data;
            L.atlas_level = atlas->level;
            L.atlas_tiles_x = atlas->tiles_x;
            L.atlas_bits = atlas->out_bits;
        }
        const int unused = atlas->tiles_x * atlas->tiles_y - dims[i][2];
        if (unused > 0) {
            const int64_t cnt = (int64_t)unused * dims[i][0] * dims[i][1];
            const int64_t g = std::max<int64_t>(1, std::min<int64_t>((int64_t)vr::num_cus() * 4, vr::ceil_div<int64_t>(cnt, kThreads)));
            zero_tiles<<<(unsigned)g, kThreads, 0, s>>>(atlas->data, atlas->out_bits,
                                                        (int64_t)atlas->tiles_x * dims[i][0], atlas->tiles_x,
                                                        dims[i][0], dims[i][1], dims[i][2], unused);
            int rc = vr::check_launch("vr_threshold_downsample: atlas tiles");
            if (rc) return rc;
        }
    }
    // 16-byte row loads need 8-voxel rows on a 16-byte base; whole 4-value level-1 stores need
    // a level-1 row of a multiple of 4 on an 8-byte base and no atlas of level 1
    const int aligned = (nx % 8 == 0) && ((reinterpret_cast<uintptr_t>(d_vol) & 15u) == 0);
    const int aligned_out = (L.nx[0] % 4 == 0) && ((reinterpret_cast<uintptr_t>(L.p[0]) & 7u) == 0) &&
                            L.atlas_level != 1;
    // 32-bit level-2 pairs: even level-2 rows on a 4-byte base, and a 16-bit atlas
    // on a 4-byte base when level 2 is the atlas level
    L.pair2 = fused >= 2 && L.nx[1] % 2 == 0 && ((reinterpret_cast<uintptr_t>(L.p[1]) & 3u) == 0) &&
              (L.atlas_level != 2 ||
               (L.atlas_bits == 16 && (reinterpret_cast<uintptr_t>(L.atlas) & 3u) == 0));
    const int tiles_x = (int)((nx + WX - 1) / WX), tiles_y = (int)((ny + TY - 1) / TY);
    const int64_t tiles = (int64_t)tiles_x * tiles_y * ((nz + TZ - 1) / TZ);
    VR_REQUIRE(tiles < (int64_t(1) << 31), VR_ERR_DIMS, "vr_threshold_downsample: volume too large");
    // one resident round of workgroups (as many per compute unit as registers and LDS allow)
    static const int per_cu[2][2] = {{occupancy<false, false>(), occupancy<false, true>()},
                                     {occupancy<true, false>(), occupancy<true, true>()}};
    int64_t grid = (int64_t)vr::num_cus() * per_cu[d_circle ? 1 : 0][sums ? 1 : 0];
    if (grid > tiles) grid = tiles;
    auto launch = [&](auto disc, auto with_sums) {
        constexpr bool D = decltype(disc)::value, SU = decltype(with_sums)::value;
        downsample_kernel<D, SU><<<(unsigned)grid, WT, 0, s>>>(d_vol, (int)nx, (int)ny, (int)nz, aligned,
                                                               aligned_out, d_keep_bits, fused, L, tiles_x, tiles_y,
                                                               (int)tiles, d_circle);
    };
    using T_ = std::true_type;
    using F_ = std::false_type;
    if (d_circle) {
        if (sums) launch(T_{}, T_{});
        else launch(T_{}, F_{});
    } else {
        if (sums) launch(F_{}, T_{});
        else launch(F_{}, F_{});
    }
    int rc = vr::check_launch("vr_threshold_downsample");
    if (rc || n_levels <= kFusedLevels) return rc;
    // levels 5..n_levels from the level-4 sums
    CoarseOut C{};
    C.s4 = h_level_sums[kFusedLevels - 1];
    C.n4x = dims[kFusedLevels - 1][0];
    C.n4y = dims[kFusedLevels - 1][1];
    C.n4z = dims[kFusedLevels - 1][2];
    C.n_coarse = n_levels - kFusedLevels;
    C.first[0] = 0;
    for (int i = 0; i < C.n_coarse; ++i) {
        const int k = kFusedLevels + 1 + i;
        C.p[i] = h_levels[k - 1];
        C.sums[i] = h_level_sums[k - 1];
        C.nx[i] = dims[k - 1][0];
        C.ny[i] = dims[k - 1][1];
        C.nz[i] = dims[k - 1][2];
        C.first[i + 1] = C.first[i] + (int64_t)C.nx[i] * C.ny[i] * C.nz[i];
    }
    VR_REQUIRE(C.first[C.n_coarse] < (int64_t(1) << 31), VR_ERR_DIMS, "vr_threshold_downsample: volume too large");
    if (atlas != nullptr && atlas->level > kFusedLevels) {
        C.atlas = atlas->data;
        C.atlas_level = atlas->level;
        C.atlas_tiles_x = atlas->tiles_x;
        C.atlas_bits = atlas->out_bits;
    }
    coarse_kernel<<<(unsigned)C.first[C.n_coarse], CT, 0, s>>>(C);
    return vr::check_launch("vr_threshold_downsample: levels past the fourth");
}

}  // namespace

extern "C" int vr_threshold_downsample(const uint16_t* d_vol, int64_t nx, int64_t ny, int64_t nz,
                                       const uint32_t* d_keep_bits, int n_levels,
                                       uint16_t* const* h_levels, uint64_t* const* h_level_sums,
                                       const vr_atlas_spec* atlas, void* stream)
{
    vr::clear_error();
    return downsample(d_vol, nx, ny, nz, d_keep_bits, nullptr, n_levels, h_levels, h_level_sums, atlas, stream);
}

extern "C" int vr_threshold_downsample_in_disc(const uint16_t* d_vol, int64_t nx, int64_t ny, int64_t nz,
                                               const uint32_t* d_keep_bits, const int32_t* d_circle,
                                               int n_levels, uint16_t* const* h_levels,
                                               uint64_t* const* h_level_sums, const vr_atlas_spec* atlas,
                                               void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_circle != nullptr, VR_ERR_NULL, "vr_threshold_downsample_in_disc: d_circle is NULL");
    VR_REQUIRE(nx <= kMaxDiscSide && ny <= kMaxDiscSide, VR_ERR_DIMS,
               "vr_threshold_downsample_in_disc: slices of %lld x %lld exceed %d x %d", (long long)nx,
               (long long)ny, kMaxDiscSide, kMaxDiscSide);
    return downsample(d_vol, nx, ny, nz, d_keep_bits, d_circle, n_levels, h_levels, h_level_sums, atlas, stream);
}
