// Device-side pieces of the fused threshold + pyramid pass shared by the
// single-volume kernel and the batched persistent kernel: level and atlas
// stores, the keep-mask interval test, and one 64 x 16 x 16 tile.
#pragma once

#include "common.h"

namespace vr {
namespace ds {

constexpr int kThreads = 256;      // threads of one tile group
constexpr int TX = 64, TY = 16, TZ = 16;
constexpr int kFusedLevels = 4;    // levels the streaming pass writes itself

struct LevelOut {
    uint16_t* p[kFusedLevels];
    int nx[kFusedLevels], ny[kFusedLevels], nz[kFusedLevels];
    uint64_t* sums[kFusedLevels];   // exact level sums (NULL: not written)
    // optional slicemap atlas of one level, written beside it
    void* atlas;
    int atlas_level, atlas_tiles_x, atlas_bits;
    int pair2;   // level 2 (and its atlas copy) may be stored as aligned voxel pairs
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// streaming 16-byte load: the volume is read once
__device__ __forceinline__ uint4 load_stream(const uint16_t* p)
{
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ void store_atlas(const LevelOut& L, int i, int x, int y, int z, uint16_t v)
{
    const int tx = z % L.atlas_tiles_x, ty = z / L.atlas_tiles_x;
    const int64_t W = (int64_t)L.atlas_tiles_x * L.nx[i];
    const int64_t a = ((int64_t)ty * L.ny[i] + y) * W + (int64_t)tx * L.nx[i] + x;
    if (L.atlas_bits == 16) {
        static_cast<uint16_t*>(L.atlas)[a] = v;
    } else {
        const uint32_t b = ((uint32_t)v + 128u) >> 8;
        static_cast<uint8_t*>(L.atlas)[a] = (uint8_t)(b > 255u ? 255u : b);
    }
}

template <bool INTERVAL>
__device__ __forceinline__ uint32_t keepv(const uint32_t* bits, uint32_t v, uint32_t T)
{
    if (INTERVAL) return v >= T ? v : 0u;
    return ((bits[v >> 5] >> (v & 31u)) & 1u) ? v : 0u;
}

__device__ __forceinline__ uint16_t round_level(uint32_t s, int k)
{
    return (uint16_t)((s + (1u << (3 * k - 1))) >> (3 * k));
}

__device__ __forceinline__ void store_level(const LevelOut& L, int k, int x, int y, int z, uint32_t s)
{
    const int i = k - 1;
    if (x < L.nx[i] && y < L.ny[i] && z < L.nz[i]) {
        const uint16_t v = round_level(s, k);
        L.p[i][((int64_t)z * L.ny[i] + y) * L.nx[i] + x] = v;
        if (k == L.atlas_level) store_atlas(L, i, x, y, z, v);
    }
}

// Per-tile LDS of a 256-thread group.
struct TileLds {
    uint32_t s1[TZ / 2][TY / 2][TX / 2];
    uint32_t s2[TZ / 4][TY / 4][TX / 4];
    uint32_t s3[TZ / 8][TY / 8][TX / 8];
};

// One 64 x 16 x 16 tile by a group of kThreads threads (thread `tid` of the
// group).  Inactive groups (active == false) take the same barriers so that
// several groups can share a workgroup.
template <bool INTERVAL>
__device__ inline void tile_body(const uint16_t* __restrict__ vol, int nx, int ny, int nz, int aligned,
                                 const uint32_t* bits, uint32_t T, int n_levels, const LevelOut& L,
                                 int tiles_x, int tiles_y, int tile, bool active, int tid, TileLds& G)
{
    auto& s1 = G.s1;
    auto& s2 = G.s2;
    auto& s3 = G.s3;
    {
        const int tx = tile % tiles_x;
        const int ty = (tile / tiles_x) % tiles_y;
        const int tz = tile / (tiles_x * tiles_y);
        const int X0 = tx * TX, Y0 = ty * TY, Z0 = tz * TZ;
        const bool interior = aligned && X0 + TX <= nx && Y0 + TY <= ny && Z0 + TZ <= nz;

        uint32_t v[2][4][8];
        if (active) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int item = tid + kThreads * j;
            const int c = item & 7, yp = (item >> 3) & 7, zp = item >> 6;
            const int x = X0 + 8 * c;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int y = Y0 + 2 * yp + (r & 1), z = Z0 + 2 * zp + (r >> 1);
                const uint16_t* row = vol + ((int64_t)z * ny + y) * nx;
                if (interior) {
                    const uint4 q = load_stream(row + x);
                    v[j][r][0] = q.x & 0xFFFFu; v[j][r][1] = q.x >> 16;
                    v[j][r][2] = q.y & 0xFFFFu; v[j][r][3] = q.y >> 16;
                    v[j][r][4] = q.z & 0xFFFFu; v[j][r][5] = q.z >> 16;
                    v[j][r][6] = q.w & 0xFFFFu; v[j][r][7] = q.w >> 16;
                } else if (y < ny && z < nz && x + 8 <= nx) {
                    // a whole piece of a row whose start is only 2-byte aligned: one
                    // 16-byte load (the device runs with unaligned access enabled)
                    typedef uint4 u32x4_a2 __attribute__((aligned(2)));
                    const uint4 q = *reinterpret_cast<const u32x4_a2*>(row + x);
                    v[j][r][0] = q.x & 0xFFFFu; v[j][r][1] = q.x >> 16;
                    v[j][r][2] = q.y & 0xFFFFu; v[j][r][3] = q.y >> 16;
                    v[j][r][4] = q.z & 0xFFFFu; v[j][r][5] = q.z >> 16;
                    v[j][r][6] = q.w & 0xFFFFu; v[j][r][7] = q.w >> 16;
                } else {
                    const bool rowok = y < ny && z < nz;
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        v[j][r][e] = (rowok && x + e < nx) ? (uint32_t)row[x + e] : 0u;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int item = tid + kThreads * j;
            const int c = item & 7, yp = (item >> 3) & 7, zp = item >> 6;
            uint32_t s[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t acc = 0;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc += keepv<INTERVAL>(bits, v[j][r][2 * q], T) + keepv<INTERVAL>(bits, v[j][r][2 * q + 1], T);
                s[q] = acc;
            }
            const int x1 = (X0 >> 1) + 4 * c, y1 = (Y0 >> 1) + yp, z1 = (Z0 >> 1) + zp;
            if (interior && (L.nx[0] & 3) == 0 && L.atlas_level != 1) {
                uint2 w;
                w.x = (uint32_t)round_level(s[0], 1) | ((uint32_t)round_level(s[1], 1) << 16);
                w.y = (uint32_t)round_level(s[2], 1) | ((uint32_t)round_level(s[3], 1) << 16);
                *reinterpret_cast<uint2*>(L.p[0] + ((int64_t)z1 * L.ny[0] + y1) * L.nx[0] + x1) = w;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) store_level(L, 1, x1 + q, y1, z1, s[q]);
            }
            if (n_levels > 1) {
#pragma unroll
                for (int q = 0; q < 4; ++q) s1[zp][yp][4 * c + q] = s[q];
            }
        }
        }   // active
        if (n_levels > 1) {
            __syncthreads();
            if (active) {   // level 2: 16 x 4 x 4 outputs, one per thread
                const int x = tid & 15, y = (tid >> 4) & 3, z = tid >> 6;
                uint32_t acc = 0;
#pragma unroll
                for (int d = 0; d < 8; ++d)
                    acc += s1[2 * z + (d >> 2)][2 * y + ((d >> 1) & 1)][2 * x + (d & 1)];
                store_level(L, 2, (X0 >> 2) + x, (Y0 >> 2) + y, (Z0 >> 2) + z, acc);
                s2[z][y][x] = acc;
            }
            if (n_levels > 2) {
                __syncthreads();
                if (active && tid < 32) {   // level 3: 8 x 2 x 2
                    const int x = tid & 7, y = (tid >> 3) & 1, z = tid >> 4;
                    uint32_t acc = 0;
#pragma unroll
                    for (int d = 0; d < 8; ++d)
                        acc += s2[2 * z + (d >> 2)][2 * y + ((d >> 1) & 1)][2 * x + (d & 1)];
                    store_level(L, 3, (X0 >> 3) + x, (Y0 >> 3) + y, (Z0 >> 3) + z, acc);
                    s3[z][y][x] = acc;
                }
                if (n_levels > 3) {
                    __syncthreads();
                    if (active && tid < 4) {   // level 4: 4 x 1 x 1
                        uint32_t acc = 0;
#pragma unroll
                        for (int d = 0; d < 8; ++d)
                            acc += s3[d >> 2][(d >> 1) & 1][2 * tid + (d & 1)];
                        store_level(L, 4, (X0 >> 4) + tid, Y0 >> 4, Z0 >> 4, acc);
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Copy the keep mask into LDS and find whether it is one interval
// [first, 65535]: returns first, or a value > 65536 when it is not.
__device__ inline uint32_t load_mask(const uint32_t* __restrict__ keep_bits, uint32_t* bits,
                                     uint32_t& s_first, uint32_t& s_bad)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) { s_first = VR_NBINS; s_bad = 0; }
    __syncthreads();
    for (int w = tid; w < VR_KEEP_WORDS; w += nt) {
        const uint32_t x = keep_bits[w];
        bits[w] = x;
        if (x) atomicMin(&s_first, (uint32_t)w * 32u + (uint32_t)__builtin_ctz(x));
    }
    __syncthreads();
    const uint32_t first = s_first;
    for (int w = tid; w < VR_KEEP_WORDS; w += nt) {
        const uint32_t lo = (uint32_t)w * 32u;
        const uint32_t want = lo + 32u <= first ? 0u : (lo >= first ? 0xFFFFFFFFu : (0xFFFFFFFFu << (first - lo)));
        if (bits[w] != want) s_bad = 1u;
    }
    __syncthreads();
    return s_bad ? 0xFFFFFFFFu : first;
}

}  // namespace ds
}  // namespace vr
