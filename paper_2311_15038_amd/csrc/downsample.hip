// Thresholding fused with the multi-resolution pyramid (Sections II, III-A,
// III-D): one streaming pass over the u16 volume writes up to four box-mean
// levels, each rounded from its own exact integer sum.
//
// A workgroup (256 threads) walks 64 x 16 x 16-voxel tiles.  Each thread owns
// two 8-voxel x-runs of a 2 x 2 (y, z) pair of rows: it loads 4 x 16 bytes per
// run (adjacent threads read adjacent 16-byte pieces of a 128-byte row), looks
// every voxel up in the keep mask held in LDS, and forms four level-1 sums.
// Level-k sums for k > 1 are reduced from the level-1 sums in LDS.  When the
// keep mask is one interval [T, 65535] (a plain threshold, or a top-slice
// filter that removed nothing above T) a voxel is kept by a compare instead
// of the LDS lookup; each workgroup detects that once from the mask.
#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr int TX = 64, TY = 16, TZ = 16;

struct LevelOut {
    uint16_t* p[VR_MAX_LEVELS];
    int nx[VR_MAX_LEVELS], ny[VR_MAX_LEVELS], nz[VR_MAX_LEVELS];
    // optional slicemap atlas of one level, written beside it
    void* atlas;
    int atlas_level, atlas_tiles_x, atlas_bits;
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

template <bool INTERVAL>
__device__ void tiles(const uint16_t* __restrict__ vol, int nx, int ny, int nz, int aligned,
                      const uint32_t* bits, uint32_t T, int n_levels, const LevelOut& L,
                      int tiles_x, int tiles_y, int n_tiles, uint32_t (*s1)[TY / 2][TX / 2],
                      uint32_t (*s2)[TY / 4][TX / 4], uint32_t (*s3)[TY / 8][TX / 8])
{
    const int tid = threadIdx.x;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int tx = tile % tiles_x;
        const int ty = (tile / tiles_x) % tiles_y;
        const int tz = tile / (tiles_x * tiles_y);
        const int X0 = tx * TX, Y0 = ty * TY, Z0 = tz * TZ;
        const bool interior = aligned && X0 + TX <= nx && Y0 + TY <= ny && Z0 + TZ <= nz;

        uint32_t v[2][4][8];
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
        if (n_levels > 1) {
            __syncthreads();
            {   // level 2: 16 x 4 x 4 outputs, one per thread
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
                if (tid < 32) {   // level 3: 8 x 2 x 2
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
                    if (tid < 4) {   // level 4: 4 x 1 x 1
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

__global__ void __launch_bounds__(kThreads)
downsample_kernel(const uint16_t* __restrict__ vol, int nx, int ny, int nz, int aligned,
                  const uint32_t* __restrict__ keep_bits, int n_levels, LevelOut L, int tiles_x,
                  int tiles_y, int n_tiles)
{
    __shared__ uint32_t bits[VR_KEEP_WORDS];
    __shared__ uint32_t s1[TZ / 2][TY / 2][TX / 2];
    __shared__ uint32_t s2[TZ / 4][TY / 4][TX / 4];
    __shared__ uint32_t s3[TZ / 8][TY / 8][TX / 8];
    __shared__ uint32_t s_first, s_bad;
    const int tid = threadIdx.x;
    if (keep_bits == nullptr) {
        tiles<true>(vol, nx, ny, nz, aligned, bits, 0u, n_levels, L, tiles_x, tiles_y, n_tiles, s1, s2, s3);
        return;
    }
    if (tid == 0) { s_first = VR_NBINS; s_bad = 0; }
    __syncthreads();
    for (int w = tid; w < VR_KEEP_WORDS; w += kThreads) {
        const uint32_t x = keep_bits[w];
        bits[w] = x;
        if (x) atomicMin(&s_first, (uint32_t)w * 32u + (uint32_t)__builtin_ctz(x));
    }
    __syncthreads();
    // is the mask exactly the interval [first, 65535]?
    const uint32_t first = s_first;
    for (int w = tid; w < VR_KEEP_WORDS; w += kThreads) {
        const uint32_t lo = (uint32_t)w * 32u;
        const uint32_t want = lo + 32u <= first ? 0u : (lo >= first ? 0xFFFFFFFFu : (0xFFFFFFFFu << (first - lo)));
        if (bits[w] != want) s_bad = 1u;
    }
    __syncthreads();
    if (s_bad == 0u)
        tiles<true>(vol, nx, ny, nz, aligned, bits, first, n_levels, L, tiles_x, tiles_y, n_tiles, s1, s2, s3);
    else
        tiles<false>(vol, nx, ny, nz, aligned, bits, 0u, n_levels, L, tiles_x, tiles_y, n_tiles, s1, s2, s3);
}

}  // namespace

extern "C" int vr_threshold_downsample(const uint16_t* d_vol, int64_t nx, int64_t ny, int64_t nz,
                                       const uint32_t* d_keep_bits, int n_levels,
                                       uint16_t* const* h_levels, const vr_atlas_spec* atlas,
                                       void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_vol && h_levels, VR_ERR_NULL, "vr_threshold_downsample: NULL pointer");
    VR_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1 && nx < (1 << 30) && ny < (1 << 30) && nz < (1 << 30),
               VR_ERR_DIMS, "vr_threshold_downsample: dims %lld x %lld x %lld", (long long)nx,
               (long long)ny, (long long)nz);
    VR_REQUIRE(n_levels >= 1 && n_levels <= VR_MAX_LEVELS, VR_ERR_RANGE,
               "vr_threshold_downsample: n_levels %d outside [1, %d]", n_levels, VR_MAX_LEVELS);
    LevelOut L{};
    for (int k = 1; k <= VR_MAX_LEVELS; ++k) {
        const int64_t d = int64_t(1) << k;
        L.nx[k - 1] = (int)((nx + d - 1) / d);
        L.ny[k - 1] = (int)((ny + d - 1) / d);
        L.nz[k - 1] = (int)((nz + d - 1) / d);
        if (k <= n_levels) {
            VR_REQUIRE(h_levels[k - 1] != nullptr, VR_ERR_NULL,
                       "vr_threshold_downsample: level %d pointer is NULL", k);
            L.p[k - 1] = h_levels[k - 1];
        } else {
            L.p[k - 1] = nullptr;
        }
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
                       (int64_t)atlas->tiles_x * atlas->tiles_y >= L.nz[i],
                   VR_ERR_RANGE, "vr_threshold_downsample: %d x %d atlas tiles cannot hold %d slices",
                   atlas->tiles_x, atlas->tiles_y, L.nz[i]);
        L.atlas = atlas->data;
        L.atlas_level = atlas->level;
        L.atlas_tiles_x = atlas->tiles_x;
        L.atlas_bits = atlas->out_bits;
        const int unused = atlas->tiles_x * atlas->tiles_y - L.nz[i];
        if (unused > 0) {
            const int64_t cnt = (int64_t)unused * L.nx[i] * L.ny[i];
            const int64_t g = std::max<int64_t>(1, std::min<int64_t>((int64_t)vr::num_cus() * 4, vr::ceil_div<int64_t>(cnt, kThreads)));
            zero_tiles<<<(unsigned)g, kThreads, 0, s>>>(atlas->data, atlas->out_bits,
                                                        (int64_t)atlas->tiles_x * L.nx[i], atlas->tiles_x,
                                                        L.nx[i], L.ny[i], L.nz[i], unused);
            int rc = vr::check_launch("vr_threshold_downsample: atlas tiles");
            if (rc) return rc;
        }
    }
    const int aligned = (nx % 8 == 0) && ((reinterpret_cast<uintptr_t>(d_vol) & 15u) == 0) &&
                        ((reinterpret_cast<uintptr_t>(L.p[0]) & 7u) == 0);
    const int tiles_x = (int)((nx + TX - 1) / TX), tiles_y = (int)((ny + TY - 1) / TY);
    const int64_t tiles = (int64_t)tiles_x * tiles_y * ((nz + TZ - 1) / TZ);
    VR_REQUIRE(tiles < (int64_t(1) << 31), VR_ERR_DIMS, "vr_threshold_downsample: volume too large");
    int64_t grid = (int64_t)vr::num_cus() * 8;
    if (grid > tiles) grid = tiles;
    downsample_kernel<<<(unsigned)grid, kThreads, 0, s>>>(
        d_vol, (int)nx, (int)ny, (int)nz, aligned, d_keep_bits, n_levels, L, tiles_x, tiles_y,
        (int)tiles);
    return vr::check_launch("vr_threshold_downsample");
}
