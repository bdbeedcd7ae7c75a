// Hollow data preview (Section II: the data preview keeps the object's outer
// geometry and drops its interior volume).  A non-zero voxel is kept when a
// voxel within city-block distance t of it is zero or lies outside the
// volume (the shell that t erosions with the 6-neighbourhood take away);
// every other voxel becomes 0.
//
// A workgroup owns a 32 x 8 x 8 tile.  It stages the tile and a halo of t
// voxels in LDS (0 outside the volume), then computes the city-block distance
// to the nearest zero, capped at t + 1, in three separable passes: along x
// for every halo row, along y for the tile's columns over the halo in z,
// then along z for the tile.  Capping keeps the decision "distance <= t"
// exact: a path of length <= t never passes through a capped value, and each
// axis step of such a path is at most t.  The volume is read once from HBM
// (halos come again from L2) and written once: the kernel is HBM-bound.
#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kTX = 32, kTY = 8, kTZ = 8;

template <int T>
struct HollowLds {
    static constexpr int RX = kTX + 2 * T, RY = kTY + 2 * T, RZ = kTZ + 2 * T;
    uint16_t v[RZ][RY][RX];     // tile and halo, 0 outside the volume
    uint8_t dx[RZ][RY][kTX];    // distance to background along x, capped at T + 1
    uint8_t dy[RZ][kTY][kTX];   // then along y
};

// Workgroup ids are dealt round-robin over the 8 XCDs; tile b of the launch
// order runs where the neighbouring tiles whose halos it shares run.
__device__ __forceinline__ int tile_of_block(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x * q + min(x, r) + i;
}

__global__ void zero_count(unsigned long long* c) { *c = 0ull; }

template <int T>
__global__ void __launch_bounds__(kThreads)
hollow_kernel(const uint16_t* __restrict__ src, int nx, int ny, int nz, int tiles_x, int tiles_y, int n_tiles,
              uint16_t* __restrict__ dst, unsigned long long* __restrict__ kept)
{
    using H = HollowLds<T>;
    __shared__ H L;
    __shared__ uint32_t wsum[kThreads / 64];
    constexpr int F = T + 1;
    const int b = tile_of_block((int)blockIdx.x, n_tiles);
    const int tx = b % tiles_x, tyz = b / tiles_x, ty = tyz % tiles_y, tz = tyz / tiles_y;
    const int x0 = tx * kTX - T, y0 = ty * kTY - T, z0 = tz * kTZ - T;   // region origin

    for (int q = threadIdx.x; q < H::RX * H::RY * H::RZ; q += kThreads) {
        const int rx = q % H::RX, r = q / H::RX, ry = r % H::RY, rz = r / H::RY;
        const int x = x0 + rx, y = y0 + ry, z = z0 + rz;
        uint16_t v = 0;
        if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz) v = src[((int64_t)z * ny + y) * nx + x];
        L.v[rz][ry][rx] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kTX * H::RY * H::RZ; q += kThreads) {
        const int ix = q % kTX, r = q / kTX, ry = r % H::RY, rz = r / H::RY;
        int d = F;
#pragma unroll
        for (int k = -T; k <= T; ++k)
            if (L.v[rz][ry][ix + T + k] == 0) d = min(d, k < 0 ? -k : k);
        L.dx[rz][ry][ix] = (uint8_t)d;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kTX * kTY * H::RZ; q += kThreads) {
        const int ix = q % kTX, r = q / kTX, iy = r % kTY, rz = r / kTY;
        int d = F;
#pragma unroll
        for (int k = -T; k <= T; ++k) d = min(d, (int)L.dx[rz][iy + T + k][ix] + (k < 0 ? -k : k));
        L.dy[rz][iy][ix] = (uint8_t)d;
    }
    __syncthreads();
    uint32_t n_keep = 0;
    for (int q = threadIdx.x; q < kTX * kTY * kTZ; q += kThreads) {
        const int ix = q % kTX, r = q / kTX, iy = r % kTY, iz = r / kTY;
        const int x = x0 + T + ix, y = y0 + T + iy, z = z0 + T + iz;
        if (x >= nx || y >= ny || z >= nz) continue;
        int d = F;
#pragma unroll
        for (int k = -T; k <= T; ++k) d = min(d, (int)L.dy[iz + T + k][iy][ix] + (k < 0 ? -k : k));
        const uint16_t v = L.v[iz + T][iy + T][ix + T];
        const bool keep = v != 0 && d <= T;
        dst[((int64_t)z * ny + y) * nx + x] = keep ? v : (uint16_t)0;
        n_keep += keep ? 1u : 0u;
    }
    if (kept == nullptr) return;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) n_keep += __shfl_xor(n_keep, off);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = n_keep;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) s += wsum[w];
        if (s) atomicAdd(kept, s);
    }
}

template <int T>
void launch(unsigned blocks, hipStream_t s, const uint16_t* src, int nx, int ny, int nz, int tiles_x, int tiles_y,
            uint16_t* dst, unsigned long long* kept)
{
    hollow_kernel<T><<<blocks, kThreads, 0, s>>>(src, nx, ny, nz, tiles_x, tiles_y, (int)blocks, dst, kept);
}

}  // namespace

extern "C" int vr_hollow(const uint16_t* d_src, int64_t nx, int64_t ny, int64_t nz, int thickness,
                         uint16_t* d_dst, uint64_t* d_kept, void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_src && d_dst, VR_ERR_NULL, "vr_hollow: NULL volume");
    VR_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1 && nx < (1 << 30) && ny < (1 << 30) && nz < (1 << 30), VR_ERR_DIMS,
               "vr_hollow: dims %lld x %lld x %lld", (long long)nx, (long long)ny, (long long)nz);
    VR_REQUIRE(thickness >= 1 && thickness <= VR_HOLLOW_MAX_THICKNESS, VR_ERR_RANGE,
               "vr_hollow: thickness %d outside [1, %d]", thickness, VR_HOLLOW_MAX_THICKNESS);
    const int64_t n = nx * ny * nz;
    const uintptr_t s0 = reinterpret_cast<uintptr_t>(d_src), d0 = reinterpret_cast<uintptr_t>(d_dst);
    VR_REQUIRE(d0 + 2 * (uint64_t)n <= s0 || s0 + 2 * (uint64_t)n <= d0, VR_ERR_RANGE,
               "vr_hollow: d_dst overlaps d_src");
    const int64_t tiles_x = (nx + kTX - 1) / kTX, tiles_y = (ny + kTY - 1) / kTY, tiles_z = (nz + kTZ - 1) / kTZ;
    const int64_t tiles = tiles_x * tiles_y * tiles_z;
    VR_REQUIRE(tiles < (int64_t(1) << 31), VR_ERR_DIMS, "vr_hollow: volume too large");
    hipStream_t s = vr::as_stream(stream);
    auto* kept = reinterpret_cast<unsigned long long*>(d_kept);
    if (kept) {
        zero_count<<<1, 1, 0, s>>>(kept);
        const int rc = vr::check_launch("vr_hollow: count");
        if (rc) return rc;
    }
    const unsigned nb = (unsigned)tiles;
    const int ix = (int)nx, iy = (int)ny, iz = (int)nz, tx = (int)tiles_x, ty = (int)tiles_y;
    switch (thickness) {
    case 1: launch<1>(nb, s, d_src, ix, iy, iz, tx, ty, d_dst, kept); break;
    case 2: launch<2>(nb, s, d_src, ix, iy, iz, tx, ty, d_dst, kept); break;
    case 3: launch<3>(nb, s, d_src, ix, iy, iz, tx, ty, d_dst, kept); break;
    case 4: launch<4>(nb, s, d_src, ix, iy, iz, tx, ty, d_dst, kept); break;
    case 5: launch<5>(nb, s, d_src, ix, iy, iz, tx, ty, d_dst, kept); break;
    case 6: launch<6>(nb, s, d_src, ix, iy, iz, tx, ty, d_dst, kept); break;
    case 7: launch<7>(nb, s, d_src, ix, iy, iz, tx, ty, d_dst, kept); break;
    default: launch<8>(nb, s, d_src, ix, iy, iz, tx, ty, d_dst, kept); break;
    }
    return vr::check_launch("vr_hollow");
}
