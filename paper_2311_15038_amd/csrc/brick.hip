// Render layout of a volume level: 4 x 4 x 4-voxel bricks (a 128-byte line
// for u16) and an occupancy grid that tells the ray caster where every tap of
// a trilinear fetch is zero.
//
// Brick (bx, by, bz) starts at element ((bz * nby + by) * nbx + bx) * 64 and
// voxel (x, y, z) sits at ((z & 3) * 16 + (y & 3) * 4 + (x & 3)) inside it.
// occupancy[b] != 0 iff some non-zero voxel is one of the eight taps of a
// trilinear fetch whose base tap (the floor corner, clamped to the volume)
// lies in brick b; a voxel at (x, y, z) is a tap for base taps
// (x - {0,1}, y - {0,1}, z - {0,1}), so it marks up to eight bricks.  A second
// grid follows the first: one byte per 4 x 4 x 4 bricks (16^3 voxels), set
// when any of its bricks is marked, so a ray can cross large empty regions in
// long steps.
#include "common.h"

namespace {

constexpr int kThreads = 256;

__global__ void __launch_bounds__(kThreads) fill_u8(uint8_t* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        p[i] = 0;
}

template <typename T>
__device__ __forceinline__ bool nonzero(T v) { return v != (T)0; }

// A workgroup converts a 64 x 4 x 4-voxel slab (16 bricks along x) at brick
// row (by, bz): thread t reads 4 voxels of volume row (t / 16) at x offset
// 4 (t % 16), which is row t / 16 of brick t % 16.  The slab goes through LDS
// in brick order so that stores are 16-byte pieces of whole bricks.  The
// occupancy marks of the slab (its 16 bricks and the neighbours at -1 in x, y
// and z) are gathered in LDS and written once per workgroup.
template <typename T>
__global__ void __launch_bounds__(kThreads)
brick_kernel(const T* __restrict__ src, int nx, int ny, int nz, int nbx, int nby,
             T* __restrict__ dst, uint8_t* __restrict__ occ, uint8_t* __restrict__ macro, int nmx,
             int nmy)
{
    __shared__ __align__(16) T slab[16 * 64];
    __shared__ uint32_t marks[17 * 2 * 2];      // (bx - 1 .. bx + 15) x (by - 1, by) x (bz - 1, bz)
    const int t = threadIdx.x;
    const int bx0 = blockIdx.x * 16, by = blockIdx.y, bz = blockIdx.z;
    if (t < 17 * 4) marks[t] = 0;
    __syncthreads();
    const int r = t >> 4, lb = t & 15;          // row inside the brick, brick within the slab
    const int y = by * 4 + (r & 3), z = bz * 4 + (r >> 2), x0 = (bx0 + lb) * 4;
    T v[4];
    const bool rowok = y < ny && z < nz;
    const T* row = src + ((int64_t)z * ny + y) * nx;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (rowok && x0 + e < nx) ? row[x0 + e] : (T)0;
#pragma unroll
    for (int e = 0; e < 4; ++e) slab[lb * 64 + r * 4 + e] = v[e];
    if (occ != nullptr) {
        bool any = false;
#pragma unroll
        for (int e = 0; e < 4; ++e) any |= nonzero(v[e]);
        if (any) {
            // a voxel at x marks the base-tap bricks of x and x - 1 (and likewise in y, z)
            const int xs[2] = {lb + 1, nonzero(v[0]) ? lb : -1};          // index into -1..15 (+1)
            const int ys[2] = {1, (r & 3) == 0 ? 0 : -1};
            const int zs[2] = {1, (r >> 2) == 0 ? 0 : -1};
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        if (xs[a] >= 0 && ys[b] >= 0 && zs[c] >= 0)
                            marks[(zs[c] * 2 + ys[b]) * 17 + xs[a]] = 1u;
        }
    }
    __syncthreads();
    // whole bricks out: 16 bricks x 64 voxels, 16 bytes per store
    constexpr int kPer = 16 / sizeof(T);
    const int nb_here = min(16, nbx - bx0);
    for (int q = t; q < 16 * 64 / kPer; q += kThreads) {
        const int e = q * kPer;
        if (e / 64 < nb_here) {
            const int64_t brick = ((int64_t)bz * nby + by) * nbx + bx0 + e / 64;
            *reinterpret_cast<uint4*>(dst + (brick << 6) + (e & 63)) =
                *reinterpret_cast<const uint4*>(slab + e);
        }
    }
    if (occ != nullptr && t < 17 * 4) {
        const int xi = t % 17, yi = (t / 17) & 1, zi = t / 34;
        const int bx = bx0 + xi - 1, byy = by + yi - 1, bzz = bz + zi - 1;
        if (marks[t] && bx >= 0 && bx < nbx && byy >= 0 && bzz >= 0) {
            occ[((int64_t)bzz * nby + byy) * nbx + bx] = 1;
            macro[((int64_t)(bzz >> 2) * nmy + (byy >> 2)) * nmx + (bx >> 2)] = 1;
        }
    }
}

}  // namespace

extern "C" int vr_brick_count(int64_t nx, int64_t ny, int64_t nz, int64_t* n_bricks,
                              int64_t* occupancy_bytes)
{
    vr::clear_error();
    VR_REQUIRE(n_bricks != nullptr, VR_ERR_NULL, "vr_brick_count: n_bricks is NULL");
    VR_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1 && nx < (1 << 30) && ny < (1 << 30) && nz < (1 << 30),
               VR_ERR_DIMS, "vr_brick_count: dims %lld x %lld x %lld", (long long)nx, (long long)ny,
               (long long)nz);
    const int64_t bx = (nx + 3) / 4, by = (ny + 3) / 4, bz = (nz + 3) / 4;
    *n_bricks = bx * by * bz;
    if (occupancy_bytes) *occupancy_bytes = bx * by * bz + ((bx + 3) / 4) * ((by + 3) / 4) * ((bz + 3) / 4);
    return VR_OK;
}

extern "C" int vr_brick_volume(const void* d_src, int dtype, int64_t nx, int64_t ny, int64_t nz,
                               void* d_bricked, uint8_t* d_occupancy, void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_src && d_bricked, VR_ERR_NULL, "vr_brick_volume: NULL pointer");
    VR_REQUIRE(dtype == VR_U16_NORM || dtype == VR_F32, VR_ERR_DTYPE, "vr_brick_volume: dtype %d",
               dtype);
    VR_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1 && nx < (1 << 30) && ny < (1 << 30) && nz < (1 << 30),
               VR_ERR_DIMS, "vr_brick_volume: dims %lld x %lld x %lld", (long long)nx, (long long)ny,
               (long long)nz);
    const int nbx = (int)((nx + 3) / 4), nby = (int)((ny + 3) / 4), nbz = (int)((nz + 3) / 4);
    const int nmx = (nbx + 3) / 4, nmy = (nby + 3) / 4, nmz = (nbz + 3) / 4;
    const int64_t bricks = (int64_t)nbx * nby * nbz;
    const int64_t occ_bytes = bricks + (int64_t)nmx * nmy * nmz;
    VR_REQUIRE(nby < 65536 && nbz < 65536, VR_ERR_DIMS, "vr_brick_volume: volume too large");
    VR_REQUIRE((reinterpret_cast<uintptr_t>(d_bricked) & 15u) == 0, VR_ERR_RANGE,
               "vr_brick_volume: d_bricked must be 16-byte aligned");
    hipStream_t s = vr::as_stream(stream);
    const int64_t cap = (int64_t)vr::num_cus() * 16;
    if (d_occupancy) {
        const int64_t g = std::min<int64_t>(cap, vr::ceil_div<int64_t>(occ_bytes, kThreads));
        fill_u8<<<(unsigned)std::max<int64_t>(g, 1), kThreads, 0, s>>>(d_occupancy, occ_bytes);
        int rc = vr::check_launch("vr_brick_volume: fill");
        if (rc) return rc;
    }
    const dim3 grid((unsigned)vr::ceil_div(nbx, 16), (unsigned)nby, (unsigned)nbz);
    if (dtype == VR_U16_NORM)
        brick_kernel<uint16_t><<<grid, kThreads, 0, s>>>(
            static_cast<const uint16_t*>(d_src), (int)nx, (int)ny, (int)nz, nbx, nby,
            static_cast<uint16_t*>(d_bricked), d_occupancy,
            d_occupancy ? d_occupancy + bricks : nullptr, nmx, nmy);
    else
        brick_kernel<float><<<grid, kThreads, 0, s>>>(
            static_cast<const float*>(d_src), (int)nx, (int)ny, (int)nz, nbx, nby,
            static_cast<float*>(d_bricked), d_occupancy,
            d_occupancy ? d_occupancy + bricks : nullptr, nmx, nmy);
    return vr::check_launch("vr_brick_volume");
}
