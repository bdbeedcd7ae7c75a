// Render layout of a volume level (layout and occupancy described in brick_dev.h).
#include <type_traits>

#include "brick_dev.h"

namespace {

using namespace vr::bk;

__global__ void __launch_bounds__(kThreads) fill_u8(uint8_t* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        p[i] = 0;
}

// Zeros in 16-byte pieces (the apron: whole bricks, 16-byte aligned).
__global__ void __launch_bounds__(kThreads) fill_16(uint4* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

template <typename T, bool PAIRS, bool VEC>
__global__ void __launch_bounds__(kThreads)
brick_kernel(const T* __restrict__ src, int nx, int ny, int nz, int nbx, int nby,
             typename ElemOf<T, PAIRS>::type* __restrict__ dst, uint8_t* __restrict__ occ,
             uint8_t* __restrict__ macro, int nmx, int nmy, uint32_t above)
{
    __shared__ SlabLds<T, PAIRS> G;
    slab_body<T, PAIRS, VEC>(src, nx, ny, nz, nbx, nby, dst, occ, macro, nmx, nmy, above, blockIdx.x * 16, blockIdx.y,
                        blockIdx.z, true, threadIdx.x, G);
}

// One separable pass of the capped Chebyshev distance over the brick grid:
// out[b] = min over |t| < kDistCap of max(|t|, in(b + t e_axis)), where in(i)
// is 0 for a marked brick and kDistCap otherwise (FROM_OCC, the first pass),
// or the previous pass's value.  Taken over x, then y, then z this is the
// distance min over marked b' of max_a |b_a - b'_a|, capped.  A workgroup is
// 64 x 4 bricks of a z-slice.  Every offset is read (no early exit), so the
// 2 (kDistCap - 1) loads of a brick are in flight together; an offset past
// the grid's edge reads the edge brick instead, whose own term, at a smaller
// offset, is already in the minimum and no smaller than this one.
template <bool FROM_OCC>
__device__ __forceinline__ int dist_in(const uint8_t* __restrict__ in, int64_t i)
{
    return FROM_OCC ? (in[i] != 0 ? 0 : kDistCap) : (int)in[i];
}

template <bool FROM_OCC>
__global__ void __launch_bounds__(256)
dist_pass(const uint8_t* __restrict__ in, uint8_t* __restrict__ out, int nbx, int nby, int nbz, int axis)
{
    const int x = (int)blockIdx.x * 64 + (int)(threadIdx.x & 63);
    const int y = (int)blockIdx.y * 4 + (int)(threadIdx.x >> 6), z = (int)blockIdx.z;
    if (x >= nbx || y >= nby) return;
    const int64_t b = ((int64_t)z * nby + y) * nbx + x;
    const int c = axis == 0 ? x : axis == 1 ? y : z;
    const int na = axis == 0 ? nbx : axis == 1 ? nby : nbz;
    const int64_t st = axis == 0 ? 1 : axis == 1 ? (int64_t)nbx : (int64_t)nbx * nby;
    int best = dist_in<FROM_OCC>(in, b);
#pragma unroll
    for (int t = 1; t < kDistCap; ++t) {
        const int up = min(c + t, na - 1) - c, dn = c - max(c - t, 0);
        best = min(best, max(t, dist_in<FROM_OCC>(in, b + up * st)));
        best = min(best, max(t, dist_in<FROM_OCC>(in, b - dn * st)));
    }
    out[b] = (uint8_t)best;
}

template <bool FROM_OCC>
void launch_dist(hipStream_t s, const uint8_t* in, uint8_t* out, int nbx, int nby, int nbz, int axis)
{
    const dim3 g((unsigned)vr::ceil_div(nbx, 64), (unsigned)vr::ceil_div(nby, 4), (unsigned)nbz);
    dist_pass<FROM_OCC><<<g, 256, 0, s>>>(in, out, nbx, nby, nbz, axis);
}

// 8^3 bricks: one thread per 8-voxel row piece (grid-stride).
template <typename T>
__global__ void __launch_bounds__(kThreads)
brick8_kernel(const T* __restrict__ src, int nx, int ny, int nz, int nbx, int nby, T* __restrict__ dst,
              uint8_t* __restrict__ occ, uint8_t* __restrict__ macro, int nmx, int nmy, uint32_t above)
{
    const int64_t n = (int64_t)nbx * (nby * 8) * ((nz + 7) / 8 * 8);
    for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < n; r += (int64_t)gridDim.x * kThreads)
        row8_body<T>(src, nx, ny, nz, nbx, nby, dst, occ, macro, nmx, nmy, above, r);
}

// Overlap layout: one group of kOvlBricks bricks along x per workgroup.
template <bool VEC>
__global__ void __launch_bounds__(kThreads)
brick_ovl_kernel(const uint16_t* __restrict__ src, int nx, int ny, int nz, int nbx, int nby,
                 uint16_t* __restrict__ dst, uint8_t* __restrict__ occ, uint8_t* __restrict__ macro, int nmx,
                 int nmy, uint32_t above)
{
    __shared__ OvlLds G;
    slab_ovl_body<VEC>(src, nx, ny, nz, nbx, nby, dst, occ, macro, nmx, nmy, above, blockIdx.x * kOvlBricks,
                       blockIdx.y, blockIdx.z, threadIdx.x, G);
}

// Rows load four voxels at a time when nx is a multiple of 4 and src is
// aligned to four voxels.
template <typename T, bool PAIRS>
void launch_brick(dim3 grid, hipStream_t s, const void* src, int nx, int ny, int nz, int nbx, int nby,
                  void* dst, uint8_t* occ, uint8_t* macro, int nmx, int nmy, uint32_t above)
{
    const bool vec = nx % 4 == 0 && reinterpret_cast<uintptr_t>(src) % (4 * sizeof(T)) == 0;
    const auto* sp = static_cast<const T*>(src);
    auto* dp = static_cast<typename ElemOf<T, PAIRS>::type*>(dst);
    if (vec)
        brick_kernel<T, PAIRS, true><<<grid, kThreads, 0, s>>>(sp, nx, ny, nz, nbx, nby, dp, occ, macro, nmx, nmy,
                                                               above);
    else
        brick_kernel<T, PAIRS, false><<<grid, kThreads, 0, s>>>(sp, nx, ny, nz, nbx, nby, dp, occ, macro, nmx, nmy,
                                                                above);
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
    if (occupancy_bytes) *occupancy_bytes = 3 * bx * by * bz + ((bx + 3) / 4) * ((by + 3) / 4) * ((bz + 3) / 4);
    return VR_OK;
}

extern "C" int vr_brick_count_layout(int layout, int64_t nx, int64_t ny, int64_t nz, int64_t* n_bricks,
                                     int64_t* elements, int64_t* occupancy_bytes)
{
    vr::clear_error();
    VR_REQUIRE(n_bricks != nullptr, VR_ERR_NULL, "vr_brick_count_layout: n_bricks is NULL");
    VR_REQUIRE(layout == VR_LAYOUT_BRICK4 || layout == VR_LAYOUT_BRICK4_PAIRS || layout == VR_LAYOUT_BRICK8 ||
                   layout == VR_LAYOUT_BRICK4_OVERLAP,
               VR_ERR_RANGE, "vr_brick_count_layout: layout %d is not a brick layout", layout);
    VR_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1 && nx < (1 << 30) && ny < (1 << 30) && nz < (1 << 30),
               VR_ERR_DIMS, "vr_brick_count_layout: dims %lld x %lld x %lld", (long long)nx, (long long)ny,
               (long long)nz);
    const int e = layout == VR_LAYOUT_BRICK8 ? 8 : 4;
    int64_t nb[3];
    brick_grid(layout, nx, ny, nz, nb);
    const int64_t bx = nb[0], by = nb[1], bz = nb[2];
    *n_bricks = bx * by * bz;
    if (elements)
        *elements = (bx * by * bz + apron_bricks(bx, by)) * e * e * e * (layout == VR_LAYOUT_BRICK4_PAIRS ? 2 : 1);
    if (occupancy_bytes) *occupancy_bytes = 3 * bx * by * bz + ((bx + 3) / 4) * ((by + 3) / 4) * ((bz + 3) / 4);
    return VR_OK;
}

extern "C" int vr_brick_volume(const void* d_src, int dtype, int layout, int64_t nx, int64_t ny,
                               int64_t nz, void* d_bricked, uint8_t* d_occupancy, int32_t mark_above,
                               void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_src && d_bricked, VR_ERR_NULL, "vr_brick_volume: NULL pointer");
    VR_REQUIRE(dtype == VR_U16_NORM || dtype == VR_F32, VR_ERR_DTYPE, "vr_brick_volume: dtype %d",
               dtype);
    VR_REQUIRE(mark_above >= 0 && mark_above <= 65535 && (dtype == VR_U16_NORM || mark_above == 0), VR_ERR_RANGE,
               "vr_brick_volume: mark_above %d (0..65535 for u16, 0 for f32)", (int)mark_above);
    const uint32_t above = (uint32_t)mark_above;
    VR_REQUIRE(layout == VR_LAYOUT_BRICK4 || layout == VR_LAYOUT_BRICK4_PAIRS || layout == VR_LAYOUT_BRICK8 ||
                   layout == VR_LAYOUT_BRICK4_OVERLAP,
               VR_ERR_RANGE, "vr_brick_volume: layout %d is not a brick layout", layout);
    VR_REQUIRE(layout != VR_LAYOUT_BRICK4_OVERLAP || dtype == VR_U16_NORM, VR_ERR_DTYPE,
               "vr_brick_volume: VR_LAYOUT_BRICK4_OVERLAP holds u16 volumes only");
    VR_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1 && nx < (1 << 30) && ny < (1 << 30) && nz < (1 << 30),
               VR_ERR_DIMS, "vr_brick_volume: dims %lld x %lld x %lld", (long long)nx, (long long)ny,
               (long long)nz);
    const int be = layout == VR_LAYOUT_BRICK8 ? 8 : 4;
    int64_t nbg[3];
    brick_grid(layout, nx, ny, nz, nbg);
    const int nbx = (int)nbg[0], nby = (int)nbg[1], nbz = (int)nbg[2];
    const int nmx = (nbx + 3) / 4, nmy = (nby + 3) / 4, nmz = (nbz + 3) / 4;
    const int64_t bricks = (int64_t)nbx * nby * nbz;
    const int64_t groups = (int64_t)nmx * nmy * nmz;
    const int64_t occ_bytes = bricks + groups;           // marks and group marks (cleared first)
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
    uint8_t* macro = d_occupancy ? d_occupancy + bricks : nullptr;
    const bool pairs = layout == VR_LAYOUT_BRICK4_PAIRS;
    const int inx = (int)nx, iny = (int)ny, inz = (int)nz;
    if (layout == VR_LAYOUT_BRICK4_OVERLAP) {
        const auto* sp = static_cast<const uint16_t*>(d_src);
        auto* dp = static_cast<uint16_t*>(d_bricked);
        const dim3 og((unsigned)vr::ceil_div(nbx, kOvlBricks), (unsigned)nby, (unsigned)nbz);
        if (nx % 4 == 0 && reinterpret_cast<uintptr_t>(d_src) % 8 == 0)
            brick_ovl_kernel<true><<<og, kThreads, 0, s>>>(sp, inx, iny, inz, nbx, nby, dp, d_occupancy, macro, nmx,
                                                           nmy, above);
        else
            brick_ovl_kernel<false><<<og, kThreads, 0, s>>>(sp, inx, iny, inz, nbx, nby, dp, d_occupancy, macro,
                                                            nmx, nmy, above);
    } else if (layout == VR_LAYOUT_BRICK8) {
        const int64_t pieces = (int64_t)nbx * (nby * 8) * (nbz * 8);
        const unsigned g8 = (unsigned)std::max<int64_t>(1, std::min<int64_t>(cap * 4, vr::ceil_div<int64_t>(pieces, kThreads)));
        if (dtype == VR_U16_NORM)
            brick8_kernel<uint16_t><<<g8, kThreads, 0, s>>>(static_cast<const uint16_t*>(d_src), inx, iny, inz, nbx,
                                                            nby, static_cast<uint16_t*>(d_bricked), d_occupancy, macro,
                                                            nmx, nmy, above);
        else
            brick8_kernel<float><<<g8, kThreads, 0, s>>>(static_cast<const float*>(d_src), inx, iny, inz, nbx, nby,
                                                         static_cast<float*>(d_bricked), d_occupancy, macro, nmx,
                                                         nmy, above);
    } else if (dtype == VR_U16_NORM) {
        if (pairs) launch_brick<uint16_t, true>(grid, s, d_src, inx, iny, inz, nbx, nby, d_bricked, d_occupancy, macro, nmx, nmy, above);
        else launch_brick<uint16_t, false>(grid, s, d_src, inx, iny, inz, nbx, nby, d_bricked, d_occupancy, macro, nmx, nmy, above);
    } else {
        if (pairs) launch_brick<float, true>(grid, s, d_src, inx, iny, inz, nbx, nby, d_bricked, d_occupancy, macro, nmx, nmy, above);
        else launch_brick<float, false>(grid, s, d_src, inx, iny, inz, nbx, nby, d_bricked, d_occupancy, macro, nmx, nmy, above);
    }
    int rc = vr::check_launch("vr_brick_volume");
    if (rc) return rc;
    {   // the apron after the last brick: zeros
        const int64_t ebytes = (dtype == VR_U16_NORM ? 2 : 4) * (pairs ? 2 : 1);
        const int64_t abytes = apron_bricks(nbx, nby) * (be * be * be) * ebytes;
        const int64_t g = std::min<int64_t>(cap, vr::ceil_div<int64_t>(abytes / 16, kThreads));
        fill_16<<<(unsigned)std::max<int64_t>(g, 1), kThreads, 0, s>>>(
            reinterpret_cast<uint4*>(static_cast<uint8_t*>(d_bricked) + bricks * (be * be * be) * ebytes),
            abytes / 16);
        rc = vr::check_launch("vr_brick_volume: apron");
        if (rc || !d_occupancy) return rc;
    }
    // the distance grid: x from the marks, y into the working bytes, z back
    uint8_t* dist = d_occupancy + bricks + groups;
    uint8_t* work = dist + bricks;
    launch_dist<true>(s, d_occupancy, dist, nbx, nby, nbz, 0);
    launch_dist<false>(s, dist, work, nbx, nby, nbz, 1);
    launch_dist<false>(s, work, dist, nbx, nby, nbz, 2);
    return vr::check_launch("vr_brick_volume: distance grid");
}

namespace {

// Inverse of the brick layout: thread (x4, y, z) copies the 4-voxel row of
// brick (x4, y >> 2, z >> 2) at in-brick row (y & 3, z & 3) to voxels
// [4 x4, 4 x4 + 4) of row (y, z) of the linear volume, clipped at nx.  VEC:
// nx is a multiple of 4 and dst is aligned to a whole row of four, so each
// row moves as one vector (brick rows are always aligned).
template <typename T, bool VEC>
__global__ void __launch_bounds__(kThreads)
unbrick_kernel(const T* __restrict__ src, int64_t nx, int64_t ny, int64_t nz, int64_t nbx, int64_t nby,
               T* __restrict__ dst)
{
    using V = typename std::conditional<sizeof(T) == 2, uint2, float4>::type;   // four voxels
    const int64_t rows = nbx * ny * nz;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < rows; t += (int64_t)gridDim.x * kThreads) {
        const int64_t bx = t % nbx, yz = t / nbx, y = yz % ny, z = yz / ny;
        const int64_t b = ((z >> 2) * nby + (y >> 2)) * nbx + bx;
        const T* row = src + b * 64 + ((z & 3) << 4) + ((y & 3) << 2);
        T* out = dst + (z * ny + y) * nx + bx * 4;
        if (VEC) {
            *reinterpret_cast<V*>(out) = *reinterpret_cast<const V*>(row);
        } else {
            const int64_t m = nx - bx * 4 < 4 ? nx - bx * 4 : 4;
            for (int64_t q = 0; q < m; ++q) out[q] = row[q];
        }
    }
}

}  // namespace

extern "C" int vr_unbrick_volume(const void* d_bricked, int dtype, int64_t nx, int64_t ny, int64_t nz,
                                 void* d_dst, void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_bricked && d_dst, VR_ERR_NULL, "vr_unbrick_volume: NULL pointer");
    VR_REQUIRE(dtype == VR_U16_NORM || dtype == VR_F32, VR_ERR_DTYPE, "vr_unbrick_volume: dtype %d",
               dtype);
    VR_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1 && nx < (1 << 30) && ny < (1 << 30) && nz < (1 << 30),
               VR_ERR_DIMS, "vr_unbrick_volume: dims %lld x %lld x %lld", (long long)nx, (long long)ny,
               (long long)nz);
    const int64_t nbx = (nx + 3) / 4, nby = (ny + 3) / 4;
    const int64_t rows = nbx * ny * nz;
    hipStream_t s = vr::as_stream(stream);
    const int64_t g = std::max<int64_t>(1, std::min<int64_t>((int64_t)vr::num_cus() * 16,
                                                             vr::ceil_div<int64_t>(rows, kThreads)));
    const int64_t esz = dtype == VR_U16_NORM ? 2 : 4;
    const bool vec = nx % 4 == 0 && (reinterpret_cast<uintptr_t>(d_dst) % (4 * esz)) == 0 &&
                     (reinterpret_cast<uintptr_t>(d_bricked) % (4 * esz)) == 0;
    const auto* su = static_cast<const uint16_t*>(d_bricked);
    const auto* sf = static_cast<const float*>(d_bricked);
    auto* du = static_cast<uint16_t*>(d_dst);
    auto* df = static_cast<float*>(d_dst);
    const unsigned gb = (unsigned)g;
    if (dtype == VR_U16_NORM) {
        if (vec) unbrick_kernel<uint16_t, true><<<gb, kThreads, 0, s>>>(su, nx, ny, nz, nbx, nby, du);
        else unbrick_kernel<uint16_t, false><<<gb, kThreads, 0, s>>>(su, nx, ny, nz, nbx, nby, du);
    } else {
        if (vec) unbrick_kernel<float, true><<<gb, kThreads, 0, s>>>(sf, nx, ny, nz, nbx, nby, df);
        else unbrick_kernel<float, false><<<gb, kThreads, 0, s>>>(sf, nx, ny, nz, nbx, nby, df);
    }
    return vr::check_launch("vr_unbrick_volume");
}
