// Slicemap atlas of a volume level (Section III: slices laid out as tiles of
// one 2D image).  A pure permutation: workgroup g copies row y of slice z
// into the atlas row segment of tile z, writing zeros for tiles past the last
// slice.  Reads and writes are both contiguous along x.
#include "common.h"

namespace {

constexpr int kThreads = 256;

template <int BITS>
__global__ void __launch_bounds__(kThreads)
pack_kernel(const uint16_t* __restrict__ L, int nx, int ny, int nz, int tiles_x, int64_t n_segments,
            void* __restrict__ atlas)
{
    for (int64_t seg = blockIdx.x; seg < n_segments; seg += gridDim.x) {
        const int y = (int)(seg % ny);
        const int z = (int)(seg / ny);                  // tile index, may be >= nz
        const int tx = z % tiles_x, ty = z / tiles_x;
        const int64_t W = (int64_t)tiles_x * nx;
        const int64_t dst = ((int64_t)ty * ny + y) * W + (int64_t)tx * nx;
        const uint16_t* src = L + ((int64_t)z * ny + y) * nx;
        for (int x = threadIdx.x; x < nx; x += kThreads) {
            const uint32_t v = z < nz ? (uint32_t)src[x] : 0u;
            if (BITS == 16) {
                static_cast<uint16_t*>(atlas)[dst + x] = (uint16_t)v;
            } else {
                const uint32_t b = (v + 128u) >> 8;
                static_cast<uint8_t*>(atlas)[dst + x] = (uint8_t)(b > 255u ? 255u : b);
            }
        }
    }
}

}  // namespace

extern "C" int vr_pack_slicemap(const uint16_t* d_level, int64_t nx, int64_t ny, int64_t nz,
                                int tiles_x, int tiles_y, int out_bits, void* d_atlas, void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_level && d_atlas, VR_ERR_NULL, "vr_pack_slicemap: NULL pointer");
    VR_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1 && nx < (1 << 30) && ny < (1 << 30) && nz < (1 << 30),
               VR_ERR_DIMS, "vr_pack_slicemap: dims %lld x %lld x %lld", (long long)nx,
               (long long)ny, (long long)nz);
    VR_REQUIRE(tiles_x >= 1 && tiles_y >= 1 && (int64_t)tiles_x * tiles_y >= nz, VR_ERR_RANGE,
               "vr_pack_slicemap: %d x %d tiles cannot hold %lld slices", tiles_x, tiles_y,
               (long long)nz);
    VR_REQUIRE(out_bits == 8 || out_bits == 16, VR_ERR_RANGE, "vr_pack_slicemap: out_bits %d",
               out_bits);
    const int64_t segs = (int64_t)tiles_x * tiles_y * ny;
    int64_t grid = (int64_t)vr::num_cus() * 16;
    if (grid > segs) grid = segs;
    hipStream_t s = vr::as_stream(stream);
    if (out_bits == 16)
        pack_kernel<16><<<(unsigned)grid, kThreads, 0, s>>>(d_level, (int)nx, (int)ny, (int)nz,
                                                            tiles_x, segs, d_atlas);
    else
        pack_kernel<8><<<(unsigned)grid, kThreads, 0, s>>>(d_level, (int)nx, (int)ny, (int)nz,
                                                           tiles_x, segs, d_atlas);
    return vr::check_launch("vr_pack_slicemap");
}
