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

__global__ void __launch_bounds__(kThreads)
downsample_kernel(const uint16_t* __restrict__ vol, int nx, int ny, int nz, int aligned,
                  const uint32_t* __restrict__ keep_bits, int n_levels, LevelOut L, int tiles_x,
                  int tiles_y, int n_tiles)
{
    __shared__ uint32_t bits[VR_KEEP_WORDS];
    __shared__ TileLds G;
    __shared__ uint32_t s_first, s_bad;
    const uint32_t T = keep_bits == nullptr ? 0u : load_mask(keep_bits, bits, s_first, s_bad);
    const int tid = threadIdx.x;
    if (T <= VR_NBINS) {
        for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x)
            tile_body<true>(vol, nx, ny, nz, aligned, bits, T, n_levels, L, tiles_x, tiles_y, tile, true, tid, G);
    } else {
        for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x)
            tile_body<false>(vol, nx, ny, nz, aligned, bits, 0u, n_levels, L, tiles_x, tiles_y, tile, true, tid, G);
    }
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
