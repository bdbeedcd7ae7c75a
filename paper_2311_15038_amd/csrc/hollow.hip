// Hollow data preview (Section II: the data preview keeps the object's outer
// geometry and drops its interior volume).  A non-zero voxel is kept when a
// voxel within city-block distance t of it is zero or lies outside the
// volume (the shell that t erosions with the 6-neighbourhood take away);
// every other voxel becomes 0.
//
// A workgroup owns a 32 x 16 x 16 tile (32 x 8 x 8 for t > 4).  It reads the
// tile with a halo of t voxels in y and z and of 4 or 8 in x (a whole number
// of 4-voxel groups, so that rows load and store 8 bytes per lane when nx is
// a multiple of 4), and keeps only the background (zero voxels and the
// outside) of each row of that region, as a 64-bit mask in LDS.  t rounds of
// dilation with the 6-neighbourhood (a row's mask shifted by one voxel either
// way, OR the masks of the four neighbouring rows) then tell, for every voxel
// of the tile, whether background lies within city-block distance t.  The
// tile's voxels are read again (from L2) for the output.  The volume comes
// from HBM once (halos and the second read from L2) and is written once: the
// kernel is HBM-bound.
#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kTX = 32;          // tile width
constexpr int kBatch = 8;        // staging loads a thread keeps in flight

template <int T>
struct Shape {
    static constexpr int TY = T <= 4 ? 16 : 8, TZ = T <= 4 ? 16 : 8;   // smaller tiles for thick halos
    static constexpr int HP = T <= 4 ? 4 : 8;                           // x halo, whole 4-voxel groups
    static constexpr int RXP = kTX + 2 * HP;                            // staged row: 40 or 48 voxels
    static constexpr int RY = TY + 2 * T, RZ = TZ + 2 * T, ROWS = RY * RZ;
};

// Workgroup ids are dealt round-robin over the 8 XCDs; tile b of the launch
// order runs where the neighbouring tiles whose halos it shares run.
__device__ __forceinline__ int tile_of_block(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x * q + min(x, r) + i;
}

__global__ void zero_count(unsigned long long* c) { *c = 0ull; }

// Voxels x .. x + W - 1 of row (y, z) (W = 4: one 8-byte load), read from a
// clamped in-volume address; in: whether they lie in the volume.
template <bool VEC>
__device__ __forceinline__ uint2 load_group(const uint16_t* __restrict__ src, int nx, int ny, int nz, int x, int y,
                                            int z, bool& in)
{
    constexpr int W = VEC ? 4 : 1;
    in = x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz;
    const int cx = min(max(x, 0), nx - W), cy = min(max(y, 0), ny - 1), cz = min(max(z, 0), nz - 1);
    const uint16_t* p = src + ((int64_t)cz * ny + cy) * nx + cx;
    if (VEC) return *reinterpret_cast<const uint2*>(p);
    return make_uint2(*p, 0u);
}

// VEC: nx is a multiple of 4 and both volumes are 8-byte aligned, so every
// 4-voxel group of a row is wholly inside or wholly outside the volume.
template <int T, bool VEC>
__global__ void __launch_bounds__(kThreads)
hollow_kernel(const uint16_t* __restrict__ src, int nx, int ny, int nz, int tiles_x, int tiles_y, int n_tiles,
              uint16_t* __restrict__ dst, unsigned long long* __restrict__ kept)
{
    using S = Shape<T>;
    __shared__ uint64_t bg[2][S::ROWS];   // background bits of each staged row (bit j: voxel j), dilated in turn
    __shared__ uint2 tile[S::TZ][S::TY][kTX / 4];   // the tile's own voxels, 4 to an element
    __shared__ uint32_t wsum[kThreads / 64];
    const int b = tile_of_block((int)blockIdx.x, n_tiles);
    const int tx = b % tiles_x, tyz = b / tiles_x, ty = tyz % tiles_y, tz = tyz / tiles_y;
    const int xs = tx * kTX - S::HP, y0 = ty * S::TY - T, z0 = tz * S::TZ - T;   // staged region origin
    for (int row = (int)threadIdx.x; row < S::ROWS; row += kThreads) bg[0][row] = 0ull;
    __syncthreads();

    // background bits of the staged region: kBatch loads in flight per thread,
    // each group's bits OR-ed into its row's mask (outside the volume: all set)
    constexpr int W = VEC ? 4 : 1;                    // voxels per load
    constexpr int G = S::RXP / W, N = S::ROWS * G, PER = (N + kThreads - 1) / kThreads;
    for (int i0 = 0; i0 < PER; i0 += kBatch) {
        uint2 val[kBatch];
        bool in[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int q = (int)threadIdx.x + (i0 + i) * kThreads;
            const int g = q % G, row = q / G, ry = row % S::RY, rz = row / S::RY;
            val[i] = load_group<VEC>(src, nx, ny, nz, xs + g * W, y0 + ry, z0 + rz, in[i]);
        }
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int q = (int)threadIdx.x + (i0 + i) * kThreads;
            if (q >= N) continue;
            const int g = q % G, row = q / G;
            const uint2 w = val[i];
            uint32_t zero;
            if (VEC)
                zero = (uint32_t)((w.x & 0xFFFFu) == 0u) | ((uint32_t)((w.x >> 16) == 0u) << 1) |
                       ((uint32_t)((w.y & 0xFFFFu) == 0u) << 2) | ((uint32_t)((w.y >> 16) == 0u) << 3);
            else
                zero = (uint32_t)(w.x == 0u);
            if (!in[i]) zero = (1u << W) - 1u;
            if (zero) atomicOr(reinterpret_cast<unsigned long long*>(&bg[0][row]),
                               (unsigned long long)zero << (g * W));
            // keep the tile's own voxels for the output
            const int ry = row % S::RY, rz = row / S::RY, ix = g * W - S::HP;
            if (ry >= T && ry < T + S::TY && rz >= T && rz < T + S::TZ && ix >= 0 && ix < kTX) {
                uint16_t* t16 = reinterpret_cast<uint16_t*>(&tile[rz - T][ry - T][0]);
                if (VEC) tile[rz - T][ry - T][ix >> 2] = w;
                else t16[ix] = (uint16_t)w.x;
            }
        }
    }
    __syncthreads();
    // t dilations with the 6-neighbourhood; after round j the bits of voxels at
    // least j from the staged region's sides are exact, and the tile's are
    // after round t (its voxels are t or more from every side)
#pragma unroll
    for (int j = 0; j < T; ++j) {
        const uint64_t* P = bg[j & 1];
        uint64_t* Q = bg[(j + 1) & 1];
        for (int row = (int)threadIdx.x; row < S::ROWS; row += kThreads) {
            const int ry = row % S::RY, rz = row / S::RY;
            const uint64_t m = P[row];
            uint64_t d = m | (m << 1) | (m >> 1);
            if (ry > 0) d |= P[row - 1];
            if (ry < S::RY - 1) d |= P[row + 1];
            if (rz > 0) d |= P[row - S::RY];
            if (rz < S::RZ - 1) d |= P[row + S::RY];
            Q[row] = d;
        }
        __syncthreads();
    }
    const uint64_t* D = bg[T & 1];
    // a non-zero voxel is kept when background lies within distance t
    uint32_t n_keep = 0;
    constexpr int GO = kTX / W;                       // output groups per tile row
    for (int q = (int)threadIdx.x; q < GO * S::TY * S::TZ; q += kThreads) {
        const int g = q % GO, r = q / GO, iy = r % S::TY, iz = r / S::TY;
        const int x = tx * kTX + g * W, y = y0 + T + iy, z = z0 + T + iz;
        if (x >= nx || y >= ny || z >= nz) continue;
        {
            const int row = (iz + T) * S::RY + (iy + T);
            const uint32_t near = (uint32_t)(D[row] >> (S::HP + g * W));
            uint16_t* o = dst + ((int64_t)z * ny + y) * nx + x;
            const uint2 w = VEC ? tile[iz][iy][g]
                                : make_uint2(reinterpret_cast<const uint16_t*>(&tile[iz][iy][0])[g], 0u);
            if (VEC) {
                const uint32_t v0 = w.x & 0xFFFFu, v1 = w.x >> 16, v2 = w.y & 0xFFFFu, v3 = w.y >> 16;
                const bool k0 = v0 && (near & 1u), k1 = v1 && (near & 2u), k2 = v2 && (near & 4u),
                           k3 = v3 && (near & 8u);
                *reinterpret_cast<uint2*>(o) = make_uint2((k0 ? v0 : 0u) | (k1 ? v1 << 16 : 0u),
                                                          (k2 ? v2 : 0u) | (k3 ? v3 << 16 : 0u));
                n_keep += (uint32_t)k0 + (uint32_t)k1 + (uint32_t)k2 + (uint32_t)k3;
            } else {
                const bool keep = w.x != 0u && (near & 1u);
                *o = keep ? (uint16_t)w.x : (uint16_t)0;
                n_keep += keep ? 1u : 0u;
            }
        }
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
int launch(hipStream_t s, const uint16_t* src, int64_t nx, int64_t ny, int64_t nz, uint16_t* dst,
           unsigned long long* kept)
{
    using S = Shape<T>;
    const int64_t tiles_x = (nx + kTX - 1) / kTX, tiles_y = (ny + S::TY - 1) / S::TY;
    const int64_t tiles_z = (nz + S::TZ - 1) / S::TZ, tiles = tiles_x * tiles_y * tiles_z;
    VR_REQUIRE(tiles < (int64_t(1) << 31), VR_ERR_DIMS, "vr_hollow: volume too large");
    const bool vec = nx % 4 == 0 && (reinterpret_cast<uintptr_t>(src) & 7u) == 0 &&
                     (reinterpret_cast<uintptr_t>(dst) & 7u) == 0;
    const unsigned nb = (unsigned)tiles;
    if (vec)
        hollow_kernel<T, true><<<nb, kThreads, 0, s>>>(src, (int)nx, (int)ny, (int)nz, (int)tiles_x, (int)tiles_y,
                                                       (int)tiles, dst, kept);
    else
        hollow_kernel<T, false><<<nb, kThreads, 0, s>>>(src, (int)nx, (int)ny, (int)nz, (int)tiles_x, (int)tiles_y,
                                                        (int)tiles, dst, kept);
    return vr::check_launch("vr_hollow");
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
    hipStream_t s = vr::as_stream(stream);
    auto* kept = reinterpret_cast<unsigned long long*>(d_kept);
    if (kept) {
        zero_count<<<1, 1, 0, s>>>(kept);
        const int rc = vr::check_launch("vr_hollow: count");
        if (rc) return rc;
    }
    switch (thickness) {
    case 1: return launch<1>(s, d_src, nx, ny, nz, d_dst, kept);
    case 2: return launch<2>(s, d_src, nx, ny, nz, d_dst, kept);
    case 3: return launch<3>(s, d_src, nx, ny, nz, d_dst, kept);
    case 4: return launch<4>(s, d_src, nx, ny, nz, d_dst, kept);
    case 5: return launch<5>(s, d_src, nx, ny, nz, d_dst, kept);
    case 6: return launch<6>(s, d_src, nx, ny, nz, d_dst, kept);
    case 7: return launch<7>(s, d_src, nx, ny, nz, d_dst, kept);
    default: return launch<8>(s, d_src, nx, ny, nz, d_dst, kept);
    }
}
