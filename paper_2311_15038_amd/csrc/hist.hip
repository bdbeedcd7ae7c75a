// 65536-bin histogram of a 16-bit volume (Section III-D: the volume histogram
// and the histogram of its first three slices).
//
// One 1024-thread workgroup per compute unit keeps a private copy of all 65536
// bins in LDS as packed 16-bit counters (two bins per 32-bit word, 128 KiB).
// A counter that reaches 0x8000 hands 0x8000 to the global 64-bit bin and
// drops back (the lane whose increment crossed the mark does both), so a
// counter never exceeds 0xFFFF and never carries into its neighbour.  A wave
// whose 64 lanes hold the same value adds 64 with one LDS atomic (ballot
// test).  At the end each workgroup adds its non-zero counters to the global
// bins; whole waves of empty words are skipped by ballot.
#include "common.h"

namespace {

constexpr int kThreads = 1024;
constexpr int kWords = VR_NBINS / 2;      // packed LDS words
constexpr int kUnroll = 4;                // 16-byte loads in flight per thread
constexpr uint32_t kMark = 0x8000u;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// streaming 16-byte load (the volume is read once; keep it out of the caches' way)
__device__ __forceinline__ uint4 load_stream(const uint4* p)
{
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

__global__ void __launch_bounds__(256) fill_u64(uint64_t* __restrict__ p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__device__ __forceinline__ void add_global(uint64_t* h, uint32_t b, uint64_t v)
{
    __hip_atomic_fetch_add(h + b, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Adds n (1..64) to bin v in the packed LDS histogram, carrying to global.
__device__ __forceinline__ void count_n(uint32_t* lds, uint64_t* gh, uint32_t v, uint32_t n)
{
    const uint32_t sh = (v & 1u) << 4;
    const uint32_t old = atomicAdd(lds + (v >> 1), n << sh);
    const uint32_t half = (old >> sh) & 0xFFFFu;
    if (half < kMark && half + n >= kMark) {
        atomicSub(lds + (v >> 1), kMark << sh);
        add_global(gh, v, kMark);
    }
}

// One voxel value per lane; waves with a single common value add once.
__device__ __forceinline__ void count_voxel(uint32_t* lds, uint64_t* gh, uint32_t v)
{
    const uint32_t v0 = __builtin_amdgcn_readfirstlane(v);
    const uint64_t same = __ballot(v == v0);
    const uint64_t act = __ballot(1);
    if (same == act) {
        if (__lane_id() == (uint32_t)__builtin_ctzll(act)) count_n(lds, gh, v0, (uint32_t)__popcll(act));
    } else {
        count_n(lds, gh, v, 1u);
    }
}

__device__ __forceinline__ void count_chunk(uint32_t* lds, uint64_t* gh, uint4 c)
{
    count_voxel(lds, gh, c.x & 0xFFFFu);
    count_voxel(lds, gh, c.x >> 16);
    count_voxel(lds, gh, c.y & 0xFFFFu);
    count_voxel(lds, gh, c.y >> 16);
    count_voxel(lds, gh, c.z & 0xFFFFu);
    count_voxel(lds, gh, c.z >> 16);
    count_voxel(lds, gh, c.w & 0xFFFFu);
    count_voxel(lds, gh, c.w >> 16);
}

// vol points at the first voxel of the range; n voxels; head = voxels before
// the first 16-byte boundary (processed one by one), then n_chunks full
// 8-voxel chunks, then the tail.
__global__ void __launch_bounds__(kThreads)
hist_kernel(const uint16_t* __restrict__ vol, int64_t n, int64_t head, int64_t n_chunks,
            uint64_t* __restrict__ gh)
{
    __shared__ uint32_t lds[kWords];
    const int tid = threadIdx.x;
    for (int w = tid * 4; w < kWords; w += kThreads * 4)
        *reinterpret_cast<uint4*>(lds + w) = make_uint4(0, 0, 0, 0);
    __syncthreads();

    const int64_t gtid = (int64_t)blockIdx.x * kThreads + tid;
    const int64_t nthr = (int64_t)gridDim.x * kThreads;

    // head and tail voxels (fewer than 8 each)
    const int64_t tail_beg = head + n_chunks * 8;
    if (gtid < head) count_n(lds, gh, vol[gtid], 1u);
    if (gtid < n - tail_beg) count_n(lds, gh, vol[tail_beg + gtid], 1u);

    const uint4* body = reinterpret_cast<const uint4*>(vol + head);
    int64_t i = gtid;
    for (; i + (kUnroll - 1) * nthr < n_chunks; i += kUnroll * nthr) {
        uint4 c[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) c[u] = load_stream(body + i + u * nthr);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) count_chunk(lds, gh, c[u]);
    }
    for (; i < n_chunks; i += nthr) count_chunk(lds, gh, load_stream(body + i));
    __syncthreads();

    // flush: non-zero counters to the global bins
    for (int w = tid; w < kWords; w += kThreads) {
        const uint32_t x = lds[w];
        if (__ballot(x != 0) == 0) continue;
        if (x & 0xFFFFu) add_global(gh, 2 * w, x & 0xFFFFu);
        if (x >> 16) add_global(gh, 2 * w + 1, x >> 16);
    }
}

}  // namespace

extern "C" int vr_histogram(const uint16_t* d_vol, int64_t nx, int64_t ny, int64_t nz, int64_t z0,
                            int64_t nz_range, uint64_t* d_hist, void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_hist != nullptr, VR_ERR_NULL, "vr_histogram: d_hist is NULL");
    VR_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1, VR_ERR_DIMS, "vr_histogram: dims %lld x %lld x %lld",
               (long long)nx, (long long)ny, (long long)nz);
    VR_REQUIRE(z0 >= 0 && nz_range >= 0 && z0 + nz_range <= nz, VR_ERR_RANGE,
               "vr_histogram: slices [%lld, %lld) outside [0, %lld)", (long long)z0,
               (long long)(z0 + nz_range), (long long)nz);
    VR_REQUIRE(nz_range == 0 || d_vol != nullptr, VR_ERR_NULL, "vr_histogram: d_vol is NULL");
    hipStream_t s = vr::as_stream(stream);

    fill_u64<<<VR_NBINS / 256, 256, 0, s>>>(d_hist, VR_NBINS);
    int rc = vr::check_launch("vr_histogram: fill");
    if (rc || nz_range == 0) return rc;

    const int64_t n = nx * ny * nz_range;
    const uint16_t* p = d_vol + z0 * nx * ny;
    int64_t head = (int64_t)(((16u - (reinterpret_cast<uintptr_t>(p) & 15u)) & 15u) / 2u);
    if (head > n) head = n;
    const int64_t n_chunks = (n - head) / 8;
    // enough voxels per workgroup to amortise zeroing and flushing 65536 bins
    int64_t blocks = n / (256 * 1024);
    const int64_t cus = vr::num_cus();
    if (blocks > cus) blocks = cus;
    if (blocks < 1) blocks = 1;
    hist_kernel<<<(unsigned)blocks, kThreads, 0, s>>>(p, n, head, n_chunks, d_hist);
    return vr::check_launch("vr_histogram");
}
