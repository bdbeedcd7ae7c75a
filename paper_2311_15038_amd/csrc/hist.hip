// 65536-bin histogram of a 16-bit volume (Section III-D: the volume histogram
// and the histogram of its first three slices).
//
// One 1024-thread workgroup per compute unit keeps a private copy of all 65536
// bins in LDS as packed 16-bit counters (two bins per 32-bit word, 128 KiB).
// A counter that reaches 0x8000 hands 0x8000 to the global 64-bit bin and
// drops back (the lane whose increment crossed the mark does both), so a
// counter never exceeds 0xFFFF and never carries into its neighbour.  A wave
// whose lanes all hold eight copies of one value (constant regions, removed
// voxels) adds them with one LDS atomic (ballot test per 8-voxel chunk).  The
// streaming loop keeps the next chunks' loads in flight while it counts the
// current ones.  At the end each workgroup adds its non-zero counters to the
// global bins; whole waves of empty words are skipped by ballot.
#include "common.h"

namespace {

constexpr int kThreads = 1024;
constexpr int kWords = VR_NBINS / 2;      // packed LDS words
constexpr int kUnroll = 4;                // 16-byte loads per thread per batch (two batches in flight)
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

// Adds n (1..512) to bin v in the packed LDS histogram, carrying to global.
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

__device__ __forceinline__ void count_chunk(uint32_t* lds, uint64_t* gh, uint4 c)
{
    // wave-uniform chunk: every lane holds eight copies of the first lane's value
    const uint32_t v0 = c.x & 0xFFFFu;
    const bool same8 = (c.x >> 16) == v0 && c.y == c.x && c.z == c.x && c.w == c.x;
    const uint32_t w0 = __builtin_amdgcn_readfirstlane(v0);
    const uint64_t act = __ballot(1);
    if (__ballot(same8 && v0 == w0) == act) {
        if (__lane_id() == (uint32_t)__builtin_ctzll(act)) count_n(lds, gh, w0, 8u * (uint32_t)__popcll(act));
        return;
    }
    count_n(lds, gh, c.x & 0xFFFFu, 1u);
    count_n(lds, gh, c.x >> 16, 1u);
    count_n(lds, gh, c.y & 0xFFFFu, 1u);
    count_n(lds, gh, c.y >> 16, 1u);
    count_n(lds, gh, c.z & 0xFFFFu, 1u);
    count_n(lds, gh, c.z >> 16, 1u);
    count_n(lds, gh, c.w & 0xFFFFu, 1u);
    count_n(lds, gh, c.w >> 16, 1u);
}

// One contiguous run of voxels and the histogram it goes to.  vol points at
// the first voxel; head = voxels before the first 16-byte boundary (counted
// one by one), then n_chunks full 8-voxel chunks, then the tail.
struct Range {
    const uint16_t* vol;
    int64_t n, head, n_chunks;
    uint64_t* hist;
    int blocks;          // workgroups given to this range
};

// Workgroups [0, a.blocks) count range a, the next b.blocks count range b
// (b.blocks may be 0): one launch for the volume and its top slices.
__global__ void __launch_bounds__(kThreads) hist_kernel(Range a, Range b)
{
    __shared__ uint32_t lds[kWords];
    const int tid = threadIdx.x;
    for (int w = tid * 4; w < kWords; w += kThreads * 4)
        *reinterpret_cast<uint4*>(lds + w) = make_uint4(0, 0, 0, 0);
    __syncthreads();

    const bool first = (int)blockIdx.x < a.blocks;
    const Range& R = first ? a : b;
    const uint16_t* vol = R.vol;
    uint64_t* gh = R.hist;
    const int64_t n = R.n, head = R.head, n_chunks = R.n_chunks;
    const int64_t gtid = (int64_t)(first ? blockIdx.x : blockIdx.x - a.blocks) * kThreads + tid;
    const int64_t nthr = (int64_t)R.blocks * kThreads;

    // head and tail voxels (fewer than 8 each)
    const int64_t tail_beg = head + n_chunks * 8;
    if (gtid < head) count_n(lds, gh, vol[gtid], 1u);
    if (gtid < n - tail_beg) count_n(lds, gh, vol[tail_beg + gtid], 1u);

    const uint4* body = reinterpret_cast<const uint4*>(vol + head);
    const int64_t stride = kUnroll * nthr;
    int64_t i = gtid;
    if (i + (kUnroll - 1) * nthr < n_chunks) {
        // software pipeline: batch k+1 is loading while batch k is counted
        uint4 cur[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) cur[u] = load_stream(body + i + u * nthr);
        for (;;) {
            const int64_t nx = i + stride;
            const bool more = nx + (kUnroll - 1) * nthr < n_chunks;
            uint4 nxt[kUnroll];
            if (more) {
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) nxt[u] = load_stream(body + nx + u * nthr);
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) count_chunk(lds, gh, cur[u]);
            i = nx;
            if (!more) break;
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) cur[u] = nxt[u];
        }
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

Range make_range(const uint16_t* p, int64_t n, uint64_t* hist)
{
    Range r{};
    r.vol = p;
    r.n = n;
    r.head = (int64_t)(((16u - (reinterpret_cast<uintptr_t>(p) & 15u)) & 15u) / 2u);
    if (r.head > n) r.head = n;
    r.n_chunks = (n - r.head) / 8;
    r.hist = hist;
    return r;
}

// enough voxels per workgroup to amortise zeroing and flushing 65536 bins
int blocks_for(int64_t n, int cap)
{
    int64_t b = n / (32 * 1024);
    if (b > cap) b = cap;
    return b < 1 ? 1 : (int)b;
}

int check_dims(int64_t nx, int64_t ny, int64_t nz, const char* who)
{
    VR_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1, VR_ERR_DIMS, "%s: dims %lld x %lld x %lld", who,
               (long long)nx, (long long)ny, (long long)nz);
    return VR_OK;
}

}  // namespace

extern "C" int vr_histogram(const uint16_t* d_vol, int64_t nx, int64_t ny, int64_t nz, int64_t z0,
                            int64_t nz_range, uint64_t* d_hist, void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_hist != nullptr, VR_ERR_NULL, "vr_histogram: d_hist is NULL");
    int rc = check_dims(nx, ny, nz, "vr_histogram");
    if (rc) return rc;
    VR_REQUIRE(z0 >= 0 && nz_range >= 0 && z0 + nz_range <= nz, VR_ERR_RANGE,
               "vr_histogram: slices [%lld, %lld) outside [0, %lld)", (long long)z0,
               (long long)(z0 + nz_range), (long long)nz);
    VR_REQUIRE(nz_range == 0 || d_vol != nullptr, VR_ERR_NULL, "vr_histogram: d_vol is NULL");
    hipStream_t s = vr::as_stream(stream);

    fill_u64<<<VR_NBINS / 256, 256, 0, s>>>(d_hist, VR_NBINS);
    rc = vr::check_launch("vr_histogram: fill");
    if (rc || nz_range == 0) return rc;

    Range a = make_range(d_vol + z0 * nx * ny, nx * ny * nz_range, d_hist);
    a.blocks = blocks_for(a.n, vr::num_cus());
    Range b{};
    hist_kernel<<<(unsigned)a.blocks, kThreads, 0, s>>>(a, b);
    return vr::check_launch("vr_histogram");
}

extern "C" int vr_histogram_with_top(const uint16_t* d_vol, int64_t nx, int64_t ny, int64_t nz,
                                     int64_t top_slices, uint64_t* d_hist, uint64_t* d_hist_top,
                                     void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_vol && d_hist && d_hist_top, VR_ERR_NULL, "vr_histogram_with_top: NULL pointer");
    int rc = check_dims(nx, ny, nz, "vr_histogram_with_top");
    if (rc) return rc;
    VR_REQUIRE(top_slices >= 1 && top_slices <= nz, VR_ERR_RANGE,
               "vr_histogram_with_top: %lld top slices of %lld", (long long)top_slices, (long long)nz);
    hipStream_t s = vr::as_stream(stream);
    fill_u64<<<VR_NBINS / 256, 256, 0, s>>>(d_hist, VR_NBINS);
    fill_u64<<<VR_NBINS / 256, 256, 0, s>>>(d_hist_top, VR_NBINS);
    rc = vr::check_launch("vr_histogram_with_top: fill");
    if (rc) return rc;
    const int cus = vr::num_cus();
    Range a = make_range(d_vol, nx * ny * nz, d_hist);
    Range b = make_range(d_vol, nx * ny * top_slices, d_hist_top);
    // the top slices get a share of the compute units in proportion to their
    // voxels (at least one workgroup), the volume the rest, all co-resident
    b.blocks = std::max(1, std::min(blocks_for(b.n, cus), (int)((int64_t)cus * b.n / a.n) + 1));
    a.blocks = std::max(1, std::min(blocks_for(a.n, cus), cus - b.blocks));
    hist_kernel<<<(unsigned)(a.blocks + b.blocks), kThreads, 0, s>>>(a, b);
    return vr::check_launch("vr_histogram_with_top");
}
