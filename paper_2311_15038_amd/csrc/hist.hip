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
#include "disc_dev.h"
#include "hist_dev.h"

namespace {

using namespace vr::hg;

// zero one or two 65536-bin histograms
__global__ void __launch_bounds__(256) fill_u64(uint64_t* __restrict__ p, uint64_t* __restrict__ q, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        p[i] = 0;
        if (q) q[i] = 0;
    }
}

// One contiguous run of voxels and the histogram it goes to.
struct Range {
    const uint16_t* vol;
    int64_t n;
    uint64_t* hist;
    int blocks;          // workgroups given to this range
};

__global__ void __launch_bounds__(kThreads) hist_kernel(Range R)
{
    __shared__ uint32_t lds[kWords];
    zero_lds(lds);
    __syncthreads();
    const int64_t gtid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    count_range(lds, R.hist, R.vol, R.n, gtid, (int64_t)R.blocks * kThreads);
    __syncthreads();
    flush_lds(lds, R.hist);
}

Range make_range(const uint16_t* p, int64_t n, uint64_t* hist)
{
    Range r{};
    r.vol = p;
    r.n = n;
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

// The voxels p[0 .. n) of one row, counted by the 64 lanes of a wave: the
// voxels before the first 16-byte boundary and after the last one by single
// lanes, the body in 16-byte chunks, four chunks per lane in flight.
__device__ __forceinline__ void count_row(uint32_t* lds, uint64_t* gh, const uint16_t* p, int64_t n, int lane)
{
    int64_t head = (int64_t)(((16u - (reinterpret_cast<uintptr_t>(p) & 15u)) & 15u) / 2u);
    if (head > n) head = n;
    const int64_t nch = (n - head) / 8, tail = head + nch * 8;
    if (lane < head) count_n(lds, gh, p[lane], 1u);
    if (lane < n - tail) count_n(lds, gh, p[tail + lane], 1u);
    const uint4* b = reinterpret_cast<const uint4*>(p + head);
    for (int64_t i = lane; i < nch; i += 4 * 64) {
        uint4 c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * 64 < nch) c[u] = load_stream(b + i + u * 64);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * 64 < nch) count_chunk(lds, gh, c[u]);
    }
}

// Rows of slices, each counted over its run inside the kept disc.
struct DiscRange {
    const uint16_t* vol;   // first row
    int64_t nx, ny, rows;
    const int32_t* rec;
    uint64_t* hist;
};

__global__ void __launch_bounds__(kThreads) hist_disc_kernel(DiscRange R)
{
    __shared__ uint32_t lds[kWords];
    zero_lds(lds);
    __syncthreads();
    const vr::disc::Disc d = vr::disc::load_disc(R.rec);
    const int lane = threadIdx.x & 63;
    const int64_t wpb = kThreads / 64, nw = (int64_t)gridDim.x * wpb;
    for (int64_t row = (int64_t)blockIdx.x * wpb + threadIdx.x / 64; row < R.rows; row += nw) {
        int64_t x0, x1;
        vr::disc::row_span(d, row % R.ny, R.nx, x0, x1);
        if (x0 <= x1) count_row(lds, R.hist, R.vol + row * R.nx + x0, x1 - x0 + 1, lane);
    }
    __syncthreads();
    flush_lds(lds, R.hist);
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

    fill_u64<<<VR_NBINS / 256, 256, 0, s>>>(d_hist, nullptr, VR_NBINS);
    rc = vr::check_launch("vr_histogram: fill");
    if (rc || nz_range == 0) return rc;

    Range a = make_range(d_vol + z0 * nx * ny, nx * ny * nz_range, d_hist);
    a.blocks = blocks_for(a.n, vr::num_cus());
    hist_kernel<<<(unsigned)a.blocks, kThreads, 0, s>>>(a);
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
    fill_u64<<<VR_NBINS / 256, 256, 0, s>>>(d_hist, d_hist_top, VR_NBINS);
    rc = vr::check_launch("vr_histogram_with_top: fill");
    if (rc) return rc;
    // two launches in stream order: the top slices on as many workgroups as their
    // size warrants, then the whole volume on every compute unit (one launch
    // sharing the compute units between the two runs measured slower)
    const int cus = vr::num_cus();
    Range b = make_range(d_vol, nx * ny * top_slices, d_hist_top);
    b.blocks = blocks_for(b.n, cus);
    hist_kernel<<<(unsigned)b.blocks, kThreads, 0, s>>>(b);
    rc = vr::check_launch("vr_histogram_with_top: top slices");
    if (rc) return rc;
    Range a = make_range(d_vol, nx * ny * nz, d_hist);
    a.blocks = blocks_for(a.n, cus);
    hist_kernel<<<(unsigned)a.blocks, kThreads, 0, s>>>(a);
    return vr::check_launch("vr_histogram_with_top");
}

extern "C" int vr_histogram_in_disc(const uint16_t* d_vol, int64_t nx, int64_t ny, int64_t nz, int64_t top_slices,
                                    const int32_t* d_circle, uint64_t* d_hist, uint64_t* d_hist_top, void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_vol && d_circle && d_hist, VR_ERR_NULL, "vr_histogram_in_disc: NULL pointer");
    int rc = check_dims(nx, ny, nz, "vr_histogram_in_disc");
    if (rc) return rc;
    VR_REQUIRE(d_hist_top == nullptr || (top_slices >= 1 && top_slices <= nz), VR_ERR_RANGE,
               "vr_histogram_in_disc: %lld top slices of %lld", (long long)top_slices, (long long)nz);
    hipStream_t s = vr::as_stream(stream);
    fill_u64<<<VR_NBINS / 256, 256, 0, s>>>(d_hist, d_hist_top, VR_NBINS);
    rc = vr::check_launch("vr_histogram_in_disc: fill");
    if (rc) return rc;
    const int cus = vr::num_cus();
    if (d_hist_top != nullptr) {
        DiscRange b{d_vol, nx, ny, ny * top_slices, d_circle, d_hist_top};
        hist_disc_kernel<<<(unsigned)blocks_for(nx * ny * top_slices, cus), kThreads, 0, s>>>(b);
        rc = vr::check_launch("vr_histogram_in_disc: top slices");
        if (rc) return rc;
    }
    DiscRange a{d_vol, nx, ny, ny * nz, d_circle, d_hist};
    hist_disc_kernel<<<(unsigned)blocks_for(nx * ny * nz, cus), kThreads, 0, s>>>(a);
    return vr::check_launch("vr_histogram_in_disc");
}
