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
// global bins; whole waves of empty words are skipped by ballot.  While every
// bin's total stays below 2^32 (fewer voxels than that), the global bins are
// kept in pairs, two 32-bit counters per 64-bit word, so one atomic adds a
// whole LDS word; a last one-workgroup pass spreads the pairs into 64-bit bins
// (the flush's atomics were a sixth of the histogram's time).
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

template <bool PAIRED>
__global__ void __launch_bounds__(kThreads) hist_kernel(Range R)
{
    __shared__ uint32_t lds[kWords];
    zero_lds(lds);
    __syncthreads();
    const int64_t gtid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    count_range<PAIRED>(lds, R.hist, R.vol, R.n, gtid, (int64_t)R.blocks * kThreads);
    __syncthreads();
    flush_lds<PAIRED>(lds, R.hist);
}

// One workgroup per histogram: the 32768 words of bin pairs are read into
// registers, then written out as 65536 64-bit bins in the same buffer.
constexpr int kPairWords = VR_NBINS / 2;
constexpr int kPairsPerThread = kPairWords / kThreads;

__global__ void __launch_bounds__(kThreads) unpack_pairs(uint64_t* __restrict__ h0, uint64_t* __restrict__ h1)
{
    uint64_t* h = blockIdx.x == 0 ? h0 : h1;
    uint64_t v[kPairsPerThread];
#pragma unroll
    for (int i = 0; i < kPairsPerThread; ++i) v[i] = h[threadIdx.x + i * kThreads];
    // every word is read before any bin is written: the fence waits for this
    // thread's loads to return, the barrier for every thread's
    __threadfence();
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kPairsPerThread; ++i) {
        const int w = threadIdx.x + i * kThreads;
        h[2 * w] = v[i] & 0xFFFFFFFFull;
        h[2 * w + 1] = v[i] >> 32;
    }
}

// Whether the bins of a run of n voxels are kept in pairs: every bin's total
// must stay below 2^32, and the run must be large enough (32 M voxels, every
// compute unit busy) for the saved flush atomics to outweigh the unpack pass.
bool paired_for(int64_t n) { return n >= (int64_t(1) << 25) && n < (int64_t(1) << 32); }

int launch_unpack(hipStream_t s, uint64_t* h0, uint64_t* h1, const char* who)
{
    unpack_pairs<<<h1 ? 2 : 1, kThreads, 0, s>>>(h0, h1);
    return vr::check_launch(who);
}

void launch_hist(const Range& r, bool paired, hipStream_t s)
{
    if (paired) hist_kernel<true><<<(unsigned)r.blocks, kThreads, 0, s>>>(r);
    else hist_kernel<false><<<(unsigned)r.blocks, kThreads, 0, s>>>(r);
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
template <bool PAIRED>
__device__ __forceinline__ void count_row(uint32_t* lds, uint64_t* gh, const uint16_t* p, int64_t n, int lane)
{
    int64_t head = (int64_t)(((16u - (reinterpret_cast<uintptr_t>(p) & 15u)) & 15u) / 2u);
    if (head > n) head = n;
    const int64_t nch = (n - head) / 8, tail = head + nch * 8;
    if (lane < head) count_n<PAIRED>(lds, gh, p[lane], 1u);
    if (lane < n - tail) count_n<PAIRED>(lds, gh, p[tail + lane], 1u);
    const uint4* b = reinterpret_cast<const uint4*>(p + head);
    for (int64_t i = lane; i < nch; i += 4 * 64) {
        uint4 c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * 64 < nch) c[u] = load_stream(b + i + u * 64);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * 64 < nch) count_chunk<PAIRED>(lds, gh, c[u]);
    }
}

// Rows of slices, each counted over its run inside the kept disc.
struct DiscRange {
    const uint16_t* vol;   // first row
    int64_t nx, ny, rows;
    const int32_t* rec;
    uint64_t* hist;
};

template <bool PAIRED>
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
        if (x0 <= x1) count_row<PAIRED>(lds, R.hist, R.vol + row * R.nx + x0, x1 - x0 + 1, lane);
    }
    __syncthreads();
    flush_lds<PAIRED>(lds, R.hist);
}

constexpr int kMaxSpanRows = 4096;       // rows of the streaming variant's span table

// The streaming variant for slabs whose rows are whole 16-byte chunks: the
// chunk sequence of the slab is walked as in hist_kernel; each thread carries
// the (column, row) of its current chunk forward by its fixed stride, and
// reads the row's kept run from a table in LDS.  Chunks outside the disc are
// not loaded, chunks across its edge are counted voxel by voxel.
struct DiscStream {
    const uint4* body;     // 16-byte aligned first voxel of the slab
    uint32_t n_chunks;     // chunks of the slab
    uint32_t ny;
    uint32_t per_row;      // chunks per row
    const int32_t* rec;
    uint64_t* hist;
};

// column and image row (row of the slab modulo ny) of a chunk
struct ChunkPos {
    uint32_t col, y;
};

// advance by a stride of dcol columns and drow rows (dcol < per_row, drow < ny)
__device__ __forceinline__ void advance(ChunkPos& p, uint32_t dcol, uint32_t drow, uint32_t per_row, uint32_t ny)
{
    p.col += dcol;
    const uint32_t carry = p.col >= per_row ? 1u : 0u;
    p.col -= carry * per_row;
    p.y += drow + carry;
    if (p.y >= ny) p.y -= ny;
}

// bits e of the chunk's voxels inside their row's kept run
__device__ __forceinline__ uint32_t chunk_keep(const ChunkPos& p, const uint32_t* spans)
{
    const int x = (int)(8u * p.col);
    const uint32_t sp = spans[p.y];
    const int lo = max((int)(sp & 0xFFFFu) - x, 0), hi = min((int)(sp >> 16) - x, 7);
    return lo > hi ? 0u : (0xFFu >> (7 - hi)) & (0xFFu << lo);
}

// The chunk's voxels whose bit is set in k, in one instruction stream for
// whole, partial and (per lane) absent chunks: eight predicated additions,
// or one addition when the wave's kept chunks are all eight copies of one value.
template <bool PAIRED>
__device__ __forceinline__ void count_kept(uint32_t* lds, uint64_t* gh, uint4 c, uint32_t k)
{
    const uint32_t v0 = c.x & 0xFFFFu;
    const bool same8 = k == 0xFFu && (c.x >> 16) == v0 && c.y == c.x && c.z == c.x && c.w == c.x;
    const uint64_t act = __ballot(k != 0u);
    if (act == 0) return;
    const uint32_t w0 = __shfl(v0, __builtin_ctzll(act));
    if (__ballot(k != 0u && same8 && v0 == w0) == act) {
        if (__lane_id() == (uint32_t)__builtin_ctzll(act)) count_n<PAIRED>(lds, gh, w0, 8u * (uint32_t)__popcll(act));
        return;
    }
    const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if ((k >> e) & 1u) count_1<PAIRED>(lds, gh, (w[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
}

template <bool PAIRED>
__global__ void __launch_bounds__(kThreads) hist_disc_stream(DiscStream S)
{
    __shared__ uint32_t lds[kWords];
    __shared__ uint32_t spans[kMaxSpanRows];
    zero_lds(lds);
    {
        const vr::disc::Disc d = vr::disc::load_disc(S.rec);
        const int64_t nx = (int64_t)S.per_row * 8;
        for (uint32_t y = threadIdx.x; y < S.ny; y += kThreads) {
            int64_t x0, x1;
            vr::disc::row_span(d, y, nx, x0, x1);
            spans[y] = x0 > x1 ? 0x0000FFFFu : (uint32_t)x0 | ((uint32_t)x1 << 16);
        }
    }
    __syncthreads();
    const uint32_t nthr = gridDim.x * kThreads;
    uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t stride = kUnroll * nthr;
    const uint32_t dcol = nthr % S.per_row, drow = (nthr / S.per_row) % S.ny;
    ChunkPos p{i % S.per_row, (i / S.per_row) % S.ny};   // position of chunk i
    if ((uint64_t)i + (kUnroll - 1) * (uint64_t)nthr < S.n_chunks) {
        uint4 cur[kUnroll];
        uint32_t kc[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            kc[u] = chunk_keep(p, spans);
            cur[u] = kc[u] ? load_stream(S.body + i + u * nthr) : make_uint4(0u, 0u, 0u, 0u);
            advance(p, dcol, drow, S.per_row, S.ny);
        }
        for (;;) {
            // p is the position of chunk i + stride here
            const uint64_t nx_ = (uint64_t)i + stride;
            const bool more = nx_ + (kUnroll - 1) * (uint64_t)nthr < S.n_chunks;
            uint4 nxt[kUnroll];
            uint32_t kn[kUnroll];
            if (more) {
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    kn[u] = chunk_keep(p, spans);
                    nxt[u] = kn[u] ? load_stream(S.body + nx_ + u * nthr) : make_uint4(0u, 0u, 0u, 0u);
                    advance(p, dcol, drow, S.per_row, S.ny);
                }
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) count_kept<PAIRED>(lds, S.hist, cur[u], kc[u]);
            i = (uint32_t)nx_;
            if (!more) break;
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                cur[u] = nxt[u];
                kc[u] = kn[u];
            }
        }
    }
    for (; i < S.n_chunks; i += nthr) {
        const uint32_t k = chunk_keep(p, spans);
        uint4 c = make_uint4(0u, 0u, 0u, 0u);
        if (k) c = load_stream(S.body + i);
        count_kept<PAIRED>(lds, S.hist, c, k);
        advance(p, dcol, drow, S.per_row, S.ny);
    }
    __syncthreads();
    flush_lds<PAIRED>(lds, S.hist);
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
    const bool paired = paired_for(a.n);
    launch_hist(a, paired, s);
    rc = vr::check_launch("vr_histogram");
    if (rc || !paired) return rc;
    return launch_unpack(s, d_hist, nullptr, "vr_histogram: unpack");
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
    const bool paired = paired_for(nx * ny * nz);
    Range b = make_range(d_vol, nx * ny * top_slices, d_hist_top);
    b.blocks = blocks_for(b.n, cus);
    launch_hist(b, paired, s);
    rc = vr::check_launch("vr_histogram_with_top: top slices");
    if (rc) return rc;
    Range a = make_range(d_vol, nx * ny * nz, d_hist);
    a.blocks = blocks_for(a.n, cus);
    launch_hist(a, paired, s);
    rc = vr::check_launch("vr_histogram_with_top");
    if (rc || !paired) return rc;
    return launch_unpack(s, d_hist, d_hist_top, "vr_histogram_with_top: unpack");
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
    // whole 16-byte chunks per row, a span table that fits, 32-bit chunk indices
    const bool stream_ok = nx % 8 == 0 && (reinterpret_cast<uintptr_t>(d_vol) & 15u) == 0 &&
                           ny <= kMaxSpanRows && nx <= 65536 && nx * ny * nz / 8 < (int64_t(1) << 31);
    const bool paired = paired_for(nx * ny * nz);
    auto launch = [&](int64_t slices, uint64_t* h) {
        const int blocks = blocks_for(nx * ny * slices, cus);
        if (stream_ok) {
            DiscStream S{reinterpret_cast<const uint4*>(d_vol), (uint32_t)(nx * ny * slices / 8), (uint32_t)ny,
                         (uint32_t)(nx / 8), d_circle, h};
            if (paired) hist_disc_stream<true><<<(unsigned)blocks, kThreads, 0, s>>>(S);
            else hist_disc_stream<false><<<(unsigned)blocks, kThreads, 0, s>>>(S);
        } else {
            DiscRange R{d_vol, nx, ny, ny * slices, d_circle, h};
            if (paired) hist_disc_kernel<true><<<(unsigned)blocks, kThreads, 0, s>>>(R);
            else hist_disc_kernel<false><<<(unsigned)blocks, kThreads, 0, s>>>(R);
        }
    };
    if (d_hist_top != nullptr) {
        launch(top_slices, d_hist_top);
        rc = vr::check_launch("vr_histogram_in_disc: top slices");
        if (rc) return rc;
    }
    launch(nz, d_hist);
    rc = vr::check_launch("vr_histogram_in_disc");
    if (rc || !paired) return rc;
    return launch_unpack(s, d_hist, d_hist_top, "vr_histogram_in_disc: unpack");
}
