// Device-side pieces of the 65536-bin histogram shared by the single-volume
// kernels and the batched persistent kernel: packed 16-bit LDS counters with
// carry to global 64-bit bins, wave-uniform chunk aggregation, the streaming
// count of a voxel run, and the flush.
#pragma once

#include "common.h"

namespace vr {
namespace hg {

constexpr int kThreads = 1024;          // threads of a histogram workgroup
constexpr int kWords = VR_NBINS / 2;      // packed LDS words
constexpr int kUnroll = 8;                // 16-byte loads per thread per batch (two batches in flight)
constexpr uint32_t kMark = 0x8000u;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// streaming 16-byte load (the volume is read once; keep it out of the caches' way)
__device__ __forceinline__ uint4 load_stream(const uint4* p)
{
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

// Global bins: one 64-bit counter per bin, or (PAIRED) bins 2w and 2w + 1 as
// the low and high 32-bit halves of word w, so that one 64-bit atomic adds
// to both (valid while every bin's total stays below 2^32; unpack_pairs then
// spreads the words into 64-bit bins).
template <bool PAIRED = false>
__device__ __forceinline__ void add_global(uint64_t* h, uint32_t b, uint64_t v)
{
    if (PAIRED) __hip_atomic_fetch_add(h + (b >> 1), v << ((b & 1u) << 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else __hip_atomic_fetch_add(h + b, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Adds n (1..512) to bin v in the packed LDS histogram, carrying to global.
template <bool PAIRED = false>
__device__ __forceinline__ void count_n(uint32_t* lds, uint64_t* gh, uint32_t v, uint32_t n)
{
    const uint32_t sh = (v & 1u) << 4;
    const uint32_t old = atomicAdd(lds + (v >> 1), n << sh);
    const uint32_t half = (old >> sh) & 0xFFFFu;
    if (half < kMark && half + n >= kMark) {
        atomicSub(lds + (v >> 1), kMark << sh);
        add_global<PAIRED>(gh, v, kMark);
    }
}

// Adds 1 to bin v: the counter crosses the mark exactly when it held 0x7FFF.
template <bool PAIRED = false>
__device__ __forceinline__ void count_1(uint32_t* lds, uint64_t* gh, uint32_t v)
{
    const uint32_t sh = (v & 1u) << 4;
    const uint32_t old = atomicAdd(lds + (v >> 1), 1u << sh);
    if (((old >> sh) & 0xFFFFu) == kMark - 1u) {
        atomicSub(lds + (v >> 1), kMark << sh);
        add_global<PAIRED>(gh, v, kMark);
    }
}

template <bool PAIRED = false>
__device__ __forceinline__ void count_chunk(uint32_t* lds, uint64_t* gh, uint4 c)
{
    // wave-uniform chunk: every lane holds eight copies of the first lane's value
    const uint32_t v0 = c.x & 0xFFFFu;
    const bool same8 = (c.x >> 16) == v0 && c.y == c.x && c.z == c.x && c.w == c.x;
    const uint32_t w0 = __builtin_amdgcn_readfirstlane(v0);
    const uint64_t act = __ballot(1);
    if (__ballot(same8 && v0 == w0) == act) {
        if (__lane_id() == (uint32_t)__builtin_ctzll(act)) count_n<PAIRED>(lds, gh, w0, 8u * (uint32_t)__popcll(act));
        return;
    }
    count_1<PAIRED>(lds, gh, c.x & 0xFFFFu);
    count_1<PAIRED>(lds, gh, c.x >> 16);
    count_1<PAIRED>(lds, gh, c.y & 0xFFFFu);
    count_1<PAIRED>(lds, gh, c.y >> 16);
    count_1<PAIRED>(lds, gh, c.z & 0xFFFFu);
    count_1<PAIRED>(lds, gh, c.z >> 16);
    count_1<PAIRED>(lds, gh, c.w & 0xFFFFu);
    count_1<PAIRED>(lds, gh, c.w >> 16);
}

// The block's share of a contiguous run of n voxels starting at vol: block
// thread `gtid` of `nthr` threads over all the blocks given to the run.
// head voxels up to the first 16-byte boundary and the tail are counted one
// by one, the body in 16-byte chunks, two batches of loads in flight.
template <bool PAIRED = false>
__device__ __forceinline__ void count_range(uint32_t* lds, uint64_t* gh, const uint16_t* vol, int64_t n,
                                            int64_t gtid, int64_t nthr)
{
    int64_t head = (int64_t)(((16u - (reinterpret_cast<uintptr_t>(vol) & 15u)) & 15u) / 2u);
    if (head > n) head = n;
    const int64_t n_chunks = (n - head) / 8;
    const int64_t tail_beg = head + n_chunks * 8;
    if (gtid < head) count_n<PAIRED>(lds, gh, vol[gtid], 1u);
    if (gtid < n - tail_beg) count_n<PAIRED>(lds, gh, vol[tail_beg + gtid], 1u);

    const uint4* body = reinterpret_cast<const uint4*>(vol + head);
    const int64_t stride = kUnroll * nthr;
    int64_t i = gtid;
    if (i + (kUnroll - 1) * nthr < n_chunks) {
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
            for (int u = 0; u < kUnroll; ++u) count_chunk<PAIRED>(lds, gh, cur[u]);
            i = nx;
            if (!more) break;
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) cur[u] = nxt[u];
        }
    }
    for (; i < n_chunks; i += nthr) count_chunk<PAIRED>(lds, gh, load_stream(body + i));
}

// Zero the block's packed LDS histogram (blockDim.x == kThreads).
__device__ __forceinline__ void zero_lds(uint32_t* lds)
{
    for (int w = threadIdx.x * 4; w < kWords; w += kThreads * 4)
        *reinterpret_cast<uint4*>(lds + w) = make_uint4(0, 0, 0, 0);
}

// Add the block's non-zero counters to the global bins; whole waves of empty
// words are skipped by ballot.  PAIRED: one atomic per word for both bins.
template <bool PAIRED = false>
__device__ __forceinline__ void flush_lds(const uint32_t* lds, uint64_t* gh)
{
    for (int w = threadIdx.x; w < kWords; w += kThreads) {
        const uint32_t x = lds[w];
        if (__ballot(x != 0) == 0) continue;
        if (PAIRED) {
            if (x) add_global<false>(gh, w, (uint64_t)(x & 0xFFFFu) | ((uint64_t)(x >> 16) << 32));
        } else {
            if (x & 0xFFFFu) add_global(gh, 2 * w, x & 0xFFFFu);
            if (x >> 16) add_global(gh, 2 * w + 1, x >> 16);
        }
    }
}

}  // namespace hg
}  // namespace vr
