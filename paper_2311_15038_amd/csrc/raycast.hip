// Emission-absorption ray casting of the reduced volume into preview frames
// (Section III-C: the volume rendered to 2D images while it turns about Z).
// The adjoint is in raycast_bwd.hip.
//
// Launch shape: a workgroup is one wave, an 8 x 8-pixel ray tile, so the 64
// rays of a wave are neighbours and their trilinear taps share cache lines.
// Ray lengths vary widely and a workgroup's slot frees only when its last
// ray ends, so one-wave workgroups keep the compute units fuller than 16 x 16
// tiles of four waves (2.70 against 3.06 ms on the 36-view 512^2 turntable
// of a 512^3 level).  Workgroup ids are remapped so that the tiles of one
// view that run at the same time sit on the same XCD (consecutive ids are
// dealt round-robin over the 8 XCDs, each with its own L2).  The transfer
// function's knots are staged in LDS (4 KiB, so LDS leaves the occupancy at
// eight waves per SIMD).  Samples are FP32 with explicit fused
// multiply-adds (the library builds with contraction off), so the forward and
// the adjoint replay bit-identical transmittances and stop at the same sample.
#include <cmath>
#include <type_traits>

#include "raycast_dev.h"
#include "raycast_staged.h"

namespace {

using namespace vr::rc;

constexpr int kThreads = 64;   // one wave: an 8 x 8-pixel tile

__global__ void __launch_bounds__(kThreads) zero_u32(uint32_t* __restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// The depth-window march with LDS staging (raycast_staged.h), same epilogue.
template <bool COUNT>
__global__ void __launch_bounds__(kThreads)
raycast_fwd_staged(const Views V, const Scene S, const float4* __restrict__ tf, float4* __restrict__ out,
                   unsigned long long* __restrict__ samples)
{
    __shared__ TfLds tf_s;
    __shared__ uint32_t grey[256];
    __shared__ __align__(16) uint16_t reg[kRegCap];
    stage_tf(tf_s, tf, (int)threadIdx.x, kThreads);
    if (S.view_hist)
        for (int q = (int)threadIdx.x; q < 256; q += kThreads) grey[q] = 0u;
    __syncthreads();
    const bool skip = can_skip(S, tf_s);
    int view, i, j;
    tile_pixel<8, 8>(S, (int)gridDim.x, view, i, j);
    uint32_t cnt = 0, evals = 0;
    const bool in = i < S.W && j < S.H;
    const float4 res = march_staged<COUNT>(S, V.v[view], static_cast<const uint16_t*>(S.data), tf_s, reg, skip, i,
                                           j, in, cnt, evals);
    if (in) out[((int64_t)(S.view0 + view) * S.H + j) * S.W + i] = res;
    if (S.view_hist) {
        vr::ent::count_grey(grey, in, vr::ent::grey_code(res));
        __syncthreads();
        for (int q = (int)threadIdx.x; q < 256; q += kThreads) {
            const uint32_t c = grey[q];
            if (c) atomicAdd(S.view_hist + (int64_t)(S.view0 + view) * 256 + q, c);
        }
    }
    if (COUNT) {
        unsigned long long c = cnt, e = evals;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            c += __shfl_xor(c, off);
            e += __shfl_xor(e, off);
        }
        if ((threadIdx.x & 63) == 0 && c) atomicAdd(samples, c);
        if ((threadIdx.x & 63) == 0 && e) atomicAdd(samples + 1, e);
    }
}

template <typename T, int LAYOUT, bool COUNT, bool WIDE>
__global__ void __launch_bounds__(kThreads)
raycast_fwd(const Views V, const Scene S, const float4* __restrict__ tf, float4* __restrict__ out,
            unsigned long long* __restrict__ samples)
{
    __shared__ TfLds tf_s;
    __shared__ uint32_t grey[256];
    stage_tf(tf_s, tf, (int)threadIdx.x, kThreads);
    if (S.view_hist)
        for (int q = (int)threadIdx.x; q < 256; q += kThreads) grey[q] = 0u;
    __syncthreads();
    const bool skip = can_skip(S, tf_s);
    int view, i, j;
    tile_pixel<8, 8>(S, (int)gridDim.x, view, i, j);
    uint32_t cnt = 0, evals = 0;
    const bool in = i < S.W && j < S.H;
    float4 res = make_float4(0.f, 0.f, 0.f, 0.f);
    if (in) {
        res = march<T, LAYOUT, COUNT, WIDE>(S, V.v[view], static_cast<const T*>(S.data), tf_s, skip, i, j, cnt,
                                            evals);
        out[((int64_t)(S.view0 + view) * S.H + j) * S.W + i] = res;
    }
    if (S.view_hist) {
        // grey-value counts of the tile for the best-view snapshot (one view per workgroup)
        vr::ent::count_grey(grey, in, vr::ent::grey_code(res));
        __syncthreads();
        for (int q = (int)threadIdx.x; q < 256; q += kThreads) {
            const uint32_t c = grey[q];
            if (c) atomicAdd(S.view_hist + (int64_t)(S.view0 + view) * 256 + q, c);
        }
    }
    if (COUNT) {
        unsigned long long c = cnt, e = evals;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            c += __shfl_xor(c, off);
            e += __shfl_xor(e, off);
        }
        if ((threadIdx.x & 63) == 0 && c) atomicAdd(samples, c);
        if ((threadIdx.x & 63) == 0 && e) atomicAdd(samples + 1, e);
    }
}

// One forward launch with the kernel variant for the volume's type, layout,
// counting and addressing width.
template <typename T, int LAYOUT>
void launch_fwd(unsigned blocks, hipStream_t s, const Views& V, const Scene& S, const float4* tf, float4* out,
                unsigned long long* cnt, bool staged)
{
    const bool wide = needs_wide(S);
    if (staged) {                // u16, 4^3 bricks with occupancy, 32-bit addressing (checked by the caller)
        if (cnt) raycast_fwd_staged<true><<<blocks, kThreads, 0, s>>>(V, S, tf, out, cnt);
        else raycast_fwd_staged<false><<<blocks, kThreads, 0, s>>>(V, S, tf, out, cnt);
        return;
    }
    if constexpr (!Lay<LAYOUT>::ovl) {   // the overlap layout takes 32-bit offsets only (checked by the scene)
        if (wide) {
            if (cnt) raycast_fwd<T, LAYOUT, true, true><<<blocks, kThreads, 0, s>>>(V, S, tf, out, cnt);
            else raycast_fwd<T, LAYOUT, false, true><<<blocks, kThreads, 0, s>>>(V, S, tf, out, cnt);
            return;
        }
    }
    if (cnt) raycast_fwd<T, LAYOUT, true, false><<<blocks, kThreads, 0, s>>>(V, S, tf, out, cnt);
    else raycast_fwd<T, LAYOUT, false, false><<<blocks, kThreads, 0, s>>>(V, S, tf, out, cnt);
}

}  // namespace

extern "C" int vr_raycast(const vr_volume* vol, const float* d_tf, const vr_camera* h_cams,
                          int n_views, const vr_render_opts* opts, float* d_rgba,
                          uint64_t* d_samples, void* stream)
{
    vr::clear_error();
    Scene S{};
    int rc = build_scene(vol, d_tf, h_cams, n_views, opts, S);
    if (rc) return rc;
    VR_REQUIRE(d_rgba != nullptr, VR_ERR_NULL, "vr_raycast: d_rgba is NULL");
    const bool staged = (opts->flags & VR_RENDER_STAGED) != 0u;
    VR_REQUIRE(!staged || (vol->dtype == VR_U16_NORM && vol->layout == VR_LAYOUT_BRICK4 && vol->occupancy != nullptr &&
                           !needs_wide(S)),
               VR_ERR_UNSUPPORTED,
               "vr_raycast: VR_RENDER_STAGED takes a u16 volume in VR_LAYOUT_BRICK4 with its occupancy "
               "(at most 2^24 bricks)");
    set_tiles<8, 8>(S);
    hipStream_t s = vr::as_stream(stream);
    if (S.view_hist) {
        const int64_t n = (int64_t)n_views * 256;
        zero_u32<<<(unsigned)vr::ceil_div<int64_t>(n, kThreads), kThreads, 0, s>>>(S.view_hist, n);
        rc = vr::check_launch("vr_raycast: view counts");
        if (rc) return rc;
    }
    for (int v0 = 0; v0 < n_views; v0 += kMaxViews) {
        const int nv = std::min(kMaxViews, n_views - v0);
        Views V{};
        rc = build_views(h_cams + v0, nv, V);
        if (rc) return rc;
        S.view0 = v0;
        const int64_t blocks = (int64_t)S.tiles_x * S.tiles_y * nv;
        VR_REQUIRE(blocks < (int64_t(1) << 31), VR_ERR_DIMS, "vr_raycast: too many tiles");
        auto* out = reinterpret_cast<float4*>(d_rgba);
        auto* cnt = reinterpret_cast<unsigned long long*>(d_samples);
        const auto* tf = reinterpret_cast<const float4*>(d_tf);
        const unsigned nb = (unsigned)blocks;
        const int L = vol->layout;
        if (vol->dtype == VR_U16_NORM) {
            if (L == VR_LAYOUT_BRICK4_PAIRS) launch_fwd<uint16_t, VR_LAYOUT_BRICK4_PAIRS>(nb, s, V, S, tf, out, cnt, false);
            else if (L == VR_LAYOUT_BRICK4) launch_fwd<uint16_t, VR_LAYOUT_BRICK4>(nb, s, V, S, tf, out, cnt, staged);
            else if (L == VR_LAYOUT_BRICK8) launch_fwd<uint16_t, VR_LAYOUT_BRICK8>(nb, s, V, S, tf, out, cnt, false);
            else if (L == VR_LAYOUT_BRICK4_OVERLAP)
                launch_fwd<uint16_t, VR_LAYOUT_BRICK4_OVERLAP>(nb, s, V, S, tf, out, cnt, false);
            else launch_fwd<uint16_t, VR_LAYOUT_LINEAR>(nb, s, V, S, tf, out, cnt, false);
        } else {
            if (L == VR_LAYOUT_BRICK4_PAIRS) launch_fwd<float, VR_LAYOUT_BRICK4_PAIRS>(nb, s, V, S, tf, out, cnt, false);
            else if (L == VR_LAYOUT_BRICK4) launch_fwd<float, VR_LAYOUT_BRICK4>(nb, s, V, S, tf, out, cnt, false);
            else if (L == VR_LAYOUT_BRICK8) launch_fwd<float, VR_LAYOUT_BRICK8>(nb, s, V, S, tf, out, cnt, false);
            else launch_fwd<float, VR_LAYOUT_LINEAR>(nb, s, V, S, tf, out, cnt, false);
        }
        rc = vr::check_launch("vr_raycast");
        if (rc) return rc;
    }
    return VR_OK;
}
