// Best-view snapshot (Section III-C, Eq. 2): the Shannon entropy of the
// 256-bin grey-value histogram of every rendered frame, and the first view of
// maximal entropy.
//
// A frame's pixels become 8-bit channel codes q = floor(255 clamp(c, 0, 1) +
// 1/2) (FP32: product, then sum) and the integer BT.601 grey value
// (77 q_r + 150 q_g + 29 q_b + 128) >> 8.  Workgroups of 256 threads count a
// share of one view's pixels in an LDS histogram (a wave whose pixels all have
// one grey value adds them with one atomic: frames hold large uniform
// regions) and add it to the view's global counts; one workgroup then forms
// -sum p log2 p in FP64, a wave per view with a fixed-order shuffle sum, and
// picks the best view.
#include <cmath>

#include "entropy_dev.h"

namespace {

constexpr int kT = 256;

__global__ void __launch_bounds__(kT) zero_u32(uint32_t* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) p[i] = 0u;
}

// grid (blocks per view, views)
__global__ void __launch_bounds__(kT)
frame_hist_kernel(const float4* __restrict__ rgba, int64_t pix, uint32_t* __restrict__ hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const int view = (int)blockIdx.y;
    const float4* f = rgba + (int64_t)view * pix;
    // four pixels per thread per round, loads first
    constexpr int kU = 4;
    const int64_t stride = (int64_t)gridDim.x * kT;
    for (int64_t i0 = (int64_t)blockIdx.x * kT + threadIdx.x; i0 - threadIdx.x < pix; i0 += kU * stride) {
        float4 px[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t i = i0 + u * stride;
            px[u] = i < pix ? f[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t i = i0 + u * stride;
            vr::ent::count_grey(h, i < pix, vr::ent::grey_code(px[u]));
        }
    }
    __syncthreads();
    const uint32_t c = h[threadIdx.x];
    if (c) atomicAdd(hist + (int64_t)view * 256 + threadIdx.x, c);
}

// one workgroup of kE threads: each wave forms the entropy of one view at a
// time (four bins per lane, a fixed-order shuffle sum), then thread 0 picks
// the first view of maximal entropy
constexpr int kE = 1024;

__global__ void __launch_bounds__(kE)
entropy_kernel(const uint32_t* __restrict__ hist, int n_views, int64_t pix, double* __restrict__ ent,
               int32_t* __restrict__ best)
{
    __shared__ double s_h[kE / 64];
    __shared__ int s_v[kE / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, waves = kE / 64;
    double best_h = -1.0;          // this wave's first view of maximal entropy
    int best_v = n_views;
    for (int v = w; v < n_views; v += waves) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t c = hist[(int64_t)v * 256 + q * 64 + lane];
            if (c) {
                const double p = (double)c / (double)pix;
                sum += -p * log2(p);
            }
        }
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
        if (lane == 0) ent[v] = sum;
        if (sum > best_h) {
            best_h = sum;
            best_v = v;
        }
    }
    if (lane == 0) {
        s_h[w] = best_h;
        s_v[w] = best_v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double bh = s_h[0];
        int bv = s_v[0];
        for (int k = 1; k < waves; ++k)
            if (s_h[k] > bh || (s_h[k] == bh && s_v[k] < bv)) {
                bh = s_h[k];
                bv = s_v[k];
            }
        best[0] = bv;
    }
}

}  // namespace

extern "C" int vr_frame_entropy(const float* d_rgba, int n_views, int width, int height, uint32_t* d_hist,
                                double* d_entropy, int32_t* d_best, void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_rgba && d_hist && d_entropy && d_best, VR_ERR_NULL, "vr_frame_entropy: NULL pointer");
    VR_REQUIRE(n_views >= 1 && width >= 1 && height >= 1, VR_ERR_DIMS,
               "vr_frame_entropy: %d views of %d x %d", n_views, width, height);
    const int64_t pix = (int64_t)width * height;
    VR_REQUIRE(pix < (int64_t(1) << 32) && n_views <= 65535, VR_ERR_DIMS,
               "vr_frame_entropy: frames too large");
    hipStream_t s = vr::as_stream(stream);
    const int64_t nh = (int64_t)n_views * 256;
    zero_u32<<<(unsigned)std::min<int64_t>(vr::ceil_div<int64_t>(nh, kT), 1024), kT, 0, s>>>(d_hist, nh);
    int rc = vr::check_launch("vr_frame_entropy: zero");
    if (rc) return rc;
    // enough workgroups per view to fill the compute units a few times over
    const int64_t want = std::max<int64_t>(1, (int64_t)vr::num_cus() * 8 / n_views);
    const int bx = (int)std::min<int64_t>(want, vr::ceil_div<int64_t>(pix, kT));
    frame_hist_kernel<<<dim3((unsigned)bx, (unsigned)n_views), kT, 0, s>>>(
        reinterpret_cast<const float4*>(d_rgba), pix, d_hist);
    rc = vr::check_launch("vr_frame_entropy: histograms");
    if (rc) return rc;
    entropy_kernel<<<1, kE, 0, s>>>(d_hist, n_views, pix, d_entropy, d_best);
    return vr::check_launch("vr_frame_entropy");
}

extern "C" int vr_entropy_from_counts(const uint32_t* d_hist, int n_views, int64_t pixels, double* d_entropy,
                                      int32_t* d_best, void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_hist && d_entropy && d_best, VR_ERR_NULL, "vr_entropy_from_counts: NULL pointer");
    VR_REQUIRE(n_views >= 1 && n_views <= 65535 && pixels >= 1 && pixels < (int64_t(1) << 32), VR_ERR_DIMS,
               "vr_entropy_from_counts: %d views of %lld pixels", n_views, (long long)pixels);
    entropy_kernel<<<1, kE, 0, vr::as_stream(stream)>>>(d_hist, n_views, pixels, d_entropy, d_best);
    return vr::check_launch("vr_entropy_from_counts");
}
