// Adjoint of the emission-absorption ray caster (the gradient of an image
// loss with respect to the density grid and the transfer-function table),
// for fitting a coarse preview volume to full-resolution renders.  Each ray
// is re-marched with the forward's samples (shared code in raycast_dev.h,
// built with contraction off), so it replays the forward's transmittances
// and stops at the same sample; nothing is stored per sample.
#include <cmath>

#include "raycast_dev.h"

namespace {

using namespace vr::rc;

// One wave per workgroup (an 8 x 8-pixel tile), as in the forward: a
// workgroup's slot frees only when its last ray ends.  Registers (over 100 per
// lane) allow four waves per SIMD, the 12 KiB of LDS thirteen workgroups per CU.
constexpr int kThreads = 64;

__device__ __forceinline__ void flush_tf(float* g, int k, float4 a0, float4 a1)
{
    atomicAdd(g + 4 * k + 0, a0.x);
    atomicAdd(g + 4 * k + 1, a0.y);
    atomicAdd(g + 4 * k + 2, a0.z);
    atomicAdd(g + 4 * k + 3, a0.w);
    atomicAdd(g + 4 * k + 4, a1.x);
    atomicAdd(g + 4 * k + 5, a1.y);
    atomicAdd(g + 4 * k + 6, a1.z);
    atomicAdd(g + 4 * k + 7, a1.w);
}

// Density-gradient atomics are performed at the memory side of the fabric (on
// this device every one of them shows in the memory-side atomic count), one
// request per cache line and instruction, so their cost follows the number
// of (instruction, line) pairs.  A lane that holds one cell's eight taps would issue eight
// instructions whose lanes hit unrelated lines.  Instead the lanes of a wave
// that flush a cell write its non-zero (offset, gradient) pairs, packed, to
// the wave's slice of LDS, and the active lanes then take consecutive
// entries: the taps of one cell (x pairs adjacent in memory) and of the
// neighbouring rays' cells go out in the same instruction and share lines.
constexpr int kFlushSlots = 64 * 8;   // entries per wave: every lane flushing one cell

__device__ __forceinline__ void wave_flush(bool f, const uint32_t (&off)[8], const float (&gc)[8],
                                           float* __restrict__ gvol, uint2* __restrict__ buf)
{
    if (__ballot(f) == 0) return;
    const uint32_t lane = __lane_id();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64u - lane));
    // the lane's non-zero entries, packed after those of the lanes below it
    int c = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) c += (f && gc[t] != 0.0f) ? 1 : 0;
    int first = 0, n = 0;
#pragma unroll
    for (int bit = 0; bit < 4; ++bit) {
        const uint64_t m = __ballot((c >> bit) & 1);
        first += __popcll(m & below) << bit;
        n += __popcll(m) << bit;
    }
    if (f) {
        int q = first;
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (gc[t] != 0.0f) buf[q++] = make_uint2(off[t], __float_as_uint(gc[t]));
    }
    // the wave's own LDS writes above are complete before any lane reads them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint64_t act = __ballot(true);
    const int n_act = __popcll(act), me = __popcll(act & below);
    for (int base = 0; base < n; base += n_act) {
        const int q = base + me;
        if (q < n) {
            const uint2 e = buf[q];
            atomicAdd(gvol + e.x, __uint_as_float(e.y));
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int LAYOUT>
__global__ void __launch_bounds__(kThreads)
raycast_bwd(const Views V, const Scene S, const float4* __restrict__ tf,
            const float4* __restrict__ fwd, const float4* __restrict__ grad, float* __restrict__ gvol,
            float* __restrict__ gtf)
{
    __shared__ float4 tf_s[256];
    __shared__ float gtf_s[256 * 4];
    __shared__ uint2 flush_s[kThreads / 64][kFlushSlots];
    uint2* const fbuf = flush_s[threadIdx.x >> 6];
    for (int q = threadIdx.x; q < 256; q += kThreads) tf_s[q] = tf[q];
    for (int q = threadIdx.x; q < 1024; q += kThreads) gtf_s[q] = 0.0f;
    __syncthreads();
    // empty bricks may be passed over when the first TF segment has zero extinction
    // (a sample at density 0 then has neither extinction nor a density gradient)
    const bool skipping = S.occ != nullptr && tf_s[0].w == 0.0f && tf_s[1].w == 0.0f && isfinite(tf_s[0].x) &&
                          isfinite(tf_s[0].y) && isfinite(tf_s[0].z);
    int view, i, j;
    tile_pixel<8, 8>(S, (int)gridDim.x, view, i, j);
    const float* vol = static_cast<const float*>(S.data);
    uint32_t cell_off[8];        // taps of the cell whose density gradient is pending
    float cell_g[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        cell_off[t] = 0xFFFFFFFFu;
        cell_g[t] = 0.0f;
    }
    if (i < S.W && j < S.H) {
        const View& v = V.v[view];
        float p[3], d[3], L;
        if (setup_ray(v, S, i, j, p, d, L)) {
            const int64_t pix = ((int64_t)(S.view0 + view) * S.H + j) * S.W + i;
            const float4 g = grad[pix];
            const float4 I = fwd[pix];
            const float ga = g.w * (1.0f - I.w);
            const int n = step_count(L, S.step);
            const float last = L - (float)(n - 1) * S.step;
            float Tr = 1.0f, Pr = 0.0f, Pg = 0.0f, Pb = 0.0f;
            int kc = -1;
            float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = a0;
            float u0[3], gr[3], ig[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                u0[a] = fmaf(p[a], S.inv_sp[a], -0.5f);
                gr[a] = d[a] * S.inv_sp[a];
                ig[a] = gr[a] != 0.0f ? 1.0f / gr[a] : 0.0f;
            }
            const SkipRay SR = skip_ray(S, u0, gr, ig, 2);
            uint32_t cur_b = 0xFFFFFFFFu;
            uint32_t cur_r = 0u;     // distance byte of brick cur_b (0: occupied)
            const float half_last = 0.5f * last;
            for (int k = 0; k < n;) {
                const bool inner = k < n - 1;
                const float len = inner ? S.step : last;
                const Cell c = cell_at(S, u0, gr, sample_mid(S, k, inner, half_last));
                if (skipping) {
                    const uint32_t b = ((c.z0 >> 2) * (uint32_t)S.nby + (c.y0 >> 2)) * (uint32_t)S.nbx + (c.x0 >> 2);
                    if (b != cur_b) {
                        cur_b = b;
                        cur_r = S.dist[b];
                    }
                    if (cur_r != 0u) {
                        // a run of samples whose eight taps are all 0: density 0, zero
                        // extinction and colour weight, so the colour, the transmittance and
                        // the density gradient are unchanged; each sample's only gradient is
                        // len * q to the first knot's extinction, added for the whole run
                        // (the run leaves the cube of empty bricks the distance grid gives)
                        const uint32_t bb[3] = {c.x0 >> 2, c.y0 >> 2, c.z0 >> 2};
                        const int next = skip_cube_ray(S, SR, gr, bb, cur_r, k, n);
                        const float lsum = next < n ? (float)(next - k) * S.step
                                                    : fmaf((float)(n - 1 - k), S.step, last);
                        const float q = g.x * (Tr * tf_s[0].x - (I.x - Pr)) + g.y * (Tr * tf_s[0].y - (I.y - Pg)) +
                                        g.z * (Tr * tf_s[0].z - (I.z - Pb)) + ga;
                        if (kc != 0) {
                            if (kc >= 0) flush_tf(gtf_s, kc, a0, a1);
                            kc = 0;
                            a0 = make_float4(0.f, 0.f, 0.f, 0.f);
                            a1 = a0;
                        }
                        a0.w = fmaf(lsum, q, a0.w);
                        k = next;
                        continue;
                    }
                }
                Sample sm;
                sample<float, LAYOUT>(S, vol, c, sm);
                const TfHit h = tf_lookup(tf_s, sm.s * tf_scale<float>());
                const float e = transmit(h.q.w, len * kNegLog2E);
                const float te = Tr * e;
                const float ta = Tr - te;     // Tr (1 - e), as the forward takes it
                Pr = fmaf(ta, h.q.x, Pr);
                Pg = fmaf(ta, h.q.y, Pg);
                Pb = fmaf(ta, h.q.z, Pb);
                // dI/drgb_i = T_i alpha_i;  dI/dsigma_i = len (T_{i+1} rgb_i - (I - P_i)) (+ alpha term)
                const float gs = len * (g.x * (te * h.q.x - (I.x - Pr)) + g.y * (te * h.q.y - (I.y - Pg)) +
                                        g.z * (te * h.q.z - (I.z - Pb)) + ga);
                const float4 G = make_float4(g.x * ta, g.y * ta, g.z * ta, gs);
                if (h.k != kc) {
                    if (kc >= 0) flush_tf(gtf_s, kc, a0, a1);
                    kc = h.k;
                    a0 = make_float4(0.f, 0.f, 0.f, 0.f);
                    a1 = a0;
                }
                const float w0 = 1.0f - h.w;
                a0.x = fmaf(w0, G.x, a0.x); a0.y = fmaf(w0, G.y, a0.y);
                a0.z = fmaf(w0, G.z, a0.z); a0.w = fmaf(w0, G.w, a0.w);
                a1.x = fmaf(h.w, G.x, a1.x); a1.y = fmaf(h.w, G.y, a1.y);
                a1.z = fmaf(h.w, G.z, a1.z); a1.w = fmaf(h.w, G.w, a1.w);
                float ds = 0.0f;
                if (sm.s >= 0.0f && sm.s <= 1.0f) {
                    const float4 ka = tf_s[h.k], kb = tf_s[h.k + 1];
                    ds = 255.0f * ((kb.x - ka.x) * G.x + (kb.y - ka.y) * G.y + (kb.z - ka.z) * G.z +
                                   (kb.w - ka.w) * G.w);
                }
                // consecutive samples of one cell add to the same eight taps: their
                // gradients are summed in registers.  When the ray moves on, the taps
                // the new cell shares with the pending one keep their sums (each old
                // tap goes to the first new tap with its offset) and only the others
                // are scattered.
                const bool change = ds != 0.0f && (sm.off[0] != cell_off[0] || sm.off[7] != cell_off[7]);
                float carry[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) carry[t] = 0.0f;
                if (change) {
#pragma unroll
                    for (int a = 0; a < 8; ++a) {
                        bool moved = false;
#pragma unroll
                        for (int t = 0; t < 8; ++t) {
                            const bool hit = !moved && cell_off[a] == sm.off[t];
                            carry[t] += hit ? cell_g[a] : 0.0f;
                            moved = moved || hit;
                        }
                        if (moved) cell_g[a] = 0.0f;
                    }
                }
                wave_flush(change && cell_off[0] != 0xFFFFFFFFu, cell_off, cell_g, gvol, fbuf);
                if (change) {
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        cell_off[t] = sm.off[t];
                        cell_g[t] = carry[t];
                    }
                }
                if (ds != 0.0f) {
                    const float ax = 1.0f - sm.wx, ay = 1.0f - sm.wy, az = 1.0f - sm.wz;
                    const float w[8] = {ax * ay * az, sm.wx * ay * az, ax * sm.wy * az, sm.wx * sm.wy * az,
                                        ax * ay * sm.wz, sm.wx * ay * sm.wz, ax * sm.wy * sm.wz,
                                        sm.wx * sm.wy * sm.wz};
#pragma unroll
                    for (int t = 0; t < 8; ++t) cell_g[t] = fmaf(w[t], ds, cell_g[t]);
                }
                Tr = te;
                ++k;
                if (Tr < S.eps) break;
            }
            if (kc >= 0) flush_tf(gtf_s, kc, a0, a1);
        }
    }
    // the last pending cell of every ray, with the whole wave converged
    wave_flush(cell_off[0] != 0xFFFFFFFFu, cell_off, cell_g, gvol, fbuf);
    __syncthreads();
    for (int q = threadIdx.x; q < 1024; q += kThreads) {
        const float x = gtf_s[q];
        if (x != 0.0f) atomicAdd(gtf + q, x);
    }
}

}  // namespace

extern "C" int vr_raycast_backward(const vr_volume* vol, const float* d_tf, const vr_camera* h_cams,
                                   int n_views, const vr_render_opts* opts,
                                   const float* d_rgba_fwd, const float* d_grad_rgba,
                                   float* d_grad_density, float* d_grad_tf, void* stream)
{
    vr::clear_error();
    Scene S{};
    int rc = build_scene(vol, d_tf, h_cams, n_views, opts, S);
    if (rc) return rc;
    set_tiles<8, 8>(S);
    VR_REQUIRE(vol->dtype == VR_F32, VR_ERR_DTYPE, "vr_raycast_backward: density must be VR_F32");
    VR_REQUIRE(vol->layout == VR_LAYOUT_LINEAR || vol->layout == VR_LAYOUT_BRICK4, VR_ERR_UNSUPPORTED,
               "vr_raycast_backward: the density gradient is produced for the linear and brick layouts only");
    // the occupancy of vr_brick_volume on the same grid, if given, lets the adjoint
    // pass over empty bricks (build_scene keeps it for the brick layouts only)
    S.occ = vol->occupancy;
    S.dist = vol->occupancy ? vol->occupancy + (int64_t)S.nbx * S.nby * S.nbz + (int64_t)S.nmx * S.nmy * S.nmz
                            : nullptr;
    VR_REQUIRE(d_rgba_fwd && d_grad_rgba && d_grad_density && d_grad_tf, VR_ERR_NULL,
               "vr_raycast_backward: NULL buffer");
    hipStream_t s = vr::as_stream(stream);
    for (int v0 = 0; v0 < n_views; v0 += kMaxViews) {
        const int nv = std::min(kMaxViews, n_views - v0);
        Views V{};
        rc = build_views(h_cams + v0, nv, V);
        if (rc) return rc;
        S.view0 = v0;
        const int64_t blocks = (int64_t)S.tiles_x * S.tiles_y * nv;
        VR_REQUIRE(blocks < (int64_t(1) << 31), VR_ERR_DIMS, "vr_raycast_backward: too many tiles");
        const auto* tf4 = reinterpret_cast<const float4*>(d_tf);
        const auto* fwd4 = reinterpret_cast<const float4*>(d_rgba_fwd);
        const auto* grad4 = reinterpret_cast<const float4*>(d_grad_rgba);
        if (vol->layout == VR_LAYOUT_BRICK4)
            raycast_bwd<VR_LAYOUT_BRICK4><<<(unsigned)blocks, kThreads, 0, s>>>(V, S, tf4, fwd4, grad4,
                                                                                d_grad_density, d_grad_tf);
        else
            raycast_bwd<VR_LAYOUT_LINEAR><<<(unsigned)blocks, kThreads, 0, s>>>(V, S, tf4, fwd4, grad4,
                                                                                d_grad_density, d_grad_tf);
        rc = vr::check_launch("vr_raycast_backward");
        if (rc) return rc;
    }
    return VR_OK;
}
