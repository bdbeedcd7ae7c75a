// Depth-window march with the voxels staged in LDS: an alternative to the
// gather march of raycast_dev.h for u16 volumes in the 4^3-brick layout with
// their occupancy (the nominal design of a brick-staging renderer; the
// library's default march reads the taps through the caches instead, and is
// the faster of the two on the turntable benchmark).
//
// A one-wave workgroup (8 x 8 rays) marches along its major axis M (the axis
// of the largest direction component, the same sign and at least a quarter
// of it on every ray, else the wave takes the gather march) in windows of D
// cells: the window starts at the cell of the wave's nearest sample still to
// be evaluated, the voxels every tap of the window's samples can reach are
// staged in LDS as a box (4-voxel brick rows, 8 bytes per lane, x aligned to
// rows), shrinking D from 4 until the box fits kRegCap voxels, and each lane
// evaluates its samples in the window from the box.  Empty bricks are left
// by the distance grid as in the gather march; a sample whose taps fall
// outside the box (or a window with no box) reads the taps through the
// caches.  Every sample is the gather march's own arithmetic on the same
// voxel values, so the frames are bit-identical.
#pragma once

#include "raycast_dev.h"

namespace vr {
namespace rc {

constexpr int kRegCap = 3072;   // voxels of the staged box (u16)

__device__ __forceinline__ int wave_min_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_min_f(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_max_f(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ uint32_t cell_axis(const Cell& c, int a) { return a == 0 ? c.x0 : a == 1 ? c.y0 : c.z0; }

// The ray's cell at sample k and its exp2 factor -log2(e) len (the march's own
// arithmetic).
__device__ __forceinline__ Cell cell_of(const Scene& S, const float u0[3], const float g[3], int k, int n, float last,
                                        float& nl2_len)
{
    const bool inner = k < n - 1;
    nl2_len = inner ? S.step * kNegLog2E : last * kNegLog2E;
    return cell_at(S, u0, g, sample_mid(S, k, inner, 0.5f * last));
}

template <bool COUNT>
__device__ float4 march_staged(const Scene& S, const View& v, const uint16_t* __restrict__ vol, const TfLds& tf,
                               uint16_t* __restrict__ reg, bool skip, int i, int j, bool in, uint32_t& cnt,
                               uint32_t& evals)
{
    float p[3] = {0.f, 0.f, 0.f}, d[3] = {1.f, 0.f, 0.f}, L = 0.f;
    const bool hit = in && setup_ray(v, S, i, j, p, d, L);
    int n = hit ? step_count(L, S.step) : 0;
    const float last = L - (float)(n - 1) * S.step;
    float u0[3], g[3], ig[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u0[a] = fmaf(p[a], S.inv_sp[a], -0.5f);
        g[a] = d[a] * S.inv_sp[a];
        ig[a] = g[a] != 0.0f ? 1.0f / g[a] : 0.0f;
    }
    const SkipRay SR = skip_ray(S, u0, g, ig, 2);
    // the wave's march axis: the largest |g| of its first ray that hits, the same sign and
    // |g_M| >= 0.25 on every ray that hits, else every lane marches through the caches
    const uint64_t hm = __ballot(hit);
    int M = 0, sgn = 1;
    bool ok = hm != 0ull;
    if (ok) {
        const int l0 = __ffsll((long long)hm) - 1;
        const float gx = __shfl(g[0], l0), gy = __shfl(g[1], l0), gz = __shfl(g[2], l0);
        M = (fabsf(gx) >= fabsf(gy) && fabsf(gx) >= fabsf(gz)) ? 0 : (fabsf(gy) >= fabsf(gz) ? 1 : 2);
        const float gm0 = M == 0 ? gx : M == 1 ? gy : gz;
        sgn = gm0 > 0.0f ? 1 : -1;
        const float gm = M == 0 ? g[0] : M == 1 ? g[1] : g[2];
        const bool good = !hit || (sgn > 0 ? gm >= 0.25f * fabsf(gm0) && gm > 0.0f : gm <= -0.25f * fabsf(gm0) && gm < 0.0f);
        ok = __ballot(good) == ~0ull;
    }
    if (!ok) {
        if (!in) return make_float4(0.f, 0.f, 0.f, 0.f);
        return march<uint16_t, VR_LAYOUT_BRICK4, COUNT, false>(S, v, vol, tf, skip, i, j, cnt, evals);
    }
    if (!hit) n = 0;
    const int nM = M == 0 ? S.nx : M == 1 ? S.ny : S.nz;
    const int A1 = M == 0 ? 1 : 0, A2 = M == 2 ? 1 : 2;      // the cross axes
    const int nA[3] = {S.nx, S.ny, S.nz};
    float Tr = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    int k = 0;
    uint32_t cur_b = 0xFFFFFFFFu, cur_r = 0u;
    while (true) {
        // advance over empty bricks to the next sample that must be evaluated
        int cm = 0;
        while (k < n) {
            float nl2_len;
            const Cell c = cell_of(S, u0, g, k, n, last, nl2_len);
            const uint32_t b = ((c.z0 >> 2) * (uint32_t)S.nby + (c.y0 >> 2)) * (uint32_t)S.nbx + (c.x0 >> 2);
            if (skip) {
                if (b != cur_b) {
                    cur_b = b;
                    cur_r = S.dist[b];
                }
                if (cur_r != 0u) {
                    const uint32_t bb[3] = {c.x0 >> 2, c.y0 >> 2, c.z0 >> 2};
                    const int next = skip_cube_ray(S, SR, g, bb, cur_r, k, n);
                    if (COUNT) cnt += (uint32_t)(next - k);
                    k = next;
                    continue;
                }
            }
            cm = (int)cell_axis(c, M);
            break;
        }
        const bool want = k < n;
        const int wfirst = sgn > 0 ? wave_min_i(want ? cm : 0x7FFFFFFF) : wave_max_i(want ? cm : -1);
        if (__ballot(want) == 0ull) break;
        // a window of D cells along M, shrunk until its box fits the LDS buffer
        int D = 4, wlo = 0, whi = 0, ox = 0, oy = 0, oz = 0, RX = 0, RY = 0, RZ = 0;
        bool staged = false;
        for (; D >= 1; D >>= 1) {
            wlo = sgn > 0 ? wfirst : max(wfirst - D + 1, 0);
            whi = sgn > 0 ? min(wfirst + D - 1, nM - 1) : wfirst;
            // the ray parameter where u_M leaves the window on its far side
            const float far = sgn > 0 ? (float)(whi + 1) : (float)wlo;
            float s0 = fmaf(0.5f, S.step, (float)k * S.step);
            float s1 = (far - u0[M]) * ig[M];
            s1 = fminf(s1, fmaf(0.5f, last, (float)(n - 1) * S.step));
            s1 = fmaxf(s1, s0);
            int lo[3], hi[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float ua = fmaf(s0, g[a], u0[a]), ub = fmaf(s1, g[a], u0[a]);
                lo[a] = (int)floorf(fminf(ua, ub)) - 1;
                hi[a] = (int)floorf(fmaxf(ua, ub)) + 2;
            }
            lo[M] = wlo;
            hi[M] = whi + 1;
            int gl[3], gh[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                gl[a] = wave_min_i(want ? lo[a] : 0x7FFFFFFF);
                gh[a] = wave_max_i(want ? hi[a] : -0x7FFFFFFF);
                gl[a] = min(max(gl[a], 0), nA[a] - 1);
                gh[a] = min(max(gh[a], 0), nA[a] - 1);
            }
            ox = gl[0] & ~3;
            oy = gl[1];
            oz = gl[2];
            RX = (gh[0] | 3) - ox + 1;
            RY = gh[1] - oy + 1;
            RZ = gh[2] - oz + 1;
            if (RX * RY * RZ <= kRegCap) {
                staged = true;
                break;
            }
        }
        if (D < 1) D = 1;
        if (staged) {
            // stage the box: each lane moves 4-voxel brick rows (8 bytes) into LDS
            const int CX = RX >> 2;
            const int nchunk = CX * RY * RZ;
            const int lane = (int)(threadIdx.x & 63);
            int x4 = lane % CX, r = lane / CX;
            const int dx4 = 64 % CX, dr = 64 / CX;
            int yy = r % RY, zz = r / RY;
            for (int q = lane; q < nchunk; q += 64) {
                const int x = ox + 4 * x4, y = oy + yy, z = oz + zz;
                const uint32_t b = ((uint32_t)(z >> 2) * (uint32_t)S.nby + (uint32_t)(y >> 2)) * (uint32_t)S.nbx +
                                   (uint32_t)(x >> 2);
                const uint2 w = *reinterpret_cast<const uint2*>(vol + ((size_t)b << 6) + ((z & 3) << 4) + ((y & 3) << 2));
                *reinterpret_cast<uint2*>(reg + (zz * RY + yy) * RX + 4 * x4) = w;
                x4 += dx4;
                int rr = dr;
                if (x4 >= CX) {
                    x4 -= CX;
                    ++rr;
                }
                yy += rr;
                while (yy >= RY) {
                    yy -= RY;
                    ++zz;
                }
            }
        }
        __syncthreads();
        // the samples of this window
        const int wcut_lo = wlo, wcut_hi = sgn > 0 ? min(wfirst + D - 1, nM - 1) : wfirst;
        while (k < n) {
            float nl2_len;
            const Cell c = cell_of(S, u0, g, k, n, last, nl2_len);
            const int cmv = (int)cell_axis(c, M);
            if (cmv < wcut_lo || cmv > wcut_hi) break;
            const uint32_t b = ((c.z0 >> 2) * (uint32_t)S.nby + (c.y0 >> 2)) * (uint32_t)S.nbx + (c.x0 >> 2);
            if (skip) {
                if (b != cur_b) {
                    cur_b = b;
                    cur_r = S.dist[b];
                }
                if (cur_r != 0u) {
                    const uint32_t bb[3] = {c.x0 >> 2, c.y0 >> 2, c.z0 >> 2};
                    const int next = skip_cube_ray(S, SR, g, bb, cur_r, k, n);
                    if (COUNT) cnt += (uint32_t)(next - k);
                    k = next;
                    continue;
                }
            }
            Corners kc;
            const uint32_t lx0 = c.x0 - (uint32_t)ox, ly0 = c.y0 - (uint32_t)oy, lz0 = c.z0 - (uint32_t)oz;
            const uint32_t lx1 = c.x1 - (uint32_t)ox, ly1 = c.y1 - (uint32_t)oy, lz1 = c.z1 - (uint32_t)oz;
            if (staged && lx0 < (uint32_t)RX && lx1 < (uint32_t)RX && ly0 < (uint32_t)RY && ly1 < (uint32_t)RY &&
                lz0 < (uint32_t)RZ && lz1 < (uint32_t)RZ) {
                const int RXY = RX * RY;
                const int a0 = (int)lz0 * RXY + (int)ly0 * RX + (int)lx0;
                const int ddx = (int)(lx1 - lx0), ddy = (int)(ly1 - ly0) * RX, ddz = (int)(lz1 - lz0) * RXY;
                kc.v[0] = (float)reg[a0];
                kc.v[1] = (float)reg[a0 + ddx];
                kc.v[2] = (float)reg[a0 + ddy];
                kc.v[3] = (float)reg[a0 + ddy + ddx];
                kc.v[4] = (float)reg[a0 + ddz];
                kc.v[5] = (float)reg[a0 + ddz + ddx];
                kc.v[6] = (float)reg[a0 + ddz + ddy];
                kc.v[7] = (float)reg[a0 + ddz + ddy + ddx];
            } else {
                load_corners<uint16_t, false>(S, vol, c, base_offset<false, uint16_t>(c, b), kc);
            }
            const float sv = interp_corners(kc, c);
            const TfHit h = tf_lookup(tf, sv * tf_scale<uint16_t>());
            const float e = transmit(h.q.w, nl2_len);
            const float te = Tr * e;   // transmittance after the sample
            const float ta = Tr - te;  // its opacity-weighted share, Tr (1 - e)
            cr = fmaf(ta, h.q.x, cr);
            cg = fmaf(ta, h.q.y, cg);
            cb = fmaf(ta, h.q.z, cb);
            Tr = te;
            if (COUNT) {
                ++cnt;
                ++evals;
            }
            ++k;
            if (Tr < S.eps) n = k;        // early termination: no further samples
        }
        __syncthreads();
    }
    if (!in) return make_float4(0.f, 0.f, 0.f, 0.f);
    if (!hit) return make_float4(S.bg[0], S.bg[1], S.bg[2], S.bg[3]);
    return make_float4(fmaf(Tr, S.bg[0], cr), fmaf(Tr, S.bg[1], cg), fmaf(Tr, S.bg[2], cb), 1.0f - Tr * (1.0f - S.bg[3]));
}

}  // namespace rc
}  // namespace vr
