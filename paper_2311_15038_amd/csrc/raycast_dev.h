// Device-side ray casting pieces shared by the single-volume kernels and the
// batched persistent kernel: the camera and scene records, trilinear sampling
// in the linear and 4^3-brick layouts, the transfer-function lookup, ray
// set-up, empty-space skipping and the front-to-back march of one ray.
// Included by translation units built with contraction off (explicit fmaf),
// so every includer computes bit-identical samples.
#pragma once

#include <algorithm>
#include <cmath>

#include "brick_dev.h"
#include "common.h"
#include "entropy_dev.h"

namespace vr {
namespace rc {

constexpr int kMaxViews = VR_MAX_VIEWS_PER_LAUNCH;

// Brick layouts: log2 of the brick edge (4 or 8 voxels); the linear layout has none.
template <int LAYOUT>
struct Lay {
    static constexpr bool bricked = LAYOUT != VR_LAYOUT_LINEAR;
    static constexpr bool ovl = LAYOUT == VR_LAYOUT_BRICK4_OVERLAP;   // 4^3 bricks, 3 cells apart in x
    static constexpr int bs = LAYOUT == VR_LAYOUT_BRICK8 ? 3 : 2;
    static constexpr uint32_t edge = 1u << bs;
    static constexpr uint32_t mask = edge - 1u;
};
inline int brick_shift(int layout) { return layout == VR_LAYOUT_BRICK8 ? 3 : 2; }

struct View {
    float eye[3];   // perspective origin, or centre of the orthographic view
    float f[3];     // unit forward
    float r[3];     // right, scaled by tan(fov/2) or by the orthographic half height
    float u[3];     // up, scaled likewise
    float persp;    // 1: perspective, 0: orthographic
};

struct Views {
    View v[kMaxViews];
};

struct Scene {
    const void* data;
    const uint8_t* occ;     // brick occupancy or NULL
    int skip_knots;         // leading TF knots a sample of an unmarked brick can reach (1..256)
    const uint8_t* dist;    // brick distance grid (with occ), or NULL: skip by 16^3 groups instead
    int nx, ny, nz;
    int nbx, nby, nbz;      // bricks per axis (4^3 or 8^3 voxels)
    uint32_t nbxy;          // bricks per brick layer, nbx * nby
    int nmx, nmy, nmz;      // groups of 4^3 bricks per axis
    uint32_t macro_off;     // byte offset of the group occupancy
    float inv_sp[3];
    float umax[3];          // n - 1 per axis: the last voxel centre in voxel coordinates
    float ext[3];
    int W, H;
    float aspect;
    float step, eps;
    float inv_step;         // 1 / step
    float skip_c;           // sample-centre offset (plus a rounding margin) in skip_to
    uint32_t row_e, slab_e; // element strides of a brick row and a brick slab (brick layouts)
    int wide;               // offsets need 64-bit addressing and full multiplies
    float bg[4];
    int view0;
    int tiles_x, tiles_y;
    uint32_t* view_hist;    // [views][256] grey-value counts of the frames, or NULL
};

// Margin, in voxel units, by which skip_to stops short of a cell boundary:
// it covers the rounding of the sample positions (a few ulp of coordinates
// below 2^13), so a sample whose computed base tap lies past the boundary is
// never passed over.
constexpr float kSkipMarginVox = 1.0f / 128.0f;

// Transfer function staged in LDS: the 256 knots (4 KiB, so that LDS does not
// bound the occupancy of one-wave workgroups).
struct TfLds {
    float4 a[256];
};

__device__ __forceinline__ void stage_tf(TfLds& t, const float4* __restrict__ tf, int tid, int nthreads)
{
    for (int q = tid; q < 256; q += nthreads) t.a[q] = tf[q];
}

__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x * q + min(x, r) + i;
}

// Ray tiles of TW x TH pixels, one workgroup each, made of 8 x 8-pixel waves
// (TW / 8 across, TH / 8 down): the tile counts of an image.
template <int TW, int TH>
inline void set_tiles(Scene& S)
{
    static_assert(TW % 8 == 0 && TH % 8 == 0, "a tile is whole 8 x 8 waves");
    S.tiles_x = (S.W + TW - 1) / TW;
    S.tiles_y = (S.H + TH - 1) / TH;
}

// Pixel (i, j) and view of this thread in a launch of TW x TH-pixel ray tiles,
// nb workgroups in all, in XCD-aware order: the tiles of one view that run
// at the same time cast neighbouring rays on one XCD.
template <int TW, int TH>
__device__ __forceinline__ void tile_pixel(const Scene& S, int nb, int& view, int& i, int& j)
{
    const int b = xcd_remap((int)blockIdx.x, nb);
    const int per_view = S.tiles_x * S.tiles_y;
    view = b / per_view;
    const int t = b - view * per_view;
    const int tx = t % S.tiles_x, ty = t / S.tiles_x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    i = tx * TW + (w % (TW / 8)) * 8 + (lane & 7);
    j = ty * TH + (w / (TW / 8)) * 8 + (lane >> 3);
}

// Everything one sample needs: the eight tap offsets, the trilinear weights
// and the interpolated voxel value (in the volume's own units: 0..65535 for
// u16, tf_scale maps it to the TF coordinate).
struct Sample {
    uint32_t off[8];   // (x, y, z) taps in order x fastest: 000 100 010 110 001 101 011 111
    float wx, wy, wz;
    float s;
};

template <typename T>
__device__ __forceinline__ float voxel(const T* p, uint32_t i);
template <>
__device__ __forceinline__ float voxel<uint16_t>(const uint16_t* p, uint32_t i) { return (float)p[i]; }
template <>
__device__ __forceinline__ float voxel<float>(const float* p, uint32_t i) { return p[i]; }

__device__ __forceinline__ float lerpf(float a, float b, float w) { return fmaf(w, b - a, a); }

// Offsets of the eight taps (x fastest: 000 100 010 110 001 101 011 111) of
// the clamped tap corners, in the linear or a brick layout.
template <int LAYOUT>
__device__ __forceinline__ void tap_offsets(const Scene& S, uint32_t x0, uint32_t x1, uint32_t y0,
                                            uint32_t y1, uint32_t z0, uint32_t z1, uint32_t off[8])
{
    uint32_t ax0, ax1, ay0, ay1, az0, az1;
    if (LAYOUT == VR_LAYOUT_LINEAR) {
        const uint32_t nx = (uint32_t)S.nx, nxy = (uint32_t)S.nx * (uint32_t)S.ny;
        ax0 = x0; ax1 = x1;
        ay0 = y0 * nx; ay1 = y1 * nx;
        az0 = z0 * nxy; az1 = z1 * nxy;
    } else {
        constexpr int B = Lay<LAYOUT>::bs;
        constexpr uint32_t M = Lay<LAYOUT>::mask;
        const uint32_t row = (uint32_t)S.nbx << (3 * B), slab = row * (uint32_t)S.nby;
        ax0 = ((x0 >> B) << (3 * B)) | (x0 & M); ax1 = ((x1 >> B) << (3 * B)) | (x1 & M);
        ay0 = (y0 >> B) * row + ((y0 & M) << B); ay1 = (y1 >> B) * row + ((y1 & M) << B);
        az0 = (z0 >> B) * slab + ((z0 & M) << (2 * B)); az1 = (z1 >> B) * slab + ((z1 & M) << (2 * B));
    }
    off[0] = az0 + ay0 + ax0; off[1] = az0 + ay0 + ax1;
    off[2] = az0 + ay1 + ax0; off[3] = az0 + ay1 + ax1;
    off[4] = az1 + ay0 + ax0; off[5] = az1 + ay0 + ax1;
    off[6] = az1 + ay1 + ax0; off[7] = az1 + ay1 + ax1;
}

// Base tap corner (clamped) and trilinear weights of the point p.
struct Cell {
    uint32_t x0, x1, y0, y1, z0, z1;
    float wx, wy, wz;
};

// The sample at ray distance off, in voxel coordinates u = u0 + off g (u0 the
// ray's start and g its direction, both divided by the spacing, u0 less half a
// voxel: voxel centres at integers), clamped to the volume's voxel centres.
__device__ __forceinline__ Cell cell_at(const Scene& S, const float u0[3], const float g[3], float off)
{
    Cell c;
    const float ux = __builtin_amdgcn_fmed3f(fmaf(off, g[0], u0[0]), 0.0f, S.umax[0]);
    const float uy = __builtin_amdgcn_fmed3f(fmaf(off, g[1], u0[1]), 0.0f, S.umax[1]);
    const float uz = __builtin_amdgcn_fmed3f(fmaf(off, g[2], u0[2]), 0.0f, S.umax[2]);
    // u >= 0 after the clamp: truncation is the floor, and the fraction
    // u - floor(u) is exact (one instruction each instead of floor, convert
    // and subtract)
    c.wx = __builtin_amdgcn_fractf(ux);
    c.wy = __builtin_amdgcn_fractf(uy);
    c.wz = __builtin_amdgcn_fractf(uz);
    c.x0 = (uint32_t)ux; c.x1 = (uint32_t)min((int)c.x0 + 1, S.nx - 1);
    c.y0 = (uint32_t)uy; c.y1 = (uint32_t)min((int)c.y0 + 1, S.ny - 1);
    c.z0 = (uint32_t)uz; c.z1 = (uint32_t)min((int)c.z0 + 1, S.nz - 1);
    return c;
}

template <typename T, int LAYOUT>
__device__ __forceinline__ void sample(const Scene& S, const T* __restrict__ vol, const Cell& c,
                                       Sample& sm)
{
    sm.wx = c.wx;
    sm.wy = c.wy;
    sm.wz = c.wz;
    tap_offsets<LAYOUT>(S, c.x0, c.x1, c.y0, c.y1, c.z0, c.z1, sm.off);
    float v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = voxel<T>(vol, sm.off[t]);
    const float c0 = lerpf(lerpf(v[0], v[1], sm.wx), lerpf(v[2], v[3], sm.wx), sm.wy);
    const float c1 = lerpf(lerpf(v[4], v[5], sm.wx), lerpf(v[6], v[7], sm.wx), sm.wy);
    sm.s = lerpf(c0, c1, sm.wz);
}

// TF coordinate per unit of voxel value: 255 / 65535 = 1 / 257 for u16
// (normalised to [0, 1], then 255 segments), 255 for f32.
template <typename T>
__device__ __forceinline__ float tf_scale() { return sizeof(T) == 2 ? 1.0f / 257.0f : 255.0f; }

struct TfHit {
    int k;
    float w;
    float4 q;
};

// TF coordinate x (255 times the normalised density), clamped to [0, 255):
// the segment k = floor(x) and the weight w = x - k, exact for x >= 0 (one
// truncation and one fract).  At x >= 255 the coordinate is the float below
// 255, so k = 254 and w = 1 - 2^-16 (the knot-255 value to a relative 2^-16
// of the last segment's rise).
constexpr float kTfXMax = 254.99998474f;   // 255 - 2^-16

__device__ __forceinline__ TfHit tf_hit(float xs)
{
    TfHit h;
    const float x = __builtin_amdgcn_fmed3f(xs, 0.0f, kTfXMax);
    h.k = (int)x;
    h.w = __builtin_amdgcn_fractf(x);
    return h;
}

__device__ __forceinline__ TfHit tf_lookup(const float4* tf, float x)
{
    TfHit h = tf_hit(x);
    const float4 a = tf[h.k], b = tf[h.k + 1];
    h.q = make_float4(lerpf(a.x, b.x, h.w), lerpf(a.y, b.y, h.w), lerpf(a.z, b.z, h.w),
                      lerpf(a.w, b.w, h.w));
    return h;
}

__device__ __forceinline__ TfHit tf_lookup(const TfLds& t, float x)
{
    TfHit h = tf_hit(x);
    const float4 a = t.a[h.k], b = t.a[h.k + 1];
    h.q = make_float4(lerpf(a.x, b.x, h.w), lerpf(a.y, b.y, h.w), lerpf(a.z, b.z, h.w), lerpf(a.w, b.w, h.w));
    return h;
}

// Ray for pixel (i, j): entry point p, unit direction d, segment length L.
__device__ __forceinline__ bool setup_ray(const View& v, const Scene& S, int i, int j, float p[3],
                                          float d[3], float& L)
{
    const float ndc_x = ((2.0f * ((float)i + 0.5f)) / (float)S.W - 1.0f) * S.aspect;
    const float ndc_y = 1.0f - (2.0f * ((float)j + 0.5f)) / (float)S.H;
    float o[3];
    if (v.persp != 0.0f) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o[a] = v.eye[a];
            d[a] = fmaf(ndc_y, v.u[a], fmaf(ndc_x, v.r[a], v.f[a]));
        }
        const float nrm = sqrtf(fmaf(d[0], d[0], fmaf(d[1], d[1], d[2] * d[2])));
        d[0] /= nrm;
        d[1] /= nrm;
        d[2] /= nrm;
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o[a] = fmaf(ndc_y, v.u[a], fmaf(ndc_x, v.r[a], v.eye[a]));
            d[a] = v.f[a];
        }
    }
    float tin = -INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0f) {
            if (o[a] < 0.0f || o[a] > S.ext[a]) return false;
            continue;
        }
        const float ta = (0.0f - o[a]) / d[a];
        const float tb = (S.ext[a] - o[a]) / d[a];
        tin = fmaxf(tin, fminf(ta, tb));
    }
    tin = fmaxf(tin, 0.0f);
#pragma unroll
    for (int a = 0; a < 3; ++a) p[a] = fmaf(tin, d[a], o[a]);
    // The clipped length is measured from the entry point to the first face
    // the ray leaves through, not as the difference of two long distances
    // from the eye: an axis-aligned ray across the box then has L = n *
    // spacing exactly, a whole number of steps when the step divides it.
    L = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0f) continue;
        const float la = ((d[a] > 0.0f ? S.ext[a] : 0.0f) - p[a]) / d[a];
        L = fminf(L, la);
    }
    return L > 0.0f;
}

// n = max(1, ceil(L/step)) midpoint samples, the last one shorter than step
// unless L is a whole number of steps.
__device__ __forceinline__ int step_count(float L, float step)
{
    return max(1, (int)ceilf(L / step));
}

constexpr float kNegLog2E = -1.44269504088896341f;   // -log2(e)

// Ray distance of the midpoint of sample k: k step + len / 2, len the step
// or, for the last sample (inner false), the remainder of the segment; one
// fma of k.
__device__ __forceinline__ float sample_mid(const Scene& S, float kf, bool inner, float half_last)
{
    return fmaf(kf, S.step, inner ? 0.5f * S.step : half_last);
}
__device__ __forceinline__ float sample_mid(const Scene& S, int k, bool inner, float half_last)
{
    return sample_mid(S, (float)k, inner, half_last);
}

// The transmittance factor exp(-sigma len) of a sample, as
// exp2(sigma (-log2(e) len)) with the second factor taken once per ray.
__device__ __forceinline__ float transmit(float sigma, float nl2_len)
{
    return __builtin_amdgcn_exp2f(sigma * nl2_len);
}

// Index of the first sample that may leave an empty box of cells (cells of
// 2^sh voxels: bricks, sh = 2, or 16^3 groups of bricks, sh = 4), cells lo..hi
// per axis.  The base tap stays in the box while u = u0 + s g lies in
// [lo << sh, (hi + 1) << sh) on every axis; a box that reaches the first or
// last cell of an axis extends to infinity there, since taps are clamped.
// Each bound is moved kSkipMarginVox into the box, which covers the rounding
// of the sample positions, and the sample-centre offset is taken off in ray
// distance; ig holds 1/g (0 where g = 0).  Samples below the returned index
// are in the box; the sample at it is checked again.
__device__ __forceinline__ int skip_span(const Scene& S, const float u0[3], const float g[3],
                                         const float ig[3], const uint32_t lo[3], const uint32_t hi[3],
                                         const int ncell[3], int sh, int k, int n)
{
    float s_exit = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool up = g[a] > 0.0f;
        const bool dn = g[a] < 0.0f;
        const uint32_t c1 = up ? hi[a] + 1u : lo[a];
        const float edge = (float)(c1 << sh);
        const float bound = edge + (up ? -kSkipMarginVox : kSkipMarginVox);
        const uint32_t open = ((uint32_t)up & (uint32_t)((int)hi[a] < ncell[a] - 1)) |
                              ((uint32_t)dn & (uint32_t)(lo[a] > 0u));
        const float sa = (bound - u0[a]) * ig[a];
        s_exit = open ? fminf(s_exit, sa) : s_exit;
    }
    const float lim = (s_exit - S.skip_c) * S.inv_step;
    int next = n;
    if (lim < (float)n) next = (int)ceilf(lim);
    return min(max(next, k + 1), n);
}

// skip_span for a single cell.
__device__ __forceinline__ int skip_to(const Scene& S, const float u0[3], const float g[3],
                                       const float ig[3], const uint32_t cell[3], const int ncell[3],
                                       int sh, int k, int n)
{
    return skip_span(S, u0, g, ig, cell, cell, ncell, sh, k, n);
}

// Per-ray constants of skip_cube_ray for bricks of e_a voxels along axis a
// (2^sh, or 3 along x in the overlap layout): on each axis the exit bound of
// the bricks below (or above) face c1 is s = c1 e_a / g + (-+margin - u0) / g,
// kept as s = (c1 - 1) ig2 + kb1 with ig2 = e_a / g and
// kb1 = ig2 + (-+margin - u0) / g; nopen is the axis's brick count less one
// (0 where g = 0: never left).
struct SkipRay {
    float kb1[3];
    float ig2[3];
    uint32_t nopen[3];
};

__device__ __forceinline__ SkipRay skip_ray(const Scene& S, const float u0[3], const float g[3], const float ig[3],
                                            float cx, float cy, float cz)
{
    SkipRay R;
    const int nb[3] = {S.nbx, S.nby, S.nbz};
    const float cell[3] = {cx, cy, cz};   // cells (voxels) per brick along each axis
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R.ig2[a] = ig[a] * cell[a];
        R.kb1[a] = fmaf((g[a] > 0.0f ? -kSkipMarginVox : kSkipMarginVox) - u0[a], ig[a], R.ig2[a]);
        R.nopen[a] = g[a] != 0.0f ? (uint32_t)(nb[a] - 1) : 0u;
    }
    return R;
}

__device__ __forceinline__ SkipRay skip_ray(const Scene& S, const float u0[3], const float g[3], const float ig[3],
                                            int sh)
{
    const float c = (float)(1 << sh);
    return skip_ray(S, u0, g, ig, c, c, c);
}

// The first sample that may leave the empty cube of cells around cell bb whose
// distance byte is r >= 1 (cells within r - 1 of bb on every axis, clipped to
// the grid), as skip_span computes it for a box, with the per-ray constants:
// the cube's exit face on an axis the ray climbs is c1 = bb + r, on one it
// descends c1 = bb + 1 - r; the face is open (not the grid's edge) when
// 1 <= c1 <= n - 1, one unsigned compare of c1 - 1, and its bound is one fma
// of c1 - 1.  Faces that are not open count as infinitely far; the nearest
// open one, less the sample-centre offset, gives the sample index, clamped
// to k + 1 .. n (indices as floats, exact below 2^24).
__device__ __forceinline__ float skip_cube_f(const Scene& S, const SkipRay& R, const float g[3],
                                             const uint32_t bb[3], uint32_t r, float kf, float nf)
{
    const int up = (int)r - 1, dn = -(int)r;      // c1 - 1 - bb climbing / descending
    float sa[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int c1m1 = (int)bb[a] + (g[a] > 0.0f ? up : dn);
        const bool open = (uint32_t)c1m1 < R.nopen[a];
        sa[a] = open ? fmaf((float)c1m1, R.ig2[a], R.kb1[a]) : INFINITY;
    }
    const float lim = (fminf(fminf(sa[0], sa[1]), sa[2]) - S.skip_c) * S.inv_step;
    // the middle of ceil(lim), k + 1 and n (lim is +inf where no face is open)
    return __builtin_amdgcn_fmed3f(ceilf(lim), kf + 1.0f, nf);
}

__device__ __forceinline__ int skip_cube_ray(const Scene& S, const SkipRay& R, const float g[3],
                                             const uint32_t bb[3], uint32_t r, int k, int n)
{
    return (int)skip_cube_f(S, R, g, bb, r, (float)k, (float)n);
}

// Whether samples of unmarked bricks may be passed over: the volume is in a
// brick layout with an occupancy grid, and every TF knot such a sample can
// reach (the first S.skip_knots: knot 0 when the marks are of non-zero voxels)
// has zero extinction and finite colour, so those samples leave colour and
// transmittance bit-for-bit unchanged.  Called by whole waves (the lanes share
// the knots out and vote).
__device__ __forceinline__ bool can_skip(const Scene& S, const TfLds& tf)
{
    if (S.occ == nullptr) return false;
    bool ok = true;
    for (int q = (int)(threadIdx.x & 63); q < S.skip_knots; q += 64) {
        const float4 a = tf.a[q];
        ok = ok && a.w == 0.0f && isfinite(a.x) && isfinite(a.y) && isfinite(a.z);
    }
    return __all(ok) != 0;
}

template <bool WIDE>
__device__ __forceinline__ uint32_t mul_idx(uint32_t a, uint32_t b)
{
    return WIDE ? a * b : __umul24(a, b);
}

// Voxel at offset o: in bytes (32-bit, so the load takes a 32-bit offset from
// the volume base), or in elements with 64-bit addressing when WIDE.
template <typename T, bool WIDE>
__device__ __forceinline__ float tap(const T* vol, uint32_t o)
{
    if (WIDE) return voxel<T>(vol, o);
    return voxel<T>(reinterpret_cast<const T*>(reinterpret_cast<const char*>(vol) + o), 0u);
}

// The eight corner voxels of a cell of a volume in the 4^3-brick layout
// whose base-tap brick is b, and the key that identifies them (the base
// offset, one per cell).  Tap offsets are the base offset plus
// per-axis steps: one voxel inside a brick, or into the next brick when the
// base tap is on a brick's last layer, or zero where the taps are clamped.
struct Corners {
    float v[8];   // x fastest: 000 100 010 110 001 101 011 111
    uint32_t key_o;   // base offset: one per cell, which also fixes the clamped axes
};

template <bool WIDE, typename P, int B = 2>
__device__ __forceinline__ uint32_t base_offset(const Cell& c, uint32_t b)
{
    constexpr uint32_t E = WIDE ? 1u : (uint32_t)sizeof(P);   // offsets in elements or bytes
    constexpr uint32_t M = (1u << B) - 1u;
    const uint32_t in0 = ((c.z0 & M) << (2 * B)) | ((c.y0 & M) << B) | (c.x0 & M);
    return ((b << (3 * B)) | in0) * E;
}

// Element of a pair-layout volume at offset o (bytes, or elements when
// WIDE): its two voxels as floats.
template <bool WIDE>
__device__ __forceinline__ void tap_pair(const uint16_t* vol, uint32_t o, float& lo, float& hi)
{
    const uint32_t w = WIDE ? reinterpret_cast<const uint32_t*>(vol)[o]
                            : *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(vol) + o);
    lo = (float)(w & 0xFFFFu);
    hi = (float)(w >> 16);
}

template <bool WIDE>
__device__ __forceinline__ void tap_pair(const float* vol, uint32_t o, float& lo, float& hi)
{
    const float2 w = WIDE ? reinterpret_cast<const float2*>(vol)[o]
                          : *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(vol) + o);
    lo = w.x;
    hi = w.y;
}

// Corners of cell c from a pair-layout volume: four loads, each bringing both
// x taps.  Where the x taps are clamped to one voxel (x1 == x0) the stored
// pair may hold the next voxel, so the low voxel is used for both.
template <typename T, bool WIDE>
__device__ __forceinline__ void load_corners_pairs(const Scene& S, const T* __restrict__ vol, const Cell& c,
                                                   uint32_t o0, Corners& k)
{
    constexpr uint32_t E = WIDE ? 1u : 2u * (uint32_t)sizeof(T);
    const uint32_t dy = (c.y1 == c.y0) ? 0u : ((c.y0 & 3u) == 3u ? (S.row_e - 12u) * E : 4u * E);
    const uint32_t dz = (c.z1 == c.z0) ? 0u : ((c.z0 & 3u) == 3u ? (S.slab_e - 48u) * E : 16u * E);
    const uint32_t o2 = o0 + dy, o4 = o0 + dz, o6 = o4 + dy;
    tap_pair<WIDE>(vol, o0, k.v[0], k.v[1]);
    tap_pair<WIDE>(vol, o2, k.v[2], k.v[3]);
    tap_pair<WIDE>(vol, o4, k.v[4], k.v[5]);
    tap_pair<WIDE>(vol, o6, k.v[6], k.v[7]);
    if (c.x1 == c.x0) {
        k.v[1] = k.v[0];
        k.v[3] = k.v[2];
        k.v[5] = k.v[4];
        k.v[7] = k.v[6];
    }
}

// A 32-bit word of the volume at byte offset o, which need only be 2-byte
// aligned (the device runs with unaligned access enabled: one load, whose word
// never crosses the 8- or 16-byte brick row it starts in, see load_corners).
__device__ __forceinline__ uint32_t word_at(const uint16_t* vol, uint32_t o)
{
    typedef uint32_t u32_a2 __attribute__((aligned(2)));
    return *reinterpret_cast<const u32_a2*>(reinterpret_cast<const char*>(vol) + o);
}

// Tap steps: one voxel inside a brick of edge e = 2^B; from a brick's last
// layer to the next brick, e^3 - (e - 1) in x, a brick row less (e - 1) e in y,
// a brick slab less (e - 1) e^2 in z.
//
// u16 volumes with 32-bit byte offsets take both x taps of a corner row in one
// 32-bit load where they lie in one brick row (x0 not on the brick's last
// layer): four loads per cell instead of eight, with the same lines touched.
// The texture path's time follows the 32-bit words it returns per lane, and a
// 16-bit load costs a whole word.  Where x0 is on the last layer, the word
// before it is loaded (x0 in its high half, inside the row) and the x1 taps,
// in the next brick, one by one.  This path takes no clamps: on the volume's
// last voxel layer (x0 = nx - 1, and likewise y, z) the far taps are read from
// the brick's padding, the next brick, brick row or layer, or the apron after
// the last brick, and have weight 0, since the position was clamped to that
// layer's voxel centre.  The other paths clamp the far taps (x1 == x0).
template <typename T, bool WIDE, int B = 2>
__device__ __forceinline__ void load_corners(const Scene& S, const T* __restrict__ vol, const Cell& c,
                                             uint32_t o0, Corners& k)
{
    constexpr uint32_t E = WIDE ? 1u : (uint32_t)sizeof(T);
    constexpr uint32_t e = 1u << B, M = e - 1u;
    if constexpr (sizeof(T) == 2 && !WIDE) {
        const uint32_t dy = (c.y0 & M) == M ? (S.row_e - M * e) * E : e * E;
        const uint32_t dz = (c.z0 & M) == M ? (S.slab_e - M * e * e) * E : e * e * E;
        const bool last = (c.x0 & M) == M;
        const uint32_t ob = last ? o0 - 2u : o0;   // start of the word of each row
        const uint32_t w0 = word_at(vol, ob), w2 = word_at(vol, ob + dy);
        const uint32_t w4 = word_at(vol, ob + dz), w6 = word_at(vol, ob + dz + dy);
        const uint32_t sh = last ? 16u : 0u;      // the x0 half of each word
        k.v[0] = (float)__builtin_amdgcn_ubfe(w0, sh, 16u);
        k.v[2] = (float)__builtin_amdgcn_ubfe(w2, sh, 16u);
        k.v[4] = (float)__builtin_amdgcn_ubfe(w4, sh, 16u);
        k.v[6] = (float)__builtin_amdgcn_ubfe(w6, sh, 16u);
        if (last) {
            constexpr uint32_t dx = (e * e * e - M) * E;
            const uint32_t o2 = o0 + dy, o4 = o0 + dz;
            k.v[1] = tap<T, WIDE>(vol, o0 + dx);
            k.v[3] = tap<T, WIDE>(vol, o2 + dx);
            k.v[5] = tap<T, WIDE>(vol, o4 + dx);
            k.v[7] = tap<T, WIDE>(vol, o4 + dy + dx);
        } else {
            k.v[1] = (float)(w0 >> 16);
            k.v[3] = (float)(w2 >> 16);
            k.v[5] = (float)(w4 >> 16);
            k.v[7] = (float)(w6 >> 16);
        }
        return;
    }
    const uint32_t dx = (c.x1 == c.x0) ? 0u : ((c.x0 & M) == M ? (e * e * e - M) * E : E);
    const uint32_t dy = (c.y1 == c.y0) ? 0u : ((c.y0 & M) == M ? (S.row_e - M * e) * E : e * E);
    const uint32_t dz = (c.z1 == c.z0) ? 0u : ((c.z0 & M) == M ? (S.slab_e - M * e * e) * E : e * e * E);
    const uint32_t o2 = o0 + dy, o4 = o0 + dz, o6 = o4 + dy;
    k.v[0] = tap<T, WIDE>(vol, o0);
    k.v[1] = tap<T, WIDE>(vol, o0 + dx);
    k.v[2] = tap<T, WIDE>(vol, o2);
    k.v[3] = tap<T, WIDE>(vol, o2 + dx);
    k.v[4] = tap<T, WIDE>(vol, o4);
    k.v[5] = tap<T, WIDE>(vol, o4 + dx);
    k.v[6] = tap<T, WIDE>(vol, o6);
    k.v[7] = tap<T, WIDE>(vol, o6 + dx);
}

// Overlap layout (u16, byte offsets): base tap offset of cell c in brick b,
// xi = x0 - 3 bx its column in the brick (0..2).
__device__ __forceinline__ uint32_t base_offset_ovl(const Cell& c, uint32_t b, uint32_t xi)
{
    return ((b << 6) | ((c.z0 & 3u) << 4) | ((c.y0 & 3u) << 2) | xi) * 2u;
}

// Corners of cell c in the overlap layout: both x taps of each corner row lie
// in one brick row (the cell's column is 0..2 of the brick's 4), so each row
// is one 32-bit load, with no special case in x.  The far taps in y and z
// follow load_corners (no clamps: on the volume's last layer they have weight 0).
__device__ __forceinline__ void load_corners_ovl(const Scene& S, const uint16_t* __restrict__ vol, const Cell& c,
                                                 uint32_t o0, Corners& k)
{
    const uint32_t dy = (c.y0 & 3u) == 3u ? (S.row_e - 12u) * 2u : 8u;
    const uint32_t dz = (c.z0 & 3u) == 3u ? (S.slab_e - 48u) * 2u : 32u;
    const uint32_t w0 = word_at(vol, o0), w2 = word_at(vol, o0 + dy);
    const uint32_t w4 = word_at(vol, o0 + dz), w6 = word_at(vol, o0 + dz + dy);
    k.v[0] = (float)(w0 & 0xFFFFu);
    k.v[1] = (float)(w0 >> 16);
    k.v[2] = (float)(w2 & 0xFFFFu);
    k.v[3] = (float)(w2 >> 16);
    k.v[4] = (float)(w4 & 0xFFFFu);
    k.v[5] = (float)(w4 >> 16);
    k.v[6] = (float)(w6 & 0xFFFFu);
    k.v[7] = (float)(w6 >> 16);
}

// Trilinear voxel value (the volume's units) from the corners of cell c.
__device__ __forceinline__ float interp_corners(const Corners& k, const Cell& c)
{
    const float c0 = lerpf(lerpf(k.v[0], k.v[1], c.wx), lerpf(k.v[2], k.v[3], c.wx), c.wy);
    const float c1 = lerpf(lerpf(k.v[4], k.v[5], c.wx), lerpf(k.v[6], k.v[7], c.wx), c.wy);
    return lerpf(c0, c1, c.wz);
}

// Front-to-back march of the ray through pixel (i, j): returns its RGBA and,
// with COUNT, adds to the counts of samples taken (cnt) and evaluated
// (evals).  WIDE selects 64-bit addressing and full multiplies for volumes
// of more than 2^24 bricks.  Empty bricks are left by the cube of empty
// bricks the distance grid gives (DIST, S.dist set), or else by their 16^3
// group when that is empty too.
template <typename T, int LAYOUT, bool COUNT, bool WIDE, bool DIST = true>
__device__ __forceinline__ float4 march(const Scene& S, const View& v, const T* __restrict__ vol,
                                        const TfLds& tf, bool skip, int i, int j, uint32_t& cnt,
                                        uint32_t& evals)
{
    float p[3], d[3], L;
    if (!setup_ray(v, S, i, j, p, d, L)) return make_float4(S.bg[0], S.bg[1], S.bg[2], S.bg[3]);
    const int n = step_count(L, S.step);
    const float last = L - (float)(n - 1) * S.step;
    float u0[3], g[3], ig[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u0[a] = fmaf(p[a], S.inv_sp[a], -0.5f);
        g[a] = d[a] * S.inv_sp[a];
        ig[a] = g[a] != 0.0f ? 1.0f / g[a] : 0.0f;
    }
    const bool skipping = skip && Lay<LAYOUT>::bricked;
    const SkipRay SR = Lay<LAYOUT>::ovl ? skip_ray(S, u0, g, ig, 3.0f, 4.0f, 4.0f)
                                        : skip_ray(S, u0, g, ig, Lay<LAYOUT>::bs);
    const float half_last = 0.5f * last;
    const float nl2_step = S.step * kNegLog2E, nl2_last = last * kNegLog2E;
    float Tr = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    uint32_t cur_b = 0xFFFFFFFFu;
    uint32_t cur_r = 0u;         // distance byte of brick cur_b (0: occupied)
    Corners kc;                  // corners of the last sampled cell (consecutive samples share
    kc.key_o = 0xFFFFFFFFu;      // a cell about half the time at half-voxel steps)
    // the sample index as a float (exact: at most 2^24 samples per ray)
    const float nf = (float)n, nf1 = (float)(n - 1);
    float kf = 0.0f;
    while (kf < nf) {
        const bool inner = kf < nf1;
        const Cell c = cell_at(S, u0, g, sample_mid(S, kf, inner, half_last));
        float sv;
        if constexpr (Lay<LAYOUT>::bricked) {
            constexpr int B = Lay<LAYOUT>::bs;
            constexpr bool OVL = Lay<LAYOUT>::ovl;
            static_assert(!OVL || (DIST && !WIDE && sizeof(T) == 2), "overlap bricks: u16, 32-bit offsets, distance grid");
            // brick x (x0 / 3 for overlapping bricks) and index: full multiplies when
            // WIDE, else two 24-bit products (fewer than 2^24 bricks) summed at once
            const uint32_t bxo = OVL ? vr::bk::ovl_bx(c.x0) : (c.x0 >> B);
            const uint32_t b = WIDE ? ((c.z0 >> B) * (uint32_t)S.nby + (c.y0 >> B)) * (uint32_t)S.nbx + bxo
                                    : __umul24(c.z0 >> B, S.nbxy) + __umul24(c.y0 >> B, (uint32_t)S.nbx) + bxo;
            if (skipping) {
                if (b != cur_b) {
                    cur_b = b;
                    cur_r = DIST ? (uint32_t)S.dist[b] : (S.occ[b] != 0 ? 0u : 1u);
                }
                if (cur_r != 0u) {
                    float next;
                    if constexpr (DIST) {
                        // empty brick: leave the cube of empty bricks around it
                        const uint32_t bb[3] = {bxo, c.y0 >> B, c.z0 >> B};
                        next = skip_cube_f(S, SR, g, bb, cur_r, kf, nf);
                    } else {
                        const int k = (int)kf;
                        // empty brick: leave its group of 4^3 bricks if that is empty too, else the brick
                        const uint32_t m[3] = {c.x0 >> (B + 2), c.y0 >> (B + 2), c.z0 >> (B + 2)};
                        const uint32_t mi = mul_idx<WIDE>(mul_idx<WIDE>(m[2], (uint32_t)S.nmy) + m[1],
                                                          (uint32_t)S.nmx) + m[0];
                        if (S.occ[S.macro_off + mi] == 0) {
                            const int nm[3] = {S.nmx, S.nmy, S.nmz};
                            next = (float)skip_to(S, u0, g, ig, m, nm, B + 2, k, n);
                        } else {
                            const uint32_t bb[3] = {c.x0 >> B, c.y0 >> B, c.z0 >> B};
                            const int nb[3] = {S.nbx, S.nby, S.nbz};
                            next = (float)skip_to(S, u0, g, ig, bb, nb, B, k, n);
                        }
                    }
                    if (COUNT) cnt += (uint32_t)(next - kf);
                    kf = next;
                    continue;
                }
            }
            constexpr bool PAIRS = LAYOUT == VR_LAYOUT_BRICK4_PAIRS;
            const uint32_t o0 = OVL     ? base_offset_ovl(c, b, c.x0 - 3u * bxo)
                                : PAIRS ? base_offset<WIDE, typename vr::bk::PairOf<T>::type>(c, b)
                                        : base_offset<WIDE, T, B>(c, b);
            if (o0 != kc.key_o) {
                if constexpr (OVL) load_corners_ovl(S, reinterpret_cast<const uint16_t*>(vol), c, o0, kc);
                else if constexpr (PAIRS) load_corners_pairs<T, WIDE>(S, vol, c, o0, kc);
                else load_corners<T, WIDE, B>(S, vol, c, o0, kc);
                kc.key_o = o0;
            }
            sv = interp_corners(kc, c);
        } else {
            Sample sm;
            sample<T, LAYOUT>(S, vol, c, sm);
            sv = sm.s;
        }
        const TfHit h = tf_lookup(tf, sv * tf_scale<T>());
        const float e = transmit(h.q.w, inner ? nl2_step : nl2_last);
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
        kf += 1.0f;
        if (Tr < S.eps) break;
    }
    return make_float4(fmaf(Tr, S.bg[0], cr), fmaf(Tr, S.bg[1], cg), fmaf(Tr, S.bg[2], cb),
                       1.0f - Tr * (1.0f - S.bg[3]));
}

// Whether a volume needs 64-bit addressing and full multiplies in march.
inline bool needs_wide(const Scene& S) { return S.wide != 0; }

// ------------------------------------------------------------ host side

// TF knots a sample can reach when all eight of its taps are at most
// `above` (u16 units): the trilinear lerps keep it at most `above` up to a few
// float roundings (a relative 2^-16 bounds them with room to spare), so its TF
// coordinate s * 255 / 65535 lies below k + 1 for the k below, and the lookup
// blends knots k and k + 1 at most.  With above = 0 the sample is exactly 0
// and the lookup returns knot 0.
inline int skip_knots(int above)
{
    if (above == 0) return 1;
    const double x = (double)above * 255.0 / 65535.0 * (1.0 + 1.0 / 65536.0);
    return std::min(254, (int)std::floor(x)) + 2;
}

inline int build_scene(const vr_volume* vol, const float* d_tf, const vr_camera* h_cams, int n_views,
                const vr_render_opts* o, Scene& S)
{
    VR_REQUIRE(vol && d_tf && h_cams && o, VR_ERR_NULL, "raycast: NULL argument");
    VR_REQUIRE(vol->data != nullptr, VR_ERR_NULL, "raycast: volume data is NULL");
    VR_REQUIRE(vol->dtype == VR_U16_NORM || vol->dtype == VR_F32, VR_ERR_DTYPE,
               "raycast: unknown dtype %d", vol->dtype);
    VR_REQUIRE(vol->layout == VR_LAYOUT_LINEAR || vol->layout == VR_LAYOUT_BRICK4 ||
                   vol->layout == VR_LAYOUT_BRICK4_PAIRS || vol->layout == VR_LAYOUT_BRICK8 ||
                   vol->layout == VR_LAYOUT_BRICK4_OVERLAP,
               VR_ERR_RANGE, "raycast: unknown layout %d", vol->layout);
    VR_REQUIRE(vol->nx >= 1 && vol->ny >= 1 && vol->nz >= 1 && vol->nx < (1 << 30) &&
                   vol->ny < (1 << 30) && vol->nz < (1 << 30),
               VR_ERR_DIMS, "raycast: volume dims %lld x %lld x %lld", (long long)vol->nx,
               (long long)vol->ny, (long long)vol->nz);
    const int bs = brick_shift(vol->layout);
    const int64_t bvox = int64_t(1) << (3 * bs);   // voxels per brick
    int64_t nb[3];
    vr::bk::brick_grid(vol->layout, vol->nx, vol->ny, vol->nz, nb);
    const bool bricked = vol->layout != VR_LAYOUT_LINEAR;
    VR_REQUIRE(vol->layout != VR_LAYOUT_BRICK4_OVERLAP || vol->dtype == VR_U16_NORM, VR_ERR_DTYPE,
               "raycast: VR_LAYOUT_BRICK4_OVERLAP holds u16 volumes only");
    const int64_t elems = bricked ? nb[0] * nb[1] * nb[2] * bvox : vol->nx * vol->ny * vol->nz;
    VR_REQUIRE(elems <= (int64_t)0xFFFFFFFFu, VR_ERR_DIMS,
               "raycast: volume of %lld elements exceeds 32-bit offsets", (long long)elems);
    for (int a = 0; a < 3; ++a)
        VR_REQUIRE(std::isfinite(vol->spacing[a]) && vol->spacing[a] > 0.0, VR_ERR_RANGE,
                   "raycast: spacing[%d] = %g", a, vol->spacing[a]);
    VR_REQUIRE(n_views >= 1, VR_ERR_DIMS, "raycast: n_views %d", n_views);
    VR_REQUIRE(o->width >= 1 && o->height >= 1 && o->width <= 32768 && o->height <= 32768,
               VR_ERR_DIMS, "raycast: image %d x %d", o->width, o->height);
    VR_REQUIRE(std::isfinite(o->step) && o->step > 0.0f, VR_ERR_RANGE, "raycast: step %g",
               (double)o->step);
    VR_REQUIRE(std::isfinite(o->ert_eps) && o->ert_eps >= 0.0f && o->ert_eps < 1.0f, VR_ERR_RANGE,
               "raycast: ert_eps %g", (double)o->ert_eps);
    {   // bound the samples per ray: the box diagonal over the step
        double diag2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double e = (double)(a == 0 ? vol->nx : a == 1 ? vol->ny : vol->nz) * vol->spacing[a];
            diag2 += e * e;
        }
        VR_REQUIRE(std::sqrt(diag2) / (double)o->step <= (double)(1 << 24), VR_ERR_RANGE,
                   "raycast: step %g gives more than 2^24 samples per ray", (double)o->step);
    }
    for (int v = 0; v < n_views; ++v) {
        const vr_camera& c = h_cams[v];
        VR_REQUIRE(c.fov_y_deg == 0.0 ? (std::isfinite(c.ortho_half_h) && c.ortho_half_h > 0.0)
                                      : (c.fov_y_deg > 0.0 && c.fov_y_deg < 180.0),
                   VR_ERR_RANGE, "raycast: camera %d has fov %g / half height %g", v, c.fov_y_deg,
                   c.ortho_half_h);
    }
    VR_REQUIRE(vol->occupancy_above >= 0 && vol->occupancy_above <= 65535 &&
                   (vol->dtype == VR_U16_NORM || vol->occupancy_above == 0),
               VR_ERR_RANGE, "raycast: occupancy_above %d (0..65535 for u16, 0 for f32)", (int)vol->occupancy_above);
    S.data = vol->data;
    S.occ = vol->occupancy;
    S.skip_knots = skip_knots(vol->occupancy_above);
    S.nbx = (int)nb[0];
    S.nby = (int)nb[1];
    S.nbz = (int)nb[2];
    S.nbxy = (uint32_t)(nb[0] * nb[1]);
    S.nmx = (S.nbx + 3) / 4;
    S.nmy = (S.nby + 3) / 4;
    S.nmz = (S.nbz + 3) / 4;
    S.macro_off = (uint32_t)(nb[0] * nb[1] * nb[2]);
    // the distance grid follows the bricks' and the groups' marks
    S.dist = vol->occupancy ? vol->occupancy + nb[0] * nb[1] * nb[2] + (int64_t)S.nmx * S.nmy * S.nmz : nullptr;
    S.nx = (int)vol->nx;
    S.ny = (int)vol->ny;
    S.nz = (int)vol->nz;
    const int64_t n[3] = {vol->nx, vol->ny, vol->nz};
    for (int a = 0; a < 3; ++a) {
        S.inv_sp[a] = (float)(1.0 / vol->spacing[a]);
        S.umax[a] = (float)(n[a] - 1);
        S.ext[a] = (float)((double)n[a] * vol->spacing[a]);
    }
    S.row_e = (uint32_t)(nb[0] * bvox);
    S.slab_e = (uint32_t)(nb[0] * nb[1] * bvox);
    S.inv_step = 1.0f / o->step;
    S.skip_c = 0.5f * o->step + o->step * (1.0f / 512.0f);
    if (!bricked) {                  // occupancy belongs to the brick layouts
        S.occ = nullptr;
        S.dist = nullptr;
    }
    {   // 32-bit byte offsets (to the end of the apron) and 24-bit brick-index products,
        // unless the volume is too large
        const int64_t bricks = nb[0] * nb[1] * nb[2];
        const int64_t elem_bytes = (vol->dtype == VR_U16_NORM ? 2 : 4) * (vol->layout == VR_LAYOUT_BRICK4_PAIRS ? 2 : 1);
        const int64_t bytes = (bricks + vr::bk::apron_bricks(nb[0], nb[1])) * bvox * elem_bytes;
        S.wide = (bricks > (int64_t(1) << 24) || bytes > (int64_t(1) << 32)) ? 1 : 0;
        VR_REQUIRE(!(bricked && S.wide && vol->layout == VR_LAYOUT_BRICK4_OVERLAP), VR_ERR_DIMS,
                   "raycast: VR_LAYOUT_BRICK4_OVERLAP needs fewer than 2^24 bricks and 4 GiB");
    }
    S.view_hist = o->view_hist;
    S.W = o->width;
    S.H = o->height;
    S.aspect = (float)((double)o->width / (double)o->height);
    S.step = o->step;
    S.eps = o->ert_eps;
    for (int c = 0; c < 4; ++c) S.bg[c] = o->bg[c];
    return VR_OK;
}

inline int build_views(const vr_camera* cams, int count, Views& V)
{
    for (int k = 0; k < count; ++k) {
        const vr_camera& c = cams[k];
        double f[3], r[3], u[3];
        for (int a = 0; a < 3; ++a) f[a] = c.target[a] - c.eye[a];
        double lf = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        VR_REQUIRE(lf > 0.0 && std::isfinite(lf), VR_ERR_RANGE, "raycast: camera eye == target");
        for (int a = 0; a < 3; ++a) f[a] /= lf;
        r[0] = f[1] * c.up[2] - f[2] * c.up[1];
        r[1] = f[2] * c.up[0] - f[0] * c.up[2];
        r[2] = f[0] * c.up[1] - f[1] * c.up[0];
        double lr = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        VR_REQUIRE(lr > 0.0 && std::isfinite(lr), VR_ERR_RANGE, "raycast: camera up is parallel to the view");
        for (int a = 0; a < 3; ++a) r[a] /= lr;
        u[0] = r[1] * f[2] - r[2] * f[1];
        u[1] = r[2] * f[0] - r[0] * f[2];
        u[2] = r[0] * f[1] - r[1] * f[0];
        const bool persp = c.fov_y_deg > 0.0;
        const double sc = persp ? std::tan(0.5 * c.fov_y_deg * M_PI / 180.0) : c.ortho_half_h;
        View& v = V.v[k];
        for (int a = 0; a < 3; ++a) {
            v.eye[a] = (float)c.eye[a];
            v.f[a] = (float)f[a];
            v.r[a] = (float)(sc * r[a]);
            v.u[a] = (float)(sc * u[a]);
        }
        v.persp = persp ? 1.0f : 0.0f;
    }
    return VR_OK;
}

}  // namespace rc
}  // namespace vr
