/*
 * FP64 emission-absorption ray caster — the oracle for the preview renders.
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product library.
 *
 * The paper's server-side rendering (Section III-C) projects the volume into
 * 2D images while rotating it about the Z axis; it gives no rendering model.
 * This file follows the reading used throughout the project:
 *   - emission-absorption model with extinction sigma per world unit;
 *   - front-to-back compositing, midpoint samples of step "step" with a
 *     last step that ends the steps exactly at t_out: n = max(1, ceil(L/step))
 *     samples for the clipped length L = t_out - t_in (see or_segment), the
 *     last one of length L - (n-1) step;
 *   - density = trilinear interpolation of cell-centred voxels, taps clamped
 *     to the volume (clamp-to-edge), u16 voxels scaled by 1/65535;
 *   - 256-entry piecewise-linear (r, g, b, sigma) transfer function.
 * Everything is evaluated in double precision, one ray at a time, with no
 * early termination; the number of samples a renderer with early termination
 * at T < ert_eps would take is counted alongside.
 *
 * Count bounds.  A renderer in lower precision takes the same two integer
 * decisions per ray, the step count ceil(L/step) and the sample at which T
 * first falls below ert_eps, from slightly different numbers.  Where either
 * decision sits within a relative margin `tol` of its boundary it may go the
 * other way, each by one sample.  Besides the count, the march therefore
 * reports [lo, hi]: the count with the threshold raised (lowered) by the
 * factor 1 + tol (1 - tol) and the step count taken from L/step - tol
 * (L/step + tol).  The transmittance before an extra sample past the last one
 * is the ray's final transmittance.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_U16 = 0, OR_F32 = 1, OR_F64 = 2 };

typedef struct {
    double eye[3], target[3], up[3];
    double fov_y_deg;     /* > 0: perspective with this vertical field of view */
    double ortho_half_h;  /* used when fov_y_deg == 0: half height of the view */
} or_camera;

typedef struct {
    const void* data;
    int dtype;
    long nx, ny, nz;
    double spacing[3];
} or_volume;

static double voxel(const or_volume* v, long x, long y, long z)
{
    size_t i = ((size_t)z * (size_t)v->ny + (size_t)y) * (size_t)v->nx + (size_t)x;
    switch (v->dtype) {
    case OR_U16: return (double)((const uint16_t*)v->data)[i] / 65535.0;
    case OR_F32: return (double)((const float*)v->data)[i];
    default:     return ((const double*)v->data)[i];
    }
}

static long clampl(long a, long lo, long hi) { return a < lo ? lo : (a > hi ? hi : a); }

/* Trilinear density at world point p (clamp-to-edge, voxel centres at i + 1/2). */
double or_density(const or_volume* v, const double p[3])
{
    const long n[3] = { v->nx, v->ny, v->nz };
    long i0[3];
    double w[3];
    for (int a = 0; a < 3; ++a) {
        double u = p[a] / v->spacing[a] - 0.5;
        double f = floor(u);
        i0[a] = (long)f;
        w[a] = u - f;
    }
    double s = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double wt = (dx ? w[0] : 1.0 - w[0]) * (dy ? w[1] : 1.0 - w[1]) *
                            (dz ? w[2] : 1.0 - w[2]);
                long x = clampl(i0[0] + dx, 0, n[0] - 1);
                long y = clampl(i0[1] + dy, 0, n[1] - 1);
                long z = clampl(i0[2] + dz, 0, n[2] - 1);
                s += wt * voxel(v, x, y, z);
            }
    return s;
}

/* Piecewise-linear transfer function over s in [0, 1], 256 knots of (r, g, b, sigma). */
void or_tf(const double* tf, double s, double out[4])
{
    double x = (s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s)) * 255.0;
    int k = (int)floor(x);
    if (k > 254) k = 254;
    double w = x - k;
    for (int c = 0; c < 4; ++c) out[c] = (1.0 - w) * tf[4 * k + c] + w * tf[4 * (k + 1) + c];
}

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void normalize3(double a[3])
{
    double l = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    a[0] /= l; a[1] /= l; a[2] /= l;
}

/* Primary ray through the centre of pixel (i, j); row j = 0 is the top row. */
void or_ray(const or_camera* c, int W, int H, int i, int j, double o[3], double d[3])
{
    double f[3], r[3], u[3];
    for (int a = 0; a < 3; ++a) f[a] = c->target[a] - c->eye[a];
    normalize3(f);
    cross3(f, c->up, r);
    normalize3(r);
    cross3(r, f, u);
    double ndc_x = (2.0 * (i + 0.5) / W - 1.0) * ((double)W / (double)H);
    double ndc_y = 1.0 - 2.0 * (j + 0.5) / H;
    if (c->fov_y_deg > 0.0) {
        double th = tan(0.5 * c->fov_y_deg * M_PI / 180.0);
        for (int a = 0; a < 3; ++a) {
            o[a] = c->eye[a];
            d[a] = f[a] + th * (ndc_x * r[a] + ndc_y * u[a]);
        }
        normalize3(d);
    } else {
        double h = c->ortho_half_h;
        for (int a = 0; a < 3; ++a) {
            o[a] = c->eye[a] + h * (ndc_x * r[a] + ndc_y * u[a]);
            d[a] = f[a];
        }
    }
}

/* The ray's segment inside the box [0, n*spacing]: *t0 = max(entry, 0) by the
 * slab test, and *L = the distance from the entry point p = o + t0 d to the
 * first face it leaves through, min over axes of (far_a - p_a) / d_a.  That
 * is t_out - t_in, evaluated from coordinates inside the box rather than as
 * the difference of two long distances from the eye, whose low bits rounding
 * would lose (an axis-aligned ray across the box then has L = n * spacing
 * exactly).  Returns 0 when the ray misses (L <= 0, or parallel to a pair of
 * faces outside them: then *L = -inf). */
int or_segment(const or_volume* v, const double o[3], const double d[3], double* t0, double* L)
{
    const double ext[3] = { v->nx * v->spacing[0], v->ny * v->spacing[1], v->nz * v->spacing[2] };
    double tin = -INFINITY;
    *t0 = 0.0;
    *L = -INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < 0.0 || o[a] > ext[a]) return 0;
            continue;
        }
        double ta = (0.0 - o[a]) / d[a];
        double tb = (ext[a] - o[a]) / d[a];
        double lo = ta < tb ? ta : tb;
        if (lo > tin) tin = lo;
    }
    if (tin < 0.0) tin = 0.0;
    double len = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) continue;
        double p = o[a] + tin * d[a];
        double la = ((d[a] > 0.0 ? ext[a] : 0.0) - p) / d[a];
        if (la < len) len = la;
    }
    *t0 = tin;
    *L = len;
    return len > 0.0;
}

/* One ray: writes rgba, returns the number of samples taken before T < ert_eps.
 * bounds: NULL, or [lo, hi] of that count under the margin tol (see above). */
long or_march(const or_volume* v, const double* tf, const double o[3], const double d[3],
              double step, double ert_eps, const double bg[4], double rgba[4], double tol,
              long bounds[2])
{
    double t0, L;
    if (!or_segment(v, o, d, &t0, &L)) {
        for (int c = 0; c < 4; ++c) rgba[c] = bg[c];
        if (bounds) {
            /* a ray missing the box by less than tol steps may graze it: one sample */
            bounds[0] = 0;
            bounds[1] = (L > -tol * step) ? 1 : 0;
        }
        return 0;
    }
    double r = L / step;
    long n = (long)ceil(r);
    if (n < 1) n = 1;
    long n_lo = (long)ceil(r - tol), n_hi = (long)ceil(r + tol);
    if (n_lo < 0) n_lo = 0;
    if (n_hi < 1) n_hi = 1;
    const double eps_hi = ert_eps * (1.0 + tol), eps_lo = ert_eps * (1.0 - tol);
    double T = 1.0, C[3] = { 0.0, 0.0, 0.0 };
    long counted = 0, lo = 0, hi = 0;
    for (long i = 0; i < n; ++i) {
        double len = (i < n - 1) ? step : L - (double)(n - 1) * step;
        double t = t0 + (double)i * step + 0.5 * len;
        double p[3] = { o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2] };
        double q[4];
        or_tf(tf, or_density(v, p), q);
        double e = exp(-q[3] * len);
        double alpha = 1.0 - e;
        if (T >= ert_eps) counted++;
        if (i < n_lo && T >= eps_hi) lo++;
        if (i < n_hi && T >= eps_lo) hi++;
        for (int c = 0; c < 3; ++c) C[c] += T * alpha * q[c];
        T *= e;
    }
    if (n_hi > n && T >= eps_lo) hi++;
    for (int c = 0; c < 3; ++c) rgba[c] = C[c] + T * bg[c];
    rgba[3] = 1.0 - T * (1.0 - bg[3]);
    if (bounds) {
        bounds[0] = lo;
        bounds[1] = hi;
    }
    return counted;
}

int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* All pixels of all views: out[view][j][i][4]; samples[view] = counted
 * samples; bounds: NULL or [view][2], the summed [lo, hi] of the counts. */
void or_render(const or_volume* v, const double* tf, const or_camera* cams, int n_views,
               int W, int H, double step, double ert_eps, const double bg[4],
               double* out, long long* samples, double tol, long long* bounds)
{
    for (int vw = 0; vw < n_views; ++vw) {
        long long cnt = 0, lo = 0, hi = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : cnt, lo, hi)
        for (int j = 0; j < H; ++j) {
            for (int i = 0; i < W; ++i) {
                double o[3], d[3];
                long b[2];
                or_ray(&cams[vw], W, H, i, j, o, d);
                double* px = out + (((size_t)vw * H + j) * W + i) * 4;
                cnt += or_march(v, tf, o, d, step, ert_eps, bg, px, tol, b);
                lo += b[0];
                hi += b[1];
            }
        }
        samples[vw] = cnt;
        if (bounds) {
            bounds[2 * vw] = lo;
            bounds[2 * vw + 1] = hi;
        }
    }
}

/* A subset of pixels given as (view, j, i) triples: out[k][4]; *samples = the
 * counted samples of all of them; counts: NULL or [k][3], per pixel the count
 * and its [lo, hi]. */
void or_render_pixels(const or_volume* v, const double* tf, const or_camera* cams,
                      int W, int H, double step, double ert_eps, const double bg[4],
                      long n_pix, const int32_t* pix, double* out, long long* samples,
                      double tol, long long* counts)
{
    long long cnt = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : cnt)
    for (long k = 0; k < n_pix; ++k) {
        double o[3], d[3];
        long b[2];
        or_ray(&cams[pix[3 * k]], W, H, pix[3 * k + 2], pix[3 * k + 1], o, d);
        long c = or_march(v, tf, o, d, step, ert_eps, bg, out + 4 * k, tol, b);
        cnt += c;
        if (counts) {
            counts[3 * k] = c;
            counts[3 * k + 1] = b[0];
            counts[3 * k + 2] = b[1];
        }
    }
    *samples = cnt;
}

/* Density at a list of world points (exposes the sampler to the tests). */
void or_density_many(const or_volume* v, long n, const double* pts, double* out)
{
    for (long k = 0; k < n; ++k) out[k] = or_density(v, pts + 3 * k);
}
