/*
 * Test helper: runs the FP64 oracle ray caster (oracle/render.c, linked in)
 * on inputs read from a file and writes the frames and sample counts to
 * another.  The test builds it with AddressSanitizer and UBSan, so every
 * read of the volume, the transfer function and the cameras is checked.
 *
 * Input (native endianness): int64 nx, ny, nz, dtype (0 u16, 1 f32),
 * n_views, W, H; float64 spacing[3], step, ert_eps, bg[4], tf[256][4],
 * cams[n_views][11]; then the voxels (nz * ny * nx of dtype), exactly sized.
 * Output: float64 rgba[n_views][H][W][4], then int64 samples[n_views].
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    double eye[3], target[3], up[3];
    double fov_y_deg;
    double ortho_half_h;
} or_camera;

typedef struct {
    const void* data;
    int dtype;
    long nx, ny, nz;
    double spacing[3];
} or_volume;

void or_render(const or_volume* v, const double* tf, const or_camera* cams, int n_views, int W, int H,
               double step, double ert_eps, const double bg[4], double* out, long long* samples,
               double tol, long long* bounds);

static void* take(FILE* f, size_t n)
{
    void* p = malloc(n ? n : 1);
    if (!p || fread(p, 1, n, f) != n) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

int main(int argc, char** argv)
{
    if (argc != 3) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t* h = take(f, 7 * sizeof(int64_t));
    const long nx = h[0], ny = h[1], nz = h[2];
    const int dtype = (int)h[3], nv = (int)h[4], W = (int)h[5], H = (int)h[6];
    double* p = take(f, 9 * sizeof(double));
    double* tf = take(f, 1024 * sizeof(double));
    double* c = take(f, (size_t)nv * 11 * sizeof(double));
    const size_t vox = (size_t)nx * ny * nz * (dtype == 0 ? 2 : 4);
    void* data = take(f, vox);
    if (fgetc(f) != EOF) return 3;
    fclose(f);
    or_camera* cams = malloc((size_t)nv * sizeof(or_camera));
    for (int k = 0; k < nv; ++k) {
        for (int a = 0; a < 3; ++a) {
            cams[k].eye[a] = c[11 * k + a];
            cams[k].target[a] = c[11 * k + 3 + a];
            cams[k].up[a] = c[11 * k + 6 + a];
        }
        cams[k].fov_y_deg = c[11 * k + 9];
        cams[k].ortho_half_h = c[11 * k + 10];
    }
    or_volume v = {data, dtype, nx, ny, nz, {p[0], p[1], p[2]}};
    double* out = malloc((size_t)nv * H * W * 4 * sizeof(double));
    long long* samples = malloc((size_t)nv * sizeof(long long));
    long long* bounds = malloc((size_t)nv * 2 * sizeof(long long));
    or_render(&v, tf, cams, nv, W, H, p[3], p[4], p + 5, out, samples, 1.0 / 1024.0, bounds);
    FILE* g = fopen(argv[2], "wb");
    if (!g) return 2;
    fwrite(out, sizeof(double), (size_t)nv * H * W * 4, g);
    fwrite(samples, sizeof(long long), (size_t)nv, g);
    fwrite(bounds, sizeof(long long), (size_t)nv * 2, g);
    fclose(g);
    free(out); free(samples); free(bounds); free(cams); free(data); free(c); free(tf); free(p); free(h);
    return 0;
}
