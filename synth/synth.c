/*
 * Seeded synthetic inputs: a blob volume and the server-side CPU ray caster
 * that turns it into a 2.5D premultiplied RGBA + depth image.
 *
 * This is input generation only.  It stands in for the server of the paper
 * (Sec. 4.1: a volume ray marcher writes a colour and a representative ray
 * parameter t_i per pixel) and holds none of the client method's arithmetic
 * (unprojection, hierarchy, sphere tracing, compositing of splats).  Both the
 * CPU oracle and the GPU path consume what it writes.
 *
 * Conventions (the paper names neither dataset nor transfer function):
 *   normalised volume coordinates [0,1]^3, n^3 voxels, voxel j centred at
 *   (j+1/2)/n, value v(x) = sum_k A_k exp(-|x-c_k|^2 / (2 sigma_k^2)),
 *   evaluated in double and stored as float, layout v[z][y][x];
 *   the volume occupies the world box [box_lo, box_lo + box_size]^3;
 *   trilinear reconstruction with clamp-to-edge;
 *   samples at t_in + (j+1/2)*dt with dt = 0.5*box_size/n (half a voxel);
 *   transfer: u = clamp(v,0,1), rgb = (u, 4u(1-u), 1-u), alpha = clamp(0.05 v,0,1),
 *   no step-size opacity correction;
 *   front-to-back: C += (1-A) a rgb, A += (1-A) a, stop at A >= 0.999;
 *   depth = the first sample t at which A >= 0.5, +inf if never.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double eye[3], forward[3], right[3], up[3];
    double tan_half_fov_y;
    int32_t width, height;
} syn_camera;

/* Sum of Gaussian blobs on an n^3 grid, separable per axis. */
int syn_make_volume(int32_t n, int32_t nblobs, const double *centres,
                    const double *sigmas, const double *amps, float *out)
{
    if (n <= 0 || nblobs < 0 || !out) return 1;
    double *fx = (double *)malloc(sizeof(double) * (size_t)n * (size_t)nblobs * 3);
    if (!fx) return 2;
    double *fy = fx + (size_t)n * nblobs, *fz = fy + (size_t)n * nblobs;
    for (int k = 0; k < nblobs; ++k) {
        double s2 = 2.0 * sigmas[k] * sigmas[k];
        for (int j = 0; j < n; ++j) {
            double p = (j + 0.5) / n;
            double dx = p - centres[3 * k + 0], dy = p - centres[3 * k + 1], dz = p - centres[3 * k + 2];
            fx[(size_t)k * n + j] = exp(-dx * dx / s2);
            fy[(size_t)k * n + j] = exp(-dy * dy / s2);
            fz[(size_t)k * n + j] = exp(-dz * dz / s2);
        }
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t zy = 0; zy < (int64_t)n * n; ++zy) {
        int z = (int)(zy / n), y = (int)(zy % n);
        double *acc = (double *)calloc((size_t)n, sizeof(double));
        for (int k = 0; k < nblobs; ++k) {
            double w = amps[k] * fy[(size_t)k * n + y] * fz[(size_t)k * n + z];
            const double *row = fx + (size_t)k * n;
            for (int x = 0; x < n; ++x) acc[x] += w * row[x];
        }
        float *dst = out + (size_t)zy * n;
        for (int x = 0; x < n; ++x) dst[x] = (float)acc[x];
        free(acc);
    }
    free(fx);
    return 0;
}

static double syn_clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

static double syn_sample(const float *vol, int n, const double p[3])
{
    double g[3], f[3];
    int i0[3], i1[3];
    for (int a = 0; a < 3; ++a) {
        g[a] = p[a] * n - 0.5;
        double fl = floor(g[a]);
        f[a] = g[a] - fl;
        int i = (int)fl;
        i0[a] = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
        i1[a] = i + 1 < 0 ? 0 : (i + 1 > n - 1 ? n - 1 : i + 1);
    }
#define V(X, Y, Z) ((double)vol[((size_t)(Z) * n + (Y)) * n + (X)])
    double c00 = V(i0[0], i0[1], i0[2]) * (1 - f[0]) + V(i1[0], i0[1], i0[2]) * f[0];
    double c10 = V(i0[0], i1[1], i0[2]) * (1 - f[0]) + V(i1[0], i1[1], i0[2]) * f[0];
    double c01 = V(i0[0], i0[1], i1[2]) * (1 - f[0]) + V(i1[0], i0[1], i1[2]) * f[0];
    double c11 = V(i0[0], i1[1], i1[2]) * (1 - f[0]) + V(i1[0], i1[1], i1[2]) * f[0];
#undef V
    double c0 = c00 * (1 - f[1]) + c10 * f[1];
    double c1 = c01 * (1 - f[1]) + c11 * f[1];
    return c0 * (1 - f[2]) + c1 * f[2];
}

/* Pinhole ray through the centre of pixel (x, y), row 0 at the top. */
static void syn_ray_dir(const syn_camera *c, int x, int y, double d[3])
{
    double aspect = (double)c->width / (double)c->height;
    double sx = ((2.0 * x + 1.0) / c->width - 1.0) * c->tan_half_fov_y * aspect;
    double sy = (1.0 - (2.0 * y + 1.0) / c->height) * c->tan_half_fov_y;
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = c->forward[a] + sx * c->right[a] + sy * c->up[a];
    double len = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int a = 0; a < 3; ++a) d[a] = v[a] / len;
}

/* Ray-march every pixel; rgba is premultiplied float [H][W][4], depth float [H][W]. */
int syn_raycast(const float *vol, int32_t n, double box_lo, double box_size, const syn_camera *cam,
                float *rgba, float *depth)
{
    if (!vol || !cam || !rgba || !depth || n <= 0 || cam->width <= 0 || cam->height <= 0 || !(box_size > 0))
        return 1;
    const int W = cam->width, H = cam->height;
    const double dt = 0.5 * box_size / n;
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            double d[3];
            syn_ray_dir(cam, x, y, d);
            double tin = 0.0, tout = INFINITY;
            for (int a = 0; a < 3; ++a) {
                double inv = 1.0 / d[a];
                double t0 = (box_lo - cam->eye[a]) * inv, t1 = (box_lo + box_size - cam->eye[a]) * inv;
                if (t0 > t1) { double s = t0; t0 = t1; t1 = s; }
                if (t0 > tin) tin = t0;
                if (t1 < tout) tout = t1;
            }
            double C[3] = {0, 0, 0}, A = 0.0, tdep = INFINITY;
            if (tin < tout) {
                for (int64_t j = 0;; ++j) {
                    double t = tin + (j + 0.5) * dt;
                    if (t >= tout) break;
                    double p[3];
                    for (int a = 0; a < 3; ++a) p[a] = (cam->eye[a] + d[a] * t - box_lo) / box_size;
                    double v = syn_sample(vol, n, p);
                    double u = syn_clampd(v, 0.0, 1.0);
                    double as = syn_clampd(0.05 * v, 0.0, 1.0);
                    double w = (1.0 - A) * as;
                    C[0] += w * u;
                    C[1] += w * 4.0 * u * (1.0 - u);
                    C[2] += w * (1.0 - u);
                    A += w;
                    if (A >= 0.5 && !isfinite(tdep)) tdep = t;
                    if (A >= 0.999) break;
                }
            }
            size_t i = (size_t)y * W + x;
            rgba[4 * i + 0] = (float)C[0];
            rgba[4 * i + 1] = (float)C[1];
            rgba[4 * i + 2] = (float)C[2];
            rgba[4 * i + 3] = (float)A;
            depth[i] = (float)tdep;
        }
    }
    return 0;
}
