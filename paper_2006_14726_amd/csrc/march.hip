// Server stage before the client path (Sec. 4.1): a volume ray marcher
// that writes, per source pixel, the front-to-back composited colour and one
// representative depth t (the first sample at which the accumulated alpha
// reaches depth_alpha), the image that splat_unproject turns into spheres;
// optionally also the depth interval [t_lo, t_hi] over which the alpha
// climbs from interval_lo to interval_hi (for the interval radius policy).
//
// One thread per pixel, 16 x 16 pixels per workgroup (four 8 x 8 waves, so a
// wave's rays stay close and its trilinear gathers hit the same cache
// lines).  Positions, weights and compositing are double precision; the
// volume is float.  Every sample is taken (no empty-space skipping), so the
// result is the marcher's definition exactly.
#include "common.h"
#include "kernels.h"

namespace splat {

constexpr int kMarchTile = 16;

__device__ inline double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

__global__ void __launch_bounds__(kMarchTile * kMarchTile)
k_raymarch(const float *__restrict__ vol, int32_t n, double lo, double size, Cam cam, double step,
           double alpha_scale, double depth_alpha, double stop_alpha, double interval_lo, double interval_hi,
           float4 *__restrict__ out_rgba, float *__restrict__ out_depth, float2 *__restrict__ out_interval)
{
    const int lx = threadIdx.x & 7, ly = (threadIdx.x >> 3) & 7, w = threadIdx.x >> 6;
    const int px = blockIdx.x * kMarchTile + (w & 1) * 8 + lx;
    const int py = blockIdx.y * kMarchTile + (w >> 1) * 8 + ly;
    if (px >= cam.w || py >= cam.h) return;
    double d[3];
    pixel_ray(cam, px, py, d);
    // the ray's interval inside the cube [lo, lo + size]^3, from t = 0
    double t_in = 0.0, t_out = INFINITY;
    for (int a = 0; a < 3; ++a) {
        const double o = cam.eye[a];
        if (d[a] == 0.0) {
            if (o < lo || o > lo + size) t_out = -1.0;
            continue;
        }
        double ta = (lo - o) / d[a], tb = (lo + size - o) / d[a];
        if (ta > tb) {
            const double s = ta;
            ta = tb;
            tb = s;
        }
        t_in = fmax(t_in, ta);
        t_out = fmin(t_out, tb);
    }
    double C0 = 0.0, C1 = 0.0, C2 = 0.0, A = 0.0, depth = INFINITY, t_lo = INFINITY, t_hi = INFINITY,
           t_last = INFINITY;
    if (t_in < t_out) {
        const double dt = step * size / (double)n;
        // position in voxel-centre units, g = (eye + t d - lo) n / size - 1/2, as base + t slope
        const double scale = (double)n / size;
        double base[3], slope[3];
        for (int a = 0; a < 3; ++a) {
            base[a] = (cam.eye[a] - lo) * scale - 0.5;
            slope[a] = d[a] * scale;
        }
        const uint32_t nn = (uint32_t)n, plane = nn * nn;  // n <= 1024: offsets fit 32 bits
        const int hi = n - 1;
        for (int64_t j = 0;; ++j) {
            const double t = t_in + ((double)j + 0.5) * dt;
            if (!(t < t_out)) break;
            // trilinear, clamp to edge
            uint32_t i0[3], i1[3];
            double f[3];
            for (int a = 0; a < 3; ++a) {
                const double g = fma(t, slope[a], base[a]);
                const double fl = floor(g);
                f[a] = g - fl;
                const double c = fmin(fmax(fl, -1.0), (double)hi);  // keeps the int conversion in range
                const int i = (int)c;
                i0[a] = (uint32_t)(i < 0 ? 0 : i);
                i1[a] = (uint32_t)(i + 1 > hi ? hi : i + 1);
            }
            const float *z0 = vol + i0[2] * plane, *z1 = vol + i1[2] * plane;
            const uint32_t y0 = i0[1] * nn, y1 = i1[1] * nn;
            const double v000 = z0[y0 + i0[0]], v100 = z0[y0 + i1[0]], v010 = z0[y1 + i0[0]], v110 = z0[y1 + i1[0]];
            const double v001 = z1[y0 + i0[0]], v101 = z1[y0 + i1[0]], v011 = z1[y1 + i0[0]], v111 = z1[y1 + i1[0]];
            const double gx = 1.0 - f[0], gy = 1.0 - f[1], gz = 1.0 - f[2];
            const double v = gz * (gy * (gx * v000 + f[0] * v100) + f[1] * (gx * v010 + f[0] * v110)) +
                             f[2] * (gy * (gx * v001 + f[0] * v101) + f[1] * (gx * v011 + f[0] * v111));
            // transfer and front-to-back compositing
            const double u = clamp01(v);
            const double s = clamp01(alpha_scale * v);
            const double wgt = (1.0 - A) * s;
            C0 += wgt * u;
            C1 += wgt * (4.0 * u * (1.0 - u));
            C2 += wgt * (1.0 - u);
            A += wgt;
            t_last = t;
            if (depth == INFINITY && A >= depth_alpha) depth = t;
            if (t_lo == INFINITY && A >= interval_lo) t_lo = t;
            if (t_hi == INFINITY && A >= interval_hi) t_hi = t;
            if (A >= stop_alpha) break;
        }
    }
    // an interval that opened but never reached interval_hi closes at the last sample
    if (t_lo != INFINITY && t_hi == INFINITY) t_hi = t_last;
    const size_t o = (size_t)py * cam.w + px;
    out_rgba[o] = make_float4((float)C0, (float)C1, (float)C2, (float)A);
    out_depth[o] = (float)depth;
    if (out_interval) out_interval[o] = make_float2((float)t_lo, (float)t_hi);
}

hipError_t launch_raymarch(const float *vol, int32_t n, double lo, double size, const Cam &cam,
                           const splat_march_opts &o, float *out_rgba, float *out_depth, float *out_interval,
                           hipStream_t s)
{
    const dim3 grid((cam.w + kMarchTile - 1) / kMarchTile, (cam.h + kMarchTile - 1) / kMarchTile);
    hipLaunchKernelGGL(k_raymarch, grid, dim3(kMarchTile * kMarchTile), 0, s, vol, n, lo, size, cam, o.step,
                       o.alpha_scale, o.depth_alpha, o.stop_alpha, o.interval_lo, o.interval_hi,
                       reinterpret_cast<float4 *>(out_rgba), out_depth, reinterpret_cast<float2 *>(out_interval));
    return hipGetLastError();
}

}  // namespace splat
