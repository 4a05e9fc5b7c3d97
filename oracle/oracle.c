/*
 * FP64 CPU oracle for the client-side splat ray-tracing path of
 * "Augmenting Image Warping-Based Remote Volume Rendering with Ray Tracing"
 * (Zellmann, arXiv 2006.14726).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code with the GPU library.
 *
 * It is deliberately plain and slow: every ray is tested against every
 * sphere, the hits are sorted, and they are composited one by one in double
 * precision.  Functions:
 *
 *   orc_unproject   Sec. 4.1, Eq. 1: p = o + d t_i per pixel, a footprint
 *                   radius, compaction of pixels without a sample.
 *   orc_unproject_policy  the same with the radius set by opacity or by a
 *                   depth interval (Sec. 7).
 *   orc_render      Sec. 4.1 / Fig. 2: the samples as coloured
 *                   semi-transparent spheres, traced from a new camera,
 *                   composited front to back, stopping at a given alpha.
 *   orc_grad        gradient of a per-pixel loss through orc_render.
 *   orc_pixels_near lists the pixels whose ray passes near a point.
 *   orc_sphere_test one ray against one sphere (exposed for closed-form pins).
 *   orc_spheroid_test  one ray against a prolate spheroid: a sample smeared
 *                   along its source ray over its depth interval (Sec. 7).
 *   orc_render_axis orc_render over spheroids (an axis and half-length per
 *                   sample); orc_render is its sphere case.
 *   orc_half_bits   double -> IEEE binary16, round to nearest even.
 *   orc_raymarch    the server stage before the path (Sec. 4.1): a volume
 *                   ray marcher writing colour and a representative depth;
 *   orc_volume_sample  its trilinear reconstruction (exposed for pins).
 *   orc_encode, orc_decode  the 64-bit sample + 32-bit colour wire format
 *                   (Sec. 4.1, Sec. 6), with per-value helpers for pins.
 *   orc_accumulate  temporal accumulation of samples across frames (Sec. 7):
 *                   which history samples survive the merge with a new frame.
 *
 * Readings of the paper (it specifies none of these):
 *   - camera: pinhole, ray through pixel centre (x+1/2, y+1/2), row 0 at top,
 *     d = normalize(F + sx R + sy U), sx = ((2x+1)/W - 1) tan(fov/2) W/H,
 *     sy = (1 - (2y+1)/H) tan(fov/2);
 *   - a source pixel holds a sample iff its depth t is finite, t > 0, A > 0;
 *     radius = s * 2 t tan(fov/2) / H_src (s times the pixel footprint at t);
 *     colour stored straight: k = clamp(C/A, 0, 1), alpha a = A;
 *   - hit: with oc = c - o, b = oc.d, v = oc - b d, q = v.v, disc = r^2 - q,
 *     sphere hit iff disc >= 0 and t0 = b - sqrt(disc) lies in (0, t_max);
 *   - order: ascending (t0, sphere id);
 *   - compositing, per hit: C += T alpha k, A += T alpha, T *= (1 - alpha),
 *     n += 1; stop after a hit iff A >= alpha_stop; background 0;
 *   - alpha = a (mode 0, constant, the paper's constant sample colour) or
 *     alpha = a (1 - q/r^2)^2 (mode 1, soft, differentiable in r and c).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double eye[3], forward[3], right[3], up[3];
    double tan_half_fov_y;
    int32_t width, height;
} orc_camera;

/* Pixel-centre ray of a pinhole camera. */
static void orc_ray(const orc_camera *c, int64_t x, int64_t y, double d[3])
{
    double aspect = (double)c->width / (double)c->height;
    double sx = ((2.0 * (double)x + 1.0) / c->width - 1.0) * c->tan_half_fov_y * aspect;
    double sy = (1.0 - (2.0 * (double)y + 1.0) / c->height) * c->tan_half_fov_y;
    double v[3];
    for (int k = 0; k < 3; ++k) v[k] = c->forward[k] + sx * c->right[k] + sy * c->up[k];
    double len = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int k = 0; k < 3; ++k) d[k] = v[k] / len;
}

/* IEEE binary16 bits of v, rounded to nearest even (rint in the default mode). */
uint16_t orc_half_bits(double v)
{
    uint16_t sign = signbit(v) ? 0x8000u : 0u;
    double a = fabs(v);
    if (isnan(v)) return 0x7e00u;
    if (a == 0.0) return sign;
    if (a >= 65520.0) return (uint16_t)(sign | 0x7c00u); /* rounds to infinity */
    int e;
    frexp(a, &e);          /* a = m 2^e, m in [0.5, 1) */
    int E = e - 1;         /* a in [2^E, 2^(E+1)) */
    if (E < -14) {         /* subnormal range: multiples of 2^-24 */
        double q = rint(ldexp(a, 24));
        return (uint16_t)(sign | (uint16_t)q); /* q == 1024 is the smallest normal */
    }
    double q = rint(ldexp(a, 10 - E)); /* in [1024, 2048] */
    if (q == 2048.0) { q = 1024.0; E += 1; }
    if (E > 15) return (uint16_t)(sign | 0x7c00u);
    return (uint16_t)(sign | (uint16_t)((E + 15) << 10) | (uint16_t)(q - 1024.0));
}

/*
 * Eq. 1 unprojection with stable compaction.  rgba: premultiplied float
 * [H][W][4]; depth: float [H][W].  Outputs sample j (j < returned count):
 * centre_radius[4j..4j+3] = (float)p, (float)r; colour straight RGBA rounded
 * once from double, either as float (col_f32) or binary16 bits (col_f16);
 * src_index[j] = row-major source pixel index.  Pixels are visited in
 * row-major order, so samples keep the pixel order.
 */
int64_t orc_unproject(const orc_camera *cam, const float *rgba, const float *depth, double radius_scale,
                      float *centre_radius, float *col_f32, uint16_t *col_f16, uint32_t *src_index)
{
    const int64_t W = cam->width, H = cam->height;
    int64_t n = 0;
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            int64_t i = y * W + x;
            double t = depth[i];
            double A = rgba[4 * i + 3];
            if (!(isfinite(t) && t > 0.0 && A > 0.0)) continue;
            double d[3];
            orc_ray(cam, x, y, d);
            for (int k = 0; k < 3; ++k) centre_radius[4 * n + k] = (float)(cam->eye[k] + d[k] * t);
            double footprint = 2.0 * t * cam->tan_half_fov_y / (double)H;
            centre_radius[4 * n + 3] = (float)(radius_scale * footprint);
            double col[4];
            for (int k = 0; k < 3; ++k) {
                double kc = (double)rgba[4 * i + k] / A;
                col[k] = kc < 0.0 ? 0.0 : (kc > 1.0 ? 1.0 : kc);
            }
            col[3] = A;
            for (int k = 0; k < 4; ++k) {
                if (col_f32) col_f32[4 * n + k] = (float)col[k];
                if (col_f16) col_f16[4 * n + k] = orc_half_bits(col[k]);
            }
            if (src_index) src_index[n] = (uint32_t)i;
            ++n;
        }
    }
    return n;
}

/*
 * Radius policies (Sec. 7 suggests varying the radius with the sample's
 * opacity, or with how uncertain its depth is, smearing uncertain samples
 * over an interval along the ray; no rule is given).  The readings here:
 *   - mode 0, footprint: as orc_unproject, r = s fp(t), fp(t) = 2 t tan(fov/2) / H;
 *   - mode 1, opacity: r = s fp(t) sqrt(max(A, a_floor)): the sphere's disc
 *     area grows in proportion to the pixel's opacity (the paper's own rule,
 *     radius 0 without opacity and the full footprint with it, is the step
 *     version of this);
 *   - mode 2, interval: the pixel's depth interval [t_lo, t_hi] (from the
 *     marcher) replaces the single depth: the centre sits at its midpoint
 *     t_c = (t_lo + t_hi) / 2 on the ray and r = max(s fp(t_c),
 *     kappa (t_hi - t_lo) / 2), so the sphere covers the interval.  A pixel
 *     holds a sample iff the depth rule holds and 0 < t_lo <= t_hi, both finite;
 *   - mode 3, spheroid: the interval's sample smeared along the ray instead of
 *     grown in every direction: centre at t_c on the ray, r = s fp(t_c) across
 *     the ray, half-length h = max(r, kappa (t_hi - t_lo) / 2) along it, axis
 *     u = the unit source ray d; axis[4n..4n+3] = (u, h), each rounded once to
 *     float.  The validity rule is mode 2's.
 * Colour, alpha, order and compaction are those of orc_unproject.
 */
int64_t orc_unproject_policy(const orc_camera *cam, const float *rgba, const float *depth, const float *interval,
                             int32_t mode, double radius_scale, double a_floor, double kappa, float *centre_radius,
                             float *col_f32, uint16_t *col_f16, uint32_t *src_index, float *axis)
{
    const int64_t W = cam->width, H = cam->height;
    int64_t n = 0;
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            const int64_t i = y * W + x;
            double t = depth[i];
            const double A = rgba[4 * i + 3];
            if (!(isfinite(t) && t > 0.0 && A > 0.0)) continue;
            double half_len = 0.0;
            if (mode == 2 || mode == 3) {
                const double lo = interval[2 * i], hi = interval[2 * i + 1];
                if (!(isfinite(lo) && isfinite(hi) && lo > 0.0 && hi >= lo)) continue;
                t = 0.5 * (lo + hi);
                half_len = 0.5 * (hi - lo);
            }
            double d[3];
            orc_ray(cam, x, y, d);
            for (int k = 0; k < 3; ++k) centre_radius[4 * n + k] = (float)(cam->eye[k] + d[k] * t);
            const double footprint = 2.0 * t * cam->tan_half_fov_y / (double)H;
            double r = radius_scale * footprint;
            if (mode == 1) r = r * sqrt(A > a_floor ? A : a_floor);
            if (mode == 2 && kappa * half_len > r) r = kappa * half_len;
            centre_radius[4 * n + 3] = (float)r;
            if (mode == 3) {
                const double h = kappa * half_len > r ? kappa * half_len : r;
                for (int k = 0; k < 3; ++k) axis[4 * n + k] = (float)d[k];
                axis[4 * n + 3] = (float)h;
            }
            double col[4];
            for (int k = 0; k < 3; ++k) {
                double kc = (double)rgba[4 * i + k] / A;
                col[k] = kc < 0.0 ? 0.0 : (kc > 1.0 ? 1.0 : kc);
            }
            col[3] = A;
            for (int k = 0; k < 4; ++k) {
                if (col_f32) col_f32[4 * n + k] = (float)col[k];
                if (col_f16) col_f16[4 * n + k] = orc_half_bits(col[k]);
            }
            if (src_index) src_index[n] = (uint32_t)i;
            ++n;
        }
    }
    return n;
}

/* One ray-sphere candidate. */
typedef struct {
    double t0;   /* entry distance */
    double q;    /* squared distance from ray to centre */
    double v[3]; /* offset from the closest ray point to the centre */
    int64_t id;
} orc_hit;

static int orc_hit_cmp(const void *pa, const void *pb)
{
    const orc_hit *a = (const orc_hit *)pa, *b = (const orc_hit *)pb;
    if (a->t0 < b->t0) return -1;
    if (a->t0 > b->t0) return 1;
    return (a->id > b->id) - (a->id < b->id);
}

/* Sphere table: [N][8] doubles = cx, cy, cz, r, k_r, k_g, k_b, a. */
#define SPH(j, f) (sph[8 * (j) + (f)])

static double orc_alpha(const double *sph, const orc_hit *h, int mode)
{
    double a = SPH(h->id, 7);
    if (mode == 0) return a;
    double r = SPH(h->id, 3);
    double u = h->q / (r * r);
    return a * (1.0 - u) * (1.0 - u);
}

/* Test every sphere; returns the number of hits (sorted) and flags grazing candidates. */
typedef struct {
    orc_hit *hits;
    int64_t nhits, cap_hits;
    double *graze_t; /* approximate position along the ray of grazing spheres */
    double *graze_r;
    int64_t ngraze, cap_graze;
    orc_hit *scratch; /* same capacity as hits */
    double *Ti, *al;  /* same capacity as hits */
    int oom;
} orc_ray_hits;

static void orc_rh_init(orc_ray_hits *rh)
{
    memset(rh, 0, sizeof(*rh));
}

static void orc_rh_free(orc_ray_hits *rh)
{
    free(rh->hits);
    free(rh->graze_t);
    free(rh->graze_r);
    free(rh->scratch);
    free(rh->Ti);
    free(rh->al);
    memset(rh, 0, sizeof(*rh));
}

static int orc_rh_grow_hits(orc_ray_hits *rh)
{
    int64_t cap = rh->cap_hits ? 2 * rh->cap_hits : 256;
    orc_hit *h = (orc_hit *)realloc(rh->hits, sizeof(orc_hit) * (size_t)cap);
    orc_hit *s = h ? (orc_hit *)realloc(rh->scratch, sizeof(orc_hit) * (size_t)cap) : NULL;
    if (h) rh->hits = h;
    if (s) rh->scratch = s;
    double *t = s ? (double *)realloc(rh->Ti, sizeof(double) * (size_t)cap) : NULL;
    if (t) rh->Ti = t;
    double *a = t ? (double *)realloc(rh->al, sizeof(double) * (size_t)cap) : NULL;
    if (a) rh->al = a;
    if (!a) { rh->oom = 1; return 1; }
    rh->cap_hits = cap;
    return 0;
}

static int orc_rh_grow_graze(orc_ray_hits *rh)
{
    int64_t cap = rh->cap_graze ? 2 * rh->cap_graze : 64;
    double *t = (double *)realloc(rh->graze_t, sizeof(double) * (size_t)cap);
    double *r = t ? (double *)realloc(rh->graze_r, sizeof(double) * (size_t)cap) : NULL;
    if (t) rh->graze_t = t;
    if (r) rh->graze_r = r;
    if (!r) { rh->oom = 1; return 1; }
    rh->cap_graze = cap;
    return 0;
}

/*
 * Ray-sphere test in the numerically robust form (the perpendicular offset v
 * is formed before squaring, instead of b^2 - |oc|^2 + r^2, which cancels).
 * out[0] = t0, out[1] = q, out[2] = disc, out[3..5] = v, out[6] = b.
 * Returns 1 iff disc >= 0 and 0 < t0 < t_max.
 */
int orc_sphere_test(const double o[3], const double d[3], const double c[3], double r, double t_max,
                    double out[7])
{
    double oc[3] = {c[0] - o[0], c[1] - o[1], c[2] - o[2]};
    double b = oc[0] * d[0] + oc[1] * d[1] + oc[2] * d[2];
    double v[3] = {oc[0] - b * d[0], oc[1] - b * d[1], oc[2] - b * d[2]};
    double q = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double disc = r * r - q;
    double t0 = disc >= 0.0 ? b - sqrt(disc) : NAN;
    out[0] = t0;
    out[1] = q;
    out[2] = disc;
    out[3] = v[0];
    out[4] = v[1];
    out[5] = v[2];
    out[6] = b;
    return disc >= 0.0 && t0 > 0.0 && t0 < t_max;
}

/*
 * Ray against a prolate spheroid (Sec. 7 suggests smearing a sample whose
 * depth is uncertain over an interval along its ray; this is that shape):
 * centre c, axis u, half-length h along u and radius r across it, the points
 * x with |x - c|^2 / r^2 + ((x - c).u)^2 (1/h^2 - 1/r^2) <= 1, u the given
 * axis scaled to unit length in double (a stored float axis is off unit length
 * by rounding, and the shape must stay a spheroid for any r / h).  The linear
 * map S y = y / r + (y.u)(1/h - 1/r) u takes it to the unit ball, and the ray
 * o + t d (d unit) to t D - L with D = S d, L = S (c - o).  The robust form of
 * the sphere test then applies in those coordinates: t_m = L.D / D.D,
 * v = L - t_m D, qq = v.v, disc = 1 - qq, t0 = t_m - sqrt(disc / D.D).
 * out[0] = t0, out[1] = disc, out[2] = t_m, out[3] = qq.
 * Returns 1 iff disc >= 0 and 0 < t0 < t_max.  With h = r this is the sphere.
 */
int orc_spheroid_test(const double o[3], const double d[3], const double c[3], double r, const double u_in[3],
                      double h, double t_max, double out[4])
{
    const double oc[3] = {c[0] - o[0], c[1] - o[1], c[2] - o[2]};
    const double w = 1.0 / h - 1.0 / r;
    const double ul = sqrt(u_in[0] * u_in[0] + u_in[1] * u_in[1] + u_in[2] * u_in[2]);
    const double u[3] = {u_in[0] / ul, u_in[1] / ul, u_in[2] / ul};
    const double du = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
    const double ou = oc[0] * u[0] + oc[1] * u[1] + oc[2] * u[2];
    double D[3], L[3];
    for (int k = 0; k < 3; ++k) {
        D[k] = d[k] / r + du * w * u[k];
        L[k] = oc[k] / r + ou * w * u[k];
    }
    const double DD = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
    const double tm = (L[0] * D[0] + L[1] * D[1] + L[2] * D[2]) / DD;
    const double v[3] = {L[0] - tm * D[0], L[1] - tm * D[1], L[2] - tm * D[2]};
    const double qq = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double disc = 1.0 - qq;
    const double t0 = disc >= 0.0 ? tm - sqrt(disc / DD) : NAN;
    out[0] = t0;
    out[1] = disc;
    out[2] = tm;
    out[3] = qq;
    return disc >= 0.0 && t0 > 0.0 && t0 < t_max;
}

/* Every sample against the ray: spheres (ax NULL), or spheroids with
 * ax[4 j..4 j + 3] = (u, h) of sample j. */
static void orc_collect(const double *sph, const double *ax, int64_t nsph, const double o[3], const double d[3],
                        double t_max, orc_ray_hits *rh)
{
    rh->nhits = 0;
    rh->ngraze = 0;
    for (int64_t j = 0; j < nsph; ++j) {
        double res[7];
        double r = SPH(j, 3);
        int hit;
        if (ax) {
            /* disc is relative to the unit ball here: the same 1e-6 band */
            double e[4];
            hit = orc_spheroid_test(o, d, &SPH(j, 0), r, &ax[4 * j], ax[4 * j + 3], t_max, e);
            res[0] = e[0];
            res[1] = e[3];
            res[2] = e[1] * r * r;
            res[3] = res[4] = res[5] = 0.0;
            res[6] = e[2];
            r = ax[4 * j + 3] > r ? ax[4 * j + 3] : r;  /* the extent along the ray, for the grazing range */
        } else {
            hit = orc_sphere_test(o, d, &SPH(j, 0), r, t_max, res);
        }
        if (fabs(res[2]) <= 1e-6 * SPH(j, 3) * SPH(j, 3)) {
            if (rh->ngraze == rh->cap_graze && orc_rh_grow_graze(rh)) return;
            rh->graze_t[rh->ngraze] = res[6];
            rh->graze_r[rh->ngraze] = r;
            rh->ngraze++;
        }
        if (!hit) continue;
        if (rh->nhits == rh->cap_hits && orc_rh_grow_hits(rh)) return;
        orc_hit *h = &rh->hits[rh->nhits++];
        h->t0 = res[0];
        h->q = res[1];
        h->v[0] = res[3];
        h->v[1] = res[4];
        h->v[2] = res[5];
        h->id = j;
    }
    qsort(rh->hits, (size_t)rh->nhits, sizeof(orc_hit), orc_hit_cmp);
}

/*
 * Composite a sorted hit list.  force_at >= 0 flips the decision taken at
 * knife-edge number force_at (0 = the first one met): a stop decision with
 * |A - alpha_stop| <= 1e-5 is reversed, a pair of consecutive hits with
 * 0 < |dt| <= 1e-12 t is swapped.  Returns the number of knife-edges met.
 */
static int orc_composite(const double *sph, const orc_hit *hits_in, int64_t nh, int mode, double alpha_stop,
                         int force_at, orc_hit *scratch, double out[4], int64_t *out_n, double *t_last)
{
    memcpy(scratch, hits_in, sizeof(orc_hit) * (size_t)nh);
    double C[3] = {0, 0, 0}, A = 0.0, T = 1.0;
    int64_t n = 0;
    int knives = 0;
    *t_last = -INFINITY;
    for (int64_t i = 0; i < nh; ++i) {
        if (i + 1 < nh) {
            double dt = scratch[i + 1].t0 - scratch[i].t0;
            if (dt != 0.0 && fabs(dt) <= 1e-12 * fabs(scratch[i].t0)) {
                if (knives == force_at) {
                    orc_hit tmp = scratch[i];
                    scratch[i] = scratch[i + 1];
                    scratch[i + 1] = tmp;
                }
                knives++;
            }
        }
        const orc_hit *h = &scratch[i];
        double al = orc_alpha(sph, h, mode);
        for (int k = 0; k < 3; ++k) C[k] += T * al * SPH(h->id, 4 + k);
        A += T * al;
        T *= (1.0 - al);
        n++;
        *t_last = h->t0;
        int stop = A >= alpha_stop;
        if (fabs(A - alpha_stop) <= 1e-5) {
            if (knives == force_at) stop = !stop;
            knives++;
        }
        if (stop) break;
    }
    out[0] = C[0];
    out[1] = C[1];
    out[2] = C[2];
    out[3] = A;
    *out_n = n;
    return knives;
}

/*
 * Brute-force render of the pixels listed in `pix` (row-major ids; NULL means
 * all W*H pixels in order).  Per output pixel: out_rgba[4], out_n, flags:
 *   bit 0: a grazing sphere (|disc| <= 1e-6 r^2) lies before the end of the
 *          composited range (exempt from the comparison);
 *   bit 1: exactly one knife-edge; alt_rgba / alt_n hold the other branch;
 *   bit 2: more than one knife-edge (exempt).
 * out_sig (nullable) receives a hash of the ordered composited sphere ids.
 * Returns 0, 1 on bad arguments, 2 when out of memory.
 */
int orc_render_axis(const double *sph, const double *ax, int64_t nsph, const orc_camera *cam, double alpha_stop,
                    double t_max, int mode, const int64_t *pix, int64_t npix, double *out_rgba, int32_t *out_n,
                    int32_t *flags, double *alt_rgba, int32_t *alt_n, uint64_t *out_sig)
{
    if (!sph && nsph > 0) return 1;
    if (ax && mode != 0) return 1; /* spheroids: constant alpha only */
    if (!cam || !out_rgba || !out_n || !flags || !alt_rgba || !alt_n) return 1;
    const int64_t W = cam->width;
    if (!pix) npix = (int64_t)cam->width * cam->height;
    int err = 0;
#pragma omp parallel
    {
        orc_ray_hits rh;
        orc_rh_init(&rh);
        orc_rh_grow_hits(&rh);
        orc_rh_grow_graze(&rh);
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npix; ++p) {
            if (rh.oom) continue;
            int64_t id = pix ? pix[p] : p;
            double d[3];
            orc_ray(cam, id % W, id / W, d);
            orc_collect(sph, ax, nsph, cam->eye, d, t_max, &rh);
            if (rh.oom) continue;
            double rgba[4], t_last;
            int64_t n;
            int knives = orc_composite(sph, rh.hits, rh.nhits, mode, alpha_stop, -1, rh.scratch, rgba, &n, &t_last);
            int32_t f = 0;
            int stopped = n < rh.nhits || (n > 0 && rgba[3] >= alpha_stop);
            for (int64_t g = 0; g < rh.ngraze; ++g) {
                double tb = rh.graze_t[g], rr = rh.graze_r[g];
                if (tb + rr <= 0.0 || tb - 1e-3 * rr >= t_max) continue; /* outside (0, t_max) */
                if (!stopped || tb - 1e-3 * rr <= t_last) f |= 1;
            }
            double alt[4] = {rgba[0], rgba[1], rgba[2], rgba[3]};
            int64_t nalt = n;
            if (knives == 1) {
                double t2;
                int k2 = orc_composite(sph, rh.hits, rh.nhits, mode, alpha_stop, 0, rh.scratch, alt, &nalt, &t2);
                f |= (k2 == 1) ? 2 : 4;
            } else if (knives > 1) {
                f |= 4;
            }
            for (int k = 0; k < 4; ++k) {
                out_rgba[4 * p + k] = rgba[k];
                alt_rgba[4 * p + k] = alt[k];
            }
            out_n[p] = (int32_t)n;
            alt_n[p] = (int32_t)nalt;
            flags[p] = f;
            if (out_sig) {
                /* FNV-1a over the composited ids, in order */
                uint64_t hsh = 1469598103934665603ull;
                for (int64_t i = 0; i < n; ++i) {
                    hsh ^= (uint64_t)rh.hits[i].id;
                    hsh *= 1099511628211ull;
                }
                out_sig[p] = hsh ^ (uint64_t)n;
            }
        }
        if (rh.oom) {
#pragma omp atomic write
            err = 2;
        }
        orc_rh_free(&rh);
    }
    return err;
}

/* orc_render_axis over spheres. */
int orc_render(const double *sph, int64_t nsph, const orc_camera *cam, double alpha_stop, double t_max, int mode,
               const int64_t *pix, int64_t npix, double *out_rgba, int32_t *out_n, int32_t *flags,
               double *alt_rgba, int32_t *alt_n, uint64_t *out_sig)
{
    return orc_render_axis(sph, NULL, nsph, cam, alpha_stop, t_max, mode, pix, npix, out_rgba, out_n, flags,
                           alt_rgba, alt_n, out_sig);
}

/*
 * Gradient of L = sum_p sum_ch g[p][ch] * I[p][ch] (a linearised loss: pass
 * g = dL/dI of the real loss) with respect to every sphere parameter.
 * out_grad [N][8] (zeroed here) = dL/d(cx, cy, cz, r, k_r, k_g, k_b, a).
 *
 * Per pixel with ordered composited hits i = 1..n (T_1 = 1,
 * T_{i+1} = T_i (1 - alpha_i)), w_i = k_i . g_C + g_A:
 *   dL/dk_i     = T_i alpha_i g_C
 *   dL/dalpha_i = T_i (w_i - R_i),  R_n = 0,
 *                 R_{i-1} = alpha_i w_i + (1 - alpha_i) R_i
 * (R_i is the remainder behind hit i composited from full transmittance).
 * Chain rule through alpha = a (1-u)^2, u = q / r^2, q = |v|^2 (soft mode):
 *   dalpha/da = (1-u)^2, dalpha/dr = 4 a (1-u) q / r^3,
 *   dalpha/dc = -4 a (1-u) v / r^2;
 * constant mode: dalpha/da = 1, no radius or centre gradient.  The order of
 * the hits is piecewise constant and carries no gradient.
 */
int orc_grad(const double *sph, int64_t nsph, const orc_camera *cam, double alpha_stop, double t_max, int mode,
             const double *grad_rgba, double *out_grad)
{
    if (!cam || !grad_rgba || !out_grad || (!sph && nsph > 0)) return 1;
    const int64_t W = cam->width, P = (int64_t)cam->width * cam->height;
    memset(out_grad, 0, sizeof(double) * 8 * (size_t)nsph);
    int err = 0;
#pragma omp parallel
    {
        orc_ray_hits rh;
        orc_rh_init(&rh);
        orc_rh_grow_hits(&rh);
        orc_rh_grow_graze(&rh);
        double *acc = (double *)calloc(8 * (size_t)(nsph > 0 ? nsph : 1), sizeof(double));
        if (!acc) rh.oom = 1;
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < P; ++p) {
            if (rh.oom) continue;
            const double *g = grad_rgba + 4 * p;
            double d[3];
            orc_ray(cam, p % W, p / W, d);
            orc_collect(sph, NULL, nsph, cam->eye, d, t_max, &rh);
            if (rh.oom) continue;
            double rgba[4], t_last;
            int64_t n;
            orc_composite(sph, rh.hits, rh.nhits, mode, alpha_stop, -1, rh.scratch, rgba, &n, &t_last);
            double T = 1.0;
            for (int64_t i = 0; i < n; ++i) {
                rh.Ti[i] = T;
                rh.al[i] = orc_alpha(sph, &rh.hits[i], mode);
                T *= (1.0 - rh.al[i]);
            }
            double R = 0.0;
            for (int64_t i = n - 1; i >= 0; --i) {
                const orc_hit *h = &rh.hits[i];
                int64_t j = h->id;
                double al = rh.al[i], Ti = rh.Ti[i];
                double w = SPH(j, 4) * g[0] + SPH(j, 5) * g[1] + SPH(j, 6) * g[2] + g[3];
                double dal = Ti * (w - R);
                for (int k = 0; k < 3; ++k) acc[8 * j + 4 + k] += Ti * al * g[k];
                if (mode == 0) {
                    acc[8 * j + 7] += dal;
                } else {
                    double a = SPH(j, 7), r = SPH(j, 3);
                    double u = h->q / (r * r);
                    acc[8 * j + 7] += dal * (1.0 - u) * (1.0 - u);
                    acc[8 * j + 3] += dal * 4.0 * a * (1.0 - u) * h->q / (r * r * r);
                    for (int k = 0; k < 3; ++k) acc[8 * j + k] += dal * (-4.0 * a * (1.0 - u) * h->v[k] / (r * r));
                }
                R = al * w + (1.0 - al) * R;
            }
        }
        if (rh.oom) {
#pragma omp atomic write
            err = 2;
        } else {
#pragma omp critical
            for (size_t k = 0; k < 8 * (size_t)nsph; ++k) out_grad[k] += acc[k];
        }
        free(acc);
        orc_rh_free(&rh);
    }
    return err;
}

/* Row-major ids of the pixels whose ray passes within `radius` of `centre`, in front of the eye. */
int64_t orc_pixels_near(const orc_camera *cam, const double centre[3], double radius, int64_t *out, int64_t cap)
{
    const int64_t W = cam->width, P = (int64_t)cam->width * cam->height;
    int64_t n = 0;
    for (int64_t p = 0; p < P; ++p) {
        double d[3];
        orc_ray(cam, p % W, p / W, d);
        double oc[3] = {centre[0] - cam->eye[0], centre[1] - cam->eye[1], centre[2] - cam->eye[2]};
        double b = oc[0] * d[0] + oc[1] * d[1] + oc[2] * d[2];
        double v[3] = {oc[0] - b * d[0], oc[1] - b * d[1], oc[2] - b * d[2]};
        double q = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        if (q <= radius * radius && b + radius > 0.0) {
            if (n < cap) out[n] = p;
            n++;
        }
    }
    return n;
}

/* ------------------------------------------------------------------ server
 * The server stage before the client path (Sec. 4.1: a ray marcher renders
 * the volume and writes, per pixel, the composited colour and one
 * representative depth t).  The paper names only a standard ray marcher and
 * a depth heuristic from earlier work; the rules written out here are the
 * reading used here:
 *   - volume v[z][y][x] of n^3 floats filling the cube [lo, lo + size]^3,
 *     voxel (i, j, k) centred at lo + (i + 1/2, j + 1/2, k + 1/2) size / n;
 *     reconstruction is trilinear with clamp-to-edge;
 *   - the pixel ray (as above) meets the cube over [t_in, t_out], t_in >= 0;
 *     samples at t_j = t_in + (j + 1/2) dt while t_j < t_out, with
 *     dt = step * size / n (step in voxels);
 *   - transfer: u = clamp(v, 0, 1), colour (u, 4u(1 - u), 1 - u), sample
 *     alpha s = clamp(alpha_scale v, 0, 1);
 *   - front to back: w = (1 - A) s, C += w colour, A += w; the depth is the
 *     first t_j at which A >= depth_alpha (infinite if never); marching
 *     stops after the sample at which A >= stop_alpha;
 *   - the depth interval (for the interval radius policy, Sec. 7): t_lo is
 *     the first t_j at which A >= interval_lo, t_hi the first at which
 *     A >= interval_hi, or the last t_j taken if A never gets there (both
 *     infinite if A never reaches interval_lo);
 *   - output: premultiplied (C, A), depth and interval, as float.
 */

/* Trilinear value at normalised position p in [0,1]^3 (clamp to edge):
 * the sum over the 8 surrounding voxel centres of value x weight. */
double orc_volume_sample(const float *vol, int32_t n, const double p[3])
{
    int64_t base[3];
    double frac[3];
    for (int a = 0; a < 3; ++a) {
        const double g = p[a] * (double)n - 0.5;  /* position in voxel-centre units */
        const double fl = floor(g);
        base[a] = (int64_t)fl;
        frac[a] = g - fl;
    }
    double sum = 0.0;
    for (int corner = 0; corner < 8; ++corner) {
        int64_t idx[3];
        double w = 1.0;
        for (int a = 0; a < 3; ++a) {
            const int up = (corner >> a) & 1;
            int64_t i = base[a] + up;
            if (i < 0) i = 0;
            if (i > n - 1) i = n - 1;
            idx[a] = i;
            w *= up ? frac[a] : 1.0 - frac[a];
        }
        sum += w * (double)vol[(idx[2] * n + idx[1]) * n + idx[0]];
    }
    return sum;
}

static double orc_clamp(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* One pixel of the marcher; returns the number of samples taken. */
static int64_t orc_march_pixel(const float *vol, int32_t n, double lo, double size, const orc_camera *cam,
                               int64_t x, int64_t y, double step, double alpha_scale, double depth_alpha,
                               double stop_alpha, double interval_lo, double interval_hi, double out[7])
{
    double d[3];
    orc_ray(cam, x, y, d);
    double t_in = 0.0, t_out = INFINITY;
    for (int a = 0; a < 3; ++a) {
        const double o = cam->eye[a];
        if (d[a] == 0.0) {
            if (o < lo || o > lo + size) t_out = -1.0;  /* parallel to the slab and outside it */
            continue;
        }
        double ta = (lo - o) / d[a], tb = (lo + size - o) / d[a];
        if (ta > tb) { const double s = ta; ta = tb; tb = s; }
        if (ta > t_in) t_in = ta;
        if (tb < t_out) t_out = tb;
    }
    double C[3] = {0.0, 0.0, 0.0}, A = 0.0, depth = INFINITY, t_lo = INFINITY, t_hi = INFINITY, t_last = INFINITY;
    int64_t taken = 0;
    if (t_in < t_out) {
        const double dt = step * size / (double)n;
        for (int64_t j = 0;; ++j) {
            const double t = t_in + ((double)j + 0.5) * dt;
            if (!(t < t_out)) break;
            double p[3];
            for (int a = 0; a < 3; ++a) p[a] = (cam->eye[a] + t * d[a] - lo) / size;
            const double v = orc_volume_sample(vol, n, p);
            const double u = orc_clamp(v, 0.0, 1.0);
            const double s = orc_clamp(alpha_scale * v, 0.0, 1.0);
            const double w = (1.0 - A) * s;
            C[0] += w * u;
            C[1] += w * (4.0 * u * (1.0 - u));
            C[2] += w * (1.0 - u);
            A += w;
            ++taken;
            t_last = t;
            if (depth == INFINITY && A >= depth_alpha) depth = t;
            if (t_lo == INFINITY && A >= interval_lo) t_lo = t;
            if (t_hi == INFINITY && A >= interval_hi) t_hi = t;
            if (A >= stop_alpha) break;
        }
    }
    /* an interval that opened but never reached interval_hi closes at the last sample taken */
    if (t_lo != INFINITY && t_hi == INFINITY) t_hi = t_last;
    out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = A; out[4] = depth; out[5] = t_lo; out[6] = t_hi;
    return taken;
}

/* The marcher over all pixels (pixels == NULL) or a list of pixel indices;
 * out is double [count][7]: C (3), A, depth, t_lo, t_hi.  Returns 0. */
int orc_raymarch(const float *vol, int32_t n, double lo, double size, const orc_camera *cam, double step,
                 double alpha_scale, double depth_alpha, double stop_alpha, double interval_lo, double interval_hi,
                 const int64_t *pixels, int64_t count, double *out)
{
    const int64_t W = cam->width;
    const int64_t total = pixels ? count : W * (int64_t)cam->height;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < total; ++k) {
        const int64_t pix = pixels ? pixels[k] : k;
        orc_march_pixel(vol, n, lo, size, cam, pix % W, pix / W, step, alpha_scale, depth_alpha, stop_alpha,
                        interval_lo, interval_hi, out + 7 * k);
    }
    return 0;
}

/* ------------------------------------------------------------------ codec
 * The sample codec of the wire format (Sec. 4.1: each object-space sample's
 * quantised coordinate is packed with its radius into 64 bits; Sec. 6: 32
 * bits per colour).  The paper leaves the bit split open; the reading here:
 *   - position: 18 bits per axis, q = clamp(floor((x - lo) / size 2^18),
 *     0, 2^18 - 1), decoded at the cell centre lo + (q + 1/2) size / 2^18;
 *   - radius: 10 bits, c = clamp(round_half_up(64 log2(r / r_unit)) + 512,
 *     0, 1023), decoded as r_unit 2^((c - 512) / 64);
 *   - word = qx | qy << 18 | qz << 36 | c << 54;
 *   - colour: 8 bits per straight channel and alpha,
 *     b = floor(clamp(v, 0, 1) 255 + 1/2), decoded as b / 255, byte 0 = red.
 */

static uint64_t orc_quant(double v, double lo, double size, int bits)
{
    const double cells = (double)((uint64_t)1 << bits);
    double q = floor((v - lo) / size * cells);
    if (!(q >= 0.0)) q = 0.0;  /* also NaN */
    if (q > cells - 1.0) q = cells - 1.0;
    return (uint64_t)q;
}

uint64_t orc_encode_position(const double c[3], double r, const double lo[3], double size, double r_unit)
{
    uint64_t w = 0;
    for (int a = 0; a < 3; ++a) w |= orc_quant(c[a], lo[a], size, 18) << (18 * a);
    double code = floor(64.0 * log2(r / r_unit) + 0.5) + 512.0;
    if (!(code >= 0.0)) code = 0.0;
    if (code > 1023.0) code = 1023.0;
    return w | ((uint64_t)code << 54);
}

void orc_decode_position(uint64_t w, const double lo[3], double size, double r_unit, double c[3], double *r)
{
    const double step = size / (double)((uint64_t)1 << 18);
    for (int a = 0; a < 3; ++a) c[a] = lo[a] + ((double)((w >> (18 * a)) & 0x3ffffu) + 0.5) * step;
    *r = r_unit * exp2(((double)(w >> 54) - 512.0) / 64.0);
}

uint32_t orc_encode_colour(const double k[4])
{
    uint32_t w = 0;
    for (int ch = 0; ch < 4; ++ch) {
        const double v = k[ch] < 0.0 ? 0.0 : (k[ch] > 1.0 ? 1.0 : (k[ch] == k[ch] ? k[ch] : 0.0));
        w |= (uint32_t)floor(v * 255.0 + 0.5) << (8 * ch);
    }
    return w;
}

void orc_decode_colour(uint32_t w, double k[4])
{
    for (int ch = 0; ch < 4; ++ch) k[ch] = (double)((w >> (8 * ch)) & 0xffu) / 255.0;
}

/* Whole arrays: spheres (n x [c, r] and n x straight rgba) -> words, and back
 * (the decoded centre and radius rounded to float, the colour to float). */
void orc_encode(const float *centre_radius, const double *rgba, int64_t n, const double lo[3], double size,
                double r_unit, uint64_t *pos, uint32_t *col)
{
    for (int64_t i = 0; i < n; ++i) {
        const double c[3] = {centre_radius[4 * i], centre_radius[4 * i + 1], centre_radius[4 * i + 2]};
        pos[i] = orc_encode_position(c, (double)centre_radius[4 * i + 3], lo, size, r_unit);
        col[i] = orc_encode_colour(rgba + 4 * i);
    }
}

void orc_decode(const uint64_t *pos, const uint32_t *col, int64_t n, const double lo[3], double size, double r_unit,
                float *centre_radius, float *rgba)
{
    for (int64_t i = 0; i < n; ++i) {
        double c[3], r, k[4];
        orc_decode_position(pos[i], lo, size, r_unit, c, &r);
        orc_decode_colour(col[i], k);
        for (int a = 0; a < 3; ++a) centre_radius[4 * i + a] = (float)c[a];
        centre_radius[4 * i + 3] = (float)r;
        for (int ch = 0; ch < 4; ++ch) rgba[4 * i + ch] = (float)k[ch];
    }
}

/*
 * Temporal accumulation (Sec. 7 names keeping samples across a few frames as
 * an extension; it gives no policy).  The reading here:
 *   - a uniform grid of `grid`^3 cells covers [lo, lo + size]^3; a centre x
 *     lies in cell q = clamp(floor((x - lo) / size grid), 0, grid - 1) per
 *     axis (centres outside the box fall into the border cells);
 *   - the merged set is the new frame's samples, in their order, with age 0,
 *     followed by the history samples, in their order, that survive: a
 *     history sample survives iff its age + 1 <= max_age and no centre of the
 *     new frame lies in its cell; it carries age + 1;
 *   - if the merged set exceeds the capacity, its first `capacity` samples
 *     are kept (the newest, since the list stays sorted by age).
 * orc_accumulate returns the number of surviving history samples and their
 * indices, ascending.  The frame's cells are sorted once and looked up by
 * binary search; everything else is one pass over the history.
 */
static uint64_t orc_cell_key(const float *cr, const double lo[3], double size, int32_t grid)
{
    uint64_t key = 0;
    for (int a = 0; a < 3; ++a) {
        double q = floor(((double)cr[a] - lo[a]) / size * (double)grid);
        if (!(q >= 0.0)) q = 0.0; /* also NaN */
        if (q > (double)(grid - 1)) q = (double)(grid - 1);
        key |= (uint64_t)q << (20 * a);
    }
    return key;
}

static int orc_key_cmp(const void *pa, const void *pb)
{
    const uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return (a > b) - (a < b);
}

int64_t orc_accumulate(const float *frame_cr, int64_t n_frame, const float *hist_cr, const uint8_t *hist_age,
                       int64_t n_hist, const double lo[3], double size, int32_t grid, int32_t max_age, int64_t *kept)
{
    uint64_t *keys = (uint64_t *)malloc((size_t)(n_frame > 0 ? n_frame : 1) * sizeof(uint64_t));
    if (!keys) return -1;
    for (int64_t i = 0; i < n_frame; ++i) keys[i] = orc_cell_key(frame_cr + 4 * i, lo, size, grid);
    qsort(keys, (size_t)n_frame, sizeof(uint64_t), orc_key_cmp);
    int64_t n_kept = 0;
    for (int64_t i = 0; i < n_hist; ++i) {
        if ((int32_t)hist_age[i] + 1 > max_age) continue;
        const uint64_t key = orc_cell_key(hist_cr + 4 * i, lo, size, grid);
        if (n_frame > 0 && bsearch(&key, keys, (size_t)n_frame, sizeof(uint64_t), orc_key_cmp)) continue;
        kept[n_kept++] = i;
    }
    free(keys);
    return n_kept;
}
