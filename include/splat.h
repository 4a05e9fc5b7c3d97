/*
 * splat.h -- C ABI of the MI355X (gfx950) splat ray tracer.
 *
 * The client side of image-warping remote volume rendering with ray tracing
 * (Zellmann, arXiv 2006.14726, Sec. 4.1 and Fig. 2): the samples of a 2.5D
 * RGBA + depth image become coloured semi-transparent spheres, a linear BVH
 * is built over them, and the view from a new camera is ray traced through
 * them with front-to-back compositing.
 *
 * Conventions shared by every entry point
 *   - Every pointer named "device" is device memory on the current HIP
 *     device; the caller allocates and owns it.  The library allocates
 *     nothing and keeps no per-call state.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *     enqueues work on it; none synchronises.  The sphere count stays in
 *     device memory, so the calls can be captured in a HIP graph.
 *   - Return value 0 on success, else one of the SPLAT_E* codes; all argument
 *     checks happen on the host before anything is enqueued, and
 *     splat_last_error() gives a thread-local message for the last failure.
 */
#ifndef SPLAT_H
#define SPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPLAT_OK 0
#define SPLAT_EINVAL 1        /* null pointer, bad size, non-orthonormal camera, bad option */
#define SPLAT_ENOSPC 2        /* capacity or workspace too small */
#define SPLAT_ENODEV 3        /* no gfx950 device, or HIP initialisation failed */
#define SPLAT_EHIP 4          /* a HIP launch or runtime call failed */
#define SPLAT_EUNSUPPORTED 5  /* unknown dtype, mode or tile shape */

#define SPLAT_F32 0           /* sphere colour stored as float4 */
#define SPLAT_F16 1           /* sphere colour stored as IEEE half4 */

#define SPLAT_ALPHA_CONSTANT 0 /* alpha = a: the paper's constant sample colour */
#define SPLAT_ALPHA_SOFT 1     /* alpha = a (1 - q/r^2)^2, q = squared ray-centre distance */

#define SPLAT_WALK_LANE 0      /* every lane walks the BVH on its own path */
#define SPLAT_WALK_PACKET 1    /* the 64 lanes of a wavefront walk it together */
#define SPLAT_WALK_FRUSTUM 2   /* a wavefront gathers its tile's candidate spheres once, breadth first
                                  through the tile's frustum; each lane tests them against its ray */

#define SPLAT_OP_UNPROJECT 0
#define SPLAT_OP_BUILD 1
#define SPLAT_OP_TRACE 2
#define SPLAT_OP_BACKWARD 3
#define SPLAT_OP_BATCHED 4
#define SPLAT_OP_ACCUMULATE 5

/*
 * Pinhole camera, all in double.  forward/right/up must be orthonormal
 * (checked to 1e-9).  Pixel (x, y), row 0 at the top, looks along
 * normalize(forward + sx right + sy up) with
 *   sx = ((2x+1)/width - 1) tan_half_fov_y width/height,
 *   sy = (1 - (2y+1)/height) tan_half_fov_y.
 * The paper ships the camera with the buffers (Sec. 4.2).
 */
typedef struct splat_camera {
    double eye[3];
    double forward[3];
    double right[3];
    double up[3];
    double tan_half_fov_y;
    int32_t width;
    int32_t height;
} splat_camera;

/*
 * Sphere set (Sec. 4.1: samples reinterpreted as semi-transparent spheres),
 * structure of arrays, `capacity` slots, the first *count used.
 *   centre_radius  device float4[capacity]: x, y, z, r (object space)
 *   rgba           device half4 or float4 [capacity]: straight colour k, alpha a
 *   rgba_dtype     SPLAT_F16 or SPLAT_F32
 *   src_index      device uint32[capacity]: source pixel of each sphere (may be NULL)
 *   count          device uint32 scalar: N
 *   axis           device float4[capacity] or NULL.  With it the samples are
 *                  prolate spheroids smeared along their source ray (Sec. 7):
 *                  axis (ux, uy, uz) and half-length h >= r along it, radius r
 *                  across it, i.e. the points x with
 *                  |x - c|^2 / r^2 + ((x - c).u)^2 (1/h^2 - 1/r^2) <= 1
 *                  (u as stored, scaled to unit length in double).  Spheroid sets are traced
 *                  with constant alpha only; the backward, the sample codec,
 *                  the accumulation and the batched trace take sphere sets.
 * Sphere ids are slot indices; they break ties between equal hit distances.
 */
typedef struct splat_spheres {
    float *centre_radius;
    void *rgba;
    int32_t rgba_dtype;
    int32_t reserved;
    uint32_t *src_index;
    uint32_t *count;
    uint32_t capacity;
    float *axis;
} splat_spheres;

/*
 * Linear BVH (Sec. 4.1, the LBVH of the paper) over at most `capacity`
 * spheres, in one device allocation of splat_bvh_bytes(capacity) bytes,
 * 256-byte aligned.  Opaque layout; valid after splat_build_bvh.
 */
typedef struct splat_bvh {
    void *mem;
    uint32_t capacity;
} splat_bvh;

/*
 * Device status word of a BVH: a uint32 at byte SPLAT_BVH_STATUS_OFFSET of
 * bvh->mem.  splat_build_bvh (also a refit) clears it; the build and every
 * trace through the BVH OR into it states that no build produces, so a
 * non-zero word after a run means a corrupt or mismatched hierarchy (the
 * kernels still end: their walks are bounded and their indices clamped).
 *   SPLAT_STATUS_CORRUPT  a trace was handed a sphere set smaller than the
 *                         one the BVH was built over (its references beyond
 *                         the set are skipped), a tile's breadth-first walk
 *                         went deeper than any built hierarchy, or the refit
 *                         met a node range or arrival count that a build
 *                         never writes
 *   SPLAT_STATUS_STACK    reserved: a traversal stack that dropped nodes
 *                         (no walk sets it: their stacks cannot overflow on
 *                         a built hierarchy, and the per-lane walk's
 *                         overflow is caught up by the packet walk)
 * Read it after the stream's work, e.g. with hipMemcpy from
 * splat_bvh_status_word(bvh).  splat_trace_batched, whose jobs hold their
 * hierarchies read-only, leaves it alone.
 */
#define SPLAT_BVH_STATUS_OFFSET 56
#define SPLAT_STATUS_CORRUPT 1u
#define SPLAT_STATUS_STACK 2u

/* Device address of the BVH's status word (host arithmetic only, no GPU
 * call); NULL for a NULL bvh or mem. */
uint32_t *splat_bvh_status_word(const splat_bvh *bvh);

/*
 * Trace options.
 *   alpha_stop  stop a ray once its accumulated alpha reaches this value
 *               (0.99 by default; 0 = the paper's first-hit query; > 1 never)
 *   t_max       hits must satisfy 0 < t0 < t_max (INFINITY for none)
 *   mode        SPLAT_ALPHA_CONSTANT or SPLAT_ALPHA_SOFT
 *   kbuf        hits gathered per traversal pass: 1, 2, 4, 6, 8 or 16 (0 = 6);
 *               the result does not depend on it
 *   tile_w/h    pixels per 64-lane wavefront: 8x8, 16x4, 32x2, 64x1 or 4x16
 *               (0x0 = 8x8); the result does not depend on it
 *   schedule    order of the tiles: 0 super-tiles of 8x8 tiles dealt round
 *               robin to the XCDs, 1 one contiguous band per XCD, 2 heaviest
 *               first (tiles ranked by the sphere centres that project near
 *               them; needs the trace workspace; images of at most 8192
 *               tiles, whose waves all fit on the GPU at once, run as 0);
 *               the result does not depend on it.  The batched launch
 *               ignores it (it has its own work queue)
 *   walk        SPLAT_WALK_LANE (each ray on its own path; the zero value),
 *               SPLAT_WALK_PACKET (a wavefront's rays as one packet) or
 *               SPLAT_WALK_FRUSTUM (the tile's candidates gathered once
 *               through its frustum, then screened per ray; a tile with more
 *               than 256 candidates, or a level of more than 128 nodes, takes
 *               the per-lane walk; the fastest on the client and large
 *               frames); the result does not depend on it
 *   event_begin, event_end
 *               hipEvent_t or NULL: recorded on the stream immediately
 *               before and after the trace kernel itself (after the tile
 *               ordering of schedule 2), to time that kernel alone.  Only
 *               splat_trace, splat_trace_noalloc and splat_trace_backward
 *               record them
 */
typedef struct splat_trace_opts {
    float alpha_stop;
    int32_t mode;
    double t_max;
    int32_t kbuf;
    int32_t tile_w;
    int32_t tile_h;
    int32_t schedule;
    int32_t walk;
    int32_t reserved;              /* 0 */
    void *event_begin;
    void *event_end;
} splat_trace_opts;

/* Per-sphere gradients, device float arrays indexed by sphere id; accumulated into (+=). */
typedef struct splat_grads {
    float *d_rgb;     /* [capacity][3] */
    float *d_alpha;   /* [capacity] */
    float *d_radius;  /* [capacity] */
    float *d_centre;  /* [capacity][3] */
} splat_grads;

/*
 * One job of a batched trace: one target view of one frame's sphere set.
 * All pointers are device pointers, as for splat_trace.
 */
typedef struct splat_batch_job {
    const void *bvh_mem;           /* splat_bvh.mem of the frame */
    const float *centre_radius;    /* spheres of the frame */
    const void *rgba;
    int32_t rgba_dtype;
    uint32_t bvh_capacity;         /* splat_bvh.capacity of the frame */
    splat_camera camera;           /* target view */
    float *out_rgba;               /* float4 [height][width] */
    uint32_t *out_hits;            /* uint32 [height][width] or NULL */
} splat_batch_job;

/* Bytes of workspace that `op` (SPLAT_OP_*) needs for the given capacity and image size
 * (SPLAT_OP_ACCUMULATE: capacity = the history's, width = the grid, height unused). */
size_t splat_workspace_bytes(int32_t op, uint32_t capacity, int32_t width, int32_t height);

/* Bytes of the BVH allocation for `capacity` spheres. */
size_t splat_bvh_bytes(uint32_t capacity);

/*
 * Volume for the server stage: n^3 floats v[z][y][x] (x fastest) filling the
 * cube [box_lo, box_lo + box_size]^3, voxel (i, j, k) centred at
 * box_lo + (i + 1/2, j + 1/2, k + 1/2) box_size / n.
 */
typedef struct splat_volume {
    const float *data;             /* device, n^3 floats */
    int32_t n;                     /* 1..1024 */
    double box_lo, box_size;       /* box_size > 0 */
} splat_volume;

/*
 * Server ray-marcher options (0 fields take the defaults in brackets).
 *   step         voxels between samples, >= 0.01 [0.5]
 *   alpha_scale  sample alpha = clamp(alpha_scale v, 0, 1) [0.05]
 *   depth_alpha  the depth is the first sample at which A >= depth_alpha [0.5]
 *   stop_alpha   marching stops after the sample at which A >= stop_alpha [0.999]
 *   interval_lo, interval_hi  the depth interval runs from the first sample
 *                at which A >= interval_lo [0.25] to the first at which
 *                A >= interval_hi [0.75], or to the last sample taken if A
 *                never gets there; 0 < interval_lo <= interval_hi
 */
typedef struct splat_march_opts {
    double step, alpha_scale, depth_alpha, stop_alpha;
    double interval_lo, interval_hi;
} splat_march_opts;

/*
 * Server stage before the client path (Sec. 4.1: the server ray-marches the
 * volume and writes colour and one representative depth per pixel).  For
 * every pixel of `cam`: samples at t_j = t_in + (j + 1/2) dt along the pixel
 * ray inside the cube (t_in >= 0, dt = step box_size / n), trilinear with
 * clamp to edge; u = clamp(v, 0, 1), colour (u, 4u(1 - u), 1 - u), sample
 * alpha s = clamp(alpha_scale v, 0, 1); front to back, w = (1 - A) s,
 * C += w colour, A += w.  Positions and compositing in double.
 *   out_rgba   device float [height][width][4]: premultiplied (C, A), the
 *              input of splat_unproject
 *   out_depth  device float [height][width]: the depth t, +inf if A never
 *              reaches depth_alpha (no sample there)
 *   out_interval  device float [height][width][2]: the depth interval
 *              (t_lo, t_hi), both +inf if A never reaches interval_lo; or
 *              NULL.  Sec. 7 suggests smearing samples whose depth is
 *              uncertain over an interval along the ray; this is that
 *              interval (splat_unproject_policy, SPLAT_RADIUS_INTERVAL)
 */
int splat_raymarch(const splat_volume *vol, const splat_camera *cam, const splat_march_opts *opts, float *out_rgba,
                   float *out_depth, float *out_interval, void *stream);

/*
 * Sample codec of the wire format (Sec. 4.1: the quantised coordinate is
 * packed with the radius into 64 bits; Sec. 6: 32 bits per colour).  The bit
 * split is this library's reading:
 *   position word = qx | qy << 18 | qz << 36 | c << 54, with
 *     q = clamp(floor((x - box_lo) / box_size 2^18), 0, 2^18 - 1) per axis,
 *     decoded at the cell centre (error <= box_size / 2^19 per axis), and
 *     c = clamp(floor(64 log2(r / r_unit) + 1/2) + 512, 0, 1023), decoded as
 *     r_unit 2^((c - 512) / 64) (relative error <= 2^(1/128) - 1);
 *   colour word = RGBA8 of the straight colour and alpha, byte 0 red,
 *     b = floor(clamp(v, 0, 1) 255 + 1/2), decoded as b / 255.
 */
typedef struct splat_codec {
    double box_lo[3];              /* quantisation box: [box_lo, box_lo + box_size] per axis */
    double box_size;               /* > 0 */
    double r_unit;                 /* radius of code 512, > 0 */
} splat_codec;

/* Encode the first *sph->count spheres (device count) into out_pos (device
 * uint64 [sph->capacity]) and out_rgba (device uint32 [sph->capacity]). */
int splat_encode_samples(const splat_spheres *sph, const splat_codec *codec, uint64_t *out_pos, uint32_t *out_rgba,
                         void *stream);

/* Decode min(*count, out->capacity) samples (count: device uint32) into the
 * sphere set `out` (its count is written on the device). */
int splat_decode_samples(const uint64_t *pos, const uint32_t *rgba, const uint32_t *count, const splat_codec *codec,
                         const splat_spheres *out, void *stream);

/*
 * Temporal accumulation options (Sec. 7 names keeping samples across a few
 * frames as an extension; the merge policy below is this library's reading).
 *   box_lo, box_size  the grid covers [box_lo, box_lo + box_size] per axis
 *   grid              cells per axis, 1..1024; a centre x lies in cell
 *                     q = clamp(floor((x - box_lo) / box_size grid), 0, grid - 1)
 *                     per axis, in double (centres outside the box fall into
 *                     the border cells)
 *   max_age           0..255: a history sample survives only while its age
 *                     after the merge is at most max_age
 */
typedef struct splat_accum_opts {
    double box_lo[3];
    double box_size;
    int32_t grid;
    int32_t max_age;
} splat_accum_opts;

/*
 * Temporal accumulation (Sec. 7).  The merged set `out` is the first
 * *frame->count samples of the new frame, in order, with age 0, followed by
 * the history samples, in order, that survive: a history sample survives iff
 * its age + 1 <= max_age and no centre of the new frame lies in its cell; it
 * carries age + 1.  *out->count = min(merged, out->capacity): the excess is
 * cut from the end, where the oldest samples are.  Centre, radius, colour and
 * src_index are copied bit for bit.  Build (not refit) the BVH of the merged
 * set before tracing it.
 *   history      NULL for none; otherwise its colour dtype equals the frame's
 *   history_age  device uint8 [history->capacity] (ignored without history)
 *   out          colour dtype equal to the frame's; out->src_index NULL, or
 *                set together with the frame's and the history's; no array of
 *                out (nor out_age) may overlap an input array (SPLAT_EINVAL)
 *   out_age      device uint8 [out->capacity]
 *   ws           device, >= splat_workspace_bytes(SPLAT_OP_ACCUMULATE,
 *                history capacity (0 without history), grid, 0): the cell
 *                map (one byte per cell: 16 MiB at grid 256, 1 GiB at 1024,
 *                cleared by every call) and per-tile survivor counts;
 *                16-byte aligned.  Calls that overlap on one workspace race.
 */
int splat_accumulate(const splat_spheres *frame, const splat_spheres *history, const uint8_t *history_age,
                     const splat_accum_opts *opts, const splat_spheres *out, uint8_t *out_age, void *ws,
                     size_t ws_bytes, void *stream);

/*
 * Unprojection (Sec. 4.1, Eq. 1).  For every source pixel whose depth t is
 * finite and positive and whose alpha A is positive: centre p = o + d t in
 * double (d the unit pixel-centre ray of `src`), radius
 * r = radius_scale * 2 t tan_half_fov_y / height (the pixel footprint at t),
 * colour k = clamp(C/A, 0, 1), a = A; each rounded once to float (half for
 * SPLAT_F16 colours).  Pixels without a sample are compacted away; the
 * spheres keep row-major pixel order (src_index ascending).
 *   rgba_premul  device float [height][width][4], premultiplied
 *   depth        device float [height][width], ray parameter along the unit ray
 *   out          out->capacity >= width*height (SPLAT_ENOSPC otherwise)
 *   ws           device, >= splat_workspace_bytes(SPLAT_OP_UNPROJECT, 0, width, height)
 */
int splat_unproject(const splat_camera *src, const float *rgba_premul, const float *depth, float radius_scale,
                    const splat_spheres *out, void *ws, size_t ws_bytes, void *stream);

/*
 * Radius policies of the unprojection (Sec. 7 suggests varying the radius
 * with the sample's opacity, or smearing a sample whose depth is uncertain
 * over an interval along the ray; the rules are this library's readings).
 * fp(t) = 2 t tan_half_fov_y / height is the source pixel's footprint at t.
 *   SPLAT_RADIUS_FOOTPRINT  r = radius_scale fp(t) (splat_unproject)
 *   SPLAT_RADIUS_OPACITY    r = radius_scale fp(t) sqrt(max(A, opacity_floor)):
 *                           the disc area in proportion to the opacity
 *   SPLAT_RADIUS_INTERVAL   with the depth interval (t_lo, t_hi) of the pixel:
 *                           the centre at t_c = (t_lo + t_hi) / 2 on the ray,
 *                           r = max(radius_scale fp(t_c), interval_scale (t_hi - t_lo) / 2);
 *                           a pixel then also needs 0 < t_lo <= t_hi, both finite
 *   SPLAT_RADIUS_SPHEROID   the same pixels and centres as the interval policy,
 *                           smeared along the ray instead of grown in every
 *                           direction: r = radius_scale fp(t_c) across the ray,
 *                           axis u = the unit pixel ray d and half-length
 *                           h = max(r, interval_scale (t_hi - t_lo) / 2) along it,
 *                           written to out->axis (required) as (u, h)
 * All in double, each output rounded once to float.
 */
#define SPLAT_RADIUS_FOOTPRINT 0
#define SPLAT_RADIUS_OPACITY 1
#define SPLAT_RADIUS_INTERVAL 2
#define SPLAT_RADIUS_SPHEROID 3

typedef struct splat_radius_policy {
    int32_t mode;           /* SPLAT_RADIUS_* */
    float radius_scale;     /* >= 0 */
    float opacity_floor;    /* (0, 1], SPLAT_RADIUS_OPACITY */
    float interval_scale;   /* >= 0, SPLAT_RADIUS_INTERVAL */
} splat_radius_policy;

/*
 * Unprojection with a radius policy: as splat_unproject (validity, colour,
 * compaction, order), with the centre and radius of the policy.
 *   interval  device float [height][width][2] (t_lo, t_hi), as written by
 *             splat_raymarch; needed by SPLAT_RADIUS_INTERVAL, else ignored
 */
int splat_unproject_policy(const splat_camera *src, const float *rgba_premul, const float *depth,
                           const float *interval, const splat_radius_policy *policy, const splat_spheres *out,
                           void *ws, size_t ws_bytes, void *stream);

/*
 * LBVH build (Sec. 4.1): scene bounds, 30-bit Morton codes of the centres,
 * stable LDS radix sort of (code, id), Karras radix-tree hierarchy, and a
 * bottom-up refit of boxes rounded outward to float.  refit_only != 0 keeps
 * the hierarchy of the previous build over the same centres and recomputes
 * the boxes and the per-leaf data (radius or colour changes).  The BVH keeps
 * its own copy of each sphere's centre, radius and alpha a, as read by the
 * last build or refit: after any change to those arrays, refit (or build)
 * before tracing.
 *   ws  device, >= splat_workspace_bytes(SPLAT_OP_BUILD, bvh->capacity, 0, 0)
 *   sph->capacity <= bvh->capacity (SPLAT_ENOSPC otherwise)
 */
/*
 * The build over received wire samples (Sec. 4.1: the client builds its LBVH
 * over the samples the server sent): decodes min(*count, out->capacity)
 * samples into the sphere set `out` inside the build's first kernel, which
 * reads the centres for the scene bounds anyway, then builds as
 * splat_build_bvh.  The path thus reads the 12-byte samples once instead of
 * a decode pass writing 24-byte spheres that the build then reads again.
 * Equal, bit for bit (spheres, count and BVH), to splat_decode_samples
 * followed by splat_build_bvh.
 *   pos, rgba, count, codec  as for splat_decode_samples
 *   out   a sphere set without axis; out->capacity <= bvh->capacity
 *   ws    device, >= splat_workspace_bytes(SPLAT_OP_BUILD, out->capacity, 0, 0)
 */
int splat_build_bvh_from_samples(const uint64_t *pos, const uint32_t *rgba, const uint32_t *count,
                                 const splat_codec *codec, const splat_spheres *out, const splat_bvh *bvh, void *ws,
                                 size_t ws_bytes, void *stream);

int splat_build_bvh(const splat_spheres *sph, const splat_bvh *bvh, int32_t refit_only, void *ws, size_t ws_bytes,
                    void *stream);

/*
 * Trace and composite (Sec. 4.1, Fig. 2).  For every pixel of `cam`: all
 * spheres hit by its ray (disc >= 0, 0 < t0 < t_max) in ascending
 * (t0, sphere id), composited front to back, C += T alpha k, A += T alpha,
 * T *= 1 - alpha, stopping after the hit at which A >= alpha_stop.  Ray,
 * sphere test and ordering are double precision; compositing is float.
 * Centres, radii and alphas come from the BVH's copy (see splat_build_bvh),
 * colours from sph->rgba.
 *   out_rgba  device float4 [height][width] (C, A), background 0
 *   out_hits  device uint32 [height][width] composited hit count, or NULL
 *   ws        device, >= splat_workspace_bytes(SPLAT_OP_TRACE, 0, width, height)
 *             with schedule 2 (SPLAT_ENOSPC otherwise); unused, and may be
 *             NULL, with schedules 0 and 1.  Calls that overlap on one
 *             workspace race.
 */
int splat_trace(const splat_bvh *bvh, const splat_spheres *sph, const splat_camera *cam, const splat_trace_opts *opts,
                float *out_rgba, uint32_t *out_hits, void *ws, size_t ws_bytes, void *stream);

/*
 * splat_trace without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, checks and result as splat_trace
 * (bit for bit); the tile-order workspace of schedule 2 is a static device
 * array of splat_trace_noalloc_max_bytes() bytes (4 MiB) that every device the
 * library runs on holds until the process ends.  No call allocates.
 *   SPLAT_ENOSPC  schedule 2 on an image whose tile order needs more than that
 *                 (splat_workspace_bytes(SPLAT_OP_TRACE, ...) > 4 MiB, about
 *                 22 M pixels); schedules 0 and 1 need no scratch
 * All calls on one device share its array: calls that overlap on one device
 * (two streams, two threads) race.  Every call clears what it reads first.
 */
int splat_trace_noalloc(const splat_bvh *bvh, const splat_spheres *sph, const splat_camera *cam,
                        const splat_trace_opts *opts, float *out_rgba, uint32_t *out_hits, void *stream);

/* Bytes of the static scratch of splat_trace_noalloc. */
size_t splat_trace_noalloc_max_bytes(void);

/*
 * Backward of splat_trace: given dL/d(out_rgba), accumulates dL/dk, dL/da,
 * dL/dr and dL/dc of every sphere into `grads` (+=; zero them first).  The
 * ordered hits are recomputed by a second traversal, not stored.  Radius
 * and centre gradients are zero in SPLAT_ALPHA_CONSTANT mode.
 *   out_rgba   device float4 [height][width]: the forward output of the same
 *              call (checked for NULL; the hits are recomputed, not read from it)
 *   grad_rgba  device float4 [height][width]
 *   ws         as for splat_trace (SPLAT_OP_BACKWARD gives the same size)
 */
int splat_trace_backward(const splat_bvh *bvh, const splat_spheres *sph, const splat_camera *cam,
                         const splat_trace_opts *opts, const float *out_rgba, const float *grad_rgba,
                         const splat_grads *grads, void *ws, size_t ws_bytes, void *stream);

/*
 * Batched trace: every job of `jobs` (device array of n_jobs splat_batch_job)
 * in ONE launch: either persistent waves that take tiles from an atomic work
 * counter, or (max_waves = SPLAT_BATCH_GRID) one workgroup per (job, tile),
 * the job found by a binary search of the tile offsets.  Each job's output
 * equals splat_trace's bit for bit.
 *   ws          device, >= splat_workspace_bytes(SPLAT_OP_BATCHED, n_jobs, 0, 0)
 *   total_tiles sum over jobs of ceil(w / tile_w) * ceil(h / tile_h)
 *   max_waves   resident waves to launch (0 = one per SIMD slot of the
 *               device), or SPLAT_BATCH_GRID
 * The host passes per-job tile offsets through `tile_offsets` (device
 * uint32[n_jobs + 1], exclusive prefix of tiles per job).
 */
#define SPLAT_BATCH_GRID (-1)
int splat_trace_batched(const splat_batch_job *jobs, const uint32_t *tile_offsets, int32_t n_jobs,
                        uint32_t total_tiles, const splat_trace_opts *opts, int32_t max_waves, void *ws,
                        size_t ws_bytes, void *stream);

/* Thread-local text for the last non-zero status. */
const char *splat_last_error(void);

/* ABI version (major * 100 + minor): 106 added splat_spheres.axis, 107 the
 * BVH status word. */
int splat_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPLAT_H */
