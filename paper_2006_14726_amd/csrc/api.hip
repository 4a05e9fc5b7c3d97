// C ABI of the splat library: argument checks on the host, then launches.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "common.h"
#include "kernels.h"

using namespace splat;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

// Device check, cached per device id: gfx950 only.
int check_device()
{
    static std::mutex mu;
    static int state[64] = {0};  // 0 unknown, 1 ok, 2 wrong arch
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return fail(SPLAT_ENODEV, "no HIP device available");
    std::lock_guard<std::mutex> lock(mu);
    if (state[dev] == 0) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) return fail(SPLAT_ENODEV, "hipGetDeviceProperties failed");
        state[dev] = std::strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
        if (state[dev] == 2) {
            snprintf(g_err, sizeof g_err, "device %d is %s, this library is built for gfx950", dev, p.gcnArchName);
            return SPLAT_ENODEV;
        }
    }
    return state[dev] == 1 ? SPLAT_OK : fail(SPLAT_ENODEV, "device %d is not gfx950", dev);
}

int check_camera(const splat_camera *c, const char *what)
{
    if (!c) return fail(SPLAT_EINVAL, "%s camera is NULL", what);
    if (c->width <= 0 || c->height <= 0 || (int64_t)c->width * c->height > (1ll << 31))
        return fail(SPLAT_EINVAL, "%s camera size %dx%d out of range", what, c->width, c->height);
    if (!(std::isfinite(c->tan_half_fov_y) && c->tan_half_fov_y > 0))
        return fail(SPLAT_EINVAL, "%s camera tan_half_fov_y must be finite and positive", what);
    const double *v[3] = {c->forward, c->right, c->up};
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(c->eye[k])) return fail(SPLAT_EINVAL, "%s camera eye is not finite", what);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double dot = v[i][0] * v[j][0] + v[i][1] * v[j][1] + v[i][2] * v[j][2];
            if (!(std::fabs(dot - (i == j ? 1.0 : 0.0)) <= 1e-9))
                return fail(SPLAT_EINVAL, "%s camera basis is not orthonormal", what);
        }
    return SPLAT_OK;
}

int check_spheres(const splat_spheres *s, bool need_colour)
{
    if (!s) return fail(SPLAT_EINVAL, "spheres is NULL");
    if (!s->centre_radius || !s->count) return fail(SPLAT_EINVAL, "spheres centre_radius/count is NULL");
    if (need_colour && !s->rgba) return fail(SPLAT_EINVAL, "spheres rgba is NULL");
    if (s->rgba_dtype != SPLAT_F16 && s->rgba_dtype != SPLAT_F32)
        return fail(SPLAT_EUNSUPPORTED, "unknown colour dtype %d", s->rgba_dtype);
    if (s->capacity == 0 || s->capacity > 0x7fffffffu) return fail(SPLAT_EINVAL, "sphere capacity out of range");
    return SPLAT_OK;
}

int check_bvh(const splat_bvh *b)
{
    if (!b || !b->mem) return fail(SPLAT_EINVAL, "bvh or bvh->mem is NULL");
    if (reinterpret_cast<uintptr_t>(b->mem) % 256) return fail(SPLAT_EINVAL, "bvh->mem must be 256-byte aligned");
    if (b->capacity == 0 || b->capacity > 0x7fffffffu) return fail(SPLAT_EINVAL, "bvh capacity out of range");
    return SPLAT_OK;
}

int resolve_opts(const splat_trace_opts *o, splat_trace_opts *out)
{
    if (!o) return fail(SPLAT_EINVAL, "opts is NULL");
    *out = *o;
    if (out->kbuf == 0) out->kbuf = 6;
    if (out->kbuf != 1 && out->kbuf != 2 && out->kbuf != 4 && out->kbuf != 6 && out->kbuf != 8 && out->kbuf != 16)
        return fail(SPLAT_EUNSUPPORTED, "kbuf %d not in {1,2,4,6,8,16}", out->kbuf);
    if (out->tile_w == 0 && out->tile_h == 0) {
        out->tile_w = 8;
        out->tile_h = 8;
    }
    const bool shape_ok = (out->tile_w == 8 && out->tile_h == 8) || (out->tile_w == 16 && out->tile_h == 4) ||
                          (out->tile_w == 32 && out->tile_h == 2) || (out->tile_w == 64 && out->tile_h == 1) ||
                          (out->tile_w == 4 && out->tile_h == 16);
    if (!shape_ok) return fail(SPLAT_EUNSUPPORTED, "tile %dx%d is not a 64-pixel shape", out->tile_w, out->tile_h);
    if (out->mode != SPLAT_ALPHA_CONSTANT && out->mode != SPLAT_ALPHA_SOFT)
        return fail(SPLAT_EUNSUPPORTED, "unknown alpha mode %d", out->mode);
    if (out->schedule != 0 && out->schedule != 1 && out->schedule != 2)
        return fail(SPLAT_EUNSUPPORTED, "unknown schedule %d", out->schedule);
    if (out->walk != SPLAT_WALK_LANE && out->walk != SPLAT_WALK_PACKET && out->walk != SPLAT_WALK_FRUSTUM)
        return fail(SPLAT_EUNSUPPORTED, "unknown walk %d", out->walk);
    if (std::isnan(out->alpha_stop)) return fail(SPLAT_EINVAL, "alpha_stop is NaN");
    if (!(out->t_max > 0)) return fail(SPLAT_EINVAL, "t_max must be positive");
    return SPLAT_OK;
}

int hip_status(hipError_t e, const char *what)
{
    if (e == hipSuccess) return SPLAT_OK;
    return fail(SPLAT_EHIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

extern "C" {

int splat_version(void) { return 107; }

uint32_t *splat_bvh_status_word(const splat_bvh *bvh)
{
    if (!bvh || !bvh->mem) return nullptr;
    return reinterpret_cast<uint32_t *>(static_cast<char *>(bvh->mem) + SPLAT_BVH_STATUS_OFFSET);
}

const char *splat_last_error(void) { return g_err; }

size_t splat_bvh_bytes(uint32_t capacity) { return BvhLayout(capacity).total; }

// Workspace of the schedule-2 tile order: enough for any 64-pixel tile shape.
static size_t trace_ws_bytes(int32_t width, int32_t height)
{
    static const int shapes[5][2] = {{8, 8}, {16, 4}, {32, 2}, {64, 1}, {4, 16}};
    size_t best = 0;
    for (const auto &sh : shapes) {
        const uint64_t t = (uint64_t)((width + sh[0] - 1) / sh[0]) * (uint64_t)((height + sh[1] - 1) / sh[1]);
        const size_t b = TileOrderLayout((uint32_t)(t < 0xffffffffu ? t : 0xffffffffu)).total;
        if (b > best) best = b;
    }
    return best;
}

size_t splat_workspace_bytes(int32_t op, uint32_t capacity, int32_t width, int32_t height)
{
    switch (op) {
    case SPLAT_OP_UNPROJECT:
        return (width > 0 && height > 0) ? unproject_ws_bytes((int64_t)width * height) : 0;
    case SPLAT_OP_BUILD: return BuildLayout(capacity).total;
    case SPLAT_OP_TRACE:
    case SPLAT_OP_BACKWARD: return (width > 0 && height > 0) ? trace_ws_bytes(width, height) : 0;
    case SPLAT_OP_BATCHED: return 256;
    case SPLAT_OP_ACCUMULATE: return (width >= 1 && width <= 1024) ? AccumLayout(width, capacity).total : 0;
    default: return 0;
    }
}

int splat_raymarch(const splat_volume *vol, const splat_camera *cam, const splat_march_opts *opts, float *out_rgba,
                   float *out_depth, float *out_interval, void *stream)
{
    int rc;
    if (!vol || !vol->data) return fail(SPLAT_EINVAL, "volume is NULL");
    if (vol->n < 1 || vol->n > 1024) return fail(SPLAT_EINVAL, "volume n %d not in 1..1024", vol->n);
    if (!std::isfinite(vol->box_lo) || !std::isfinite(vol->box_size) || !(vol->box_size > 0))
        return fail(SPLAT_EINVAL, "volume box must be finite with box_size > 0");
    if ((rc = check_camera(cam, "source"))) return rc;
    if (!out_rgba || !out_depth) return fail(SPLAT_EINVAL, "out_rgba/out_depth is NULL");
    splat_march_opts o = {0.5, 0.05, 0.5, 0.999, 0.25, 0.75};
    if (opts) {
        if (opts->step != 0) o.step = opts->step;
        if (opts->alpha_scale != 0) o.alpha_scale = opts->alpha_scale;
        if (opts->depth_alpha != 0) o.depth_alpha = opts->depth_alpha;
        if (opts->stop_alpha != 0) o.stop_alpha = opts->stop_alpha;
        if (opts->interval_lo != 0) o.interval_lo = opts->interval_lo;
        if (opts->interval_hi != 0) o.interval_hi = opts->interval_hi;
    }
    if (!std::isfinite(o.interval_lo) || !std::isfinite(o.interval_hi) || !(o.interval_lo > 0) ||
        o.interval_hi < o.interval_lo)
        return fail(SPLAT_EINVAL, "march interval alphas must satisfy 0 < interval_lo <= interval_hi");
    // the sample count per ray is at most sqrt(3) n / step
    if (!std::isfinite(o.step) || o.step < 0.01) return fail(SPLAT_EINVAL, "march step must be >= 0.01 voxel");
    if (!std::isfinite(o.alpha_scale) || o.alpha_scale < 0 || !std::isfinite(o.depth_alpha) ||
        !std::isfinite(o.stop_alpha))
        return fail(SPLAT_EINVAL, "march alpha options must be finite, alpha_scale >= 0");
    if ((rc = check_device())) return rc;
    return hip_status(launch_raymarch(vol->data, vol->n, vol->box_lo, vol->box_size, make_cam(*cam), o, out_rgba,
                                      out_depth, out_interval, static_cast<hipStream_t>(stream)),
                      "raymarch launch");
}

static int check_codec(const splat_codec *c)
{
    if (!c) return fail(SPLAT_EINVAL, "codec is NULL");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(c->box_lo[k])) return fail(SPLAT_EINVAL, "codec box_lo is not finite");
    if (!std::isfinite(c->box_size) || !(c->box_size > 0)) return fail(SPLAT_EINVAL, "codec box_size must be > 0");
    if (!std::isfinite(c->r_unit) || !(c->r_unit > 0)) return fail(SPLAT_EINVAL, "codec r_unit must be > 0");
    return SPLAT_OK;
}

int splat_encode_samples(const splat_spheres *sph, const splat_codec *codec, uint64_t *out_pos, uint32_t *out_rgba,
                         void *stream)
{
    int rc;
    if ((rc = check_spheres(sph, true))) return rc;
    if (sph->axis) return fail(SPLAT_EUNSUPPORTED, "the sample codec takes sphere sets (no axis)");
    if ((rc = check_codec(codec))) return rc;
    if (!out_pos || !out_rgba) return fail(SPLAT_EINVAL, "out_pos/out_rgba is NULL");
    if ((rc = check_device())) return rc;
    return hip_status(launch_encode(*sph, *codec, out_pos, out_rgba, static_cast<hipStream_t>(stream)),
                      "encode launch");
}

int splat_decode_samples(const uint64_t *pos, const uint32_t *rgba, const uint32_t *count, const splat_codec *codec,
                         const splat_spheres *out, void *stream)
{
    int rc;
    if (!pos || !rgba || !count) return fail(SPLAT_EINVAL, "pos/rgba/count is NULL");
    if ((rc = check_spheres(out, true))) return rc;
    if (out->axis) return fail(SPLAT_EUNSUPPORTED, "the sample codec takes sphere sets (no axis)");
    if ((rc = check_codec(codec))) return rc;
    if ((rc = check_device())) return rc;
    return hip_status(launch_decode(pos, rgba, count, *codec, *out, static_cast<hipStream_t>(stream)),
                      "decode launch");
}

namespace {
struct Span {
    const void *p;
    size_t bytes;
};
bool overlaps(const Span &a, const Span &b)
{
    if (!a.p || !b.p || !a.bytes || !b.bytes) return false;
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a.p), b0 = reinterpret_cast<uintptr_t>(b.p);
    return a0 < b0 + b.bytes && b0 < a0 + a.bytes;
}
size_t colour_bytes(const splat_spheres &s) { return (size_t)s.capacity * (s.rgba_dtype == SPLAT_F16 ? 8 : 16); }
}  // namespace

int splat_accumulate(const splat_spheres *frame, const splat_spheres *history, const uint8_t *history_age,
                     const splat_accum_opts *opts, const splat_spheres *out, uint8_t *out_age, void *ws,
                     size_t ws_bytes, void *stream)
{
    int rc;
    if ((rc = check_spheres(frame, true))) return rc;
    if ((rc = check_spheres(out, true))) return rc;
    if (history) {
        if ((rc = check_spheres(history, true))) return rc;
        if (!history_age) return fail(SPLAT_EINVAL, "history_age is NULL");
        if (history->rgba_dtype != frame->rgba_dtype)
            return fail(SPLAT_EINVAL, "history and frame colour dtypes differ");
    }
    if (out->rgba_dtype != frame->rgba_dtype) return fail(SPLAT_EINVAL, "out and frame colour dtypes differ");
    if (frame->axis || out->axis || (history && history->axis))
        return fail(SPLAT_EUNSUPPORTED, "the accumulation takes sphere sets (no axis)");
    if (!out_age) return fail(SPLAT_EINVAL, "out_age is NULL");
    if (out->src_index && (!frame->src_index || (history && !history->src_index)))
        return fail(SPLAT_EINVAL, "out->src_index needs src_index on the frame and the history");
    if (!opts) return fail(SPLAT_EINVAL, "accumulation opts is NULL");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(opts->box_lo[k])) return fail(SPLAT_EINVAL, "accumulation box_lo is not finite");
    if (!std::isfinite(opts->box_size) || !(opts->box_size > 0))
        return fail(SPLAT_EINVAL, "accumulation box_size must be > 0");
    if (opts->grid < 1 || opts->grid > 1024) return fail(SPLAT_EINVAL, "accumulation grid %d not in 1..1024", opts->grid);
    if (opts->max_age < 0 || opts->max_age > 255)
        return fail(SPLAT_EINVAL, "accumulation max_age %d not in 0..255", opts->max_age);
    const uint32_t hcap = history ? history->capacity : 0u;
    const Span outs[5] = {{out->centre_radius, (size_t)out->capacity * 16}, {out->rgba, colour_bytes(*out)},
                          {out->src_index, out->src_index ? (size_t)out->capacity * 4 : 0}, {out->count, 4},
                          {out_age, out->capacity}};
    const Span ins[9] = {{frame->centre_radius, (size_t)frame->capacity * 16},
                         {frame->rgba, colour_bytes(*frame)},
                         {frame->src_index, frame->src_index ? (size_t)frame->capacity * 4 : 0},
                         {frame->count, 4},
                         {history ? history->centre_radius : nullptr, (size_t)hcap * 16},
                         {history ? history->rgba : nullptr, history ? colour_bytes(*history) : 0},
                         {history ? history->src_index : nullptr, history && history->src_index ? (size_t)hcap * 4 : 0},
                         {history ? history->count : nullptr, 4},
                         {history ? history_age : nullptr, hcap}};
    for (const Span &o : outs)
        for (const Span &i : ins)
            if (overlaps(o, i)) return fail(SPLAT_EINVAL, "an output array of the accumulation overlaps an input");
    const size_t need = AccumLayout(opts->grid, hcap).total;
    if (!ws || ws_bytes < need) return fail(SPLAT_ENOSPC, "accumulation workspace needs %zu bytes", need);
    if (reinterpret_cast<uintptr_t>(ws) % 16) return fail(SPLAT_EINVAL, "accumulation workspace must be 16-byte aligned");
    if ((rc = check_device())) return rc;
    return hip_status(launch_accumulate(*frame, history, history_age, *opts, *out, out_age, ws,
                                        static_cast<hipStream_t>(stream)),
                      "accumulate launch");
}

int splat_unproject_policy(const splat_camera *src, const float *rgba_premul, const float *depth,
                           const float *interval, const splat_radius_policy *policy, const splat_spheres *out,
                           void *ws, size_t ws_bytes, void *stream)
{
    int rc;
    if ((rc = check_camera(src, "source"))) return rc;
    if (!rgba_premul || !depth) return fail(SPLAT_EINVAL, "rgba_premul/depth is NULL");
    if ((rc = check_spheres(out, true))) return rc;
    if (!policy) return fail(SPLAT_EINVAL, "radius policy is NULL");
    if (policy->mode != SPLAT_RADIUS_FOOTPRINT && policy->mode != SPLAT_RADIUS_OPACITY &&
        policy->mode != SPLAT_RADIUS_INTERVAL && policy->mode != SPLAT_RADIUS_SPHEROID)
        return fail(SPLAT_EUNSUPPORTED, "unknown radius policy %d", policy->mode);
    if (policy->mode == SPLAT_RADIUS_SPHEROID && !out->axis)
        return fail(SPLAT_EINVAL, "the spheroid policy needs out->axis");
    if (!std::isfinite(policy->radius_scale) || policy->radius_scale < 0)
        return fail(SPLAT_EINVAL, "radius_scale must be >= 0");
    if (policy->mode == SPLAT_RADIUS_OPACITY && !(policy->opacity_floor > 0 && policy->opacity_floor <= 1))
        return fail(SPLAT_EINVAL, "opacity_floor must be in (0, 1]");
    if (policy->mode == SPLAT_RADIUS_INTERVAL || policy->mode == SPLAT_RADIUS_SPHEROID) {
        if (!interval) return fail(SPLAT_EINVAL, "the interval policies need the depth interval");
        if (!std::isfinite(policy->interval_scale) || policy->interval_scale < 0)
            return fail(SPLAT_EINVAL, "interval_scale must be >= 0");
    }
    const int64_t pixels = (int64_t)src->width * src->height;
    if ((int64_t)out->capacity < pixels)
        return fail(SPLAT_ENOSPC, "sphere capacity %u < %lld source pixels", out->capacity, (long long)pixels);
    const size_t need = unproject_ws_bytes(pixels);
    if (!ws || ws_bytes < need) return fail(SPLAT_ENOSPC, "unproject workspace needs %zu bytes", need);
    if ((rc = check_device())) return rc;
    return hip_status(launch_unproject(make_cam(*src), rgba_premul, depth, interval, *policy, *out, ws,
                                       static_cast<hipStream_t>(stream)),
                      "unproject launch");
}

int splat_unproject(const splat_camera *src, const float *rgba_premul, const float *depth, float radius_scale,
                    const splat_spheres *out, void *ws, size_t ws_bytes, void *stream)
{
    const splat_radius_policy policy = {SPLAT_RADIUS_FOOTPRINT, radius_scale, 1.0f, 0.0f};
    return splat_unproject_policy(src, rgba_premul, depth, nullptr, &policy, out, ws, ws_bytes, stream);
}

int splat_build_bvh(const splat_spheres *sph, const splat_bvh *bvh, int32_t refit_only, void *ws, size_t ws_bytes,
                    void *stream)
{
    int rc;
    if ((rc = check_spheres(sph, true))) return rc;
    if ((rc = check_bvh(bvh))) return rc;
    if (sph->capacity > bvh->capacity)
        return fail(SPLAT_ENOSPC, "sphere capacity %u exceeds bvh capacity %u", sph->capacity, bvh->capacity);
    if (!refit_only) {
        const size_t need = BuildLayout(sph->capacity).total;
        if (!ws || ws_bytes < need) return fail(SPLAT_ENOSPC, "build workspace needs %zu bytes", need);
    }
    if ((rc = check_device())) return rc;
    return hip_status(launch_build(*sph, *bvh, refit_only != 0, ws, static_cast<hipStream_t>(stream)),
                      "build launch");
}

int splat_build_bvh_from_samples(const uint64_t *pos, const uint32_t *rgba, const uint32_t *count,
                                 const splat_codec *codec, const splat_spheres *out, const splat_bvh *bvh, void *ws,
                                 size_t ws_bytes, void *stream)
{
    int rc;
    if (!pos || !rgba || !count) return fail(SPLAT_EINVAL, "pos/rgba/count is NULL");
    if ((rc = check_spheres(out, true))) return rc;
    if (out->axis) return fail(SPLAT_EUNSUPPORTED, "the sample codec takes sphere sets (no axis)");
    if ((rc = check_codec(codec))) return rc;
    if ((rc = check_bvh(bvh))) return rc;
    if (out->capacity > bvh->capacity)
        return fail(SPLAT_ENOSPC, "sphere capacity %u exceeds bvh capacity %u", out->capacity, bvh->capacity);
    const size_t need = BuildLayout(out->capacity).total;
    if (!ws || ws_bytes < need) return fail(SPLAT_ENOSPC, "build workspace needs %zu bytes", need);
    if ((rc = check_device())) return rc;
    const SampleSource src = {pos, rgba, count, *codec};
    return hip_status(launch_build(*out, *bvh, false, ws, static_cast<hipStream_t>(stream), &src),
                      "build launch");
}

static int trace_common(const splat_bvh *bvh, const splat_spheres *sph, const splat_camera *cam,
                        const splat_trace_opts *opts, TraceArgs &a)
{
    int rc;
    if ((rc = check_bvh(bvh))) return rc;
    if ((rc = check_spheres(sph, true))) return rc;
    if ((rc = check_camera(cam, "target"))) return rc;
    splat_trace_opts o;
    if ((rc = resolve_opts(opts, &o))) return rc;
    if (sph->axis && o.mode != SPLAT_ALPHA_CONSTANT)
        return fail(SPLAT_EUNSUPPORTED, "spheroid sets are traced with constant alpha only");
    std::memset(&a, 0, sizeof a);
    a.bvh_mem = bvh->mem;
    a.status = reinterpret_cast<uint32_t *>(static_cast<char *>(bvh->mem) + SPLAT_BVH_STATUS_OFFSET);
    a.bvh_capacity = bvh->capacity < sph->capacity ? bvh->capacity : sph->capacity;
    a.layout_cap = bvh->capacity;
    a.centre_radius = reinterpret_cast<const float4 *>(sph->centre_radius);
    a.axis = reinterpret_cast<const float4 *>(sph->axis);
    a.rgba = sph->rgba;
    a.half = sph->rgba_dtype == SPLAT_F16;
    a.cam = make_cam(*cam);
    a.alpha_stop = o.alpha_stop;
    a.mode = o.mode;
    a.t_max = o.t_max;
    a.kbuf = o.kbuf;
    a.tile_w = o.tile_w;
    a.tile_h = o.tile_h;
    a.schedule = o.schedule;
    a.walk = o.walk;
    return SPLAT_OK;
}

// Schedule 2 orders the tiles in the workspace, which must then be large enough.
static int check_trace_ws(const TraceArgs &a, void *ws, size_t ws_bytes)
{
    if (a.schedule != 2) return SPLAT_OK;
    const size_t need = trace_ws_bytes(a.cam.w, a.cam.h);
    if (!ws || ws_bytes < need)
        return fail(SPLAT_ENOSPC, "schedule 2 needs a workspace of %zu bytes (got %zu)", need, ws ? ws_bytes : 0);
    return SPLAT_OK;
}

int splat_trace(const splat_bvh *bvh, const splat_spheres *sph, const splat_camera *cam, const splat_trace_opts *opts,
                float *out_rgba, uint32_t *out_hits, void *ws, size_t ws_bytes, void *stream)
{
    TraceArgs a;
    int rc;
    if ((rc = trace_common(bvh, sph, cam, opts, a))) return rc;
    if (!out_rgba) return fail(SPLAT_EINVAL, "out_rgba is NULL");
    if ((rc = check_trace_ws(a, ws, ws_bytes))) return rc;
    a.out = reinterpret_cast<float4 *>(out_rgba);
    a.hits = out_hits;
    if ((rc = check_device())) return rc;
    return hip_status(launch_trace(a, false, ws, static_cast<hipStream_t>(stream),
                                   static_cast<hipEvent_t>(opts->event_begin), static_cast<hipEvent_t>(opts->event_end)),
                      "trace launch");
}

// Scratch of splat_trace_noalloc: the tile-order workspace of the heaviest-first
// schedule, in a device array instead of a caller's buffer.  Every device the
// library runs on holds its own copy until the process ends.  In host code the
// array's name is only a stand-in: the device address comes from
// hipGetSymbolAddress, once per device, and only that address reaches a kernel.
constexpr size_t kNoAllocScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static int scratch_address(void **out)
{
    static std::mutex mu;
    static void *addr[64] = {nullptr};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(SPLAT_ENODEV, "no HIP device available");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(SPLAT_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        addr[dev] = p;
    }
    *out = addr[dev];
    return SPLAT_OK;
}

size_t splat_trace_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

int splat_trace_noalloc(const splat_bvh *bvh, const splat_spheres *sph, const splat_camera *cam,
                        const splat_trace_opts *opts, float *out_rgba, uint32_t *out_hits, void *stream)
{
    TraceArgs a;
    int rc;
    if ((rc = trace_common(bvh, sph, cam, opts, a))) return rc;
    if (!out_rgba) return fail(SPLAT_EINVAL, "out_rgba is NULL");
    if (a.schedule == 2) {
        const size_t need = trace_ws_bytes(a.cam.w, a.cam.h);
        if (need > kNoAllocScratchBytes)
            return fail(SPLAT_ENOSPC, "a %dx%d image needs %zu bytes of tile-order scratch; splat_trace_noalloc holds %zu",
                        a.cam.w, a.cam.h, need, kNoAllocScratchBytes);
    }
    a.out = reinterpret_cast<float4 *>(out_rgba);
    a.hits = out_hits;
    if ((rc = check_device())) return rc;
    void *ws = nullptr;
    if ((rc = scratch_address(&ws))) return rc;
    return hip_status(launch_trace(a, false, ws, static_cast<hipStream_t>(stream),
                                   static_cast<hipEvent_t>(opts->event_begin), static_cast<hipEvent_t>(opts->event_end)),
                      "trace launch");
}

int splat_trace_backward(const splat_bvh *bvh, const splat_spheres *sph, const splat_camera *cam,
                         const splat_trace_opts *opts, const float *out_rgba, const float *grad_rgba,
                         const splat_grads *grads, void *ws, size_t ws_bytes, void *stream)
{
    TraceArgs a;
    int rc;
    if ((rc = trace_common(bvh, sph, cam, opts, a))) return rc;
    if (!out_rgba || !grad_rgba) return fail(SPLAT_EINVAL, "out_rgba/grad_rgba is NULL");
    if ((rc = check_trace_ws(a, ws, ws_bytes))) return rc;
    if (sph->axis) return fail(SPLAT_EUNSUPPORTED, "the backward takes sphere sets (no axis)");
    if (!grads || !grads->d_rgb || !grads->d_alpha) return fail(SPLAT_EINVAL, "grads d_rgb/d_alpha is NULL");
    if (a.mode == SPLAT_ALPHA_SOFT && (!grads->d_radius || !grads->d_centre))
        return fail(SPLAT_EINVAL, "soft mode needs d_radius and d_centre");
    a.grad = reinterpret_cast<const float4 *>(grad_rgba);
    a.d_rgb = grads->d_rgb;
    a.d_alpha = grads->d_alpha;
    a.d_radius = grads->d_radius;
    a.d_centre = grads->d_centre;
    if ((rc = check_device())) return rc;
    return hip_status(launch_trace(a, true, ws, static_cast<hipStream_t>(stream),
                                   static_cast<hipEvent_t>(opts->event_begin), static_cast<hipEvent_t>(opts->event_end)),
                      "backward launch");
}

int splat_trace_batched(const splat_batch_job *jobs, const uint32_t *tile_offsets, int32_t n_jobs,
                        uint32_t total_tiles, const splat_trace_opts *opts, int32_t max_waves, void *ws,
                        size_t ws_bytes, void *stream)
{
    int rc;
    if (!jobs || !tile_offsets) return fail(SPLAT_EINVAL, "jobs/tile_offsets is NULL");
    if (n_jobs <= 0) return fail(SPLAT_EINVAL, "n_jobs must be positive");
    splat_trace_opts o;
    if ((rc = resolve_opts(opts, &o))) return rc;
    if (!ws || ws_bytes < 256) return fail(SPLAT_ENOSPC, "batched workspace needs 256 bytes");
    if (max_waves < 0 && max_waves != SPLAT_BATCH_GRID)
        return fail(SPLAT_EINVAL, "max_waves must be >= 0 or SPLAT_BATCH_GRID");
    if (max_waves == SPLAT_BATCH_GRID && total_tiles > 0x7fffffffu)
        return fail(SPLAT_EINVAL, "a grid launch holds at most 2^31 - 1 tiles");
    if ((rc = check_device())) return rc;
    int waves = max_waves;
    if (waves == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return fail(SPLAT_EHIP, "cannot query compute units");
        waves = cus * 16;
    }
    return hip_status(launch_trace_batched(jobs, tile_offsets, n_jobs, total_tiles, o, waves, ws,
                                           static_cast<hipStream_t>(stream)),
                      "batched launch");
}

}  // extern "C"
