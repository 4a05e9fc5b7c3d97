// Host-side launchers implemented by the kernel translation units.
#pragma once

#include "common.h"

namespace splat {

struct TraceArgs {
    const void *bvh_mem;
    uint32_t bvh_capacity;      // spheres that may be referenced: min(BVH, sphere-array capacity)
    uint32_t layout_cap;        // capacity the BVH allocation was laid out for
    const float4 *centre_radius;
    const void *rgba;
    int32_t half;               // colour dtype is half4
    Cam cam;
    float alpha_stop;
    int32_t mode;
    double t_max;
    int32_t kbuf;
    int32_t tile_w, tile_h;
    int32_t schedule;           // tile -> XCD assignment (0 super-tiles, 1 bands)
    int32_t walk;               // SPLAT_WALK_LANE, SPLAT_WALK_PACKET or SPLAT_WALK_FRUSTUM
    const uint32_t *order;      // schedule 2: item of each block, heaviest first (else NULL): tile << 3 | part
    uint32_t order_items;       // schedule 2: items of the order
    float4 *out;                // forward output
    uint32_t *hits;             // nullable
    // backward only
    const float4 *grad;         // dL/d out
    float *d_rgb, *d_alpha, *d_radius, *d_centre;
    const float4 *axis;         // spheroid sets: (u, h) per sample; NULL for spheres
    uint32_t *status;           // the BVH's status word (SPLAT_STATUS_* bits)
};

hipError_t launch_raymarch(const float *vol, int32_t n, double lo, double size, const Cam &cam,
                           const splat_march_opts &o, float *out_rgba, float *out_depth, float *out_interval,
                           hipStream_t s);

hipError_t launch_encode(const splat_spheres &sph, const splat_codec &c, uint64_t *pos, uint32_t *col,
                         hipStream_t s);
hipError_t launch_decode(const uint64_t *pos, const uint32_t *col, const uint32_t *count, const splat_codec &c,
                         const splat_spheres &out, hipStream_t s);

// Exclusive scan of n per-tile counts in place (one workgroup); the total to *total.
hipError_t launch_tile_scan(uint32_t *counts, uint32_t n, uint32_t *total, hipStream_t s);

// Temporal accumulation: frame first, then the history samples that survive.
hipError_t launch_accumulate(const splat_spheres &frame, const splat_spheres *history, const uint8_t *history_age,
                             const splat_accum_opts &o, const splat_spheres &out, uint8_t *out_age, void *ws,
                             hipStream_t s);

hipError_t launch_unproject(const Cam &cam, const float *rgba, const float *depth, const float *interval,
                            const splat_radius_policy &policy, const splat_spheres &out, void *ws, hipStream_t s);

// Wire samples that a build decodes into its sphere set as it reads them.
struct SampleSource {
    const uint64_t *pos;
    const uint32_t *col;
    const uint32_t *count;
    splat_codec codec;
};

hipError_t launch_build(const splat_spheres &sph, const splat_bvh &bvh, bool refit_only, void *ws,
                        hipStream_t s, const SampleSource *samples = nullptr);

hipError_t launch_trace(const TraceArgs &a, bool backward, void *ws, hipStream_t s, hipEvent_t ev_begin,
                        hipEvent_t ev_end);

// Schedule 2: computes the heaviest-first order of trace items into the
// workspace (the heaviest tiles as four quadrant items each).
hipError_t launch_tile_order(const TraceArgs &a, int tiles_x, int tiles_y, void *ws, hipStream_t s,
                             const uint32_t **order_out, uint32_t *items_out);

hipError_t launch_trace_batched(const splat_batch_job *jobs, const uint32_t *tile_offsets, int32_t n_jobs,
                                uint32_t total_tiles, const splat_trace_opts &o, int32_t waves, void *ws,
                                hipStream_t s);

}  // namespace splat
