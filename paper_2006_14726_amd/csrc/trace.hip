// Ray tracing of the sphere set with exact front-to-back compositing
// (Sec. 3.1 and Fig. 2: the client renders the samples as coloured
// semi-transparent spheres from the current camera).
//
// One 64-lane wavefront traces one tile of pixels as a packet: the BVH walk
// is wave-uniform (node fetched once per wave with scalar loads, stack of
// node indices in LDS, a child is visited if any lane's ray meets its box),
// while each lane keeps its own ordered hit buffer.  Per traversal pass a
// lane gathers the K hits with the smallest keys (t0, sphere id) greater than
// the last key it composited; nodes beyond the K-th key, or beyond the hit
// at which the alpha stop is already certain, are pruned.  If a pass fills
// the buffer without reaching the stop, the lane composites it and runs
// another pass from its last key, so there is no cap on hits and the result
// does not depend on K, the tile shape or the other lanes of the wave.
//
// Precision: ray and sphere test in double (exact enough to settle hits at
// relative discriminants far below 1e-6), keys in double, boxes in float
// with a conservative margin, compositing in float with explicitly rounded
// operations so that every pass performs the same arithmetic.
#include "common.h"
#include "kernels.h"

namespace splat {

// ---------------------------------------------------------------- helpers

__device__ inline uint32_t ufirst(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline float ffirst(float v) { return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v))); }

struct Key {
    double t;
    uint32_t id;
};
__device__ inline bool key_less(double ta, uint32_t ia, double tb, uint32_t ib)
{
    return ta < tb || (ta == tb && ia < ib);
}

// One compositing step; the alpha part is shared by pruning and compositing.
__device__ inline void alpha_step(float alpha, float &A, float &T, float &w)
{
    w = __fmul_rn(T, alpha);
    A = __fadd_rn(A, w);
    T = __fmul_rn(T, __fsub_rn(1.0f, alpha));
}

__device__ inline float4 load_colour(const void *rgba, int half, uint32_t id)
{
    if (half) {
        const ushort4 h = reinterpret_cast<const ushort4 *>(rgba)[id];
        return make_float4(half_to_float(h.x), half_to_float(h.y), half_to_float(h.z), half_to_float(h.w));
    }
    return reinterpret_cast<const float4 *>(rgba)[id];
}

// Per-lane ray state.
struct Ray {
    double d[3];     // unit direction, double
    float df[3];     // float copy of d
    float inv[3];    // 1 / df
};

// Wave-uniform ray state.
struct Eye {
    double o[3];
    float of[3];
    float oP[3], oM[3];  // float eye moved by +margin / -margin (padded-box slab test)
    float E;             // bound on float sphere-distance error
};

// ---------------------------------------------------------------- one tile

template <int K, bool BWD>
__device__ void trace_tile(const TraceArgs &a, const Node *__restrict__ nodes, const BvhHeader *__restrict__ hdr,
                           int tile_x, int tile_y, uint32_t *stack)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int px = tile_x * a.tile_w + (lane % a.tile_w);
    const int py = tile_y * a.tile_h + (lane / a.tile_w);
    const bool inside = px >= 0 && py >= 0 && px < a.cam.w && py < a.cam.h;
    // the header count is clamped to the allocation, so even a BVH that was
    // never built cannot send the walk outside it
    const uint32_t n_spheres = min(ufirst(hdr->n), a.bvh_capacity);
    const uint32_t n_nodes = n_spheres > 1 ? n_spheres - 1 : 1;
    const int half = a.half;
    const float stop = a.alpha_stop;
    const int soft = a.mode == SPLAT_ALPHA_SOFT;

    // ---- rays
    Ray ray;
    {
        double d[3];
        pixel_ray(a.cam, inside ? px : 0, inside ? py : 0, d);
        for (int k = 0; k < 3; ++k) {
            ray.d[k] = d[k];
            float f = (float)d[k];
            if (f == 0.0f) f = copysignf(1e-30f, (float)d[k] + 0.0f);
            ray.df[k] = f;
            ray.inv[k] = 1.0f / f;
        }
    }
    Eye eye;
    {
        // margin: bounds the distance between the float ray and the double
        // ray anywhere inside the scene box, plus float rounding of the tests
        double ext = 0.0, onorm = 0.0;
        for (int k = 0; k < 3; ++k) {
            eye.o[k] = a.cam.eye[k];
            eye.of[k] = (float)a.cam.eye[k];
            const double lo = hdr->scene_lo[k], hi = hdr->scene_hi[k];
            ext += fmax(fabs(lo - eye.o[k]), fabs(hi - eye.o[k]));
            onorm = fmax(onorm, fabs(eye.o[k]));
        }
        const float m = (float)(0x1p-20 * (onorm + 4.0 * ext)) + 1e-30f;
        for (int k = 0; k < 3; ++k) {
            eye.oP[k] = eye.of[k] + m;
            eye.oM[k] = eye.of[k] - m;
        }
        eye.E = m;
    }
    // near-first order per split axis, from the first lane's ray
    const uint32_t neg_mask = ufirst((ray.d[0] < 0.0 ? 1u : 0u) | (ray.d[1] < 0.0 ? 2u : 0u) |
                                     (ray.d[2] < 0.0 ? 4u : 0u));

    // ---- compositing state
    float C[3] = {0.0f, 0.0f, 0.0f}, A = 0.0f, T = 1.0f;
    uint32_t n_hit = 0;
    double lo_t = 0.0;        // keys must exceed (lo_t, lo_id)
    uint32_t lo_id = 0xffffffffu;
    bool active = inside && n_spheres > 0;

    // backward state
    float4 g = make_float4(0, 0, 0, 0);
    float G = 0.0f, P = 0.0f;  // total and running sum of T alpha (k.gC + gA)
    if (BWD && inside) {
        g = a.grad[(size_t)py * a.cam.w + px];
        const float4 f = a.fwd[(size_t)py * a.cam.w + px];
        G = f.x * g.x + f.y * g.y + f.z * g.z + f.w * g.w;
    }

    while (__ballot(active)) {
        // ---- one traversal pass
        double kt[K];
        uint32_t kid[K];
        float kal[K];
#pragma unroll
        for (int j = 0; j < K; ++j) { kt[j] = INFINITY; kid[j] = 0xffffffffu; kal[j] = 0.0f; }
        uint32_t m = 0;
        double pr_t = active ? a.t_max : -1.0;  // prune key
        uint32_t pr_id = 0;
        float pr_f = active ? (float)(pr_t * (1.0 + 0x1p-20)) : -INFINITY;
        if (active && !(pr_f < INFINITY)) pr_f = INFINITY;
        const float lo_f = (float)(lo_t * (1.0 - 0x1p-20));
        const float A0 = A, T0 = T;

        int sp = 0;
        uint32_t node = 0;
        // a pass visits every node at most once; the cap only matters for a
        // corrupt hierarchy, where it turns a cycle into an early exit
        for (uint32_t visits = 0; visits <= n_nodes; ++visits) {
            const Node *nd = nodes + node;
            float f[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) f[k] = nd->f[k];
            bool hit[2] = {false, false};
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const uint32_t ref = __float_as_uint(f[12 + side]);
                const float *s = f + 6 * side;
                if (ref == kEmpty) continue;
                if (ref & kLeafBit) {
                    if (!active || (ref & ~kLeafBit) >= n_spheres) continue;
                    // float prefilter: certain miss if the ray passes farther than r + E
                    const float ox = s[0] - eye.of[0], oy = s[1] - eye.of[1], oz = s[2] - eye.of[2];
                    const float bf = ox * ray.df[0] + oy * ray.df[1] + oz * ray.df[2];
                    const float vx = ox - bf * ray.df[0], vy = oy - bf * ray.df[1], vz = oz - bf * ray.df[2];
                    const float qf = vx * vx + vy * vy + vz * vz;
                    const float rE = s[3] + eye.E;
                    if (qf > rE * rE) continue;
                    // exact test in double
                    const double oc0 = (double)s[0] - eye.o[0], oc1 = (double)s[1] - eye.o[1],
                                 oc2 = (double)s[2] - eye.o[2];
                    const double b = oc0 * ray.d[0] + oc1 * ray.d[1] + oc2 * ray.d[2];
                    const double v0 = oc0 - b * ray.d[0], v1 = oc1 - b * ray.d[1], v2 = oc2 - b * ray.d[2];
                    const double q = v0 * v0 + v1 * v1 + v2 * v2;
                    const double r = (double)s[3];
                    const double disc = r * r - q;
                    if (disc < 0.0) continue;
                    const double t0 = b - sqrt(disc);
                    const uint32_t id = ref & ~kLeafBit;
                    if (!(t0 > 0.0)) continue;
                    if (!key_less(lo_t, lo_id, t0, id)) continue;
                    if (!key_less(t0, id, pr_t, pr_id)) continue;
                    float al = s[4];
                    if (soft) {
                        const double u = q / (r * r);
                        al = (float)((double)s[4] * (1.0 - u) * (1.0 - u));
                    }
                    // insert into the sorted buffer
#pragma unroll
                    for (int j = K - 1; j >= 1; --j) {
                        const bool shift = key_less(t0, id, kt[j - 1], kid[j - 1]);
                        const bool here = !shift && key_less(t0, id, kt[j], kid[j]);
                        kt[j] = shift ? kt[j - 1] : (here ? t0 : kt[j]);
                        kid[j] = shift ? kid[j - 1] : (here ? id : kid[j]);
                        kal[j] = shift ? kal[j - 1] : (here ? al : kal[j]);
                    }
                    if (key_less(t0, id, kt[0], kid[0])) { kt[0] = t0; kid[0] = id; kal[0] = al; }
                    m = m < K ? m + 1 : K;
                    // new prune key: the hit at which the stop is certain, else the K-th
                    double nt = m == K ? kt[K - 1] : a.t_max;
                    uint32_t ni = m == K ? kid[K - 1] : 0u;
                    float As = A0, Ts = T0, w;
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        if ((uint32_t)j < m) {
                            alpha_step(kal[j], As, Ts, w);
                            if (As >= stop) {
                                nt = kt[j];
                                ni = kid[j];
                                break;
                            }
                        }
                    }
                    pr_t = nt;
                    pr_id = ni;
                    pr_f = (float)(pr_t * (1.0 + 0x1p-20));
                    if (!(pr_f < INFINITY)) pr_f = INFINITY;
                } else {
                    // padded-box slab test in float
                    const float t1x = (s[0] - eye.oP[0]) * ray.inv[0], t2x = (s[3] - eye.oM[0]) * ray.inv[0];
                    const float t1y = (s[1] - eye.oP[1]) * ray.inv[1], t2y = (s[4] - eye.oM[1]) * ray.inv[1];
                    const float t1z = (s[2] - eye.oP[2]) * ray.inv[2], t2z = (s[5] - eye.oM[2]) * ray.inv[2];
                    const float tn = fmaxf(fmaxf(fminf(t1x, t2x), fminf(t1y, t2y)), fminf(t1z, t2z));
                    const float tf = fminf(fminf(fmaxf(t1x, t2x), fmaxf(t1y, t2y)), fmaxf(t1z, t2z)) * 1.0000005f;
                    hit[side] = tn <= tf && tf >= lo_f && tn <= pr_f && ref < n_nodes;
                }
            }
            const uint64_t b0 = __ballot(hit[0]), b1 = __ballot(hit[1]);
            const uint32_t r0 = __float_as_uint(f[12]), r1 = __float_as_uint(f[13]);
            if (b0 && b1) {
                const uint32_t axis = __float_as_uint(f[14]);
                const bool second_first = axis < 3 && ((neg_mask >> axis) & 1u);
                // depth <= 63 for 62-bit (code, position) keys, so 64 slots never overflow
                if (sp < 64) {
                    if (lane == 0) stack[sp] = second_first ? r0 : r1;
                    ++sp;
                }
                node = second_first ? r1 : r0;
            } else if (b0) {
                node = r0;
            } else if (b1) {
                node = r1;
            } else {
                if (sp == 0) break;
                --sp;
                node = ufirst(stack[sp]);
            }
        }

        // ---- composite this pass
        if (active) {
            bool done = false;
            uint32_t used = 0;
            float Tj[K];
            float4 col[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                if ((uint32_t)j < m && !done) {
                    col[j] = load_colour(a.rgba, half, kid[j]);
                    Tj[j] = T;
                    float w;
                    alpha_step(kal[j], A, T, w);
                    C[0] = __fadd_rn(C[0], __fmul_rn(w, col[j].x));
                    C[1] = __fadd_rn(C[1], __fmul_rn(w, col[j].y));
                    C[2] = __fadd_rn(C[2], __fmul_rn(w, col[j].z));
                    ++n_hit;
                    ++used;
                    if (A >= stop) done = true;
                }
            }
            const bool more = !done && m == K;
            if (BWD) {
                // remainder behind the last hit of this pass, from full transmittance
                float Pend = P;
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    if ((uint32_t)j < used) {
                        const float wj = col[j].x * g.x + col[j].y * g.y + col[j].z * g.z + g.w;
                        Pend += Tj[j] * kal[j] * wj;
                    }
                }
                float R = more && T > 0.0f ? (G - Pend) / T : 0.0f;
#pragma unroll
                for (int j = K - 1; j >= 0; --j) {
                    if ((uint32_t)j < used) {
                        const uint32_t id = kid[j];
                        const float al = kal[j];
                        const float wj = col[j].x * g.x + col[j].y * g.y + col[j].z * g.z + g.w;
                        const float dal = Tj[j] * (wj - R);
                        const float ta = Tj[j] * al;
                        unsafeAtomicAdd(&a.d_rgb[3 * (size_t)id + 0], ta * g.x);
                        unsafeAtomicAdd(&a.d_rgb[3 * (size_t)id + 1], ta * g.y);
                        unsafeAtomicAdd(&a.d_rgb[3 * (size_t)id + 2], ta * g.z);
                        if (!soft) {
                            unsafeAtomicAdd(&a.d_alpha[id], dal);
                        } else {
                            const float4 c = a.centre_radius[id];
                            const double oc0 = (double)c.x - eye.o[0], oc1 = (double)c.y - eye.o[1],
                                         oc2 = (double)c.z - eye.o[2];
                            const double b = oc0 * ray.d[0] + oc1 * ray.d[1] + oc2 * ray.d[2];
                            const double v0 = oc0 - b * ray.d[0], v1 = oc1 - b * ray.d[1], v2 = oc2 - b * ray.d[2];
                            const double q = v0 * v0 + v1 * v1 + v2 * v2;
                            const double r = (double)c.w;
                            const double u = q / (r * r);
                            const double aa = (double)col[j].w;
                            const double dd = (double)dal;
                            unsafeAtomicAdd(&a.d_alpha[id], (float)(dd * (1.0 - u) * (1.0 - u)));
                            unsafeAtomicAdd(&a.d_radius[id], (float)(dd * 4.0 * aa * (1.0 - u) * q / (r * r * r)));
                            const double cc = -dd * 4.0 * aa * (1.0 - u) / (r * r);
                            unsafeAtomicAdd(&a.d_centre[3 * (size_t)id + 0], (float)(cc * v0));
                            unsafeAtomicAdd(&a.d_centre[3 * (size_t)id + 1], (float)(cc * v1));
                            unsafeAtomicAdd(&a.d_centre[3 * (size_t)id + 2], (float)(cc * v2));
                        }
                        R = al * wj + (1.0f - al) * R;
                    }
                }
                P = Pend;
            }
            if (more) {
                lo_t = kt[K - 1];
                lo_id = kid[K - 1];
            } else {
                active = false;
            }
        }
    }
    if (!BWD && inside) {
        a.out[(size_t)py * a.cam.w + px] = make_float4(C[0], C[1], C[2], A);
        if (a.hits) a.hits[(size_t)py * a.cam.w + px] = n_hit;
    }
}

// ---------------------------------------------------------------- kernels

// One wave per block; block b -> XCD b % 8.  Each XCD gets a contiguous band
// of tiles so that neighbouring tiles share that XCD's L2.
template <int K, bool BWD>
__global__ void __launch_bounds__(64) k_trace(TraceArgs a, int tiles_x, int tiles)
{
    __shared__ uint32_t stack[64];
    const int per_xcd = (tiles + 7) / 8;
    const int tile = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (tile >= tiles) return;
    const char *mem = static_cast<const char *>(a.bvh_mem);
    const BvhLayout L(0);
    const BvhHeader *hdr = reinterpret_cast<const BvhHeader *>(mem);
    const Node *nodes = reinterpret_cast<const Node *>(mem + L.nodes);
    trace_tile<K, BWD>(a, nodes, hdr, tile % tiles_x, tile / tiles_x, stack);
}

// Persistent batched trace: waves pull tiles from one atomic counter until
// the batch is drained; every wave reaches the exit test.
template <int K>
__global__ void __launch_bounds__(64)
k_trace_batched(const splat_batch_job *__restrict__ jobs, const uint32_t *__restrict__ tile_offsets, int n_jobs,
                uint32_t total_tiles, float alpha_stop, int mode, double t_max, int tile_w, int tile_h,
                uint32_t *__restrict__ counter)
{
    __shared__ uint32_t stack[64];
    __shared__ uint32_t item_s;
    const BvhLayout L(0);
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t item = ufirst(item_s);
        __syncthreads();
        if (item >= total_tiles) break;
        // job of this tile: last offset <= item (binary search, uniform)
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tile_offsets[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        const splat_batch_job &j = jobs[lo];
        TraceArgs a;
        a.bvh_mem = j.bvh_mem;
        a.bvh_capacity = j.bvh_capacity;
        a.centre_radius = reinterpret_cast<const float4 *>(j.centre_radius);
        a.rgba = j.rgba;
        a.half = j.rgba_dtype == SPLAT_F16;
        for (int k = 0; k < 3; ++k) {
            a.cam.eye[k] = j.camera.eye[k];
            a.cam.fwd[k] = j.camera.forward[k];
            a.cam.right[k] = j.camera.right[k];
            a.cam.up[k] = j.camera.up[k];
        }
        a.cam.tan_half = j.camera.tan_half_fov_y;
        a.cam.w = j.camera.width;
        a.cam.h = j.camera.height;
        a.alpha_stop = alpha_stop;
        a.mode = mode;
        a.t_max = t_max;
        a.kbuf = K;
        a.tile_w = tile_w;
        a.tile_h = tile_h;
        a.out = reinterpret_cast<float4 *>(j.out_rgba);
        a.hits = j.out_hits;
        a.fwd = nullptr;
        a.grad = nullptr;
        a.d_rgb = a.d_alpha = a.d_radius = a.d_centre = nullptr;
        const int tiles_x = (a.cam.w + tile_w - 1) / tile_w;
        const int64_t t64 = (int64_t)item - (int64_t)tile_offsets[lo];
        const int t = t64 < 0 ? 0x7fffffff : (int)min(t64, (int64_t)0x7fffffff);
        const char *mem = static_cast<const char *>(j.bvh_mem);
        trace_tile<K, false>(a, reinterpret_cast<const Node *>(mem + L.nodes), reinterpret_cast<const BvhHeader *>(mem),
                             t % tiles_x, t / tiles_x, stack);
    }
}

__global__ void k_zero_counter(uint32_t *c)
{
    if (threadIdx.x == 0) *c = 0u;
}

template <bool BWD>
static hipError_t launch_k(const TraceArgs &a, int K, dim3 grid, int tiles_x, int tiles, hipStream_t s)
{
    switch (K) {
    case 1: hipLaunchKernelGGL((k_trace<1, BWD>), grid, dim3(64), 0, s, a, tiles_x, tiles); break;
    case 2: hipLaunchKernelGGL((k_trace<2, BWD>), grid, dim3(64), 0, s, a, tiles_x, tiles); break;
    case 4: hipLaunchKernelGGL((k_trace<4, BWD>), grid, dim3(64), 0, s, a, tiles_x, tiles); break;
    case 8: hipLaunchKernelGGL((k_trace<8, BWD>), grid, dim3(64), 0, s, a, tiles_x, tiles); break;
    case 16: hipLaunchKernelGGL((k_trace<16, BWD>), grid, dim3(64), 0, s, a, tiles_x, tiles); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_trace(const TraceArgs &a, bool backward, hipStream_t s)
{
    const int tiles_x = (a.cam.w + a.tile_w - 1) / a.tile_w;
    const int tiles_y = (a.cam.h + a.tile_h - 1) / a.tile_h;
    const int tiles = tiles_x * tiles_y;
    const int per_xcd = (tiles + 7) / 8;
    const dim3 grid(per_xcd * 8);
    return backward ? launch_k<true>(a, a.kbuf, grid, tiles_x, tiles, s)
                    : launch_k<false>(a, a.kbuf, grid, tiles_x, tiles, s);
}

hipError_t launch_trace_batched(const splat_batch_job *jobs, const uint32_t *tile_offsets, int32_t n_jobs,
                                uint32_t total_tiles, const splat_trace_opts &o, int32_t waves, void *ws,
                                hipStream_t s)
{
    uint32_t *counter = static_cast<uint32_t *>(ws);
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, counter);
    const dim3 grid(waves), block(64);
    switch (o.kbuf) {
    case 1: hipLaunchKernelGGL(k_trace_batched<1>, grid, block, 0, s, jobs, tile_offsets, n_jobs, total_tiles,
                               o.alpha_stop, o.mode, o.t_max, o.tile_w, o.tile_h, counter); break;
    case 2: hipLaunchKernelGGL(k_trace_batched<2>, grid, block, 0, s, jobs, tile_offsets, n_jobs, total_tiles,
                               o.alpha_stop, o.mode, o.t_max, o.tile_w, o.tile_h, counter); break;
    case 4: hipLaunchKernelGGL(k_trace_batched<4>, grid, block, 0, s, jobs, tile_offsets, n_jobs, total_tiles,
                               o.alpha_stop, o.mode, o.t_max, o.tile_w, o.tile_h, counter); break;
    case 8: hipLaunchKernelGGL(k_trace_batched<8>, grid, block, 0, s, jobs, tile_offsets, n_jobs, total_tiles,
                               o.alpha_stop, o.mode, o.t_max, o.tile_w, o.tile_h, counter); break;
    case 16: hipLaunchKernelGGL(k_trace_batched<16>, grid, block, 0, s, jobs, tile_offsets, n_jobs, total_tiles,
                                o.alpha_stop, o.mode, o.t_max, o.tile_w, o.tile_h, counter); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace splat
