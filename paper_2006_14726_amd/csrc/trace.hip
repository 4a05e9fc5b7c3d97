// Ray tracing of the sphere set with exact front-to-back compositing
// (Sec. 4.1 and Fig. 2: the client renders the samples as coloured
// semi-transparent spheres from the current camera).
//
// One 64-lane wavefront traces one tile of pixels as a packet: the BVH walk
// is wave-uniform (node fetched once per wave with scalar loads, stack of
// node indices in LDS, a child is visited if any lane's ray meets its box),
// while each lane gathers its own hits.  A visit costs the wave its whole
// instruction stream whatever the number of lanes that need it, so the walk
// keeps it short: slot kinds come precomputed with the node, child order is
// chosen with scalar selects, and the spheres that pass a lane's float
// prefilter are queued and settled by the exact test in batches.
//
// Per traversal pass a lane keeps the K hits with the smallest keys
// (t0, sphere id) greater than the last key it composited, sorted in
// registers.  Nodes beyond the hit at which the alpha stop is already
// certain, or beyond the largest key of a full buffer, are pruned.  At the
// end of the pass the buffer is composited; if it was full and the alpha
// stop was not reached, the lane runs another pass from its last key.  So
// there is no cap on hits, and the result depends neither on K, nor on the
// tile shape, nor on the other lanes of the wave.
//
// Precision: ray and sphere test in double (hits are settled far below a
// relative discriminant of 1e-6), keys in double, boxes in float with a
// conservative margin, compositing in float with explicitly rounded
// operations so that every pass performs the same arithmetic.
#include "common.h"
#include "kernels.h"

namespace splat {

// ---------------------------------------------------------------- helpers

// Direction signs shared by every tracing lane of a wave: bit k set when the
// rays run towards -k.  kMixedSigns: the lanes differ (or a direction is
// too close to an axis plane for the shortcut below).
template <int S>
struct SignTag {
    static constexpr int value = S;
};
constexpr int kMixedSigns = 8;

__device__ inline uint32_t ufirst(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline bool key_less(double ta, uint32_t ia, double tb, uint32_t ib)
{
    return ta < tb || (ta == tb && ia < ib);
}

// One compositing step of the alpha channel.
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

__device__ inline float load_alpha(const void *rgba, int half, uint32_t id)
{
    if (half) return half_to_float(reinterpret_cast<const ushort4 *>(rgba)[id].w);
    return reinterpret_cast<const float4 *>(rgba)[id].w;
}

__device__ inline double wdot(const float4 &k, const float4 &g)
{
    return (double)k.x * g.x + (double)k.y * g.y + (double)k.z * g.z + (double)g.w;
}

// Per-lane ray state.
struct Ray {
    double d[3];     // unit direction, double
    float df[3];     // float copy of d
    float inv[3];    // 1 / df
    float oPi[3];    // (eye + margin) / df
    float oMi[3];    // (eye - margin) / df
};

// Wave-uniform ray state.
struct Eye {
    double o[3];
    float of[3];
    float oP[3], oM[3];  // float eye moved by +margin / -margin (padded-box slab test)
    float E;             // bound on the float ray-to-centre distance error
};

constexpr int kStack = 128;  // wave traversal stack (entries)
constexpr int kQueue = 8;    // leaf candidates queued per lane (at least the 4 slots of one node)
constexpr uint32_t kLaneStack = 16;  // per-lane walk: stack entries per lane (a power of 2)

constexpr uint32_t kFront = 128;  // frustum walk: nodes of one level of the breadth-first walk
constexpr uint32_t kTileCand = 256;  // frustum walk: candidate spheres of one tile
// spheroid sets: the depth-first frustum walk's stack, and its candidates
// screened and tested a chunk at a time
constexpr uint32_t kStackS = 512;
constexpr uint32_t kChunk = 128;

// Frustum walk: the two levels of the breadth-first walk, and per candidate
// sphere of the tile its screen disc (centre X, Y and squared radius in the
// tangent units of the pixel grid), its depth range [tmin, tmax] along any
// ray of the tile, and its slot, (wide node index << 2) | slot.
template <bool SPH>
struct FrustumLds {
    uint32_t front[2][kFront];
    float4 disc[kTileCand];   // X, Y, rho^2, tmin
    float2 far_ref[kTileCand];  // tmax, slot (bits)
};
// Spheroid sets walk the tile's frustum depth first, with the stack of
// nodes still to visit; per candidate of the current chunk the screen
// capsule (one end of its screen segment with the squared radius and tmin,
// the segment to the other end with tmax and the id) and what the exact
// test reads: centre and radius, axis as stored and half-length, opacity.
template <>
struct FrustumLds<true> {
    uint32_t stack[kStackS];
    float4 scr[kChunk];       // Xa, Ya, rho^2, tmin
    float4 seg[kChunk];       // dX, dY, tmax, id (bits)
    float4 geo[kChunk];       // cx, cy, cz, r
    float4 ax[kChunk];        // axis, h
    float alpha[kChunk];
};

// LDS of one wave: the leaf candidates awaiting the exact test (a column per
// lane) and the traversal stacks; with the frustum walk also its lists.  The
// per-lane stacks are only used by a frustum-walk tile that fell back to the
// per-lane walk, when its lists are no longer needed, so the two share
// memory.  The other walks do without the lists (their waves fit more per CU).
template <bool FR, bool SPH = false>
struct WaveLds {
    uint32_t cand[kQueue][kWave];            // (wide node index << 2) | slot
    uint32_t lstack[kLaneStack][kWave];      // per-lane walk: a stack per lane
    uint32_t stack[kStack];                  // packet walk: one stack per wave
};
template <bool SPH>
struct WaveLds<true, SPH> {
    uint32_t cand[kQueue][kWave];
    union {
        uint32_t lstack[kLaneStack][kWave];
        FrustumLds<SPH> fr;
    };
    uint32_t stack[kStack];
};

// A lane's hits of one pass, sorted by key, in registers (every index is a
// compile-time constant).  Empty entries hold the key (+inf, ~0), which is
// above every hit.
template <int K>
struct HitBuf {
    double t[K];  // hit distance; in the backward, the transmittance before the hit
    uint32_t id[K];
    float al[K];
};

// ---------------------------------------------------------------- one tile

// Region of a tile, in pixel columns [x0, x1) and rows [y0, y1) of the
// tile: the lanes outside it take no part.  The heaviest-first order gives
// the heaviest tiles to four waves, one per quadrant, so that they run side
// by side instead of on one wave at the end of the launch.
struct TileRegion {
    int x0, x1, y0, y1;
};

// Traces the pixels of one region of a tile; the frustum walk falls back to
// the per-lane walk for a region whose candidate lists overflow.
// SPH: the set is a spheroid set (an axis per sample); its kernels are
// compiled apart, so that the sphere kernels carry none of its code.
template <int K, bool BWD, int WALK, bool SPH = false>
__device__ void trace_tile(const TraceArgs &a, const WideNode *__restrict__ nodes, const BvhHeader *__restrict__ hdr,
                           int tile_x, int tile_y, WaveLds<WALK == SPLAT_WALK_FRUSTUM, SPH> &L, TileRegion rg)
{
    constexpr bool FRUSTUM = WALK == SPLAT_WALK_FRUSTUM;
    constexpr bool LANE = WALK == SPLAT_WALK_LANE || FRUSTUM;
    const int lane = threadIdx.x & (kWave - 1);
    const int lx = lane % a.tile_w, ly = lane / a.tile_w;
    const int px = tile_x * a.tile_w + lx;
    const int py = tile_y * a.tile_h + ly;
    const bool inside = px >= 0 && py >= 0 && px < a.cam.w && py < a.cam.h && lx >= rg.x0 && lx < rg.x1 &&
                        ly >= rg.y0 && ly < rg.y1;
    // the header count is clamped to the allocation, so even a BVH that was
    // never built cannot send the walk outside it
    const uint32_t n_spheres = min(ufirst(hdr->n), a.bvh_capacity);
    const uint32_t n_nodes = n_spheres > 1 ? n_spheres - 1 : 1;
    // a hierarchy over more samples than the set holds references samples
    // beyond it (skipped, and clamped to the nodes of the smaller count)

    const int half = a.half;
    const float stop = a.alpha_stop;
    const int soft = a.mode == SPLAT_ALPHA_SOFT;

    // ---- rays
    Ray ray;
    {
        double d[3];
        pixel_ray(a.cam, max(min(px, a.cam.w - 1), 0), max(min(py, a.cam.h - 1), 0), d);
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
            ray.oPi[k] = eye.oP[k] * ray.inv[k];
            ray.oMi[k] = eye.oM[k] * ray.inv[k];
        }
        eye.E = m;
    }
    // near-first order per split axis, from the first lane's ray
    const uint32_t neg_mask = ufirst((ray.d[0] < 0.0 ? 1u : 0u) | (ray.d[1] < 0.0 ? 2u : 0u) |
                                     (ray.d[2] < 0.0 ? 4u : 0u));
    // signs of 1/d shared by every lane that traces (lanes outside the image
    // carry a stand-in ray and take no part), for the per-lane walk's box
    // test; a 1/d beyond 2^40 could overflow the slab products, so such a
    // wave keeps the general test
    uint32_t sign_pattern = kMixedSigns;
    if (WALK == SPLAT_WALK_LANE && K <= 8 && !SPH) {
        const bool part = inside && n_spheres > 0;
        uint32_t neg = 0, pos = 0;
        bool tame = true;
        for (int k = 0; k < 3; ++k) {
            neg |= __ballot(part && ray.inv[k] < 0.0f) ? 1u << k : 0u;
            pos |= __ballot(part && !(ray.inv[k] < 0.0f)) ? 1u << k : 0u;
            tame &= __ballot(part && !(fabsf(ray.inv[k]) <= 0x1p40f)) == 0;
        }
        if ((neg & pos) == 0 && tame) sign_pattern = neg;
    }

    // ---- compositing state
    float C[3] = {0.0f, 0.0f, 0.0f}, A = 0.0f, T = 1.0f;
    uint32_t n_hit = 0;
    double lo_t = 0.0;        // keys must exceed (lo_t, lo_id)
    uint32_t lo_id = 0xffffffffu;
    bool active = inside && n_spheres > 0;

    // backward state.  A pixel whose hits fit one pass gets its gradients
    // back to front from that pass alone.  Otherwise (phase 1) the remaining
    // passes first sum G = sum_j T_j alpha_j w_j in double; then (phase 2)
    // the passes are repeated from the first hit, and the remainder behind
    // each pass is (G - P) / T with the prefix P and T in double.
    float4 g = make_float4(0, 0, 0, 0);
    int phase = 0;
    double G64 = 0.0, P64 = 0.0, T64 = 1.0;
    if (BWD && inside) g = a.grad[(size_t)py * a.cam.w + px];

    // ---- frustum walk, once per tile: the spheres that the tile's frustum
    // may meet.  The four side planes pass through the eye and two adjacent
    // corner rays of the tile; every pixel ray of the tile is a convex
    // combination of the corner rays, so a box or sphere wholly outside one
    // plane (by more than the float margin) meets none of them.  Levels of
    // the 4-wide hierarchy are walked breadth first, 16 nodes per round (a
    // lane per slot).  Each sphere that passes is entered in the tile's
    // candidate list with its screen disc: a ray with screen coordinates
    // (sx, sy) that hits the sphere satisfies |(sx, sy) - (X, Y)| <= rho with
    // (X, Y) = (x, y) / z and rho = r sqrt(1 + X^2 + Y^2) / (z - r), where
    // (x, y, z) is the centre in the camera basis (right, up, forward)
    // relative to the eye, as long as z - r > 0.  If a level or the list
    // overflows, the tile falls back to the per-lane walk.
    uint32_t n_cand = 0;  // wave-uniform
    bool fb = !FRUSTUM;   // wave-uniform: the tile uses the per-lane walk
    float sxl = 0.0f, syl = 0.0f;
    if constexpr (FRUSTUM && !SPH) {
        {
            const double aspect = (double)a.cam.w / (double)a.cam.h;
            const int cx = max(min(px, a.cam.w - 1), 0), cy = max(min(py, a.cam.h - 1), 0);
            sxl = (float)(((2.0 * cx + 1.0) / (double)a.cam.w - 1.0) * a.cam.tan_half * aspect);
            syl = (float)((1.0 - (2.0 * cy + 1.0) / (double)a.cam.h) * a.cam.tan_half);
        }
        const int tw = a.tile_w;  // the region's corner lanes, clockwise on the screen
        const int corner[4] = {rg.y0 * tw + rg.x0, rg.y0 * tw + rg.x1 - 1, (rg.y1 - 1) * tw + rg.x1 - 1,
                               (rg.y1 - 1) * tw + rg.x0};
        double cd[4][3];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int k = 0; k < 3; ++k) cd[c][k] = __shfl(ray.d[k], corner[c], kWave);
        const double cen[3] = {cd[0][0] + cd[1][0] + cd[2][0] + cd[3][0], cd[0][1] + cd[1][1] + cd[2][1] + cd[3][1],
                               cd[0][2] + cd[1][2] + cd[2][2] + cd[3][2]};
        // plane i: pp[i] . x + pc[i] >= -slack, split into the positive and
        // negative parts of the normal for the box test (the corner of the box
        // farthest along the normal)
        float pp[4][3], pn[4][3], pc[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double *u = cd[i], *v = cd[(i + 1) & 3];
            double n0 = u[1] * v[2] - u[2] * v[1], n1 = u[2] * v[0] - u[0] * v[2], n2 = u[0] * v[1] - u[1] * v[0];
            const double len = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
            const double sg = (n0 * cen[0] + n1 * cen[1] + n2 * cen[2]) < 0.0 ? -1.0 : 1.0;
            // two equal corners (a one-row tile) give no plane: it is left out
            const double inv = len > 1e-300 ? sg / len : 0.0;
            const float f0 = (float)(n0 * inv), f1 = (float)(n1 * inv), f2 = (float)(n2 * inv);
            pp[i][0] = fmaxf(f0, 0.0f); pp[i][1] = fmaxf(f1, 0.0f); pp[i][2] = fmaxf(f2, 0.0f);
            pn[i][0] = fminf(f0, 0.0f); pn[i][1] = fminf(f1, 0.0f); pn[i][2] = fminf(f2, 0.0f);
            pc[i] = (float)(-((double)f0 * eye.o[0] + (double)f1 * eye.o[1] + (double)f2 * eye.o[2]));
        }
        // the margin bounds the float rounding of the plane tests
        const float slack = 4.0f * eye.E;
        const float bR[3] = {(float)a.cam.right[0], (float)a.cam.right[1], (float)a.cam.right[2]};
        const float bU[3] = {(float)a.cam.up[0], (float)a.cam.up[1], (float)a.cam.up[2]};
        const float bF[3] = {(float)a.cam.fwd[0], (float)a.cam.fwd[1], (float)a.cam.fwd[2]};
        const bool any = __ballot(active) != 0;
        uint32_t cur = 0, n_front = any ? 1u : 0u;
        if (lane == 0) L.fr.front[0][0] = 0u;  // the root
        fb = false;
        // the top cut, one entry per lane, in place of the first three levels
        const uint32_t n_cut = any ? min(ufirst(hdr->n_cut), kCut) : 0u;
        if (n_cut > 0) {
            const CutEntry *cut = reinterpret_cast<const CutEntry *>(reinterpret_cast<const char *>(a.bvh_mem) +
                                                                     BvhLayout(a.layout_cap).cut);
            const bool valid = (uint32_t)lane < n_cut;
            const float4 e0 = valid ? reinterpret_cast<const float4 *>(cut + lane)[0] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            const float4 e1 = valid ? reinterpret_cast<const float4 *>(cut + lane)[1] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            const float q0 = e0.x, q1 = e0.y, q2 = e0.z, q3 = e0.w, q4 = e1.x, q5 = e1.y;
            const uint32_t ref = __float_as_uint(e1.z), origin = __float_as_uint(e1.w);
            const bool is_leaf = valid && (ref & kLeafBit) != 0u, is_int = valid && (ref & kLeafBit) == 0u;
            bool pass = is_leaf || is_int;
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) {
                // box: its corner farthest along the normal; sphere: its centre, moved r along it
                const float bx = fmaf(pp[pl][0], q3, fmaf(pn[pl][0], q0, pc[pl]));
                const float vb = fmaf(pp[pl][2], q5, fmaf(pn[pl][2], q2, fmaf(pp[pl][1], q4, fmaf(pn[pl][1], q1, bx))));
                const float vs = fmaf(pp[pl][0] + pn[pl][0], q0, fmaf(pp[pl][1] + pn[pl][1], q1,
                                 fmaf(pp[pl][2] + pn[pl][2], q2, pc[pl]))) + q3;
                pass = pass && (is_leaf ? vs : vb) >= -slack;
            }
            const uint64_t mi = __ballot(pass && is_int), ml = __ballot(pass && is_leaf);
            const uint32_t below_i = (uint32_t)__popcll(mi & ((1ull << lane) - 1ull));
            const uint32_t below_l = (uint32_t)__popcll(ml & ((1ull << lane) - 1ull));
            if (pass && is_int && below_i < kFront) L.fr.front[0][below_i] = ref;
            if (pass && is_leaf && below_l < kTileCand) {
                // the candidate's screen disc and depth range, in float with
                // outward slack (relative 2^-12 on rho, 2^-18 absolute in tangent
                // units, 2^-20 relative on depths plus the margin); the hardware
                // reciprocal and square root, within a few ulps on normal
                // operands, stay far inside it
                const float ox = q0 - eye.of[0], oy = q1 - eye.of[1], oz = q2 - eye.of[2];
                const float x = ox * bR[0] + oy * bR[1] + oz * bR[2];
                const float y = ox * bU[0] + oy * bU[1] + oz * bU[2];
                const float z = ox * bF[0] + oy * bF[1] + oz * bF[2];
                const float dist = __builtin_amdgcn_sqrtf(ox * ox + oy * oy + oz * oz);
                const float zr = z - q3;
                float X = 0.0f, Y = 0.0f, rho2 = INFINITY;
                if (zr > 0x1p-10f * dist && zr > 0x1p-100f) {
                    const float iz = __builtin_amdgcn_rcpf(z);
                    X = x * iz;
                    Y = y * iz;
                    const float rho = q3 * __builtin_amdgcn_sqrtf(1.0f + X * X + Y * Y) * __builtin_amdgcn_rcpf(zr);
                    const float rs = rho * (1.0f + 0x1p-12f) + 0x1p-18f * (1.0f + fabsf(X) + fabsf(Y));
                    rho2 = rs * rs;
                }
                const float tmin = (dist - q3) * (1.0f - 0x1p-20f) - slack;
                const float tmax = dist * (1.0f + 0x1p-20f) + slack;
                L.fr.disc[below_l] = make_float4(X, Y, rho2, tmin);
                L.fr.far_ref[below_l] = make_float2(tmax, __uint_as_float(origin));
            }
            n_front = (uint32_t)__popcll(mi);
            n_cand = (uint32_t)__popcll(ml);
        }
        // a hierarchy over 62-bit (code, position) keys is at most 64 binary
        // levels deep; more levels only occur in a corrupt one
        for (uint32_t level = 0; n_front > 0; ++level) {
            __builtin_amdgcn_wave_barrier();
            if (level > 40) {
                if (lane == 0) flag_status(a.status, SPLAT_STATUS_CORRUPT);
                fb = true;
                break;
            }
            uint32_t n_next = 0;
            for (uint32_t base = 0; base < n_front; base += kWave / 4) {
                const uint32_t i = base + (uint32_t)lane / 4u, sl = (uint32_t)lane & 3u;
                const bool valid = i < n_front;
                const uint32_t node = valid ? min(L.fr.front[cur][i], n_nodes - 1) : 0u;
                const float *f = nodes[node].f;
                const uint32_t kinds = valid ? __float_as_uint(f[31]) : 0u;
                const bool is_leaf = (kinds >> sl) & 1u, is_int = (kinds >> (4u + sl)) & 1u;
                const float *q = f + 6 * sl;
                const float q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3], q4 = q[4], q5 = q[5];
                const uint32_t ref = __float_as_uint(f[24 + sl]);
                bool pass = is_leaf || is_int;
#pragma unroll
                for (int pl = 0; pl < 4; ++pl) {
                    // box: its corner farthest along the normal; sphere: its centre, moved r along it
                    const float bx = fmaf(pp[pl][0], q3, fmaf(pn[pl][0], q0, pc[pl]));
                    const float vb = fmaf(pp[pl][2], q5, fmaf(pn[pl][2], q2, fmaf(pp[pl][1], q4, fmaf(pn[pl][1], q1, bx))));
                    const float vs = fmaf(pp[pl][0] + pn[pl][0], q0, fmaf(pp[pl][1] + pn[pl][1], q1,
                                     fmaf(pp[pl][2] + pn[pl][2], q2, pc[pl]))) + q3;
                    pass = pass && (is_leaf ? vs : vb) >= -slack;
                }
                const uint64_t mi = __ballot(pass && is_int), ml = __ballot(pass && is_leaf);
                const uint32_t below_i = (uint32_t)__popcll(mi & ((1ull << lane) - 1ull));
                const uint32_t below_l = (uint32_t)__popcll(ml & ((1ull << lane) - 1ull));
                if (pass && is_int && n_next + below_i < kFront) L.fr.front[cur ^ 1u][n_next + below_i] = ref;
                if (pass && is_leaf && n_cand + below_l < kTileCand) {
                    // the candidate's screen disc and depth range, in float with
                    // outward slack (relative 2^-12 on rho, 2^-18 absolute in tangent
                    // units, 2^-20 relative on depths plus the margin); the hardware
                    // reciprocal and square root, within a few ulps on normal
                    // operands, stay far inside it
                    const float ox = q0 - eye.of[0], oy = q1 - eye.of[1], oz = q2 - eye.of[2];
                    const float x = ox * bR[0] + oy * bR[1] + oz * bR[2];
                    const float y = ox * bU[0] + oy * bU[1] + oz * bU[2];
                    const float z = ox * bF[0] + oy * bF[1] + oz * bF[2];
                    const float dist = __builtin_amdgcn_sqrtf(ox * ox + oy * oy + oz * oz);
                    const float zr = z - q3;
                    float X = 0.0f, Y = 0.0f, rho2 = INFINITY;
                    if (zr > 0x1p-10f * dist && zr > 0x1p-100f) {
                        const float iz = __builtin_amdgcn_rcpf(z);
                        X = x * iz;
                        Y = y * iz;
                        const float rho = q3 * __builtin_amdgcn_sqrtf(1.0f + X * X + Y * Y) * __builtin_amdgcn_rcpf(zr);
                        const float rs = rho * (1.0f + 0x1p-12f) + 0x1p-18f * (1.0f + fabsf(X) + fabsf(Y));
                        rho2 = rs * rs;
                    }
                    const float tmin = (dist - q3) * (1.0f - 0x1p-20f) - slack;
                    const float tmax = dist * (1.0f + 0x1p-20f) + slack;
                    L.fr.disc[n_cand + below_l] = make_float4(X, Y, rho2, tmin);
                    L.fr.far_ref[n_cand + below_l] = make_float2(tmax, __uint_as_float((node << 2) | sl));
                }
                n_next += (uint32_t)__popcll(mi);
                n_cand += (uint32_t)__popcll(ml);
            }
            if (n_next > kFront || n_cand > kTileCand) {
                fb = true;
                break;
            }
            cur ^= 1u;
            n_front = n_next;
        }
        __builtin_amdgcn_wave_barrier();
    }

    HitBuf<K> B;
    while (__ballot(active)) {
        // ---- one traversal pass
#pragma unroll
        for (int k = 0; k < K; ++k) {
            B.t[k] = INFINITY;
            B.id[k] = 0xffffffffu;
            B.al[k] = 0.0f;
        }
        uint32_t m = 0;                          // buffered hits
        double pr_t = active ? a.t_max : -1.0;   // prune key: hits must be below it
        uint32_t pr_id = 0;
        float pr_f = active ? (float)(pr_t * (1.0 + 0x1p-20)) : -INFINITY;
        if (active && !(pr_f < INFINITY)) pr_f = INFINITY;
        const float lo_f = (float)(lo_t * (1.0 - 0x1p-20));
        uint32_t nc = 0;                         // queued leaf candidates
        bool redo = false;                       // spheres may be tested a second time
        bool from_chunk = false;                 // spheroid frustum walk: the queue holds chunk indices

        // The exact test of the queued candidates.  A leaf slot holds the
        // sphere's centre, radius and opacity as stored by the last build or
        // refit; the node was fetched moments ago, so the slot is read from
        // cache.  A hit below the prune key is filed in key order; a full
        // buffer drops its largest key, and its new largest key becomes the
        // prune key.  Afterwards the prune key moves down to the hit at which
        // the alpha stop is already certain (the same float steps as the
        // compositing below).
        // The slots of kFlushGroup queue entries are loaded together before
        // any of them is tested, so a flush waits for memory once per group
        // (entries past a lane's queue read slot 0 of node 0, never used).
        // The frustum walk tests one entry at a time: its kernel keeps fewer
        // registers that way, and more of its waves fit a SIMD.  Spheroid sets
        // also load each entry's axis, a second dependent load, so they keep
        // the groups.
        constexpr int kFlushGroup = (FRUSTUM && !SPH) ? 1 : 4;
        auto flush = [&]() {
            bool changed = false;
            for (uint32_t j0 = 0; j0 < (uint32_t)kQueue; j0 += kFlushGroup) {
              if (!__ballot(j0 < nc)) break;
              float2 p01[kFlushGroup], p23[kFlushGroup];
              float pa[kFlushGroup], ph[kFlushGroup];
              float4 pax[kFlushGroup];
              uint32_t pid[kFlushGroup];
              bool loaded = false;
              if constexpr (SPH && FRUSTUM) {
                  if (from_chunk) {
                      // everything from the chunk in LDS
#pragma unroll
                      for (int u = 0; u < kFlushGroup; ++u) {
                          const uint32_t e = j0 + u < nc ? L.cand[j0 + u][lane] : 0u;
                          const float4 gc = L.fr.geo[e];
                          pax[u] = L.fr.ax[e];
                          p01[u] = make_float2(gc.x, gc.y);
                          p23[u] = make_float2(gc.z, gc.w);
                          pa[u] = L.fr.alpha[e];
                          ph[u] = pax[u].w;
                          pid[u] = __float_as_uint(L.fr.seg[e].w);
                      }
                      loaded = true;
                  }
              }
              if (!loaded) {
#pragma unroll
              for (int u = 0; u < kFlushGroup; ++u) {
                  const uint32_t e = j0 + u < nc ? L.cand[j0 + u][lane] : 0u;
                  const float *s = nodes[e >> 2].f + 6 * (e & 3u);
                  p01[u] = *reinterpret_cast<const float2 *>(s);
                  p23[u] = *reinterpret_cast<const float2 *>(s + 2);
                  pa[u] = s[4];
                  if constexpr (SPH) ph[u] = s[5];
                  pid[u] = __float_as_uint(nodes[e >> 2].f[24 + (e & 3u)]) & ~kLeafBit;
              }
              if constexpr (SPH) {
#pragma unroll
                  for (int u = 0; u < kFlushGroup; ++u)
                      pax[u] = (j0 + u < nc && ph[u] > 0.0f && pid[u] < n_spheres) ? a.axis[pid[u]]
                                                                                    : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
              }
              }
#pragma unroll
              for (int u = 0; u < kFlushGroup; ++u) {
                if (j0 + u >= nc) continue;
                const float2 s01 = p01[u], s23 = p23[u];
                const float ca = pa[u];
                const uint32_t id = pid[u];
                if (id >= n_spheres) continue;
                const double oc0 = (double)s01.x - eye.o[0], oc1 = (double)s01.y - eye.o[1],
                             oc2 = (double)s23.x - eye.o[2];
                const double r = (double)s23.y;
                const double b = oc0 * ray.d[0] + oc1 * ray.d[1] + oc2 * ray.d[2];
                const double v0 = oc0 - b * ray.d[0], v1 = oc1 - b * ray.d[1], v2 = oc2 - b * ray.d[2];
                const double q = v0 * v0 + v1 * v1 + v2 * v2;
                double disc = r * r - q, tc = b;
                if constexpr (SPH) {
                    if (ph[u] > 0.0f) {
                        // spheroid (axis u scaled to unit length, half-length h
                        // along it, r across): y -> y + (y.u)(r/h - 1) u maps it to
                        // the ball of radius r and the ray to t D - L, D the image of
                        // d and L that of c - o; then the robust sphere form:
                        // t_m = L.D / D.D, w = L - t_m D, t0 = t_m - sqrt((r^2 - w.w) / D.D)
                        const float4 ua = pax[u];
                        const double il = 1.0 / sqrt((double)ua.x * ua.x + (double)ua.y * ua.y + (double)ua.z * ua.z);
                        const double u0 = ua.x * il, u1 = ua.y * il, u2 = ua.z * il;
                        const double h = (double)ph[u];
                        const double k = (r - h) / h;
                        const double du = (ray.d[0] * u0 + ray.d[1] * u1 + ray.d[2] * u2) * k;
                        const double ou = (oc0 * u0 + oc1 * u1 + oc2 * u2) * k;
                        const double D0 = ray.d[0] + du * u0, D1 = ray.d[1] + du * u1, D2 = ray.d[2] + du * u2;
                        const double L0 = oc0 + ou * u0, L1 = oc1 + ou * u1, L2 = oc2 + ou * u2;
                        const double iDD = 1.0 / (D0 * D0 + D1 * D1 + D2 * D2);
                        const double tm = (L0 * D0 + L1 * D1 + L2 * D2) * iDD;
                        const double w0 = L0 - tm * D0, w1 = L1 - tm * D1, w2 = L2 - tm * D2;
                        const double ds = r * r - (w0 * w0 + w1 * w1 + w2 * w2);
                        disc = ds < 0.0 ? ds : ds * iDD;
                        tc = tm;
                    }
                }
                if (disc < 0.0) continue;
                const double t0 = tc - sqrt(disc);
                if (!(t0 > 0.0)) continue;
                if (!key_less(lo_t, lo_id, t0, id)) continue;
                if (!key_less(t0, id, pr_t, pr_id)) continue;
                if (redo) {
                    // a second walk over the same nodes: keys are unique, so an
                    // equal key is this sphere already filed
                    bool dup = false;
#pragma unroll
                    for (int k = 0; k < K; ++k) dup |= B.t[k] == t0 && B.id[k] == id;
                    if (dup) continue;
                }
                float al = ca;
                if (soft) {
                    const double u = q / (r * r);
                    al = (float)((double)al * (1.0 - u) * (1.0 - u));
                }
                // insertion network: entry k takes entry k - 1 when the new key is
                // below that, the new hit when it lands at k, else stays
                bool lt[K];
#pragma unroll
                for (int k = 0; k < K; ++k) lt[k] = key_less(t0, id, B.t[k], B.id[k]);
#pragma unroll
                for (int k = K - 1; k > 0; --k) {
                    const bool here = lt[k] && !lt[k - 1];
                    B.t[k] = lt[k - 1] ? B.t[k - 1] : (here ? t0 : B.t[k]);
                    B.id[k] = lt[k - 1] ? B.id[k - 1] : (here ? id : B.id[k]);
                    B.al[k] = lt[k - 1] ? B.al[k - 1] : (here ? al : B.al[k]);
                }
                if (lt[0]) {
                    B.t[0] = t0;
                    B.id[0] = id;
                    B.al[0] = al;
                }
                m = m < K ? m + 1 : K;
                changed = true;
                if (key_less(B.t[K - 1], B.id[K - 1], pr_t, pr_id)) {
                    // full: later candidates must beat the new largest key
                    pr_t = B.t[K - 1];
                    pr_id = B.id[K - 1];
                    pr_f = (float)(pr_t * (1.0 + 0x1p-20));
                }
              }
            }
            nc = 0;
            if (changed) {
                float As = A, Ts = T, w;
                bool found = false;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (!found && (uint32_t)k < m) {
                        alpha_step(B.al[k], As, Ts, w);
                        if (As >= stop) {
                            found = true;
                            pr_t = B.t[k];
                            pr_id = B.id[k];
                            pr_f = (float)(pr_t * (1.0 + 0x1p-20));
                        }
                    }
                }
            }
        };
        // Leaf slots of a node: float prefilter, certain misses only (the ray
        // passes farther than r + E from the centre, or the sphere lies wholly
        // beyond the prune key or before the last composited key: t0 lies in
        // [b - r, b], and E bounds the error of the float b).  A survivor is
        // queued for the exact test.  `pf` is the lane's prune bound (-inf for
        // a lane that takes no part).
        auto queue_leaves = [&](const float *f, uint32_t node, uint32_t kinds, float pf) {
#pragma unroll
            for (int side = 0; side < 4; ++side) {
                if (!((kinds >> side) & 1u)) continue;
                const float *s = f + 6 * side;
                const float ox = s[0] - eye.of[0], oy = s[1] - eye.of[1], oz = s[2] - eye.of[2];
                const float bf = ox * ray.df[0] + oy * ray.df[1] + oz * ray.df[2];
                const float vx = ox - bf * ray.df[0], vy = oy - bf * ray.df[1], vz = oz - bf * ray.df[2];
                const float qf = vx * vx + vy * vy + vz * vz;
                // a spheroid (word 5: its half-length h, which is at least r) lies
                // in the ball of radius h around its centre, and its entry in
                // [b - h, b + h]; a sphere's (word 5: 0) in [b - r, b]
                const float rE = (SPH ? fmaxf(s[3], s[5]) : s[3]) + eye.E;
                bool may = (qf <= rE * rE) & (bf - rE <= pf) & ((SPH ? bf + s[5] : bf) + eye.E >= lo_f);
                if constexpr (SPH) {
                    // a spheroid with h > r: the ray's distance to the capsule's
                    // segment c + s u, |s| <= h - r, at s clamped from the
                    // minimiser over the line (a ray nearly along the axis keeps
                    // the ball test: there the clamped minimiser's rounding could
                    // exceed the margins)
                    const uint32_t id = __float_as_uint(f[24 + side]) & ~kLeafBit;
                    if (may && s[5] > s[3] && id < n_spheres) {
                        const float4 ua = a.axis[id];
                        const float il = rsqrtf(fmaf(ua.x, ua.x, fmaf(ua.y, ua.y, ua.z * ua.z)));
                        const float u0 = ua.x * il, u1 = ua.y * il, u2 = ua.z * il;
                        const float ha = s[5] - s[3];
                        const float du = u0 * ray.df[0] + u1 * ray.df[1] + u2 * ray.df[2];
                        const float wu = ox * u0 + oy * u1 + oz * u2;
                        const float den = 1.0f - du * du;
                        if (den >= 0x1p-6f) {
                            const float sd = fminf(fmaxf((bf * du - wu) / den, -ha), ha);
                            const float gx = fmaf(sd, u0, ox), gy = fmaf(sd, u1, oy), gz = fmaf(sd, u2, oz);
                            const float gb = gx * ray.df[0] + gy * ray.df[1] + gz * ray.df[2];
                            const float wx = gx - gb * ray.df[0], wy = gy - gb * ray.df[1], wz = gz - gb * ray.df[2];
                            const float rc = s[3] + 2.0f * eye.E + ha * 0x1p-20f;
                            may = wx * wx + wy * wy + wz * wz <= rc * rc;
                        }
                    }
                }
                // nc < kQueue here: the queue is flushed once a lane could overflow
                L.cand[nc][lane] = (node << 2) | (uint32_t)side;
                nc += may ? 1u : 0u;
            }
        };
        // Internal slots: padded-box slab test in float, (x - o) / d as
        // fma(x, 1/d, -o/d): the rounding of o/d moves the eye by at most
        // eps |o|, far inside the margin.  Bit s of the result: this lane's
        // ray meets the box of slot s before its prune bound.
        auto box_hits = [&](const float *f, uint32_t kinds, float pf) -> uint32_t {
            uint32_t hits = 0;
#pragma unroll
            for (int side = 0; side < 4; ++side) {
                if (!((kinds >> (4 + side)) & 1u)) continue;
                const float *s = f + 6 * side;
                const float t1x = fmaf(s[0], ray.inv[0], -ray.oPi[0]), t2x = fmaf(s[3], ray.inv[0], -ray.oMi[0]);
                const float t1y = fmaf(s[1], ray.inv[1], -ray.oPi[1]), t2y = fmaf(s[4], ray.inv[1], -ray.oMi[1]);
                const float t1z = fmaf(s[2], ray.inv[2], -ray.oPi[2]), t2z = fmaf(s[5], ray.inv[2], -ray.oMi[2]);
                const float tn = fmaxf(fmaxf(fminf(t1x, t2x), fminf(t1y, t2y)), fminf(t1z, t2z));
                const float tf = fminf(fminf(fmaxf(t1x, t2x), fmaxf(t1y, t2y)), fmaxf(t1z, t2z)) * 1.0000005f;
                hits |= (fmaxf(tn, lo_f) <= fminf(tf, pf)) ? 1u << side : 0u;
            }
            return hits;
        };
        // Near-first order of the four slots: the near child of the node, within
        // it the near grandchild (split axes against the ray signs in `neg`),
        // as four 2-bit slot numbers.
        auto slot_order = [](const float *f, uint32_t neg) -> uint32_t {
            const uint32_t ax = __float_as_uint(f[28]), a0 = __float_as_uint(f[29]), a1 = __float_as_uint(f[30]);
            const uint32_t cn = ax < 3u ? (neg >> ax) & 1u : 0u;
            const uint32_t axn = cn ? a1 : a0, axf = cn ? a0 : a1;
            const uint32_t gn = axn < 3u ? (neg >> axn) & 1u : 0u;
            const uint32_t gf = axf < 3u ? (neg >> axf) & 1u : 0u;
            const uint32_t o0 = 2u * cn + gn, o2 = 2u * (1u - cn) + gf;
            return o0 | ((o0 ^ 1u) << 2) | (o2 << 4) | ((o2 ^ 1u) << 6);
        };
        // per lane: hit mask and entry distance of each slot.  Nearly every
        // step has an internal slot at every position in some lane, so the
        // four tests run unconditionally and the slot kinds mask the result
        // once (a sphere slot's words make a meaningless box, never used;
        // its entry distance only reorders slots that are not pushed).
        // With the direction signs known for the wave, the near and far plane
        // of each axis are known too: for a box with lo <= hi and a positive
        // 1/d, fma(lo, 1/d, -(o+m)/d) <= fma(hi, 1/d, -(o-m)/d) by monotone
        // rounding, so the per-axis min and max give exactly these values.
        auto box_hits_tn = [&](auto sign, const float *f, uint32_t kinds, float pf, float tn_out[4]) -> uint32_t {
            constexpr int S = decltype(sign)::value;
            uint32_t hits = 0;
#pragma unroll
            for (int side = 0; side < 4; ++side) {
                const float *s = f + 6 * side;
                const float t1x = fmaf(s[0], ray.inv[0], -ray.oPi[0]), t2x = fmaf(s[3], ray.inv[0], -ray.oMi[0]);
                const float t1y = fmaf(s[1], ray.inv[1], -ray.oPi[1]), t2y = fmaf(s[4], ray.inv[1], -ray.oMi[1]);
                const float t1z = fmaf(s[2], ray.inv[2], -ray.oPi[2]), t2z = fmaf(s[5], ray.inv[2], -ray.oMi[2]);
                float tn, tf;
                if constexpr (S == kMixedSigns) {
                    tn = fmaxf(fmaxf(fminf(t1x, t2x), fminf(t1y, t2y)), fminf(t1z, t2z));
                    tf = fminf(fminf(fmaxf(t1x, t2x), fmaxf(t1y, t2y)), fmaxf(t1z, t2z)) * 1.0000005f;
                } else {
                    tn = fmaxf(fmaxf((S & 1) ? t2x : t1x, (S & 2) ? t2y : t1y), (S & 4) ? t2z : t1z);
                    tf = fminf(fminf((S & 1) ? t1x : t2x, (S & 2) ? t1y : t2y), (S & 4) ? t1z : t2z) * 1.0000005f;
                }
                // tn <= tf, tf >= lo_f and tn <= pf in one comparison (lo_f <= pf for a lane
                // taking part; pf = -inf for one that does not)
                const bool h = fmaxf(tn, lo_f) <= fminf(tf, pf);
                hits |= h ? 1u << side : 0u;
                tn_out[side] = h ? tn : INFINITY;
            }
            return hits & (kinds >> 4) & 0xfu;
        };
        auto slot_ref = [](const float *f, uint32_t o) -> uint32_t {
            // two levels of selects on the slot's bits (no branches for a per-lane slot)
            const uint32_t r01 = (o & 1u) ? __float_as_uint(f[25]) : __float_as_uint(f[24]);
            const uint32_t r23 = (o & 1u) ? __float_as_uint(f[27]) : __float_as_uint(f[26]);
            return (o & 2u) ? r23 : r01;
        };

        bool overflow = false;  // the lane's own stack dropped entries
        // Per-lane walk: every lane follows its own ray through the tree
        // (vector loads of its node; stack in its own LDS column, a ring of
        // kLaneStack entries; children entered nearest box entry first).  A
        // wave costs the longest path of its lanes rather than the union of
        // their paths.  One copy per sign pattern of the wave.
        auto lane_walk = [&](auto sign) {
            uint32_t node = 0, top = 0, depth = 0, steps = 0;
            bool walking = active;
            // steps run in an inner loop that ends when some lane's queue may
            // overflow; the flush (which rewrites the hit buffer) stays out of
            // it, so the buffer's registers are not copied at every step
            while (__ballot(walking)) {
              do {
                if (walking) {
                    const float4 *np = reinterpret_cast<const float4 *>(nodes + node);
                    float f[32];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const float4 v = np[k];
                        f[4 * k] = v.x;
                        f[4 * k + 1] = v.y;
                        f[4 * k + 2] = v.z;
                        f[4 * k + 3] = v.w;
                    }
                    const uint32_t kinds = __float_as_uint(f[31]);
                    queue_leaves(f, node, kinds, pr_f);
                    float tn[4];
                    const uint32_t boxes = box_hits_tn(sign, f, kinds, pr_f, tn);
                    if (boxes) {
                        // sort the slots by entry distance (misses last)
                        uint32_t sl[4] = {0u, 1u, 2u, 3u};
                        auto cx = [&](int i, int j) {
                            const bool sw = tn[j] < tn[i];
                            const float ti = tn[i], tj = tn[j];
                            const uint32_t si = sl[i], sj = sl[j];
                            tn[i] = sw ? tj : ti; tn[j] = sw ? ti : tj;
                            sl[i] = sw ? sj : si; sl[j] = sw ? si : sj;
                        };
                        cx(0, 1); cx(2, 3); cx(0, 2); cx(1, 3); cx(1, 2);
                        uint32_t next = kEmpty;
#pragma unroll
                        for (int i = 3; i >= 0; --i) {
                            const uint32_t o = sl[i];
                            if (!((boxes >> o) & 1u)) continue;
                            if (next != kEmpty) {
                                // a full ring drops its oldest entry; the packet walk
                                // below then settles this lane
                                L.lstack[top][lane] = next;
                                top = (top + 1u) & (kLaneStack - 1u);
                                if (depth < kLaneStack) ++depth;
                                else overflow = true;
                            }
                            next = slot_ref(f, o);
                        }
                        node = next;
                    } else if (depth > 0) {
                        top = (top - 1u) & (kLaneStack - 1u);
                        node = L.lstack[top][lane];
                        --depth;
                    } else {
                        walking = false;
                    }
                    // only a corrupt hierarchy can name a node outside the array
                    // or take more steps than there are nodes
                    node = min(node, n_nodes - 1);
                    if (++steps > n_nodes) walking = false;
                }
              } while (__ballot(walking) && !__ballot(nc > (uint32_t)kQueue - 4u));
                if (__ballot(nc > (uint32_t)kQueue - 4u)) flush();
            }
        };
        // Frustum walk: the tile's candidates against the lane's ray.  The
        // screen test is the disc above; the depth range must reach below the
        // prune key and past the last composited key, as in the per-lane
        // prefilter.  Survivors are queued for the exact test, as in the walks.
        // kCandGroup candidates per round, their records read together.
        constexpr int kCandGroup = 2;
        auto cand_pass = [&](auto &F) {
            for (uint32_t j = 0; j < n_cand; j += kCandGroup) {
                float4 dc[kCandGroup];
                float2 fr[kCandGroup];
#pragma unroll
                for (int u = 0; u < kCandGroup; ++u) {
                    const uint32_t i = min(j + (uint32_t)u, n_cand - 1u);
                    dc[u] = F.disc[i];
                    fr[u] = F.far_ref[i];
                }
#pragma unroll
                for (int u = 0; u < kCandGroup; ++u) {
                    const float du = sxl - dc[u].x, dv = syl - dc[u].y;
                    const bool may = (j + u < n_cand) & (fmaf(du, du, dv * dv) <= dc[u].z) & (dc[u].w <= pr_f) &
                                     (fr[u].x >= lo_f);
                    // nc <= kQueue - kCandGroup at the start of a round: the
                    // queue is flushed once a lane could overflow it
                    L.cand[nc][lane] = __float_as_uint(fr[u].y);
                    nc += may ? 1u : 0u;
                }
                if (__ballot(nc > (uint32_t)(kQueue - kCandGroup))) flush();
            }
        };
        // Spheroid sets: the tile's frustum walked depth first, sixteen nodes a
        // step (one slot per lane) from a stack in LDS.  A box that lies wholly
        // beyond every lane's prune key is dropped, which the stop at the alpha
        // threshold makes common behind an opaque layer.  Each spheroid the
        // frustum meets goes into the current chunk with its screen capsule and
        // what the exact test reads; a chunk is screened per lane and tested
        // when it fills, so no list bounds the walk.  A stack overflow or a
        // corrupt hierarchy sets fb: the tile then takes the per-lane walk.
        auto frustum_dfs = [&]() {
          if constexpr (FRUSTUM && SPH) {
            {
                const double aspect = (double)a.cam.w / (double)a.cam.h;
                const int cx = max(min(px, a.cam.w - 1), 0), cy = max(min(py, a.cam.h - 1), 0);
                sxl = (float)(((2.0 * cx + 1.0) / (double)a.cam.w - 1.0) * a.cam.tan_half * aspect);
                syl = (float)((1.0 - (2.0 * cy + 1.0) / (double)a.cam.h) * a.cam.tan_half);
            }
            // the tile's four side planes, as for the breadth-first walk
            const int tw = a.tile_w;
            const int corner[4] = {rg.y0 * tw + rg.x0, rg.y0 * tw + rg.x1 - 1, (rg.y1 - 1) * tw + rg.x1 - 1,
                                   (rg.y1 - 1) * tw + rg.x0};
            double cd[4][3];
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int k = 0; k < 3; ++k) cd[c][k] = __shfl(ray.d[k], corner[c], kWave);
            const double cen[3] = {cd[0][0] + cd[1][0] + cd[2][0] + cd[3][0], cd[0][1] + cd[1][1] + cd[2][1] + cd[3][1],
                                   cd[0][2] + cd[1][2] + cd[2][2] + cd[3][2]};
            float pp[4][3], pn[4][3], pc[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double *u = cd[i], *v = cd[(i + 1) & 3];
                double n0 = u[1] * v[2] - u[2] * v[1], n1 = u[2] * v[0] - u[0] * v[2], n2 = u[0] * v[1] - u[1] * v[0];
                const double len = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
                const double sg = (n0 * cen[0] + n1 * cen[1] + n2 * cen[2]) < 0.0 ? -1.0 : 1.0;
                const double inv = len > 1e-300 ? sg / len : 0.0;
                const float f0 = (float)(n0 * inv), f1 = (float)(n1 * inv), f2 = (float)(n2 * inv);
                pp[i][0] = fmaxf(f0, 0.0f); pp[i][1] = fmaxf(f1, 0.0f); pp[i][2] = fmaxf(f2, 0.0f);
                pn[i][0] = fminf(f0, 0.0f); pn[i][1] = fminf(f1, 0.0f); pn[i][2] = fminf(f2, 0.0f);
                pc[i] = (float)(-((double)f0 * eye.o[0] + (double)f1 * eye.o[1] + (double)f2 * eye.o[2]));
            }
            const float slack = 4.0f * eye.E;
            const float bR[3] = {(float)a.cam.right[0], (float)a.cam.right[1], (float)a.cam.right[2]};
            const float bU[3] = {(float)a.cam.up[0], (float)a.cam.up[1], (float)a.cam.up[2]};
            const float bF[3] = {(float)a.cam.fwd[0], (float)a.cam.fwd[1], (float)a.cam.fwd[2]};
            auto wave_max = [](float v) {
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
                return v;
            };
            float wmax = wave_max(pr_f);  // lanes taking no part hold -inf
            // The chunk's screening: the point of the capsule's screen segment
            // nearest the pixel, to the rounding of its parameter (an error far
            // inside the slack); a segment whose squared length underflows gives
            // a NaN or infinite parameter, which the clamp turns into an end
            // point, and any of its points will do.  Then the chunk is tested
            // before it is overwritten.
            auto chunk_pass = [&](uint32_t n) {
                from_chunk = true;
                for (uint32_t j = 0; j < n; j += kCandGroup) {
                    float4 dc[kCandGroup], sg[kCandGroup];
#pragma unroll
                    for (int u = 0; u < kCandGroup; ++u) {
                        const uint32_t i = min(j + (uint32_t)u, n - 1u);
                        dc[u] = L.fr.scr[i];
                        sg[u] = L.fr.seg[i];
                    }
#pragma unroll
                    for (int u = 0; u < kCandGroup; ++u) {
                        float du = sxl - dc[u].x, dv = syl - dc[u].y;
                        const float l2 = fmaf(sg[u].x, sg[u].x, sg[u].y * sg[u].y);
                        const float w = fminf(fmaxf(fmaf(du, sg[u].x, dv * sg[u].y) * __builtin_amdgcn_rcpf(l2), 0.0f),
                                              1.0f);
                        du = fmaf(-w, sg[u].x, du);
                        dv = fmaf(-w, sg[u].y, dv);
                        const bool may = (j + u < n) & (fmaf(du, du, dv * dv) <= dc[u].z) & (dc[u].w <= pr_f) &
                                         (sg[u].z >= lo_f);
                        L.cand[nc][lane] = j + (uint32_t)u;
                        nc += may ? 1u : 0u;
                    }
                    if (__ballot(nc > (uint32_t)(kQueue - kCandGroup))) flush();
                }
                if (__ballot(nc > 0u)) flush();
                from_chunk = false;
                wmax = wave_max(pr_f);
            };
            uint32_t top = __ballot(active) ? 1u : 0u;  // wave-uniform
            if (lane == 0) L.fr.stack[0] = 0u;          // the root
            uint32_t n_chunk = 0, visits = 0;
            while (top > 0u) {
                __builtin_amdgcn_wave_barrier();
                const uint32_t take = min(top, (uint32_t)kWave / 4u);
                // a pass visits every node at most once; more visits only
                // occur in a corrupt hierarchy
                visits += take;
                if (visits > n_nodes + (uint32_t)kWave) {
                    fb = true;
                    break;
                }
                const uint32_t base = top - take;
                const uint32_t i = (uint32_t)lane / 4u, sl = (uint32_t)lane & 3u;
                const bool valid = i < take;
                const uint32_t node = valid ? min(L.fr.stack[base + i], n_nodes - 1) : 0u;
                top = base;
                const float *f = nodes[node].f;
                const uint32_t kinds = valid ? __float_as_uint(f[31]) : 0u;
                const bool is_leaf = (kinds >> sl) & 1u, is_int = (kinds >> (4u + sl)) & 1u;
                const float *q = f + 6 * sl;
                const float q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3], q4 = q[4], q5 = q[5];
                const uint32_t ref = __float_as_uint(f[24 + sl]);
                const uint32_t id = ref & ~kLeafBit;
                // an id beyond the set is never tested (only a corrupt or
                // mismatched hierarchy has one)
                bool pass = is_int || (is_leaf && id < n_spheres);
#pragma unroll
                for (int pl = 0; pl < 4; ++pl) {
                    // box: its corner farthest along the normal; spheroid: the
                    // ball of radius max(r, h) around its centre
                    const float bx = fmaf(pp[pl][0], q3, fmaf(pn[pl][0], q0, pc[pl]));
                    const float vb = fmaf(pp[pl][2], q5, fmaf(pn[pl][2], q2, fmaf(pp[pl][1], q4, fmaf(pn[pl][1], q1, bx))));
                    const float vs = fmaf(pp[pl][0] + pn[pl][0], q0, fmaf(pp[pl][1] + pn[pl][1], q1,
                                     fmaf(pp[pl][2] + pn[pl][2], q2, pc[pl]))) + fmaxf(q3, q5);
                    pass = pass && (is_leaf ? vs : vb) >= -slack;
                }
                if (pass && is_int) {
                    // the eye's distance to the box bounds every entry in it
                    const float ex = fmaxf(fmaxf(q0 - eye.of[0], eye.of[0] - q3), 0.0f);
                    const float ey = fmaxf(fmaxf(q1 - eye.of[1], eye.of[1] - q4), 0.0f);
                    const float ez = fmaxf(fmaxf(q2 - eye.of[2], eye.of[2] - q5), 0.0f);
                    pass = sqrtf(ex * ex + ey * ey + ez * ez) * (1.0f - 0x1p-20f) - slack <= wmax;
                }
                // a spheroid with h > r lies in the capsule of radius r around
                // the segment c +- (h - r) u (at a distance x from c along u its
                // half-width r sqrt(1 - x^2 / h^2) stays within the capsule's);
                // the capsule meets the half-space of a plane with unit normal n
                // when n.c + (h - r)|n.u| + r does, with margins for the float
                // axis and end points.  A sample with 0 < h <= r lies in its ball.
                float4 ua = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                float u0 = 0.0f, u1 = 0.0f, u2 = 0.0f, ha = 0.0f;
                if (pass && is_leaf && q5 > 0.0f) {
                    ua = a.axis[id];
                    if (q5 > q3) {
                        const float il = rsqrtf(fmaf(ua.x, ua.x, fmaf(ua.y, ua.y, ua.z * ua.z)));
                        u0 = ua.x * il;
                        u1 = ua.y * il;
                        u2 = ua.z * il;
                        ha = q5 - q3;
                        const float rr = q3 + eye.E + ha * 0x1p-20f;
#pragma unroll
                        for (int pl = 0; pl < 4; ++pl) {
                            const float n0 = pp[pl][0] + pn[pl][0], n1 = pp[pl][1] + pn[pl][1],
                                        n2 = pp[pl][2] + pn[pl][2];
                            const float sc = fmaf(n0, q0, fmaf(n1, q1, fmaf(n2, q2, pc[pl])));
                            const float nu = fabsf(fmaf(n0, u0, fmaf(n1, u1, n2 * u2)));
                            pass = pass && fmaf(ha, nu, sc + rr) >= -slack;
                        }
                    }
                }
                const uint64_t mi = __ballot(pass && is_int), ml = __ballot(pass && is_leaf);
                const uint32_t below_i = (uint32_t)__popcll(mi & ((1ull << lane) - 1ull));
                const uint32_t below_l = (uint32_t)__popcll(ml & ((1ull << lane) - 1ull));
                if (pass && is_int && top + below_i < kStackS) L.fr.stack[top + below_i] = ref;
                if (pass && is_leaf) {
                    // n_chunk <= kChunk - 64 here: a fuller chunk is tested first.
                    // The screen capsule: the balls of radius rr centred on the
                    // segment project into discs whose centres run along the
                    // screen segment between the projected end points A, B and
                    // whose radii rr sqrt(1 + X^2 + Y^2) / (z - rr) are convex
                    // along it (z is affine in the segment's parameter, 1 / z
                    // affine along the screen segment), so at most the larger of
                    // the two ends' radii, the smaller z and the larger
                    // sqrt(1 + X^2 + Y^2) taken together.  Depths: the entry lies
                    // no nearer than the eye's distance to the segment minus rr,
                    // and no farther than dist + max(r, h).  A sample with h <= r
                    // is the capsule with ha = 0.
                    const uint32_t slot = n_chunk + below_l;
                    const float ox = q0 - eye.of[0], oy = q1 - eye.of[1], oz = q2 - eye.of[2];
                    const float x = ox * bR[0] + oy * bR[1] + oz * bR[2];
                    const float y = ox * bU[0] + oy * bU[1] + oz * bU[2];
                    const float z = ox * bF[0] + oy * bF[1] + oz * bF[2];
                    const float dist = sqrtf(ox * ox + oy * oy + oz * oz);
                    const float rr = q3 + eye.E + ha * 0x1p-20f;
                    const float ux = u0 * bR[0] + u1 * bR[1] + u2 * bR[2];
                    const float uy = u0 * bU[0] + u1 * bU[1] + u2 * bU[2];
                    const float uz = u0 * bF[0] + u1 * bF[1] + u2 * bF[2];
                    const float xa = fmaf(-ha, ux, x), ya = fmaf(-ha, uy, y), za = fmaf(-ha, uz, z);
                    const float xb = fmaf(ha, ux, x), yb = fmaf(ha, uy, y), zb = fmaf(ha, uz, z);
                    const float zr = fminf(za, zb) - rr;
                    float Xa = 0.0f, Ya = 0.0f, rho2 = INFINITY, dX = 0.0f, dY = 0.0f;
                    if (zr > 0x1p-10f * dist && zr > 0x1p-100f) {
                        // the hardware reciprocal and square root (a few ulps on
                        // normal operands) stay far inside the slack below
                        const float ia = __builtin_amdgcn_rcpf(za), ib = __builtin_amdgcn_rcpf(zb);
                        Xa = xa * ia;
                        Ya = ya * ia;
                        const float Xb = xb * ib, Yb = yb * ib;
                        const float m2 = fmaxf(1.0f + Xa * Xa + Ya * Ya, 1.0f + Xb * Xb + Yb * Yb);
                        const float rho = rr * __builtin_amdgcn_sqrtf(m2) * __builtin_amdgcn_rcpf(zr);
                        const float rs = rho * (1.0f + 0x1p-12f) +
                                         0x1p-18f * (1.0f + fmaxf(fabsf(Xa), fabsf(Xb)) + fmaxf(fabsf(Ya), fabsf(Yb)));
                        rho2 = rs * rs;
                        dX = Xb - Xa;
                        dY = Yb - Ya;
                    }
                    const float sd = fminf(fmaxf(-(ox * u0 + oy * u1 + oz * u2), -ha), ha);
                    const float wx = fmaf(sd, u0, ox), wy = fmaf(sd, u1, oy), wz = fmaf(sd, u2, oz);
                    const float dmin = sqrtf(wx * wx + wy * wy + wz * wz);
                    const float tmin = (dmin - rr) * (1.0f - 0x1p-20f) - slack;
                    const float tmax = (dist + fmaxf(q3, q5) + eye.E) * (1.0f + 0x1p-20f) + slack;
                    L.fr.scr[slot] = make_float4(Xa, Ya, rho2, tmin);
                    L.fr.seg[slot] = make_float4(dX, dY, tmax, __uint_as_float(id));
                    L.fr.geo[slot] = make_float4(q0, q1, q2, q3);
                    L.fr.ax[slot] = make_float4(ua.x, ua.y, ua.z, q5);
                    L.fr.alpha[slot] = q4;
                }
                top += (uint32_t)__popcll(mi);
                n_chunk += (uint32_t)__popcll(ml);
                if (top > kStackS) {
                    fb = true;
                    break;
                }
                if (n_chunk > kChunk - (uint32_t)kWave) {
                    chunk_pass(n_chunk);
                    n_chunk = 0;
                }
            }
            if (!fb && n_chunk > 0u) chunk_pass(n_chunk);
          }
        };
        if constexpr (FRUSTUM && SPH) {
            bool partial = false;
            if (!fb) {
                frustum_dfs();
                partial = fb;
            }
            if (fb) {
                // a walk cut short has filed hits that the per-lane walk finds again
                redo = partial;
                lane_walk(SignTag<kMixedSigns>{});
                redo = partial || overflow;
            }
        } else if constexpr (FRUSTUM) {
            if (!fb) {
                cand_pass(L.fr);
            } else {
                lane_walk(SignTag<kMixedSigns>{});
                redo = overflow;
            }
        } else if constexpr (LANE && (K > 8 || SPH)) {
            // a large buffer leaves no registers for copies of the walk (and a
            // spheroid set keeps to the general one)
            lane_walk(SignTag<kMixedSigns>{});
            redo = overflow;
        } else if (LANE) {
            switch (sign_pattern) {
            case 0: lane_walk(SignTag<0>{}); break;
            case 1: lane_walk(SignTag<1>{}); break;
            case 2: lane_walk(SignTag<2>{}); break;
            case 3: lane_walk(SignTag<3>{}); break;
            case 4: lane_walk(SignTag<4>{}); break;
            case 5: lane_walk(SignTag<5>{}); break;
            case 6: lane_walk(SignTag<6>{}); break;
            case 7: lane_walk(SignTag<7>{}); break;
            default: lane_walk(SignTag<kMixedSigns>{}); break;
            }
            redo = overflow;
        }
        if (!LANE || __ballot(overflow)) {
            // Packet walk (all lanes, or the lanes whose stack overflowed): the
            // node is fetched once per wave with scalar loads and visited when
            // any taking part lane's ray meets its box.
            int sp = 0;
            uint32_t node = 0;
            // a pass visits every node at most once; the cap only matters for a
            // corrupt hierarchy, where it turns a cycle into an early exit
            for (uint32_t visits = 0; visits <= n_nodes; ++visits) {
                const WideNode *nd = nodes + node;
                float f[32];
#pragma unroll
                for (int k = 0; k < 32; ++k) f[k] = nd->f[k];
                const uint32_t kinds = __float_as_uint(f[31]);  // bits 0-3 leaf slots, 4-7 internal slots
                if (kinds & 0xfu) {
                    queue_leaves(f, node, kinds, (!LANE || overflow) ? pr_f : -INFINITY);
                    if (__ballot(nc > (uint32_t)kQueue - 4u)) flush();
                }
                uint32_t boxes = 0;  // slots whose box some lane's ray meets
                {
                    const uint32_t mine = box_hits(f, kinds, (!LANE || overflow) ? pr_f : -INFINITY);
#pragma unroll
                    for (int side = 0; side < 4; ++side)
                        if (__ballot((mine >> side) & 1u)) boxes |= 1u << side;
                }
                if (boxes) {
                    const uint32_t order = slot_order(f, neg_mask);
                    // descend into the nearest slot hit; push the others, farthest first
                    uint32_t next = kEmpty;
#pragma unroll
                    for (int i = 3; i >= 0; --i) {
                        const uint32_t o = (order >> (2 * i)) & 3u;
                        if (!((boxes >> o) & 1u)) continue;
                        if (next != kEmpty) {
                            // a wide level pushes at most 3 entries and the wide depth is
                            // at most 32 for 62-bit (code, position) keys: 128 slots suffice
                            if (sp < kStack) {
                                if (lane == 0) L.stack[sp] = next;
                                ++sp;
                            }
                        }
                        next = slot_ref(f, o);
                    }
                    node = next;
                } else {
                    if (sp == 0) break;
                    --sp;
                    node = ufirst(L.stack[sp]);
                }
                // only a corrupt hierarchy can name a node outside the array
                node = min(node, n_nodes - 1);
            }
        }
        if (__ballot(nc > 0)) flush();
        if (!active) continue;
        // the last key, where a further pass starts
        const double last_t = B.t[K - 1];
        const uint32_t last_id = B.id[K - 1];

        // ---- composite this pass
        bool done = false;
        uint32_t used = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if ((uint32_t)k < m && !done) {
                const float al = B.al[k];
                const float4 col = load_colour(a.rgba, half, B.id[k]);
                float w;
                alpha_step(al, A, T, w);
                C[0] = __fadd_rn(C[0], __fmul_rn(w, col.x));
                C[1] = __fadd_rn(C[1], __fmul_rn(w, col.y));
                C[2] = __fadd_rn(C[2], __fmul_rn(w, col.z));
                if (BWD) {
                    B.t[k] = T64;  // transmittance before hit k, for the gradients
                    T64 *= 1.0 - (double)al;
                }
                ++n_hit;
                ++used;
                if (A >= stop) done = true;
            }
        }
        const bool more = !done && m == K;
        if (BWD) {
            // sum over this pass of T_j alpha_j w_j, w_j = k_j . g_C + g_A
            double Pc = 0.0;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if ((uint32_t)k < used)
                    Pc += B.t[k] * (double)B.al[k] * wdot(load_colour(a.rgba, half, B.id[k]), g);
            if (phase == 0 && more) {
                phase = 1;  // the total G is needed: sweep the rest first
                G64 = Pc;
            } else if (phase == 1) {
                G64 += Pc;
                if (!more) {
                    // G known: start over from the first hit and emit gradients
                    phase = 2;
                    A = 0.0f; T = 1.0f; C[0] = C[1] = C[2] = 0.0f;
                    n_hit = 0; T64 = 1.0; P64 = 0.0;
                    lo_t = 0.0; lo_id = 0xffffffffu;
                    continue;
                }
            } else {
                // remainder behind this pass, composited from full transmittance
                double R = (more && T64 > 0.0) ? (G64 - (P64 + Pc)) / T64 : 0.0;
#pragma unroll
                for (int k = K - 1; k >= 0; --k) {
                    if ((uint32_t)k >= used) continue;
                    const uint32_t id = B.id[k];
                    const double al = (double)B.al[k];
                    const double Tj = B.t[k];
                    const float4 col = load_colour(a.rgba, half, id);
                    const double wj = wdot(col, g);
                    const double dal = Tj * (wj - R);
                    const double ta = Tj * al;
                    unsafeAtomicAdd(&a.d_rgb[3 * (size_t)id + 0], (float)(ta * g.x));
                    unsafeAtomicAdd(&a.d_rgb[3 * (size_t)id + 1], (float)(ta * g.y));
                    unsafeAtomicAdd(&a.d_rgb[3 * (size_t)id + 2], (float)(ta * g.z));
                    if (!soft) {
                        unsafeAtomicAdd(&a.d_alpha[id], (float)dal);
                    } else {
                        const float4 c = a.centre_radius[id];
                        const double oc0 = (double)c.x - eye.o[0], oc1 = (double)c.y - eye.o[1],
                                     oc2 = (double)c.z - eye.o[2];
                        const double b = oc0 * ray.d[0] + oc1 * ray.d[1] + oc2 * ray.d[2];
                        const double v0 = oc0 - b * ray.d[0], v1 = oc1 - b * ray.d[1], v2 = oc2 - b * ray.d[2];
                        const double q = v0 * v0 + v1 * v1 + v2 * v2;
                        const double r = (double)c.w;
                        const double u = q / (r * r);
                        const double aa = (double)col.w;
                        unsafeAtomicAdd(&a.d_alpha[id], (float)(dal * (1.0 - u) * (1.0 - u)));
                        unsafeAtomicAdd(&a.d_radius[id], (float)(dal * 4.0 * aa * (1.0 - u) * q / (r * r * r)));
                        const double cc = -dal * 4.0 * aa * (1.0 - u) / (r * r);
                        unsafeAtomicAdd(&a.d_centre[3 * (size_t)id + 0], (float)(cc * v0));
                        unsafeAtomicAdd(&a.d_centre[3 * (size_t)id + 1], (float)(cc * v1));
                        unsafeAtomicAdd(&a.d_centre[3 * (size_t)id + 2], (float)(cc * v2));
                    }
                    R = al * wj + (1.0 - al) * R;
                }
                P64 += Pc;
            }
        }
        if (more) {
            lo_t = last_t;
            lo_id = last_id;
        } else {
            active = false;
        }
    }
    if (!BWD && inside) {
        a.out[(size_t)py * a.cam.w + px] = make_float4(C[0], C[1], C[2], A);
        if (a.hits) a.hits[(size_t)py * a.cam.w + px] = n_hit;
    }
    // a hierarchy over more samples than the set holds references samples
    // beyond it (skipped, and clamped to the nodes of the smaller count)
    if (lane == 0 && ufirst(hdr->n) > a.bvh_capacity) flag_status(a.status, SPLAT_STATUS_CORRUPT);
}

// ---------------------------------------------------------------- kernels

// Tile of a block.  Consecutive blocks are dealt round robin to the 8 XCDs
// (block b runs on XCD b % 8).  Schedule 0: the image is cut into
// super-tiles of 8 x 8 tiles, dealt round robin to the XCDs; each XCD walks
// its super-tiles tile by tile, so neighbouring tiles share an L2 while
// every XCD gets a spread of the image (balanced load).  Schedule 1: each
// XCD takes one contiguous band of tiles.  Schedule 2 reads the tile of each
// block from the heaviest-first order (schedule.hip).
__device__ inline bool tile_of_block(uint32_t b, int tiles_x, int tiles_y, int schedule, int &tx, int &ty)
{
    const int xcd = (int)(b % 8), i = (int)(b / 8);
    if (schedule == 1) {
        const int tiles = tiles_x * tiles_y, per_xcd = (tiles + 7) / 8;
        const int t = xcd * per_xcd + i;
        tx = t % tiles_x;
        ty = t / tiles_x;
        return t < tiles;
    }
    const int sx_n = (tiles_x + 7) / 8, sy_n = (tiles_y + 7) / 8;
    const int s = xcd + 8 * (i / 64), w = i % 64;
    if (s >= sx_n * sy_n) return false;
    tx = (s % sx_n) * 8 + w % 8;
    ty = (s / sx_n) * 8 + w / 8;
    return tx < tiles_x && ty < tiles_y;
}

__host__ inline uint32_t blocks_for(int tiles_x, int tiles_y, int schedule)
{
    if (schedule == 1) return (uint32_t)(((tiles_x * tiles_y + 7) / 8) * 8);
    const int s = ((tiles_x + 7) / 8) * ((tiles_y + 7) / 8);
    return (uint32_t)(((s + 7) / 8) * 8 * 64);
}

template <int K, bool BWD, int WALK, bool SPH>
__global__ void __launch_bounds__(64) k_trace(TraceArgs a, int tiles_x, int tiles_y)
{
    __shared__ WaveLds<WALK == SPLAT_WALK_FRUSTUM, SPH> lds;
    int tx, ty;
    TileRegion rg = {0, a.tile_w, 0, a.tile_h};
    if (a.order) {
        // an item of the heaviest-first order: tile << 3 | part, part 4 the
        // whole tile, 0..3 one of its quadrants
        if (blockIdx.x >= a.order_items) return;
        const uint32_t item = a.order[blockIdx.x], t = item >> 3, part = item & 7u;
        if (t >= (uint32_t)(tiles_x * tiles_y)) return;
        tx = (int)(t % (uint32_t)tiles_x);
        ty = (int)(t / (uint32_t)tiles_x);
        if (part < 4u) {
            const int nx = a.tile_w >= 2 ? 2 : 1, ny = a.tile_h >= 2 ? 2 : 1;
            const int rx = (int)(part & 1u) % nx, ry = (int)(part >> 1) % ny;
            // a one-row or one-column tile has two parts; the others are empty
            if ((int)(part & 1u) >= nx || (int)(part >> 1) >= ny) return;
            rg = {rx * a.tile_w / nx, (rx + 1) * a.tile_w / nx, ry * a.tile_h / ny, (ry + 1) * a.tile_h / ny};
        }
    } else if (!tile_of_block(blockIdx.x, tiles_x, tiles_y, a.schedule, tx, ty)) {
        return;
    }
    const char *mem = static_cast<const char *>(a.bvh_mem);
    const BvhLayout L(a.layout_cap);
    const BvhHeader *hdr = reinterpret_cast<const BvhHeader *>(mem);
    const WideNode *nodes = reinterpret_cast<const WideNode *>(mem + L.wide);
    trace_tile<K, BWD, WALK, SPH>(a, nodes, hdr, tx, ty, lds, rg);
}

// Trace arguments of one job of a batch.
template <int K, int WALK>
__device__ inline TraceArgs batch_args(const splat_batch_job &j, float alpha_stop, int mode, double t_max, int tile_w,
                                       int tile_h)
{
    TraceArgs a;
    a.bvh_mem = j.bvh_mem;
    a.status = nullptr;  // a job's hierarchy is read-only here
    a.bvh_capacity = j.bvh_capacity;
    a.layout_cap = j.bvh_capacity;
    a.centre_radius = reinterpret_cast<const float4 *>(j.centre_radius);
    a.axis = nullptr;
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
    a.schedule = 0;
    a.walk = WALK;
    a.order = nullptr;
    a.order_items = 0;
    a.out = reinterpret_cast<float4 *>(j.out_rgba);
    a.hits = j.out_hits;
    a.grad = nullptr;
    a.d_rgb = a.d_alpha = a.d_radius = a.d_centre = nullptr;
    return a;
}

// Persistent batched trace: waves pull tiles from one atomic counter until
// the batch is drained.  A wave claims its next tile before it traces the
// current one, so the atomic's round trip overlaps the tile's first node
// loads; every claimed tile below the total is traced by the wave that
// claimed it, and a wave exits at its first claim at or past the total.
template <int K, int WALK>
__global__ void __launch_bounds__(64)
k_trace_batched(const splat_batch_job *__restrict__ jobs, const uint32_t *__restrict__ tile_offsets, int n_jobs,
                uint32_t total_tiles, float alpha_stop, int mode, double t_max, int tile_w, int tile_h,
                uint32_t *__restrict__ counter)
{
    __shared__ WaveLds<WALK == SPLAT_WALK_FRUSTUM> lds;
    uint32_t claim = 0;
    if (threadIdx.x == 0) claim = atomicAdd(counter, 1u);
    uint32_t item = ufirst(claim);
    int lo = 0;  // job of the wave's last tile
    for (;;) {
        if (item >= total_tiles) break;
        claim = 0;
        if (threadIdx.x == 0) claim = atomicAdd(counter, 1u);
        // job of this tile: the last offset <= item.  A wave's claims only
        // grow, so the scan starts at the job of its previous tile
        while (lo + 1 < n_jobs && tile_offsets[lo + 1] <= item) ++lo;
        const splat_batch_job &j = jobs[lo];
        TraceArgs a;
        a.bvh_mem = j.bvh_mem;
        a.status = nullptr;  // a job's hierarchy is read-only here
        a.bvh_capacity = j.bvh_capacity;
        a.layout_cap = j.bvh_capacity;
        const BvhLayout L(a.layout_cap);
        a.centre_radius = reinterpret_cast<const float4 *>(j.centre_radius);
        a.axis = nullptr;
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
        a.schedule = 0;
        a.walk = WALK;
        a.order = nullptr;
        a.order_items = 0;
        a.out = reinterpret_cast<float4 *>(j.out_rgba);
        a.hits = j.out_hits;
        a.grad = nullptr;
        a.d_rgb = a.d_alpha = a.d_radius = a.d_centre = nullptr;
        const int tiles_x = (a.cam.w + tile_w - 1) / tile_w;
        const int64_t t64 = (int64_t)item - (int64_t)tile_offsets[lo];
        const int t = t64 < 0 ? 0x7fffffff : (int)min(t64, (int64_t)0x7fffffff);
        const char *mem = static_cast<const char *>(j.bvh_mem);
        const TileRegion whole = {0, tile_w, 0, tile_h};
        trace_tile<K, false, WALK>(a, reinterpret_cast<const WideNode *>(mem + L.wide), reinterpret_cast<const BvhHeader *>(mem),
                             t % tiles_x, t / tiles_x, lds, whole);
        item = ufirst(claim);
    }
}

// Batched trace as one grid: workgroup b traces item b, the tile b minus the
// offset of its job (the last offset <= b, by binary search).  No loop and no
// counter: the kernel is compiled like the plain one.
template <int K, int WALK>
__global__ void __launch_bounds__(64)
k_trace_grid(const splat_batch_job *__restrict__ jobs, const uint32_t *__restrict__ tile_offsets, int n_jobs,
             uint32_t total_tiles, float alpha_stop, int mode, double t_max, int tile_w, int tile_h)
{
    __shared__ WaveLds<WALK == SPLAT_WALK_FRUSTUM> lds;
    const uint32_t item = blockIdx.x;
    if (item >= total_tiles) return;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (tile_offsets[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    const splat_batch_job &j = jobs[lo];
    const TraceArgs a = batch_args<K, WALK>(j, alpha_stop, mode, t_max, tile_w, tile_h);
    const BvhLayout L(a.layout_cap);
    const int tiles_x = (a.cam.w + tile_w - 1) / tile_w;
    const int t = (int)(item - min(tile_offsets[lo], item));
    const char *mem = static_cast<const char *>(j.bvh_mem);
    const TileRegion whole = {0, tile_w, 0, tile_h};
    trace_tile<K, false, WALK>(a, reinterpret_cast<const WideNode *>(mem + L.wide), reinterpret_cast<const BvhHeader *>(mem),
                               t % tiles_x, t / tiles_x, lds, whole);
}

__global__ void k_zero_counter(uint32_t *c)
{
    if (threadIdx.x == 0) *c = 0u;
}

template <bool BWD, int WALK, bool SPH = false>
static hipError_t launch_k(const TraceArgs &a, int K, dim3 grid, int tiles_x, int tiles_y, hipStream_t s)
{
    switch (K) {
    case 1: hipLaunchKernelGGL((k_trace<1, BWD, WALK, SPH>), grid, dim3(64), 0, s, a, tiles_x, tiles_y); break;
    case 2: hipLaunchKernelGGL((k_trace<2, BWD, WALK, SPH>), grid, dim3(64), 0, s, a, tiles_x, tiles_y); break;
    case 4: hipLaunchKernelGGL((k_trace<4, BWD, WALK, SPH>), grid, dim3(64), 0, s, a, tiles_x, tiles_y); break;
    case 6: hipLaunchKernelGGL((k_trace<6, BWD, WALK, SPH>), grid, dim3(64), 0, s, a, tiles_x, tiles_y); break;
    case 8: hipLaunchKernelGGL((k_trace<8, BWD, WALK, SPH>), grid, dim3(64), 0, s, a, tiles_x, tiles_y); break;
    case 16: hipLaunchKernelGGL((k_trace<16, BWD, WALK, SPH>), grid, dim3(64), 0, s, a, tiles_x, tiles_y); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_trace(const TraceArgs &args, bool backward, void *ws, hipStream_t s, hipEvent_t ev_begin,
                        hipEvent_t ev_end)
{
    TraceArgs a = args;
    const int tiles_x = (a.cam.w + a.tile_w - 1) / a.tile_w;
    const int tiles_y = (a.cam.h + a.tile_h - 1) / a.tile_h;
    a.order = nullptr;
    a.order_items = 0;
    // with few tiles every wave is resident from the start and the order
    // cannot pay for its kernels: schedule 0 then
    if (a.schedule == 2 && tiles_x * tiles_y <= kOrderMinTiles) a.schedule = 0;
    if (a.schedule == 2) {
        const hipError_t e = launch_tile_order(a, tiles_x, tiles_y, ws, s, &a.order, &a.order_items);
        if (e != hipSuccess) return e;
    }
    const dim3 grid(a.order ? a.order_items : blocks_for(tiles_x, tiles_y, a.schedule));
    // optional events bracketing the trace kernel alone (not the tile ordering)
    if (ev_begin) {
        const hipError_t e = hipEventRecord(ev_begin, s);
        if (e != hipSuccess) return e;
    }
    hipError_t e;
    if (a.axis) {
        // spheroid sets: forward only (the API refuses their backward)
        if (backward) return hipErrorInvalidValue;
        if (a.walk == SPLAT_WALK_PACKET)
            e = launch_k<false, SPLAT_WALK_PACKET, true>(a, a.kbuf, grid, tiles_x, tiles_y, s);
        else if (a.walk == SPLAT_WALK_FRUSTUM)
            e = launch_k<false, SPLAT_WALK_FRUSTUM, true>(a, a.kbuf, grid, tiles_x, tiles_y, s);
        else
            e = launch_k<false, SPLAT_WALK_LANE, true>(a, a.kbuf, grid, tiles_x, tiles_y, s);
    } else if (a.walk == SPLAT_WALK_PACKET)
        e = backward ? launch_k<true, SPLAT_WALK_PACKET>(a, a.kbuf, grid, tiles_x, tiles_y, s)
                     : launch_k<false, SPLAT_WALK_PACKET>(a, a.kbuf, grid, tiles_x, tiles_y, s);
    else if (a.walk == SPLAT_WALK_FRUSTUM)
        e = backward ? launch_k<true, SPLAT_WALK_FRUSTUM>(a, a.kbuf, grid, tiles_x, tiles_y, s)
                     : launch_k<false, SPLAT_WALK_FRUSTUM>(a, a.kbuf, grid, tiles_x, tiles_y, s);
    else
        e = backward ? launch_k<true, SPLAT_WALK_LANE>(a, a.kbuf, grid, tiles_x, tiles_y, s)
                     : launch_k<false, SPLAT_WALK_LANE>(a, a.kbuf, grid, tiles_x, tiles_y, s);
    if (e == hipSuccess && ev_end) e = hipEventRecord(ev_end, s);
    return e;
}

hipError_t launch_trace_batched(const splat_batch_job *jobs, const uint32_t *tile_offsets, int32_t n_jobs,
                                uint32_t total_tiles, const splat_trace_opts &o, int32_t waves, void *ws,
                                hipStream_t s)
{
    if (waves < 0) {
        // one workgroup per (job, tile)
        if (total_tiles == 0) return hipSuccess;
        const dim3 grid(total_tiles), block(64);
#define SPLAT_GRID(KK)                                                                                           \
    if (o.walk == SPLAT_WALK_PACKET)                                                                             \
        hipLaunchKernelGGL((k_trace_grid<KK, SPLAT_WALK_PACKET>), grid, block, 0, s, jobs, tile_offsets, n_jobs,   \
                           total_tiles, o.alpha_stop, o.mode, o.t_max, o.tile_w, o.tile_h);                      \
    else if (o.walk == SPLAT_WALK_FRUSTUM)                                                                       \
        hipLaunchKernelGGL((k_trace_grid<KK, SPLAT_WALK_FRUSTUM>), grid, block, 0, s, jobs, tile_offsets, n_jobs,  \
                           total_tiles, o.alpha_stop, o.mode, o.t_max, o.tile_w, o.tile_h);                      \
    else                                                                                                         \
        hipLaunchKernelGGL((k_trace_grid<KK, SPLAT_WALK_LANE>), grid, block, 0, s, jobs, tile_offsets, n_jobs,     \
                           total_tiles, o.alpha_stop, o.mode, o.t_max, o.tile_w, o.tile_h);
        switch (o.kbuf) {
        case 1: SPLAT_GRID(1) break;
        case 2: SPLAT_GRID(2) break;
        case 4: SPLAT_GRID(4) break;
        case 6: SPLAT_GRID(6) break;
        case 8: SPLAT_GRID(8) break;
        case 16: SPLAT_GRID(16) break;
        default: return hipErrorInvalidValue;
        }
#undef SPLAT_GRID
        return hipGetLastError();
    }
    uint32_t *counter = static_cast<uint32_t *>(ws);
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, counter);
    const dim3 grid(waves), block(64);
#define SPLAT_BATCHED(KK)                                                                                        \
    if (o.walk == SPLAT_WALK_PACKET)                                                                             \
        hipLaunchKernelGGL((k_trace_batched<KK, SPLAT_WALK_PACKET>), grid, block, 0, s, jobs, tile_offsets,      \
                           n_jobs, total_tiles, o.alpha_stop, o.mode, o.t_max, o.tile_w, o.tile_h, counter);      \
    else if (o.walk == SPLAT_WALK_FRUSTUM)                                                                       \
        hipLaunchKernelGGL((k_trace_batched<KK, SPLAT_WALK_FRUSTUM>), grid, block, 0, s, jobs, tile_offsets,     \
                           n_jobs, total_tiles, o.alpha_stop, o.mode, o.t_max, o.tile_w, o.tile_h, counter);      \
    else                                                                                                         \
        hipLaunchKernelGGL((k_trace_batched<KK, SPLAT_WALK_LANE>), grid, block, 0, s, jobs, tile_offsets,        \
                           n_jobs, total_tiles, o.alpha_stop, o.mode, o.t_max, o.tile_w, o.tile_h, counter);
    switch (o.kbuf) {
    case 1: SPLAT_BATCHED(1) break;
    case 2: SPLAT_BATCHED(2) break;
    case 4: SPLAT_BATCHED(4) break;
    case 6: SPLAT_BATCHED(6) break;
    case 8: SPLAT_BATCHED(8) break;
    case 16: SPLAT_BATCHED(16) break;
    default: return hipErrorInvalidValue;
    }
#undef SPLAT_BATCHED
    return hipGetLastError();
}

}  // namespace splat
