// Unprojection of a 2.5D RGBA + depth image into spheres (Sec. 4.1, Eq. 1),
// with stable compaction of the pixels that carry a sample (the paper moves
// zero-radius samples aside before sending; here it is a GPU scan).
//
// Three launches, all sized for width*height so they can be graph-captured:
//   count   one block per 1024-pixel tile: number of valid pixels
//   scan    one block: exclusive prefix of the tile counts, total -> *count
//   write   one block per tile: rank of each valid pixel, FP64 Eq. 1, stores
#include "common.h"
#include "kernels.h"

namespace splat {

// With a depth interval (interval policy) a pixel also needs 0 < t_lo <= t_hi, both finite.
__device__ inline bool pixel_valid(const float *__restrict__ rgba, const float *__restrict__ depth,
                                   const float *__restrict__ interval, int64_t p)
{
    const float t = depth[p];
    const float A = rgba[4 * p + 3];
    if (!(isfinite(t) && t > 0.0f && A > 0.0f)) return false;
    if (!interval) return true;
    const float2 iv = reinterpret_cast<const float2 *>(interval)[p];
    return isfinite(iv.x) && isfinite(iv.y) && iv.x > 0.0f && iv.y >= iv.x;
}

__global__ void __launch_bounds__(kUnprojBlock)
k_unproject_count(const float *__restrict__ rgba, const float *__restrict__ depth, const float *__restrict__ interval,
                  int64_t pixels, uint32_t *__restrict__ tile_counts)
{
    const int64_t base = (int64_t)blockIdx.x * kUnprojTile;
    int c = 0;
#pragma unroll
    for (int i = 0; i < kUnprojItems; ++i) {
        const int64_t p = base + i * kUnprojBlock + threadIdx.x;
        if (p < pixels && pixel_valid(rgba, depth, interval, p)) ++c;
    }
    // wave reduction, then across the 4 waves of the block
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
    __shared__ int wsum[kUnprojBlock / kWave];
    if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < kUnprojBlock / kWave; ++w) s += wsum[w];
        tile_counts[blockIdx.x] = (uint32_t)s;
    }
}

// Single block of 1024 threads: exclusive scan of `n` tile counts in place; total to *count.
__global__ void __launch_bounds__(1024) k_unproject_scan(uint32_t *__restrict__ tile_counts, uint32_t n,
                                                         uint32_t *__restrict__ count)
{
    __shared__ uint32_t part[1024];
    const uint32_t per = (n + 1023) / 1024;
    const uint32_t lo = threadIdx.x * per, hi = min(n, lo + per);
    uint32_t s = 0;
    for (uint32_t i = lo; i < hi; ++i) s += tile_counts[i];
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over 1024 partial sums
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    for (uint32_t i = lo; i < hi; ++i) {
        const uint32_t c = tile_counts[i];
        tile_counts[i] = run;
        run += c;
    }
    if (threadIdx.x == 1023) *count = part[1023];
}

// MODE: SPLAT_RADIUS_FOOTPRINT, SPLAT_RADIUS_OPACITY, SPLAT_RADIUS_INTERVAL or
// SPLAT_RADIUS_SPHEROID (the interval's sample smeared along its ray: axis the
// unit pixel ray, half-length max(r, kappa half-interval), r the footprint)
template <bool HALF, int MODE>
__global__ void __launch_bounds__(kUnprojBlock)
k_unproject_write(Cam cam, const float *__restrict__ rgba, const float *__restrict__ depth,
                  const float *__restrict__ interval, int64_t pixels, double radius_scale, double a_floor,
                  double kappa, const uint32_t *__restrict__ tile_offsets, float4 *__restrict__ centre_radius,
                  void *__restrict__ colour, uint32_t *__restrict__ src_index, float4 *__restrict__ axis)
{
    constexpr bool ITV = MODE == SPLAT_RADIUS_INTERVAL || MODE == SPLAT_RADIUS_SPHEROID;
    __shared__ uint32_t wcount[kUnprojItems][kUnprojBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kUnprojTile;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    bool valid[kUnprojItems];
    uint32_t rank_in_wave[kUnprojItems];
#pragma unroll
    for (int i = 0; i < kUnprojItems; ++i) {
        const int64_t p = base + i * kUnprojBlock + threadIdx.x;
        valid[i] = p < pixels && pixel_valid(rgba, depth, ITV ? interval : nullptr, p);
        const uint64_t m = __ballot(valid[i]);
        rank_in_wave[i] = (uint32_t)__popcll(m & ((1ull << lane) - 1));
        if (lane == 0) wcount[i][wave] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    // pixel order inside the tile is item-major, then thread: prefix over (item, wave)
    uint32_t run = tile_offsets[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kUnprojItems; ++i) {
        uint32_t before = run;
        for (int w = 0; w < wave; ++w) before += wcount[i][w];
        for (int w = 0; w < kUnprojBlock / kWave; ++w) run += wcount[i][w];
        if (!valid[i]) continue;
        const int64_t p = base + i * kUnprojBlock + threadIdx.x;
        const uint32_t j = before + rank_in_wave[i];
        const int x = (int)(p % cam.w), y = (int)(p / cam.w);
        double d[3];
        pixel_ray(cam, x, y, d);
        double t = (double)depth[p], half_len = 0.0;
        if (ITV) {
            // the interval's midpoint replaces the depth; the sample covers kappa times its half length
            const float2 iv = reinterpret_cast<const float2 *>(interval)[p];
            t = 0.5 * ((double)iv.x + (double)iv.y);
            half_len = 0.5 * ((double)iv.y - (double)iv.x);
        }
        const float4 src = reinterpret_cast<const float4 *>(rgba)[p];
        float4 cr;
        cr.x = (float)(cam.eye[0] + d[0] * t);
        cr.y = (float)(cam.eye[1] + d[1] * t);
        cr.z = (float)(cam.eye[2] + d[2] * t);
        double r = radius_scale * (2.0 * t * cam.tan_half / (double)cam.h);
        if (MODE == SPLAT_RADIUS_OPACITY) {
            // disc area in proportion to the opacity
            const double A = (double)src.w;
            r = r * sqrt(A > a_floor ? A : a_floor);
        }
        if (MODE == SPLAT_RADIUS_INTERVAL && kappa * half_len > r) r = kappa * half_len;
        cr.w = (float)r;
        centre_radius[j] = cr;
        if (MODE == SPLAT_RADIUS_SPHEROID) {
            const double h = kappa * half_len > r ? kappa * half_len : r;
            axis[j] = make_float4((float)d[0], (float)d[1], (float)d[2], (float)h);
        }
        const double A = (double)src.w;
        double k[3] = {(double)src.x / A, (double)src.y / A, (double)src.z / A};
#pragma unroll
        for (int c = 0; c < 3; ++c) k[c] = k[c] < 0.0 ? 0.0 : (k[c] > 1.0 ? 1.0 : k[c]);
        if (HALF) {
            ushort4 h;
            h.x = half_bits_rne(k[0]);
            h.y = half_bits_rne(k[1]);
            h.z = half_bits_rne(k[2]);
            h.w = half_bits_rne(A);
            reinterpret_cast<ushort4 *>(colour)[j] = h;
        } else {
            reinterpret_cast<float4 *>(colour)[j] = make_float4((float)k[0], (float)k[1], (float)k[2], src.w);
        }
        if (src_index) src_index[j] = (uint32_t)p;
    }
}

hipError_t launch_tile_scan(uint32_t *counts, uint32_t n, uint32_t *total, hipStream_t s)
{
    hipLaunchKernelGGL(k_unproject_scan, dim3(1), dim3(1024), 0, s, counts, n, total);
    return hipGetLastError();
}

template <int MODE>
static void launch_write(const Cam &cam, const float *rgba, const float *depth, const float *interval, int64_t pixels,
                         uint32_t tiles, const splat_radius_policy &pol, const uint32_t *tile_counts,
                         const splat_spheres &out, hipStream_t s)
{
    const double rs = pol.radius_scale, fl = pol.opacity_floor, ka = pol.interval_scale;
    if (out.rgba_dtype == SPLAT_F16)
        hipLaunchKernelGGL((k_unproject_write<true, MODE>), dim3(tiles), dim3(kUnprojBlock), 0, s, cam, rgba, depth,
                           interval, pixels, rs, fl, ka, tile_counts, reinterpret_cast<float4 *>(out.centre_radius),
                           out.rgba, out.src_index, reinterpret_cast<float4 *>(out.axis));
    else
        hipLaunchKernelGGL((k_unproject_write<false, MODE>), dim3(tiles), dim3(kUnprojBlock), 0, s, cam, rgba, depth,
                           interval, pixels, rs, fl, ka, tile_counts, reinterpret_cast<float4 *>(out.centre_radius),
                           out.rgba, out.src_index, reinterpret_cast<float4 *>(out.axis));
}

hipError_t launch_unproject(const Cam &cam, const float *rgba, const float *depth, const float *interval,
                            const splat_radius_policy &policy, const splat_spheres &out, void *ws, hipStream_t s)
{
    const int64_t pixels = (int64_t)cam.w * cam.h;
    const uint32_t tiles = (uint32_t)((pixels + kUnprojTile - 1) / kUnprojTile);
    uint32_t *tile_counts = static_cast<uint32_t *>(ws);
    const float *itv =
        policy.mode == SPLAT_RADIUS_INTERVAL || policy.mode == SPLAT_RADIUS_SPHEROID ? interval : nullptr;
    hipLaunchKernelGGL(k_unproject_count, dim3(tiles), dim3(kUnprojBlock), 0, s, rgba, depth, itv, pixels,
                       tile_counts);
    hipLaunchKernelGGL(k_unproject_scan, dim3(1), dim3(1024), 0, s, tile_counts, tiles, out.count);
    switch (policy.mode) {
    case SPLAT_RADIUS_OPACITY:
        launch_write<SPLAT_RADIUS_OPACITY>(cam, rgba, depth, itv, pixels, tiles, policy, tile_counts, out, s);
        break;
    case SPLAT_RADIUS_INTERVAL:
        launch_write<SPLAT_RADIUS_INTERVAL>(cam, rgba, depth, itv, pixels, tiles, policy, tile_counts, out, s);
        break;
    case SPLAT_RADIUS_SPHEROID:
        launch_write<SPLAT_RADIUS_SPHEROID>(cam, rgba, depth, itv, pixels, tiles, policy, tile_counts, out, s);
        break;
    default:
        launch_write<SPLAT_RADIUS_FOOTPRINT>(cam, rgba, depth, itv, pixels, tiles, policy, tile_counts, out, s);
    }
    return hipGetLastError();
}

}  // namespace splat
