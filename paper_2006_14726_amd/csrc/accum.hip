// Temporal accumulation of samples across frames (Sec. 7 names it as an
// extension; the merge policy is this library's reading).  The merged set is
// the new frame's samples with age 0, then the history samples, in order, whose
// age + 1 stays within the limit and whose grid cell holds no centre of the
// new frame, each with age + 1.
//
// Five launches, all sized by capacities so they can be graph-captured:
//   clear    zero the occupancy map, one byte per cell (a fill kernel, not a
//            memset node)
//   frame    one thread per frame sample: store 1 in its cell's byte (all
//            writers store the same value, so plain stores suffice; a bit
//            map would need device-scope atomics, which cost several times
//            more here) and copy the sample to the front of out
//   count    one block per 1024 history samples: survivors per tile
//   scan     one block: exclusive prefix of the tile counts, total to ws
//   scatter  one block per tile: rank of each survivor, copy with age + 1,
//            and the merged count
// A cell is q = clamp(floor((x - lo) / size grid), 0, grid - 1) per axis in
// double, so every keep/drop decision is the definition's exactly.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace splat {

struct AccumGrid {
    double lo[3];
    double size;
    int32_t grid;
};

__device__ inline uint32_t accum_cell(const float4 c, const AccumGrid &g)
{
    const float v[3] = {c.x, c.y, c.z};
    uint32_t q3[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double q = floor(((double)v[a] - g.lo[a]) / g.size * (double)g.grid);
        if (!(q >= 0.0)) q = 0.0;  // also NaN
        if (q > (double)(g.grid - 1)) q = (double)(g.grid - 1);
        q3[a] = (uint32_t)q;
    }
    const uint32_t n = (uint32_t)g.grid;
    return (q3[2] * n + q3[1]) * n + q3[0];  // < 2^30 for grid <= 1024
}

__global__ void __launch_bounds__(kUnprojBlock) k_accum_clear(uint4 *__restrict__ map, uint32_t chunks)
{
    for (uint32_t i = blockIdx.x * kUnprojBlock + threadIdx.x; i < chunks; i += gridDim.x * kUnprojBlock)
        map[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Colour rows are copied as raw bits: 8 bytes (half4) or 16 bytes (float4).
template <bool HALF>
struct Row {
    using T = typename std::conditional<HALF, uint2, uint4>::type;
};

template <bool HALF>
__global__ void __launch_bounds__(kUnprojBlock)
k_accum_frame(const float4 *__restrict__ cr, const void *__restrict__ rgba, const uint32_t *__restrict__ src,
              const uint32_t *__restrict__ count, uint32_t cap, AccumGrid g, uint8_t *__restrict__ map,
              float4 *__restrict__ out_cr, void *__restrict__ out_rgba, uint32_t *__restrict__ out_src,
              uint8_t *__restrict__ out_age, uint32_t out_cap)
{
    using RowT = typename Row<HALF>::T;
    const uint32_t n = min(*count, cap);
    const uint32_t i = blockIdx.x * kUnprojBlock + threadIdx.x;
    const bool valid = i < n;
    const bool copy = valid && i < out_cap;
    // all loads first, so that the cell and its atomic do not wait for the copy's stores
    float4 c = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    RowT row{};
    uint32_t s = 0;
    if (valid) c = cr[i];
    if (copy) {
        row = reinterpret_cast<const RowT *>(rgba)[i];
        if (out_src) s = src[i];
    }
    // one byte per cell: every writer stores the same 1, so no atomic is needed
    if (valid) map[accum_cell(c, g)] = 1u;
    if (copy) {
        out_cr[i] = c;
        reinterpret_cast<RowT *>(out_rgba)[i] = row;
        if (out_src) out_src[i] = s;
        out_age[i] = 0;
    }
}

__device__ inline bool accum_survives(const float4 *__restrict__ cr, const uint8_t *__restrict__ age, uint32_t i,
                                      const AccumGrid &g, int max_age, const uint8_t *__restrict__ map)
{
    if ((int)age[i] + 1 > max_age) return false;
    return map[accum_cell(cr[i], g)] == 0u;
}

__global__ void __launch_bounds__(kUnprojBlock)
k_accum_count(const float4 *__restrict__ cr, const uint8_t *__restrict__ age, const uint32_t *__restrict__ count,
              uint32_t cap, AccumGrid g, int max_age, const uint8_t *__restrict__ map,
              uint32_t *__restrict__ tile_counts)
{
    const uint32_t n = count ? min(*count, cap) : 0u;
    const uint32_t base = blockIdx.x * kUnprojTile;
    int c = 0;
#pragma unroll
    for (int k = 0; k < kUnprojItems; ++k) {
        const uint32_t i = base + k * kUnprojBlock + threadIdx.x;
        if (i < n && accum_survives(cr, age, i, g, max_age, map)) ++c;
    }
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

template <bool HALF>
__global__ void __launch_bounds__(kUnprojBlock)
k_accum_scatter(const float4 *__restrict__ cr, const void *__restrict__ rgba, const uint32_t *__restrict__ src,
                const uint8_t *__restrict__ age, const uint32_t *__restrict__ count, uint32_t cap, AccumGrid g,
                int max_age, const uint8_t *__restrict__ map, const uint32_t *__restrict__ tile_offsets,
                const uint32_t *__restrict__ total, const uint32_t *__restrict__ frame_count, uint32_t frame_cap,
                float4 *__restrict__ out_cr, void *__restrict__ out_rgba, uint32_t *__restrict__ out_src,
                uint8_t *__restrict__ out_age, uint32_t out_cap, uint32_t *__restrict__ out_count)
{
    using RowT = typename Row<HALF>::T;
    __shared__ uint32_t wcount[kUnprojItems][kUnprojBlock / kWave];
    const uint32_t n = count ? min(*count, cap) : 0u;
    const uint32_t nf = min(*frame_count, frame_cap);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint64_t merged = (uint64_t)nf + *total;
        *out_count = (uint32_t)(merged < out_cap ? merged : out_cap);
    }
    const uint32_t base = blockIdx.x * kUnprojTile;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    bool keep[kUnprojItems];
    uint32_t rank_in_wave[kUnprojItems];
#pragma unroll
    for (int k = 0; k < kUnprojItems; ++k) {
        const uint32_t i = base + k * kUnprojBlock + threadIdx.x;
        keep[k] = i < n && accum_survives(cr, age, i, g, max_age, map);
        const uint64_t m = __ballot(keep[k]);
        rank_in_wave[k] = (uint32_t)__popcll(m & ((1ull << lane) - 1));
        if (lane == 0) wcount[k][wave] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    // history order inside the tile is item-major, then thread: prefix over (item, wave)
    uint64_t run = (uint64_t)nf + tile_offsets[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kUnprojItems; ++k) {
        uint64_t before = run;
        for (int w = 0; w < wave; ++w) before += wcount[k][w];
        for (int w = 0; w < kUnprojBlock / kWave; ++w) run += wcount[k][w];
        if (!keep[k]) continue;
        const uint64_t j = before + rank_in_wave[k];
        if (j >= out_cap) continue;
        const uint32_t i = base + k * kUnprojBlock + threadIdx.x;
        out_cr[j] = cr[i];
        reinterpret_cast<RowT *>(out_rgba)[j] = reinterpret_cast<const RowT *>(rgba)[i];
        if (out_src) out_src[j] = src[i];
        out_age[j] = (uint8_t)(age[i] + 1);
    }
}

template <bool HALF>
static hipError_t accumulate_launches(const splat_spheres &frame, const splat_spheres *history, const uint8_t *history_age,
                                const AccumGrid &g, int max_age, const splat_spheres &out, uint8_t *out_age,
                                const AccumLayout &L, char *w, hipStream_t s)
{
    uint8_t *map = reinterpret_cast<uint8_t *>(w + L.map);
    uint32_t *tile_counts = reinterpret_cast<uint32_t *>(w + L.tile_counts);
    uint32_t *total = reinterpret_cast<uint32_t *>(w + L.total_slot);
    const uint32_t clear_blocks = min((L.chunks + kUnprojBlock - 1) / kUnprojBlock, 8192u);
    hipLaunchKernelGGL(k_accum_clear, dim3(clear_blocks), dim3(kUnprojBlock), 0, s, reinterpret_cast<uint4 *>(map),
                       L.chunks);
    const uint32_t frame_blocks = (frame.capacity + kUnprojBlock - 1) / kUnprojBlock;
    hipLaunchKernelGGL(k_accum_frame<HALF>, dim3(frame_blocks), dim3(kUnprojBlock), 0, s,
                       reinterpret_cast<const float4 *>(frame.centre_radius), frame.rgba, frame.src_index, frame.count,
                       frame.capacity, g, map, reinterpret_cast<float4 *>(out.centre_radius), out.rgba,
                       out.src_index, out_age, out.capacity);
    const float4 *hcr = history ? reinterpret_cast<const float4 *>(history->centre_radius) : nullptr;
    const void *hrgba = history ? history->rgba : nullptr;
    const uint32_t *hsrc = history ? history->src_index : nullptr;
    const uint32_t *hcount = history ? history->count : nullptr;
    const uint32_t hcap = history ? history->capacity : 0u;
    hipLaunchKernelGGL(k_accum_count, dim3(L.tiles), dim3(kUnprojBlock), 0, s, hcr, history_age, hcount, hcap, g,
                       max_age, map, tile_counts);
    const hipError_t e = launch_tile_scan(tile_counts, L.tiles, total, s);  // also reports the launches above
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_accum_scatter<HALF>, dim3(L.tiles), dim3(kUnprojBlock), 0, s, hcr, hrgba, hsrc, history_age,
                       hcount, hcap, g, max_age, map, tile_counts, total, frame.count, frame.capacity,
                       reinterpret_cast<float4 *>(out.centre_radius), out.rgba, out.src_index, out_age, out.capacity,
                       out.count);
    return hipGetLastError();
}

hipError_t launch_accumulate(const splat_spheres &frame, const splat_spheres *history, const uint8_t *history_age,
                             const splat_accum_opts &o, const splat_spheres &out, uint8_t *out_age, void *ws,
                             hipStream_t s)
{
    AccumGrid g;
    for (int a = 0; a < 3; ++a) g.lo[a] = o.box_lo[a];
    g.size = o.box_size;
    g.grid = o.grid;
    const AccumLayout L(o.grid, history ? history->capacity : 0u);
    char *w = static_cast<char *>(ws);
    if (frame.rgba_dtype == SPLAT_F16)
        return accumulate_launches<true>(frame, history, history_age, g, o.max_age, out, out_age, L, w, s);
    return accumulate_launches<false>(frame, history, history_age, g, o.max_age, out, out_age, L, w, s);
}

}  // namespace splat
