// Heaviest-first tile order for the trace (schedule 2).
//
// A wave's time is set by its slowest ray, and the slow rays are the ones
// that graze the sphere sheet: they meet many boxes along a long stretch.
// Where the sheet is seen edge-on, many sphere centres project into few
// pixels, so the number of centres projecting into a tile, maximised over
// the tile's neighbourhood (a grazing ray spreads over neighbouring tiles),
// ranks the tiles by cost well enough.  Launching the heavy tiles first
// keeps them off the end of the launch, where they would run with the GPU
// mostly idle.  The order only changes when a tile runs, never what it
// computes.
//
//   zero     per-tile counts, the bucket histogram and the bucket cursors
//   count    one thread per stride-th sphere: project the centre (float;
//            only a ranking) and count it in its tile; neighbouring spheres
//            share tiles, so a wave adds once per distinct tile
//   keys     one thread per tile, 16 x 16 tiles per block through LDS:
//            neighbourhood maximum (separable) -> log bucket (bucket 0 =
//            heaviest) and the bucket histogram
//   scatter  one thread per tile: its slot in the order, buckets ascending;
//            the heaviest tiles as four quadrant items each
#include "common.h"
#include "kernels.h"

namespace splat {

constexpr int kOrderBlock = 256;
constexpr int kReach = 3;   // neighbourhood: (2 kReach + 1)^2 tiles
// Every stride-th sphere is counted (log-scale keys do not need all): a stride
// of 8, growing with the capacity beyond 2^20 spheres up to 32, so that about
// 2^17 centres are projected (measured: on 735 k spheres a stride of 16 orders
// worse; on 4.4 M spheres 32 orders as well as 8 and costs less).
constexpr uint32_t kSampleMin = 8, kSampleMax = 32;

__global__ void __launch_bounds__(kOrderBlock)
k_tile_zero(uint32_t *__restrict__ counts, uint32_t tiles, uint32_t *__restrict__ hist)
{
    const uint32_t i = blockIdx.x * kOrderBlock + threadIdx.x;
    if (i < tiles) counts[i] = 0u;
    if (i < (uint32_t)(2 * kOrderBuckets)) hist[i] = 0u;  // histogram, then cursors
}

__global__ void __launch_bounds__(kOrderBlock)
k_tile_count(const float4 *__restrict__ cr, const uint32_t *__restrict__ count, uint32_t cap, uint32_t stride, Cam cam,
             int tile_w, int tile_h, int tiles_x, int tiles_y, uint32_t *__restrict__ counts)
{
    const uint32_t n = min(*count, cap);
    const uint64_t i = ((uint64_t)blockIdx.x * kOrderBlock + threadIdx.x) * stride;
    uint32_t tile = 0xffffffffu;
    if (i < n) {
        const float4 c = cr[i];
        const float vx = c.x - (float)cam.eye[0], vy = c.y - (float)cam.eye[1], vz = c.z - (float)cam.eye[2];
        const float z = vx * (float)cam.fwd[0] + vy * (float)cam.fwd[1] + vz * (float)cam.fwd[2];
        const float th = (float)cam.tan_half, aspect = (float)cam.w / (float)cam.h;
        const float x = (vx * (float)cam.right[0] + vy * (float)cam.right[1] + vz * (float)cam.right[2]) /
                        (z * th * aspect);
        const float y = (vx * (float)cam.up[0] + vy * (float)cam.up[1] + vz * (float)cam.up[2]) / (z * th);
        const float px = (x + 1.0f) * 0.5f * (float)cam.w, py = (1.0f - y) * 0.5f * (float)cam.h;
        if (z > 0.0f && px >= 0.0f && py >= 0.0f && px < (float)cam.w && py < (float)cam.h) {
            const int tx = min((int)px / tile_w, tiles_x - 1), ty = min((int)py / tile_h, tiles_y - 1);
            tile = (uint32_t)ty * (uint32_t)tiles_x + (uint32_t)tx;
        }
    }
    // one atomic per distinct tile of the wave: the lowest pending lane adds
    // the number of pending lanes that share its tile; each round retires at
    // least that lane, so the loop ends within 64 rounds
    bool pending = tile != 0xffffffffu;
    for (uint64_t pend = __ballot(pending); pend != 0; pend = __ballot(pending)) {
        const int leader = __ffsll((unsigned long long)pend) - 1;
        const uint32_t first = __shfl(tile, leader, kWave);
        const bool mine = pending && tile == first;
        const uint64_t same = __ballot(mine);
        if (mine && (int)__lane_id() == leader) atomicAdd(&counts[first], (uint32_t)__popcll(same));
        if (mine) pending = false;
    }
}

// A block keys a kKeyTile x kKeyTile patch of tiles: the counts of the patch
// and its kReach halo go to LDS, the neighbourhood maximum is taken along x
// (into LDS), then along y.
constexpr int kKeyTile = 16;
constexpr int kKeyHalo = kKeyTile + 2 * kReach;

__global__ void __launch_bounds__(kOrderBlock)
k_tile_keys(const uint32_t *__restrict__ counts, int tiles_x, int tiles_y, uint32_t *__restrict__ bucket,
            uint32_t *__restrict__ hist)
{
    static_assert(kKeyTile * kKeyTile == kOrderBlock, "one thread per tile of the patch");
    __shared__ uint32_t h[kOrderBuckets];
    __shared__ uint32_t c[kKeyHalo][kKeyHalo];   // counts of the patch and its halo (0 outside the image)
    __shared__ uint32_t rx[kKeyHalo][kKeyTile];  // maximum along x over 2 kReach + 1 tiles
    if (threadIdx.x < (unsigned)kOrderBuckets) h[threadIdx.x] = 0u;
    const int x0 = (int)blockIdx.x * kKeyTile - kReach, y0 = (int)blockIdx.y * kKeyTile - kReach;
    for (int i = threadIdx.x; i < kKeyHalo * kKeyHalo; i += kOrderBlock) {
        const int x = x0 + i % kKeyHalo, y = y0 + i / kKeyHalo;
        c[i / kKeyHalo][i % kKeyHalo] =
            (x >= 0 && y >= 0 && x < tiles_x && y < tiles_y) ? counts[(size_t)y * tiles_x + x] : 0u;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kKeyHalo * kKeyTile; i += kOrderBlock) {
        const int row = i / kKeyTile, col = i % kKeyTile;
        uint32_t m = 0;
        for (int k = 0; k <= 2 * kReach; ++k) m = max(m, c[row][col + k]);
        rx[row][col] = m;
    }
    __syncthreads();
    const int lx = threadIdx.x % kKeyTile, ly = threadIdx.x / kKeyTile;
    const int tx = (int)blockIdx.x * kKeyTile + lx, ty = (int)blockIdx.y * kKeyTile + ly;
    if (tx < tiles_x && ty < tiles_y) {
        uint32_t key = 0;
        for (int k = 0; k <= 2 * kReach; ++k) key = max(key, rx[ly + k][lx]);
        // four buckets per octave of the key, heaviest first
        const int level = (int)(4.0f * log2f(1.0f + (float)key));
        const uint32_t b = (uint32_t)(kOrderBuckets - 1 - min(level, kOrderBuckets - 1));
        bucket[(size_t)ty * tiles_x + tx] = b;
        atomicAdd(&h[b], 1u);
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)kOrderBuckets && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Every block scans the bucket histogram itself (64 entries, one wave);
// positions are reserved per block and bucket with one atomic on the
// bucket's cursor, then handed out within the block.  The order inside a
// bucket is arbitrary.  A tile at position p < split becomes the four items
// 4p .. 4p + 3 (tile << 3 | quadrant); a later one the item p + 3 split
// (tile << 3 | 4, the whole tile).
__global__ void __launch_bounds__(kOrderBlock)
k_tile_scatter(const uint32_t *__restrict__ bucket, uint32_t tiles, uint32_t split, uint32_t *__restrict__ hist,
               uint32_t *__restrict__ order)
{
    static_assert(kOrderBuckets == kWave, "one bucket per lane");
    __shared__ uint32_t cnt[kOrderBuckets], base[kOrderBuckets], start[kOrderBuckets];
    uint32_t *cursor = hist + kOrderBuckets;
    if (threadIdx.x < (unsigned)kOrderBuckets) {
        cnt[threadIdx.x] = 0u;
        const uint32_t v = hist[threadIdx.x];
        uint32_t incl = v;
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t o = __shfl_up(incl, off, kWave);
            if ((int)threadIdx.x >= off) incl += o;
        }
        start[threadIdx.x] = incl - v;
    }
    __syncthreads();
    const uint32_t t = blockIdx.x * kOrderBlock + threadIdx.x;
    uint32_t b = 0, rank = 0;
    if (t < tiles) {
        b = bucket[t];
        rank = atomicAdd(&cnt[b], 1u);
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)kOrderBuckets && cnt[threadIdx.x])
        base[threadIdx.x] = start[threadIdx.x] + atomicAdd(&cursor[threadIdx.x], cnt[threadIdx.x]);
    __syncthreads();
    if (t < tiles) {
        const uint32_t pos = base[b] + rank;
        if (pos < split) {
            for (uint32_t q = 0; q < 4; ++q) order[4 * pos + q] = (t << 3) | q;
        } else {
            order[pos + 3 * split] = (t << 3) | 4u;
        }
    }
}

hipError_t launch_tile_order(const TraceArgs &a, int tiles_x, int tiles_y, void *ws, hipStream_t s,
                             const uint32_t **order_out, uint32_t *items_out)
{
    const uint32_t tiles = (uint32_t)tiles_x * (uint32_t)tiles_y;
    const TileOrderLayout W(tiles);
    char *w = static_cast<char *>(ws);
    uint32_t *counts = reinterpret_cast<uint32_t *>(w + W.counts);
    uint32_t *bucket = reinterpret_cast<uint32_t *>(w + W.bucket);
    uint32_t *order = reinterpret_cast<uint32_t *>(w + W.order);
    uint32_t *hist = reinterpret_cast<uint32_t *>(w + W.hist);
    const uint32_t tile_blocks = (tiles + kOrderBlock - 1) / kOrderBlock;
    const uint32_t cap = a.bvh_capacity;
    const uint32_t stride = min(max(cap >> 17, kSampleMin), kSampleMax);
    const uint32_t samples = (cap + stride - 1) / stride;
    const uint32_t sphere_blocks = samples ? (samples + kOrderBlock - 1) / kOrderBlock : 1;
    // the sphere count of the hierarchy (clamped by cap below)
    const uint32_t *n = &static_cast<const BvhHeader *>(a.bvh_mem)->n;
    hipLaunchKernelGGL(k_tile_zero, dim3(tile_blocks > 0 ? tile_blocks : 1), dim3(kOrderBlock), 0, s, counts, tiles,
                       hist);
    hipLaunchKernelGGL(k_tile_count, dim3(sphere_blocks), dim3(kOrderBlock), 0, s, a.centre_radius, n, cap, stride, a.cam,
                       a.tile_w, a.tile_h, tiles_x, tiles_y, counts);
    const dim3 key_grid((tiles_x + kKeyTile - 1) / kKeyTile, (tiles_y + kKeyTile - 1) / kKeyTile);
    hipLaunchKernelGGL(k_tile_keys, key_grid, dim3(kOrderBlock), 0, s, counts, tiles_x, tiles_y, bucket, hist);
    // quadrant items pay off only with the frustum walk, whose costly tiles
    // are the ones whose frustum meets a long stretch of the sphere sheet
    const uint32_t split = a.walk == SPLAT_WALK_FRUSTUM ? order_split(tiles) : 0u;
    hipLaunchKernelGGL(k_tile_scatter, dim3(tile_blocks), dim3(kOrderBlock), 0, s, bucket, tiles, split, hist, order);
    *order_out = order;
    *items_out = tiles + 3 * split;
    return hipGetLastError();
}

}  // namespace splat
