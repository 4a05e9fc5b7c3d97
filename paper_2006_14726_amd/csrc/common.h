// Device-side definitions shared by the splat kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "splat.h"

namespace splat {

constexpr int kWave = 64;

// ---------------------------------------------------------------- camera

// Camera as kernels see it (same fields as splat_camera, passed by value).
struct Cam {
    double eye[3], fwd[3], right[3], up[3];
    double tan_half;
    int32_t w, h;
};

__host__ inline Cam make_cam(const splat_camera &c)
{
    Cam k;
    for (int a = 0; a < 3; ++a) {
        k.eye[a] = c.eye[a];
        k.fwd[a] = c.forward[a];
        k.right[a] = c.right[a];
        k.up[a] = c.up[a];
    }
    k.tan_half = c.tan_half_fov_y;
    k.w = c.width;
    k.h = c.height;
    return k;
}

// Unit direction of the ray through the centre of pixel (x, y), in double.
__device__ inline void pixel_ray(const Cam &c, int x, int y, double d[3])
{
    const double aspect = (double)c.w / (double)c.h;
    const double sx = ((2.0 * x + 1.0) / (double)c.w - 1.0) * c.tan_half * aspect;
    const double sy = (1.0 - (2.0 * y + 1.0) / (double)c.h) * c.tan_half;
    double v0 = c.fwd[0] + sx * c.right[0] + sy * c.up[0];
    double v1 = c.fwd[1] + sx * c.right[1] + sy * c.up[1];
    double v2 = c.fwd[2] + sx * c.right[2] + sy * c.up[2];
    const double len = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    d[0] = v0 / len;
    d[1] = v1 / len;
    d[2] = v2 / len;
}

// ---------------------------------------------------------------- half

// IEEE binary16 bits of a double, round to nearest even, by integer
// manipulation of the binary64 encoding (one rounding, no float detour).
__device__ inline uint16_t half_bits_rne(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint16_t sign = (uint16_t)((b >> 48) & 0x8000u);
    const int e = (int)((b >> 52) & 0x7ff);
    uint64_t m = b & 0xfffffffffffffull;
    if (e == 0x7ff) return (uint16_t)(sign | (m ? 0x7e00u : 0x7c00u));
    if (e == 0) return sign;                 // binary64 subnormals underflow to zero
    const int E = e - 1023;                  // value = 1.m * 2^E
    if (E > 15) return (uint16_t)(sign | 0x7c00u);
    m |= 1ull << 52;                         // 53-bit significand
    int shift;                               // bits dropped from the 53-bit significand
    uint32_t exp_field;
    if (E >= -14) {
        shift = 42;                          // keep 11 bits (implicit + 10)
        exp_field = (uint32_t)(E + 15);
    } else {
        shift = 42 + (-14 - E);              // subnormal: fewer bits kept
        exp_field = 0;
        if (shift > 63) return sign;
    }
    uint64_t kept = m >> shift;
    const uint64_t rem = m & ((1ull << shift) - 1);
    const uint64_t half = 1ull << (shift - 1);
    if (rem > half || (rem == half && (kept & 1))) kept += 1;
    uint32_t bits;
    if (exp_field == 0) {
        bits = (uint32_t)kept;               // may carry into the smallest normal: still right
    } else {
        if (kept == (1ull << 11)) {          // significand overflow
            kept >>= 1;
            exp_field += 1;
            if (exp_field >= 31) return (uint16_t)(sign | 0x7c00u);
        }
        bits = (exp_field << 10) | (uint32_t)(kept & 0x3ff);
    }
    return (uint16_t)(sign | bits);
}

__device__ inline float half_to_float(uint16_t h)
{
    return (float)__builtin_bit_cast(_Float16, h);  // exact widening
}

// ---------------------------------------------------------------- BVH layout

// Child references in a node.
constexpr uint32_t kLeafBit = 0x80000000u;
constexpr uint32_t kEmpty = 0xffffffffu;

// Node: two child slots of 6 floats each, then two references and metadata.
//   internal child: lo.xyz, hi.xyz of its box (float, rounded outward)
//   leaf child:     centre.xyz, radius, alpha a, unused
//   f[12], f[13]:   child references (node index, kLeafBit | sphere id, kEmpty)
//   f[14]:          split axis of the node (0 x, 1 y, 2 z, 3 none)
struct __align__(64) Node {
    float f[16];
};

// Wide node of internal node X: the four grandchildren of X (two per internal
// child of X; a leaf child of X takes one slot and leaves the next empty).
//   f[0..23]:  four slots of 6 floats, as in Node
//   f[24..27]: slot references (binary node index of an internal grandchild,
//              whose own wide node is wide[index]; kLeafBit | sphere id; kEmpty)
//   f[28..30]: split axes of X, of X's child 0 and of X's child 1 (3 = none)
//   f[31]:     slot kinds (uint32): bit s marks slot s as a sphere of the
//              set, bit 4 + s as an internal node of the hierarchy
//   A sphere slot holds the centre, radius and opacity of the sphere (as
//   read at the last build or refit) and 0.
struct __align__(128) WideNode {
    float f[32];
};

// Top cut of the hierarchy: the slots met by expanding the root's wide node
// and the internal slots below it down to three wide levels (the slots of
// the wide nodes at depth 2, and any sphere slot above them), at most 64.
// A tile's breadth-first walk starts from the cut with one load instead of
// three dependent node fetches.
//   f[0..5]: the slot's words (a box, or a sphere's centre, radius, opacity, h)
//   f[6]:    its reference (node index, or kLeafBit | sphere id)
//   f[7]:    its origin, (wide node << 2) | slot (for the exact test)
constexpr uint32_t kCut = 64;
struct __align__(32) CutEntry {
    float f[8];
};

struct __align__(256) BvhHeader {
    uint32_t n;            // spheres at build time
    uint32_t n_entry;      // refit: entries of the top tree (treelet roots and leaves under top nodes)
    float scene_lo[3];     // box of all leaves (root box)
    float scene_hi[3];
    float cen_lo[3];       // bounds of the centres (Morton quantisation)
    float cen_hi[3];
    uint32_t status;       // SPLAT_STATUS_* bits: cleared by a build or refit, set by kernels
    uint32_t n_cut;        // entries of the top cut (CutEntry)
    uint32_t pad[48];
};
static_assert(sizeof(BvhHeader) == 256, "header size");
static_assert(offsetof(BvhHeader, status) == SPLAT_BVH_STATUS_OFFSET, "status word offset");

// Marks an impossible device state in the BVH's status word (rare paths only).
__device__ inline void flag_status(uint32_t *status, uint32_t bits)
{
    if (status) atomicOr(status, bits);
}

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Offsets inside splat_bvh.mem.
struct BvhLayout {
    size_t header, nodes, leaf_parent, node_parent, leaf_ids, flags, ranges, entries, wide, cut, total;
    __host__ __device__ explicit BvhLayout(uint32_t cap)
    {
        const size_t c = cap < 1 ? 1 : cap;
        header = 0;
        nodes = align256(sizeof(BvhHeader));
        leaf_parent = align256(nodes + c * sizeof(Node));
        node_parent = align256(leaf_parent + c * 4);
        leaf_ids = align256(node_parent + c * 4);
        flags = align256(leaf_ids + c * 4);
        ranges = align256(flags + c * 4);       // first/last sorted leaf of each internal node
        entries = align256(ranges + c * 8);     // refit entries of the top tree (at most 2 per top node)
        wide = align256(entries + c * 8);       // WideNode per internal node (what the trace reads)
        cut = align256(wide + c * sizeof(WideNode));
        total = align256(cut + kCut * sizeof(CutEntry));
    }
};

// Radix-sort layout in the build workspace.
constexpr int kSortBits = 8;
constexpr int kSortBins = 1 << kSortBits;
constexpr int kSortBlock = 1024;                 // threads per sort block
constexpr int kSortItems = 2;                    // keys per thread
constexpr int kSortTile = kSortBlock * kSortItems;
constexpr int kMortonBits = 30;

constexpr int kTreelet = 2048;                   // most leaves of a treelet (refit by one workgroup)

struct BuildLayout {
    size_t keys_a, vals_a, keys_b, vals_b, hist, partial, totals, total;
    uint32_t tiles;
    __host__ __device__ explicit BuildLayout(uint32_t cap)
    {
        const size_t c = cap < 1 ? 1 : cap;
        tiles = (uint32_t)((c + kSortTile - 1) / kSortTile);
        keys_a = 0;
        vals_a = align256(keys_a + c * 4);
        keys_b = align256(vals_a + c * 4);
        vals_b = align256(keys_b + c * 4);
        hist = align256(vals_b + c * 4);
        partial = align256(hist + (size_t)kSortBins * tiles * 4);
        totals = align256(partial + 1024 * 8 * sizeof(float));
        total = align256(totals + kSortBins * 4);
    }
};

// Trace workspace of the heaviest-first tile order (schedule 2).
constexpr int kOrderBuckets = 64;
constexpr int kOrderMinTiles = 8192;  // fewer tiles: the order is skipped (schedule 0)

// With the frustum walk, the heaviest tiles of the order are traced as four
// quadrant items each: the first order_split(tiles) tiles (1/32 of them, at
// most 1024).
__host__ __device__ inline uint32_t order_split(uint32_t tiles) { return tiles / 32 < 1024 ? tiles / 32 : 1024; }

struct TileOrderLayout {
    size_t counts, bucket, order, hist, total;
    __host__ __device__ explicit TileOrderLayout(uint32_t tiles)
    {
        const size_t t = tiles < 1 ? 1 : tiles;
        counts = 0;
        bucket = align256(counts + t * 4);
        order = align256(bucket + t * 4);
        hist = align256(order + (t + 3 * (size_t)order_split(tiles)) * 4);  // the items
        total = align256(hist + 2 * kOrderBuckets * 4);  // histogram, then cursors
    }
};

// Unprojection workspace: per-block valid counts and their exclusive scan.
constexpr int kUnprojBlock = 256;
constexpr int kUnprojItems = 4;
constexpr int kUnprojTile = kUnprojBlock * kUnprojItems;

__host__ __device__ inline size_t unproject_ws_bytes(int64_t pixels)
{
    const size_t blocks = (size_t)((pixels + kUnprojTile - 1) / kUnprojTile);
    return align256((blocks + 1) * 4);
}

// Temporal accumulation workspace: the occupancy map of the grid (one byte
// per cell, cleared in 16-byte chunks), the per-tile survivor counts of the
// history and their scan, and the survivor total.  Tiles are kUnprojTile
// history samples.
struct AccumLayout {
    size_t map, tile_counts, total_slot, total;
    uint32_t chunks, tiles;
    __host__ __device__ AccumLayout(int32_t grid, uint32_t history_capacity)
    {
        const uint64_t cells = (uint64_t)grid * (uint64_t)grid * (uint64_t)grid;
        chunks = (uint32_t)((cells + 15) / 16);
        tiles = history_capacity ? (history_capacity + kUnprojTile - 1) / kUnprojTile : 1;
        map = 0;
        tile_counts = align256(map + (size_t)chunks * 16);
        total_slot = align256(tile_counts + (size_t)tiles * 4);
        total = align256(total_slot + 4);
    }
};

}  // namespace splat
