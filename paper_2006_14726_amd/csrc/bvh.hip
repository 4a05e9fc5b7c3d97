// LBVH construction over the spheres (Sec. 4.1: the client builds a linear
// BVH over the received samples).
//
//   bounds   block partial min/max of the centres
//   morton   every block folds the partials; 30-bit Morton code per centre
//            and the tile histogram of the first digit
//   sort     stable LSD radix sort of (code, id), 8-bit digits, 4 passes:
//            tile histograms -> per-digit scans -> stable LDS scatter
//   karras   radix-tree hierarchy: one thread per internal node finds its
//            key range and split from common-prefix lengths of the sorted
//            codes (ties broken by the sorted position)
//   refit    bottom-up: each leaf writes its sphere into its parent; the
//            second thread to reach a node unions the two child boxes and
//            climbs on.  The hierarchy is cut into treelets (subtrees of at
//            most kTreelet leaves, refit by one workgroup each in LDS) and
//            the top tree above them (finished by one workgroup)
//
// All sizes are read from device memory (the sphere count), so the sequence
// can be captured in a HIP graph.
#include "codec.h"
#include "common.h"
#include "kernels.h"

namespace splat {

constexpr int kBoundsBlocks = 1024;

__device__ inline float wave_min(float v)
{
    for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, kWave));
    return v;
}
__device__ inline float wave_max(float v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
    return v;
}

// Block partials of the centre box.  The first thread also sets the header's
// sphere count and empties the list of refit entries of the new hierarchy.
// DECODE: the spheres come from wire samples, decoded here into the set (as
// splat_decode_samples does) while their centres are read for the bounds.
template <bool DECODE>
__global__ void __launch_bounds__(256)
k_bounds_partial(const float4 *__restrict__ cr, const uint32_t *__restrict__ count, uint32_t cap,
                 float *__restrict__ partial, BvhHeader *__restrict__ hdr, SampleSource src, float4 *__restrict__ out_cr,
                 void *__restrict__ out_rgba, int half, uint32_t *__restrict__ out_count)
{
    const uint32_t n = min(*(DECODE ? src.count : count), cap);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        hdr->n = n;
        hdr->n_entry = 0u;
        hdr->status = 0u;
        if (DECODE) *out_count = n;
    }
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        float4 c;
        if constexpr (DECODE) {
            c = decode_position(src.pos[i], src.codec.box_lo[0], src.codec.box_lo[1], src.codec.box_lo[2],
                                src.codec.box_size, src.codec.r_unit);
            out_cr[i] = c;
            decode_colour(src.col[i], out_rgba, half, i);
        } else {
            c = cr[i];
        }
        lo[0] = fminf(lo[0], c.x); lo[1] = fminf(lo[1], c.y); lo[2] = fminf(lo[2], c.z);
        hi[0] = fmaxf(hi[0], c.x); hi[1] = fmaxf(hi[1], c.y); hi[2] = fmaxf(hi[2], c.z);
    }
    __shared__ float s[4][6];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int a = 0; a < 3; ++a) {
        lo[a] = wave_min(lo[a]);
        hi[a] = wave_max(hi[a]);
    }
    if (lane == 0)
        for (int a = 0; a < 3; ++a) { s[w][a] = lo[a]; s[w][3 + a] = hi[a]; }
    __syncthreads();
    if (threadIdx.x < 6) {
        float v = s[0][threadIdx.x];
        for (int k = 1; k < 4; ++k) v = threadIdx.x < 3 ? fminf(v, s[k][threadIdx.x]) : fmaxf(v, s[k][threadIdx.x]);
        partial[blockIdx.x * 8 + threadIdx.x] = v;
    }
}

__device__ inline uint32_t expand_bits10(uint32_t v)
{
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Morton codes of one sort tile.  Every block folds the block partials into
// the centre box itself (block 0 also stores it in the header), quantises its
// kSortTile centres to 10 bits per axis and interleaves them (bit 3k+2 of a
// code is x, 3k+1 is y, 3k is z), and writes the tile's histogram of the
// first digit, so the first sort pass needs no histogram launch.
static_assert(kBoundsBlocks <= kSortBlock, "one bound partial per thread");

__global__ void __launch_bounds__(kSortBlock)
k_morton(const float4 *__restrict__ cr, const uint32_t *__restrict__ count, uint32_t cap,
         const float *__restrict__ partial, BvhHeader *__restrict__ hdr, uint32_t *__restrict__ keys,
         uint32_t *__restrict__ vals, uint32_t *__restrict__ hist, uint32_t tiles)
{
    constexpr int kWaves = kSortBlock / kWave;
    __shared__ float s[kWaves][6];
    __shared__ float box[6];
    __shared__ uint32_t h[kSortBins];
    for (int d = threadIdx.x; d < kSortBins; d += kSortBlock) h[d] = 0;
    float v[6];
    if (threadIdx.x < kBoundsBlocks) {
        for (int k = 0; k < 6; ++k) v[k] = partial[threadIdx.x * 8 + k];
    } else {
        for (int k = 0; k < 3; ++k) { v[k] = INFINITY; v[3 + k] = -INFINITY; }
    }
    for (int k = 0; k < 3; ++k) {
        v[k] = wave_min(v[k]);
        v[3 + k] = wave_max(v[3 + k]);
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0)
        for (int k = 0; k < 6; ++k) s[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        float r = s[0][threadIdx.x];
        for (int q = 1; q < kWaves; ++q) r = threadIdx.x < 3 ? fminf(r, s[q][threadIdx.x]) : fmaxf(r, s[q][threadIdx.x]);
        box[threadIdx.x] = r;
        if (blockIdx.x == 0) {
            if (threadIdx.x < 3) hdr->cen_lo[threadIdx.x] = r;
            else hdr->cen_hi[threadIdx.x - 3] = r;
        }
    }
    __syncthreads();
    const uint32_t n = min(*count, cap);
    const uint32_t base = blockIdx.x * kSortTile;
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const uint32_t i = base + it * kSortBlock + threadIdx.x;
        if (i >= n) continue;
        const float4 c = cr[i];
        const float p[3] = {c.x, c.y, c.z};
        uint32_t q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float ext = box[3 + a] - box[a];
            const float u = ext > 0.0f ? (p[a] - box[a]) / ext : 0.0f;
            int vq = (int)(u * 1024.0f);
            q[a] = (uint32_t)(vq < 0 ? 0 : (vq > 1023 ? 1023 : vq));
        }
        const uint32_t code = (expand_bits10(q[0]) << 2) | (expand_bits10(q[1]) << 1) | expand_bits10(q[2]);
        keys[i] = code;
        vals[i] = i;
        atomicAdd(&h[code & (kSortBins - 1)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kSortBins; d += kSortBlock) hist[(size_t)d * tiles + blockIdx.x] = h[d];
}

// ---------------------------------------------------------------- radix sort

__global__ void __launch_bounds__(kSortBlock)
k_sort_hist(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ count, uint32_t cap, int shift,
            uint32_t *__restrict__ hist, uint32_t tiles)
{
    __shared__ uint32_t h[kSortBins];
    for (int d = threadIdx.x; d < kSortBins; d += kSortBlock) h[d] = 0;
    __syncthreads();
    const uint32_t n = min(*count, cap);
    const uint32_t base = blockIdx.x * kSortTile;
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const uint32_t i = base + it * kSortBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kSortBins - 1)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kSortBins; d += kSortBlock) hist[(size_t)d * tiles + blockIdx.x] = h[d];
}

// One block per digit: exclusive scan of that digit's per-tile counts (a
// contiguous row of the digit-major histogram) in place, and the digit total.
__global__ void __launch_bounds__(256)
k_scan_digits(uint32_t *__restrict__ hist, uint32_t tiles, uint32_t *__restrict__ totals)
{
    __shared__ uint32_t wsum[4];
    uint32_t *row = hist + (size_t)blockIdx.x * tiles;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < tiles; base += 1024) {
        uint32_t v[4], s = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t i = base + threadIdx.x * 4 + k;
            v[k] = i < tiles ? row[i] : 0u;
            s += v[k];
        }
        uint32_t incl = s;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(incl, off, 64);
            if (lane >= off) incl += o;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        uint32_t before = carry;
        for (int k = 0; k < w; ++k) before += wsum[k];
        uint32_t run = before + incl - s;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t i = base + threadIdx.x * 4 + k;
            if (i < tiles) row[i] = run;
            run += v[k];
        }
        carry += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Stable scatter of one tile.  Wave w owns the contiguous keys
// [base + w*64*kSortItems, +64*kSortItems), visited in 64-key rounds; lanes
// holding the same digit find each other with 8 ballots and rank by lane.
__global__ void __launch_bounds__(kSortBlock)
k_sort_scatter(const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in,
               uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out, const uint32_t *__restrict__ count,
               uint32_t cap, int shift, const uint32_t *__restrict__ hist, const uint32_t *__restrict__ totals,
               uint32_t tiles)
{
    constexpr int kWaves = kSortBlock / kWave;
    __shared__ uint32_t cnt[kWaves][kSortBins];
    __shared__ uint32_t local_start[kSortBins];
    __shared__ uint32_t global_start[kSortBins];
    __shared__ uint32_t digit_base[kSortBins];
    __shared__ uint32_t skeys[kSortTile];
    __shared__ uint32_t svals[kSortTile];

    const uint32_t n = min(*count, cap);
    const uint32_t base = blockIdx.x * kSortTile;
    if (base >= n) return;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int d = threadIdx.x; d < kWaves * kSortBins; d += kSortBlock) (&cnt[0][0])[d] = 0;
    __syncthreads();

    uint32_t key[kSortItems], val[kSortItems], rank[kSortItems];
    const uint64_t lt = (1ull << lane) - 1;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint32_t i = base + (uint32_t)(w * kSortItems + r) * kWave + lane;
        const bool ok = i < n;
        key[r] = ok ? keys_in[i] : 0u;
        val[r] = ok ? vals_in[i] : 0u;
        const uint32_t d = (key[r] >> shift) & (kSortBins - 1);
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < kSortBits; ++b) {
            const uint64_t bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t before = cnt[w][d];
        rank[r] = before + (uint32_t)__popcll(peers & lt);
        const bool leader = ok && (peers & lt) == 0;
        if (leader) cnt[w][d] = before + (uint32_t)__popcll(peers);
        if (!ok) rank[r] = 0xffffffffu;
    }
    __syncthreads();
    // digit totals: exclusive prefix over waves (in place), then over digits
    if (threadIdx.x < kSortBins) {
        const int d = threadIdx.x;
        uint32_t run = 0;
        for (int k = 0; k < kWaves; ++k) {
            const uint32_t t = cnt[k][d];
            cnt[k][d] = run;
            run += t;
        }
        local_start[d] = run;  // tile total of the digit, scanned below
        digit_base[d] = totals[d];
    }
    __syncthreads();
    if (threadIdx.x < kWave) {
        // exclusive scans over the 256 digits, by one wave, 4 digits per lane:
        // of this tile's digit totals, and of the global digit totals
        uint32_t v[4], u[4], s = 0, t = 0;
        for (int k = 0; k < 4; ++k) {
            v[k] = local_start[threadIdx.x * 4 + k];
            u[k] = digit_base[threadIdx.x * 4 + k];
            s += v[k];
            t += u[k];
        }
        uint32_t incl = s, incl2 = t;
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t o = __shfl_up(incl, off, kWave);
            const uint32_t o2 = __shfl_up(incl2, off, kWave);
            if (threadIdx.x >= (unsigned)off) { incl += o; incl2 += o2; }
        }
        uint32_t run = incl - s, run2 = incl2 - t;
        for (int k = 0; k < 4; ++k) {
            const int d = threadIdx.x * 4 + k;
            local_start[d] = run;
            global_start[d] = run2 + hist[(size_t)d * tiles + blockIdx.x];
            run += v[k];
            run2 += u[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        if (rank[r] == 0xffffffffu) continue;
        const uint32_t d = (key[r] >> shift) & (kSortBins - 1);
        const uint32_t pos = local_start[d] + cnt[w][d] + rank[r];
        skeys[pos] = key[r];
        svals[pos] = val[r];
    }
    __syncthreads();
    const uint32_t m = min((uint32_t)kSortTile, n - base);
    for (uint32_t i = threadIdx.x; i < m; i += kSortBlock) {
        const uint32_t k = skeys[i];
        const uint32_t d = (k >> shift) & (kSortBins - 1);
        const uint32_t o = global_start[d] + i - local_start[d];
        keys_out[o] = k;
        vals_out[o] = svals[i];
    }
}

// ---------------------------------------------------------------- hierarchy

// The keys around a block's nodes, staged in LDS: most nodes are low in the
// tree, and their searches stay within a few hundred positions.
constexpr int kKarrasBlock = 256;
constexpr int kKarrasHalo = 256;
constexpr int kKarrasSpan = kKarrasBlock + 2 * kKarrasHalo;

struct StagedKeys {
    const uint32_t *keys;  // all sorted keys
    const uint32_t *lds;   // keys [first, first + kKarrasSpan), where they exist
    int first;
    __device__ uint32_t operator[](int j) const
    {
        const int k = j - first;
        return (k >= 0 && k < kKarrasSpan) ? lds[k] : keys[j];
    }
};

__device__ inline int common_prefix(const StagedKeys &keys, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    const uint32_t a = keys[i], b = keys[j];
    if (a != b) return __clz(a ^ b);
    return 32 + __clz((uint32_t)i ^ (uint32_t)j);
}

__device__ inline void set_ref(Node *nodes, uint32_t node, int side, uint32_t ref)
{
    nodes[node].f[12 + side] = __uint_as_float(ref);
}

__global__ void __launch_bounds__(kKarrasBlock)
k_karras(const uint32_t *__restrict__ sorted_keys, const uint32_t *__restrict__ vals, const uint32_t *__restrict__ count,
         uint32_t cap,
         Node *__restrict__ nodes, uint32_t *__restrict__ leaf_parent, uint32_t *__restrict__ node_parent,
         uint32_t *__restrict__ leaf_ids, uint32_t *__restrict__ flags, uint2 *__restrict__ ranges,
         uint32_t *__restrict__ entries, BvhHeader *__restrict__ hdr)
{
    __shared__ uint32_t skeys[kKarrasSpan];
    const int n = (int)min(*count, cap);
    const int first = (int)blockIdx.x * kKarrasBlock - kKarrasHalo;
    for (int k = threadIdx.x; k < kKarrasSpan; k += kKarrasBlock) {
        const int j = first + k;
        skeys[k] = (j >= 0 && j < n) ? sorted_keys[j] : 0u;
    }
    __syncthreads();
    const StagedKeys keys{sorted_keys, skeys, first};
    const int i = blockIdx.x * kKarrasBlock + threadIdx.x;
    if (i < n) leaf_ids[i] = vals[i];
    if (n == 1 && i == 0) {
        // a single sphere: a root with one leaf and one empty child
        set_ref(nodes, 0, 0, kLeafBit | vals[0]);
        set_ref(nodes, 0, 1, kEmpty);
        nodes[0].f[14] = __uint_as_float(3u);
        leaf_parent[0] = 0u;
        node_parent[0] = kEmpty;
        flags[0] = 0u;
        ranges[0] = make_uint2(0u, 0u);
        entries[atomicAdd(&hdr->n_entry, 1u)] = 0u;  // the root is the one treelet
        return;
    }
    if (i >= n - 1) return;
    flags[i] = 0u;
    const int d = common_prefix(keys, n, i, i + 1) > common_prefix(keys, n, i, i - 1) ? 1 : -1;
    const int dmin = common_prefix(keys, n, i, i - d);
    int lmax = 2;
    while (common_prefix(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (common_prefix(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = common_prefix(keys, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (common_prefix(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int gamma = i + s * d + (d < 0 ? -1 : 0);
    const int lo = min(i, j), hi = max(i, j);
    ranges[i] = make_uint2((uint32_t)lo, (uint32_t)hi);
    const bool left_leaf = lo == gamma, right_leaf = hi == gamma + 1;
    set_ref(nodes, i, 0, left_leaf ? (kLeafBit | vals[gamma]) : (uint32_t)gamma);
    set_ref(nodes, i, 1, right_leaf ? (kLeafBit | vals[gamma + 1]) : (uint32_t)(gamma + 1));
    uint32_t axis = 3u;
    if (dnode < 32) axis = 2u - (uint32_t)((31 - dnode) % 3);
    nodes[i].f[14] = __uint_as_float(axis);
    if (left_leaf) leaf_parent[gamma] = (uint32_t)i << 1;
    else node_parent[gamma] = (uint32_t)i << 1;
    if (right_leaf) leaf_parent[gamma + 1] = ((uint32_t)i << 1) | 1u;
    else node_parent[gamma + 1] = ((uint32_t)i << 1) | 1u;
    if (i == 0) node_parent[0] = kEmpty;
    // Refit entries.  A node of more than kTreelet leaves belongs to the top
    // tree; each of its children that is a treelet root (an internal node of
    // at most kTreelet leaves) or a leaf is an entry of the top tree.  A root
    // of at most kTreelet leaves is itself the one treelet.
    const int size = hi - lo + 1;
    if (size > kTreelet) {
        const int lsize = gamma - lo + 1, rsize = hi - gamma;
        if (left_leaf) entries[atomicAdd(&hdr->n_entry, 1u)] = kLeafBit | (uint32_t)gamma;
        else if (lsize <= kTreelet) entries[atomicAdd(&hdr->n_entry, 1u)] = (uint32_t)gamma;
        if (right_leaf) entries[atomicAdd(&hdr->n_entry, 1u)] = kLeafBit | (uint32_t)(gamma + 1);
        else if (rsize <= kTreelet) entries[atomicAdd(&hdr->n_entry, 1u)] = (uint32_t)(gamma + 1);
    } else if (i == 0) {
        entries[atomicAdd(&hdr->n_entry, 1u)] = 0u;
    }
}

__global__ void __launch_bounds__(256) k_zero_flags(uint32_t *__restrict__ flags, const uint32_t *__restrict__ count,
                                                    uint32_t cap)
{
    const uint32_t n = min(*count, cap);
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < (n > 1 ? n - 1 : 1)) flags[i] = 0u;
}

// Box of a sample, rounded outward to float: c +- r for a sphere; for a
// spheroid (axis set: unit axis u, half-length h along it, r across) its
// exact extent along each coordinate axis, sqrt(r^2 + (h^2 - r^2) u_k^2), in
// double, then rounded outward by one more float step.
__device__ inline void leaf_box(float cx, float cy, float cz, float r, float h, const float4 *__restrict__ axis,
                                uint32_t id, float lo[3], float hi[3])
{
    const float c[3] = {cx, cy, cz};
    if (!axis) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = nextafterf(c[k] - r, -INFINITY);
            hi[k] = nextafterf(c[k] + r, INFINITY);
        }
        return;
    }
    const float4 u = axis[id];
    const double ul = sqrt((double)u.x * u.x + (double)u.y * u.y + (double)u.z * u.z);
    const double un[3] = {u.x / ul, u.y / ul, u.z / ul};
    const double rr = (double)r * r, hh = (double)h * h;
    for (int k = 0; k < 3; ++k) {
        const double e = sqrt(rr + (hh - rr) * un[k] * un[k]);
        lo[k] = nextafterf((float)((double)c[k] - e), -INFINITY);
        hi[k] = nextafterf((float)((double)c[k] + e), INFINITY);
    }
}

// Box of a child slot: the stored box of an internal child, or the sample's
// box (leaf_box) for a leaf child.
__device__ inline void slot_box(const Node &nd, int side, const float4 *__restrict__ axis, float lo[3], float hi[3])
{
    const uint32_t ref = __float_as_uint(nd.f[12 + side]);
    const float *s = nd.f + 6 * side;
    if (ref == kEmpty) {
        for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    } else if (ref & kLeafBit) {
        leaf_box(s[0], s[1], s[2], s[3], s[5], axis, ref & ~kLeafBit, lo, hi);
    } else {
        for (int a = 0; a < 3; ++a) { lo[a] = s[a]; hi[a] = s[3 + a]; }
    }
}

__device__ inline float sphere_alpha_a(const void *rgba, int half, uint32_t id)
{
    if (half) return half_to_float(reinterpret_cast<const ushort4 *>(rgba)[id].w);
    return reinterpret_cast<const float4 *>(rgba)[id].w;
}

// Box of node p from its two slots, written into its parent's slot (or the
// header for the root).  Returns the parent reference (kEmpty at the root).
__device__ inline uint32_t lift_box(Node *nodes, uint32_t p, const uint32_t *__restrict__ node_parent,
                                    const float4 *__restrict__ axis, BvhHeader *__restrict__ hdr)
{
    const Node nd = nodes[p];
    float lo0[3], hi0[3], lo1[3], hi1[3];
    slot_box(nd, 0, axis, lo0, hi0);
    slot_box(nd, 1, axis, lo1, hi1);
    float lo[3], hi[3];
    for (int k = 0; k < 3; ++k) { lo[k] = fminf(lo0[k], lo1[k]); hi[k] = fmaxf(hi0[k], hi1[k]); }
    const uint32_t pp = node_parent[p];
    if (pp == kEmpty) {
        for (int k = 0; k < 3; ++k) { hdr->scene_lo[k] = lo[k]; hdr->scene_hi[k] = hi[k]; }
        return kEmpty;
    }
    float *s = nodes[pp >> 1].f + 6 * (pp & 1u);
    s[0] = lo[0]; s[1] = lo[1]; s[2] = lo[2]; s[3] = hi[0]; s[4] = hi[1]; s[5] = hi[2];
    return pp;
}

// Refit, phase 1: one workgroup per treelet.  The internal nodes of a
// subtree whose leaves are the sorted positions lo..hi have indices in
// [lo, hi], so the treelet's arrival counters, the box of each node's first
// arrival and the parent references live in LDS, indexed from lo; the
// second-arrival handshake needs only workgroup scope.  Node slots are
// written to HBM for the wide-node gather and for phase 2.  The thread that
// finishes the treelet root writes its box into the root's parent (a node of
// the top tree) or, for a root of the whole hierarchy, into the header.
constexpr int kRefitThreads = 1024;

__global__ void __launch_bounds__(kRefitThreads)
k_refit_local(const float4 *__restrict__ cr, const float4 *__restrict__ axis, const void *__restrict__ rgba, int half,
              const uint32_t *__restrict__ count, uint32_t cap, Node *nodes, const uint32_t *__restrict__ leaf_parent,
              const uint32_t *__restrict__ node_parent, const uint32_t *__restrict__ leaf_ids,
              const uint2 *__restrict__ ranges, const uint32_t *__restrict__ entries, BvhHeader *hdr)
{
    __shared__ float lbox[kTreelet][2][6];  // child boxes of each node
    __shared__ uint32_t lcnt[kTreelet];   // arrivals per node
    __shared__ uint32_t lpar[kTreelet];   // parent references
    const uint32_t n = min(*count, cap);
    const uint32_t n_nodes = n > 1 ? n - 1 : 1;
    const uint32_t m = min(hdr->n_entry, 2 * cap);
    for (uint32_t e_i = blockIdx.x; e_i < m; e_i += gridDim.x) {
        const uint32_t r = entries[e_i];
        if ((r & kLeafBit) || r >= n_nodes) continue;  // a leaf entry of the top tree
        const uint2 rng = ranges[r];
        const uint32_t lo = rng.x, hi = min(rng.y, n - 1);
        if (lo > hi || hi - lo + 1 > (uint32_t)kTreelet) {  // only a corrupt hierarchy
            if (threadIdx.x == 0) flag_status(&hdr->status, SPLAT_STATUS_CORRUPT);
            continue;
        }
        __syncthreads();  // the previous treelet's LDS is no longer read
        for (uint32_t k = threadIdx.x; k <= hi - lo; k += kRefitThreads) {
            const uint32_t i = lo + k;
            lcnt[k] = 0u;
            lpar[k] = (i < n_nodes && n > 1) ? node_parent[i] : kEmpty;
        }
        __syncthreads();
        for (uint32_t j = lo + threadIdx.x; j <= hi; j += kRefitThreads) {
            const uint32_t id = leaf_ids[j];
            if (id >= n) continue;  // only after a refit of a hierarchy that was never built
            const float4 c = cr[id];
            const float a = sphere_alpha_a(rgba, half, id);
            // slot word 5: the spheroid's half-length along its axis (0 for a sphere)
            const float h = axis ? axis[id].w : 0.0f;
            uint32_t pp = leaf_parent[j];
            uint32_t p = pp >> 1;
            if (p >= n_nodes) continue;
            {
                float *sl = nodes[p].f + 6 * (pp & 1u);
                sl[0] = c.x; sl[1] = c.y; sl[2] = c.z; sl[3] = c.w; sl[4] = a; sl[5] = h;
            }
            if (n == 1) {
                float *sl = nodes[0].f + 6;
                for (int k = 0; k < 3; ++k) { sl[k] = INFINITY; sl[3 + k] = -INFINITY; }
                lift_box(nodes, 0, node_parent, axis, hdr);
                continue;
            }
            float bl[3], bh[3];
            leaf_box(c.x, c.y, c.z, c.w, h, axis, id, bl, bh);
            // (bl, bh) is the box of the child in slot (pp & 1) of node p
            for (;;) {
                if (p < lo || p > hi) {  // only a corrupt hierarchy leaves the treelet
                    flag_status(&hdr->status, SPLAT_STATUS_CORRUPT);
                    break;
                }
                const uint32_t lp = p - lo, side = pp & 1u;
                for (int k = 0; k < 3; ++k) {
                    lbox[lp][side][k] = bl[k];
                    lbox[lp][side][3 + k] = bh[k];
                }
                const uint32_t old = __hip_atomic_fetch_add(&lcnt[lp], 1u, __ATOMIC_ACQ_REL,
                                                            __HIP_MEMORY_SCOPE_WORKGROUP);
                // first arrival: the sibling subtree is not finished and its thread
                // continues; a count above 1 only occurs in a corrupt hierarchy
                if (old != 1u) {
                    if (old > 1u) flag_status(&hdr->status, SPLAT_STATUS_CORRUPT);
                    break;
                }
                for (int k = 0; k < 3; ++k) {
                    bl[k] = fminf(bl[k], lbox[lp][side ^ 1u][k]);
                    bh[k] = fmaxf(bh[k], lbox[lp][side ^ 1u][3 + k]);
                }
                pp = lpar[lp];
                if (pp == kEmpty) {
                    for (int k = 0; k < 3; ++k) { hdr->scene_lo[k] = bl[k]; hdr->scene_hi[k] = bh[k]; }
                    break;
                }
                const uint32_t up = pp >> 1;
                if (up >= n_nodes) break;
                float *sl = nodes[up].f + 6 * (pp & 1u);
                sl[0] = bl[0]; sl[1] = bl[1]; sl[2] = bl[2]; sl[3] = bh[0]; sl[4] = bh[1]; sl[5] = bh[2];
                if (p == r) break;  // the treelet is done; its parent is a node of the top tree
                p = up;
            }
        }
    }
}

// Refit, phase 2: one workgroup finishes the top tree.  Its entries are the
// treelet roots (boxes already written by phase 1) and the leaves hanging
// directly from top nodes.  Every top node is reached only by threads of this
// workgroup, so workgroup-scope ordering suffices; the boxes written by phase
// 1 are visible across the kernel boundary.
constexpr int kTopThreads = 1024;

// A top tree of at most 3/4 of kTopHash nodes climbs in LDS: a hash table
// keyed by node index holds each node's arrival count and the box of its
// first arrival, so the handshake needs no global round trip; each thread
// loads the next parent before its handshake.  Larger top trees climb through
// the global arrival counters.
constexpr uint32_t kTopHash = 2048;

__global__ void __launch_bounds__(kTopThreads)
k_refit_top(const float4 *__restrict__ cr, const float4 *__restrict__ axis, const void *__restrict__ rgba, int half,
            const uint32_t *__restrict__ count, uint32_t cap, Node *nodes, const uint32_t *__restrict__ leaf_parent,
            const uint32_t *__restrict__ node_parent, const uint32_t *__restrict__ leaf_ids, uint32_t *flags,
            const uint32_t *__restrict__ entries, BvhHeader *hdr)
{
    __shared__ uint32_t hkey[kTopHash], hcnt[kTopHash];
    __shared__ float hbox[kTopHash][2][6];
    const uint32_t n = min(*count, cap);
    const uint32_t n_nodes = n > 1 ? n - 1 : 1;
    const uint32_t m = min(hdr->n_entry, 2 * cap);
    // m entries hang from m - 1 top nodes
    const bool in_lds = m <= kTopHash / 4 * 3;
    if (in_lds) {
        for (uint32_t i = threadIdx.x; i < kTopHash; i += kTopThreads) {
            hkey[i] = kEmpty;
            hcnt[i] = 0u;
        }
        __syncthreads();
    }
    for (uint32_t e_i = threadIdx.x; e_i < m; e_i += kTopThreads) {
        const uint32_t e = entries[e_i];
        uint32_t pp;
        float bl[3], bh[3];
        if (e & kLeafBit) {
            const uint32_t j = e & ~kLeafBit;
            if (j >= n) continue;
            const uint32_t id = leaf_ids[j];
            if (id >= n) continue;
            const float4 c = cr[id];
            pp = leaf_parent[j];
            if ((pp >> 1) >= n_nodes) continue;
            float *sl = nodes[pp >> 1].f + 6 * (pp & 1u);
            const float h = axis ? axis[id].w : 0.0f;
            sl[0] = c.x; sl[1] = c.y; sl[2] = c.z; sl[3] = c.w; sl[4] = sphere_alpha_a(rgba, half, id);
            sl[5] = h;
            if (in_lds) leaf_box(c.x, c.y, c.z, c.w, h, axis, id, bl, bh);
        } else {
            if (e >= n_nodes) continue;
            pp = node_parent[e];
            if (pp == kEmpty) continue;  // the root treelet: phase 1 wrote the header
            if (in_lds) {
                // the treelet root's box, written into its parent's slot by phase 1
                const float *sl = nodes[pp >> 1].f + 6 * (pp & 1u);
                for (int k = 0; k < 3; ++k) { bl[k] = sl[k]; bh[k] = sl[3 + k]; }
            }
        }
        uint32_t p = pp >> 1;
        if (!in_lds) {
            while (p < n_nodes) {
                const uint32_t old = __hip_atomic_fetch_add(&flags[p], 1u, __ATOMIC_ACQ_REL,
                                                            __HIP_MEMORY_SCOPE_WORKGROUP);
                if (old != 1u) {
                    if (old > 1u) flag_status(&hdr->status, SPLAT_STATUS_CORRUPT);  // only a corrupt hierarchy
                    break;
                }
                const uint32_t up = lift_box(nodes, p, node_parent, axis, hdr);
                if (up == kEmpty) break;
                p = up >> 1;
            }
            continue;
        }
        while (p < n_nodes) {
            const uint32_t up = node_parent[p];
            uint32_t h = (p * 2654435761u) >> 21, key = kEmpty;
            for (uint32_t probe = 0; probe < kTopHash; ++probe) {
                key = atomicCAS(&hkey[h], kEmpty, p);
                if (key == kEmpty || key == p) break;
                h = (h + 1u) & (kTopHash - 1u);
            }
            if (key != kEmpty && key != p) {  // a full table: only a corrupt hierarchy
                flag_status(&hdr->status, SPLAT_STATUS_CORRUPT);
                break;
            }
            const uint32_t side = pp & 1u;
            for (int k = 0; k < 3; ++k) {
                hbox[h][side][k] = bl[k];
                hbox[h][side][3 + k] = bh[k];
            }
            // the handshake orders the LDS boxes; the global slots written
            // below are read by later kernels only
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
            const uint32_t old = __hip_atomic_fetch_add(&hcnt[h], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old != 1u) {
                if (old > 1u) flag_status(&hdr->status, SPLAT_STATUS_CORRUPT);  // only a corrupt hierarchy
                break;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
            for (int k = 0; k < 3; ++k) {
                bl[k] = fminf(bl[k], hbox[h][side ^ 1u][k]);
                bh[k] = fmaxf(bh[k], hbox[h][side ^ 1u][3 + k]);
            }
            if (up == kEmpty) {
                for (int k = 0; k < 3; ++k) { hdr->scene_lo[k] = bl[k]; hdr->scene_hi[k] = bh[k]; }
                break;
            }
            float *sl = nodes[up >> 1].f + 6 * (up & 1u);
            sl[0] = bl[0]; sl[1] = bl[1]; sl[2] = bl[2]; sl[3] = bh[0]; sl[4] = bh[1]; sl[5] = bh[2];
            pp = up;
            p = up >> 1;
        }
    }
}

// Wide nodes: internal node X gathers the slots of its internal children (its
// grandchildren) and keeps its leaf children, so that the traversal descends
// two levels per node fetch.  Runs after every refit (it copies boxes).
__global__ void __launch_bounds__(256)
k_gather_wide(const uint32_t *__restrict__ count, uint32_t cap, const Node *__restrict__ nodes,
              WideNode *__restrict__ wide)
{
    const uint32_t n = min(*count, cap);
    const uint32_t n_nodes = n > 1 ? n - 1 : 1;
    const uint32_t x = blockIdx.x * 256 + threadIdx.x;
    if (n == 0 || x >= n_nodes) return;
    const Node X = nodes[x];
    float w[32];
    w[28] = X.f[14];
    for (int c = 0; c < 2; ++c) {
        const uint32_t ref = __float_as_uint(X.f[12 + c]);
        if (ref != kEmpty && !(ref & kLeafBit) && ref < n_nodes) {
            const Node C = nodes[ref];
            for (int k = 0; k < 12; ++k) w[12 * c + k] = C.f[k];
            w[24 + 2 * c] = C.f[12];
            w[25 + 2 * c] = C.f[13];
            w[29 + c] = C.f[14];
        } else {
            for (int k = 0; k < 6; ++k) w[12 * c + k] = X.f[6 * c + k];
            for (int k = 6; k < 12; ++k) w[12 * c + k] = 0.0f;
            w[24 + 2 * c] = __uint_as_float(ref == kEmpty || (ref & kLeafBit) ? ref : kEmpty);
            w[25 + 2 * c] = __uint_as_float(kEmpty);
            w[29 + c] = __uint_as_float(3u);
        }
    }
    uint32_t kinds = 0;
    for (int s = 0; s < 4; ++s) {
        const uint32_t ref = __float_as_uint(w[24 + s]);
        if (ref == kEmpty) continue;
        if (ref & kLeafBit) kinds |= ((ref & ~kLeafBit) < n ? 1u : 0u) << s;
        else kinds |= (ref < n_nodes ? 1u : 0u) << (4 + s);
    }
    w[31] = __uint_as_float(kinds);
    float4 *dst = reinterpret_cast<float4 *>(wide + x);
    for (int k = 0; k < 8; ++k) dst[k] = make_float4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
}

// The top cut (CutEntry), by one wave once the wide nodes are written: three
// levels of expansion from the root, sixteen nodes at a time with one slot
// per lane; sphere slots and the slots of the third level are emitted in
// lane order.
__global__ void __launch_bounds__(64)
k_cut(const uint32_t *__restrict__ count, uint32_t cap, const WideNode *__restrict__ wide, CutEntry *__restrict__ cut,
      BvhHeader *__restrict__ hdr)
{
    __shared__ uint32_t level[2][16];
    const uint32_t n = min(*count, cap);
    const uint32_t n_nodes = n > 1 ? n - 1 : 1;
    const int lane = threadIdx.x;
    uint32_t n_level = n > 0 ? 1u : 0u, n_out = 0;
    if (lane == 0) level[0][0] = 0u;  // the root
    __syncthreads();
    for (int d = 0; d < 3; ++d) {
        const uint32_t i = (uint32_t)lane / 4u, sl = (uint32_t)lane & 3u;
        const bool valid = i < n_level;
        const uint32_t x = valid ? min(level[d & 1][i], n_nodes - 1) : 0u;
        const float *f = wide[x].f;
        const uint32_t kinds = valid ? __float_as_uint(f[31]) : 0u;
        const bool is_leaf = (kinds >> sl) & 1u, is_int = (kinds >> (4u + sl)) & 1u;
        const bool expand = is_int && d < 2, emit = is_leaf || (is_int && d == 2);
        const uint32_t ref = __float_as_uint(f[24 + sl]);
        const uint64_t me = __ballot(expand), mo = __ballot(emit);
        const uint64_t below = (1ull << lane) - 1ull;
        __syncthreads();  // this level's list is read
        if (expand) level[(d + 1) & 1][__popcll(me & below)] = ref;
        // at most 64 entries from a built hierarchy; the bound only matters
        // for a corrupt one
        const uint32_t at = n_out + (uint32_t)__popcll(mo & below);
        if (emit && at < kCut) {
            CutEntry e;
            for (int k = 0; k < 6; ++k) e.f[k] = f[6 * sl + k];
            e.f[6] = __uint_as_float(ref);
            e.f[7] = __uint_as_float((x << 2) | sl);
            cut[at] = e;
        }
        n_out = min(n_out + (uint32_t)__popcll(mo), kCut);
        n_level = (uint32_t)__popcll(me);
        __syncthreads();
    }
    if (lane == 0) hdr->n_cut = n_out;
}

// Header count of a refit (an empty sphere set traces as background) and a
// clear status word; the refit entries of the hierarchy stay.  A build sets
// both in k_bounds_partial.
__global__ void k_header_count(const uint32_t *__restrict__ count, uint32_t cap, BvhHeader *__restrict__ hdr)
{
    if (threadIdx.x == 0) {
        hdr->n = min(*count, cap);
        hdr->status = 0u;
    }
}

hipError_t launch_build(const splat_spheres &sph, const splat_bvh &bvh, bool refit_only, void *ws, hipStream_t s,
                        const SampleSource *samples)
{
    const uint32_t cap = sph.capacity;
    const BvhLayout L(bvh.capacity);
    char *mem = static_cast<char *>(bvh.mem);
    BvhHeader *hdr = reinterpret_cast<BvhHeader *>(mem + L.header);
    Node *nodes = reinterpret_cast<Node *>(mem + L.nodes);
    uint32_t *leaf_parent = reinterpret_cast<uint32_t *>(mem + L.leaf_parent);
    uint32_t *node_parent = reinterpret_cast<uint32_t *>(mem + L.node_parent);
    uint32_t *leaf_ids = reinterpret_cast<uint32_t *>(mem + L.leaf_ids);
    uint32_t *flags = reinterpret_cast<uint32_t *>(mem + L.flags);
    uint2 *ranges = reinterpret_cast<uint2 *>(mem + L.ranges);
    uint32_t *entries = reinterpret_cast<uint32_t *>(mem + L.entries);
    const float4 *cr = reinterpret_cast<const float4 *>(sph.centre_radius);
    const int half = sph.rgba_dtype == SPLAT_F16;
    const uint32_t blocks = (cap + 255) / 256 > 0 ? (cap + 255) / 256 : 1;
    // one refit workgroup per CU (its LDS takes most of the CU's); they share out the treelets
    const uint32_t refit_blocks = 256;

    if (!refit_only) {
        const BuildLayout B(cap);
        char *w = static_cast<char *>(ws);
        uint32_t *ka = reinterpret_cast<uint32_t *>(w + B.keys_a), *va = reinterpret_cast<uint32_t *>(w + B.vals_a);
        uint32_t *kb = reinterpret_cast<uint32_t *>(w + B.keys_b), *vb = reinterpret_cast<uint32_t *>(w + B.vals_b);
        uint32_t *hist = reinterpret_cast<uint32_t *>(w + B.hist);
        uint32_t *totals = reinterpret_cast<uint32_t *>(w + B.totals);
        float *partial = reinterpret_cast<float *>(w + B.partial);
        if (samples)
            hipLaunchKernelGGL(k_bounds_partial<true>, dim3(kBoundsBlocks), dim3(256), 0, s, cr, sph.count, cap, partial,
                               hdr, *samples, const_cast<float4 *>(cr), sph.rgba, half, sph.count);
        else
            hipLaunchKernelGGL(k_bounds_partial<false>, dim3(kBoundsBlocks), dim3(256), 0, s, cr, sph.count, cap,
                               partial, hdr, SampleSource{}, nullptr, nullptr, half, nullptr);
        hipLaunchKernelGGL(k_morton, dim3(B.tiles), dim3(kSortBlock), 0, s, cr, sph.count, cap, partial, hdr, ka, va,
                           hist, B.tiles);
        for (int shift = 0; shift < kMortonBits; shift += kSortBits) {
            if (shift > 0)  // the first digit's histogram comes from k_morton
                hipLaunchKernelGGL(k_sort_hist, dim3(B.tiles), dim3(kSortBlock), 0, s, ka, sph.count, cap, shift,
                                   hist, B.tiles);
            hipLaunchKernelGGL(k_scan_digits, dim3(kSortBins), dim3(256), 0, s, hist, B.tiles, totals);
            hipLaunchKernelGGL(k_sort_scatter, dim3(B.tiles), dim3(kSortBlock), 0, s, ka, va, kb, vb, sph.count, cap,
                               shift, hist, totals, B.tiles);
            uint32_t *t = ka; ka = kb; kb = t;
            t = va; va = vb; vb = t;
        }
        hipLaunchKernelGGL(k_karras, dim3(blocks), dim3(kKarrasBlock), 0, s, ka, va, sph.count, cap, nodes, leaf_parent,
                           node_parent, leaf_ids, flags, ranges, entries, hdr);
    } else {
        hipLaunchKernelGGL(k_header_count, dim3(1), dim3(64), 0, s, sph.count, cap, hdr);
        hipLaunchKernelGGL(k_zero_flags, dim3(blocks), dim3(256), 0, s, flags, sph.count, cap);
    }
    const float4 *axis = reinterpret_cast<const float4 *>(sph.axis);
    hipLaunchKernelGGL(k_refit_local, dim3(refit_blocks), dim3(kRefitThreads), 0, s, cr, axis, sph.rgba, half,
                       sph.count, cap, nodes, leaf_parent, node_parent, leaf_ids, ranges, entries, hdr);
    hipLaunchKernelGGL(k_refit_top, dim3(1), dim3(kTopThreads), 0, s, cr, axis, sph.rgba, half, sph.count, cap, nodes,
                       leaf_parent, node_parent, leaf_ids, flags, entries, hdr);
    hipLaunchKernelGGL(k_gather_wide, dim3(blocks), dim3(256), 0, s, sph.count, cap, nodes,
                       reinterpret_cast<WideNode *>(mem + L.wide));
    hipLaunchKernelGGL(k_cut, dim3(1), dim3(64), 0, s, sph.count, cap, reinterpret_cast<const WideNode *>(mem + L.wide),
                       reinterpret_cast<CutEntry *>(mem + L.cut), hdr);
    return hipGetLastError();
}

}  // namespace splat
