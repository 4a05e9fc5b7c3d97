// Sample codec of the wire format between server and client (Sec. 4.1: each
// object-space sample's quantised coordinate is packed with its radius into
// 64 bits; Sec. 6: 32 bits per colour).  The paper leaves the bit split
// open; this library uses
//   word   = qx | qy << 18 | qz << 36 | c << 54,
//   q      = clamp(floor((x - lo) / size 2^18), 0, 2^18 - 1) per axis,
//            decoded at the cell centre lo + (q + 1/2) size / 2^18,
//   c      = clamp(floor(64 log2(r / r_unit) + 1/2) + 512, 0, 1023),
//            decoded as r_unit 2^((c - 512) / 64),
//   colour = RGBA8 of the straight colour and alpha, b = floor(clamp(v) 255 + 1/2),
//            byte 0 red, decoded as b / 255.
// One thread per sample; all arithmetic in double, rounded once to float on
// decode.  12 bytes per sample on the wire instead of 24 (float centre and
// radius + half colour).
#include "codec.h"
#include "common.h"
#include "kernels.h"

namespace splat {

constexpr int kCodecBlock = 256;

__device__ inline uint64_t quant18(double v, double lo, double size)
{
    const double cells = 262144.0;
    double q = floor((v - lo) / size * cells);
    if (!(q >= 0.0)) q = 0.0;  // also NaN
    if (q > cells - 1.0) q = cells - 1.0;
    return (uint64_t)q;
}

__device__ inline uint32_t byte_of(double v)
{
    v = v == v ? (v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v)) : 0.0;
    return (uint32_t)floor(v * 255.0 + 0.5);
}

__global__ void __launch_bounds__(kCodecBlock)
k_encode(const float4 *__restrict__ cr, const void *__restrict__ rgba, int half, const uint32_t *__restrict__ count,
         uint32_t cap, double lo0, double lo1, double lo2, double size, double r_unit, uint64_t *__restrict__ pos,
         uint32_t *__restrict__ col)
{
    const uint32_t n = min(*count, cap);
    const uint32_t i = blockIdx.x * kCodecBlock + threadIdx.x;
    if (i >= n) return;
    const float4 c = cr[i];
    uint64_t w = quant18(c.x, lo0, size) | quant18(c.y, lo1, size) << 18 | quant18(c.z, lo2, size) << 36;
    double code = floor(64.0 * log2((double)c.w / r_unit) + 0.5) + 512.0;
    if (!(code >= 0.0)) code = 0.0;
    if (code > 1023.0) code = 1023.0;
    pos[i] = w | (uint64_t)code << 54;
    float4 k;
    if (half) {
        const ushort4 h = reinterpret_cast<const ushort4 *>(rgba)[i];
        k = make_float4(half_to_float(h.x), half_to_float(h.y), half_to_float(h.z), half_to_float(h.w));
    } else {
        k = reinterpret_cast<const float4 *>(rgba)[i];
    }
    col[i] = byte_of(k.x) | byte_of(k.y) << 8 | byte_of(k.z) << 16 | byte_of(k.w) << 24;
}

__global__ void __launch_bounds__(kCodecBlock)
k_decode(const uint64_t *__restrict__ pos, const uint32_t *__restrict__ col, const uint32_t *__restrict__ count,
         uint32_t max_count, double lo0, double lo1, double lo2, double size, double r_unit, float4 *__restrict__ cr,
         void *__restrict__ rgba, int half, uint32_t *__restrict__ out_count)
{
    const uint32_t n = min(*count, max_count);
    const uint32_t i = blockIdx.x * kCodecBlock + threadIdx.x;
    if (i == 0) *out_count = n;
    if (i >= n) return;
    cr[i] = decode_position(pos[i], lo0, lo1, lo2, size, r_unit);
    decode_colour(col[i], rgba, half, i);
}

hipError_t launch_encode(const splat_spheres &sph, const splat_codec &c, uint64_t *pos, uint32_t *col,
                         hipStream_t s)
{
    const uint32_t blocks = sph.capacity ? (sph.capacity + kCodecBlock - 1) / kCodecBlock : 1;
    hipLaunchKernelGGL(k_encode, dim3(blocks), dim3(kCodecBlock), 0, s,
                       reinterpret_cast<const float4 *>(sph.centre_radius), sph.rgba, sph.rgba_dtype == SPLAT_F16 ? 1 : 0,
                       sph.count, sph.capacity, c.box_lo[0], c.box_lo[1], c.box_lo[2], c.box_size, c.r_unit, pos, col);
    return hipGetLastError();
}

hipError_t launch_decode(const uint64_t *pos, const uint32_t *col, const uint32_t *count, const splat_codec &c,
                         const splat_spheres &out, hipStream_t s)
{
    const uint32_t blocks = out.capacity ? (out.capacity + kCodecBlock - 1) / kCodecBlock : 1;
    hipLaunchKernelGGL(k_decode, dim3(blocks), dim3(kCodecBlock), 0, s, pos, col, count, out.capacity,
                       c.box_lo[0], c.box_lo[1], c.box_lo[2], c.box_size, c.r_unit,
                       reinterpret_cast<float4 *>(out.centre_radius), out.rgba, out.rgba_dtype == SPLAT_F16 ? 1 : 0,
                       out.count);
    return hipGetLastError();
}

}  // namespace splat
