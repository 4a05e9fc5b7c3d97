// Decoding of one wire sample (the bit split of codec.hip), shared by the
// decode kernel and the build that consumes the samples directly.
#pragma once

#include "common.h"

namespace splat {

// Centre and radius of sample word w: the quantisation cell's centre, and
// r_unit 2^((c - 512) / 64), in double, rounded once to float.
__device__ inline float4 decode_position(uint64_t w, double lo0, double lo1, double lo2, double size, double r_unit)
{
    const double step = size / 262144.0;
    const double x = lo0 + ((double)(w & 0x3ffffu) + 0.5) * step;
    const double y = lo1 + ((double)((w >> 18) & 0x3ffffu) + 0.5) * step;
    const double z = lo2 + ((double)((w >> 36) & 0x3ffffu) + 0.5) * step;
    const double r = r_unit * exp2(((double)(w >> 54) - 512.0) / 64.0);
    return make_float4((float)x, (float)y, (float)z, (float)r);
}

// Colour word c (RGBA8, byte 0 red) as b / 255 per channel, stored as half
// (rounded to nearest even) or float at index i of rgba.
__device__ inline void decode_colour(uint32_t c, void *rgba, int half, uint32_t i)
{
    const double k[4] = {(double)(c & 0xffu) / 255.0, (double)((c >> 8) & 0xffu) / 255.0,
                         (double)((c >> 16) & 0xffu) / 255.0, (double)(c >> 24) / 255.0};
    if (half) {
        reinterpret_cast<ushort4 *>(rgba)[i] =
            make_ushort4(half_bits_rne(k[0]), half_bits_rne(k[1]), half_bits_rne(k[2]), half_bits_rne(k[3]));
    } else {
        reinterpret_cast<float4 *>(rgba)[i] = make_float4((float)k[0], (float)k[1], (float)k[2], (float)k[3]);
    }
}

}  // namespace splat
