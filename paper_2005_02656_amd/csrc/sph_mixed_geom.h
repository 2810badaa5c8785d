// sph_mixed_geom.h -- the FP32 pair displacement of the mixed-precision passes.
//
// A mixed-precision position is a cell index (of the last cell build) plus an
// FP32 offset from that cell's origin, so the displacement b - a along one
// axis is (cell difference) x (cell edge) + (offset difference), formed in
// FP32 from small numbers.  On a periodic axis of nax cells (length
// L = nax x edge) the minimum image is taken on the cell difference.  At a
// cell difference of exactly nax/2 the two images are L/2 + off and
// -L/2 + off apart, and the nearer one depends on the sign of the offset
// difference, not on the sign of the cell difference.  (With off = 0 both are
// L/2 away; no such pair is within reach, since 4h < L.)
//
// Host and device: the kernels use it, and a host check compares it with the
// FP64 minimum image.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sph {

__host__ __device__ inline float axis_disp(int ca, int cb, float oa, float ob, float ce, bool per,
                                           int nax)
{
    int dc = cb - ca;
    const float off = ob - oa;
    if (per) {
        // nax is a power of two: dc mod nax, represented in [-nax/2, nax/2)
        // when off >= 0 and in (-nax/2, nax/2] when off < 0, so that at
        // |dc| = nax/2 the image taken is the one of sign opposite to off's
        const int s = (int)(__builtin_bit_cast(uint32_t, off) >> 31);
        const int half = nax >> 1;
        dc = ((dc + half - s) & (nax - 1)) - half + s;
    }
    return (float)dc * ce + off;
}

}  // namespace sph
