// sph_mixed_geom.h -- the FP32 pair displacement of the mixed-precision passes.
//
// A mixed-precision position is a cell index (of the last cell build) plus an
// FP32 offset from that cell's origin, so the displacement b - a along one
// axis is (cell difference) x (cell edge) + (offset difference), formed in
// FP32 from small numbers.  On a periodic axis of nax cells (length
// L = nax x edge) the minimum image is taken on the cell difference.  The
// half-open image interval (-L/2, L/2] of the FP64 path decides the tie at a
// cell difference of exactly nax/2: there the two images are L/2 + off and
// -L/2 + off apart, and the nearer one depends on the sign of the offset
// difference, not on the sign of the cell difference.
//
// Host and device: the kernels use it, and a host check compares it with the
// FP64 minimum image.
#pragma once

#include <hip/hip_runtime.h>

namespace sph {

__host__ __device__ inline float axis_disp(int ca, int cb, float oa, float ob, float ce, bool per,
                                           int nax)
{
    int dc = cb - ca;
    const float off = ob - oa;
    if (per) {
        const int half = nax / 2;
        if (dc > half) dc -= nax;
        else if (dc < -half) dc += nax;
        // |dc| = nax/2 (nax is even: a power of two): keep the image nearer a
        if (dc == half && off > 0.0f) dc -= nax;
        else if (dc == -half && off < 0.0f) dc += nax;
    }
    return (float)dc * ce + off;
}

}  // namespace sph
