// sph_mixed_geom.h -- the FP32 pair displacement of the mixed-precision passes.
//
// A mixed-precision position is a 32-bit fixed-point coordinate per axis,
// counted from the key domain's low corner.  On a periodic axis of length L
// there are 2^32 units per L, so the difference of two coordinates taken
// modulo 2^32 as a signed integer is the minimum image (at a difference of
// exactly L/2 both images are equally near; no such pair is within reach,
// since 4h < L).  On an open axis there are 2^31 - 1 units over the domain's
// extent, so every difference fits a signed integer as it is.  The
// displacement b - a along an axis is that integer, exact, converted to FP32
// and multiplied by the FP32 unit length: three instructions, and relative
// errors of a few 2^-24 plus two units.
//
// Host and device: the kernels use it, and a host check compares it with the
// FP64 minimum image.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace sph {

// units per length and the FP32 length of one unit for an axis [lo, hi)
// (both 0 on an axis of zero extent, where every coordinate is 0)
__host__ __device__ inline void fix_axis(double lo, double hi, bool per, double& units,
                                         float& unit)
{
    const double ext = hi - lo;
    if (!(ext > 0.0)) {
        units = 0.0;
        unit = 0.0f;
        return;
    }
    const double span = per ? 4294967296.0 : 2147483647.0;
    units = span / ext;
    unit = (float)(ext / span);
}

// the coordinate of pos: on a periodic axis taken modulo 2^32 (any number of
// periods away), on an open one clamped to [0, 2^31 - 1]
__host__ __device__ inline uint32_t fix_coord(double pos, double lo, double units, bool per)
{
    const double t = floor((pos - lo) * units);
    if (per) return (uint32_t)(uint64_t)(int64_t)t;
    return (uint32_t)fmin(fmax(t, 0.0), 2147483647.0);
}

// displacement b - a along the axis
__host__ __device__ inline float fix_disp(uint32_t qa, uint32_t qb, float unit)
{
    return (float)(int32_t)(qb - qa) * unit;
}

}  // namespace sph
