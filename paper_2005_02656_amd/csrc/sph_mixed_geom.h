// sph_mixed_geom.h -- the FP32 pair displacement of the mixed-precision passes.
//
// A mixed-precision position is a 32-bit fixed-point coordinate per axis.
// On a periodic axis of length L it counts 2^32 units per L from the box's
// low corner, so the difference of two coordinates taken modulo 2^32 as a
// signed integer is the minimum image (at a difference of exactly L/2 both
// images are equally near; no such pair is within reach, since 4h < L).  On
// an open axis it counts 2^31 - 1 units over the key domain's extent E and
// one more E on either side (positions packed after particles moved past the
// bounding box of the last build stay exact; an axis of zero extent takes the
// domain's largest extent for E), so every difference fits a signed integer
// as it is.  The displacement b - a along an axis is that integer, exact,
// converted to FP32 and multiplied by the FP32 unit length: three
// instructions, and relative errors of a few 2^-24 plus two units.
//
// Host and device: the kernels use it, and a host check compares it with the
// FP64 minimum image.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace sph {

// the origin, the units per length and the FP32 length of one unit for an
// axis [lo, hi); emax is the domain's largest extent (> 0), the length an
// open axis of zero extent takes
__host__ __device__ inline void fix_axis(double lo, double hi, bool per, double emax,
                                         double& origin, double& units, float& unit)
{
    const double ext = (hi - lo > 0.0) ? hi - lo : emax;
    const double len = per ? ext : 3.0 * ext;
    const double span = per ? 4294967296.0 : 2147483647.0;
    origin = per ? lo : lo - ext;
    units = span / len;
    unit = (float)(len / span);
}

// the coordinate of pos: on a periodic axis taken modulo 2^32 (any number of
// periods away), on an open one clamped to [0, 2^31 - 1]
__host__ __device__ inline uint32_t fix_coord(double pos, double origin, double units, bool per)
{
    const double t = floor((pos - origin) * units);
    if (per) return (uint32_t)(uint64_t)(int64_t)t;
    return (uint32_t)fmin(fmax(t, 0.0), 2147483647.0);
}

// the largest extent of the domain [lo, hi), 1 when every axis has zero extent
__host__ __device__ inline double fix_emax(const double lo[3], const double hi[3])
{
    double e = 0.0;
    for (int k = 0; k < 3; ++k) e = fmax(e, hi[k] - lo[k]);
    return e > 0.0 ? e : 1.0;
}

// displacement b - a along the axis
__host__ __device__ inline float fix_disp(uint32_t qa, uint32_t qb, float unit)
{
    return (float)(int32_t)(qb - qa) * unit;
}

}  // namespace sph
