// Host check of the mixed-precision pair displacement (sph::fix_coord,
// sph::fix_disp) against the FP64 displacement: the minimum image with the
// half-open interval (-L/2, L/2] on a periodic axis, the plain difference on
// an open one.
//
// For each axis case, particles are drawn uniformly (on a periodic axis up to
// two periods outside the box on either side, on an open one up to one extent
// outside the bounding box, as positions that left it would be; an axis of
// zero extent spreads them over the domain's extent), quantised,
// and every pair displacement the FP32 form gives is
// compared with the FP64 one.  Prints one line per case:
//   case pairs wrong worst_error_over_bound
// for the bound 4 x 2^-24 |d| + 3 units, and exits with status 1 if any pair
// took the wrong image or erred by more than the bound.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "sph_mixed_geom.h"

static uint64_t g_state = 0x9e3779b97f4a7c15ull;
static double uniform01()   // splitmix64
{
    uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1p-53;
}

struct Case {
    bool per;
    double lo, ext;
    double emax;   // the domain's largest extent (an open axis of zero extent takes it)
};

int main()
{
    const Case cases[] = {
        {true, 0.0, 1.0, 1.0},      {true, -0.5, 1.0, 1.0},   {true, 12.3, 0.37, 0.37},
        {true, -7.0, 1000.0, 1000.0}, {false, 0.0, 1.0, 1.0},  {false, -3.25, 1e-3, 1e-3},
        {false, 100.0, 1e4, 1e4},   {false, 2.0, 0.0, 0.5},
    };
    int bad_total = 0;
    for (int ci = 0; ci < (int)(sizeof(cases) / sizeof(cases[0])); ++ci) {
        const Case& c = cases[ci];
        double origin, units;
        float unit;
        sph::fix_axis(c.lo, c.lo + c.ext, c.per, c.emax, origin, units, unit);
        const double len = c.ext > 0.0 ? c.ext : c.emax;
        const int np = 600;
        double x[np];
        uint32_t q[np];
        for (int i = 0; i < np; ++i) {
            const double u = c.per ? 5.0 * uniform01() - 2.0 : 3.0 * uniform01() - 1.0;
            x[i] = c.lo + u * len;
            q[i] = sph::fix_coord(x[i], origin, units, c.per);
        }
        const double L = c.ext;
        long pairs = 0, wrong = 0;
        double worst = 0.0;
        for (int a = 0; a < np; ++a)
            for (int b = 0; b < np; ++b) {
                double d = x[b] - x[a];
                if (c.per) {
                    d -= L * floor(d / L);   // [0, L)
                    if (d > 0.5 * L) d -= L;
                    // image tie: either is right
                    if (fabs(fabs(d) - 0.5 * L) < 1e-5 * L) continue;
                }
                const float f = sph::fix_disp(q[a], q[b], unit);
                const double err = fabs((double)f - d);
                const double u1 = 1.0 / units;
                const double bound = 4.0 * 0x1p-24 * fabs(d) + 3.0 * u1;
                ++pairs;
                if (err > bound) ++wrong;
                if (err / bound > worst) worst = err / bound;
            }
        printf("%d %ld %ld %.3e\n", ci, pairs, wrong, worst);
        bad_total += wrong > 0;
    }
    return bad_total ? 1 : 0;
}
