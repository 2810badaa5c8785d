// Host check of the mixed-precision pair displacement (sph::axis_disp) against
// the FP64 minimum image with the half-open interval (-L/2, L/2].
//
// For each number of cells per axis given on the command line, particles are
// drawn uniformly on a periodic axis of length L = nax x edge, split into a
// cell index and an FP32 offset, and every pair displacement the FP32 form
// gives is compared with the FP64 one.  Prints one line per nax:
//   nax pairs wrong worst_relative_error
// and exits with status 1 if any pair took the wrong image or erred by more
// than the rounding bound.
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

int main(int argc, char** argv)
{
    int bad_total = 0;
    for (int ai = 1; ai < argc; ++ai) {
        const int nax = atoi(argv[ai]);
        const double ce = 1.0 / nax;   // unit box
        const double L = nax * ce;
        const int np = 600;
        double x[np];
        int c[np];
        float o[np];
        for (int i = 0; i < np; ++i) {
            x[i] = uniform01() * L;
            int ci = (int)floor(x[i] / ce);
            if (ci > nax - 1) ci = nax - 1;
            c[i] = ci;
            o[i] = (float)(x[i] - ci * ce);
        }
        long pairs = 0, wrong = 0;
        double worst = 0.0;
        for (int a = 0; a < np; ++a)
            for (int b = 0; b < np; ++b) {
                double d = x[b] - x[a];
                if (d > 0.5 * L) d -= L;
                else if (d <= -0.5 * L) d += L;
                if (fabs(fabs(d) - 0.5 * L) < 1e-5 * L) continue;   // image tie: either is right
                const float f = sph::axis_disp(c[a], c[b], o[a], o[b], (float)ce, true, nax);
                const double err = fabs((double)f - d);
                const double bound = 8.0 * 0x1p-24 * (fabs(d) + ce);
                ++pairs;
                if (err > bound) ++wrong;
                const double rel = err / (fabs(d) + ce);
                if (rel > worst) worst = rel;
            }
        printf("%d %ld %ld %.3e\n", nax, pairs, wrong, worst);
        bad_total += wrong > 0;
    }
    return bad_total ? 1 : 0;
}
