// sph_search.hip -- smoothing-length Newton update and neighbour search.
//
// One thread per target slot; consecutive slots are Morton-consecutive, so the
// 64 lanes of a wavefront sit in one or two cells and walk the same candidate
// cells in lockstep: candidate positions are same-address loads across lanes
// (one request per distinct cell) served from L1/L2.  Candidate cells are
// culled by the distance from the target to the cell box, per axis, with a
// margin that covers the rounding of the key quantisation.
#include "sph_common.h"

namespace sph {
namespace {

constexpr double kCullMargin = 1e-9;  // relative to the cell edge

struct AxisWalk {
    int lo, hi;      // offsets (or absolute cells when `all`)
    bool all;        // every cell of a periodic axis, no culling
    bool empty;      // zero-extent axis: only cell 0
    int c0;          // target's cell
    double f;        // target position inside its cell
    double ce;       // cell edge
};

__device__ __forceinline__ AxisWalk axis_walk(const Params& P, const Domain& D, int k, double pos,
                                              double R)
{
    AxisWalk a;
    const int nax = D.ncell_axis;
    const int sh = kKeyBits - D.level;
    uint32_t q = quantize(pos, D.lo[k], D.scale[k]);
    a.c0 = (int)(q >> sh);
    a.ce = D.cell[k];
    a.all = false;
    a.empty = !(a.ce > 0.0);
    if (a.empty) {
        a.lo = a.hi = 0;
        a.f = 0.0;
        return a;
    }
    a.f = (pos - D.lo[k]) - (double)a.c0 * a.ce;
    double Kd = ceil(R / a.ce);
    int K = (Kd < (double)nax) ? (int)Kd : nax;
    if (P.periodic[k]) {
        if (2 * K + 1 >= nax) {
            a.all = true;
            a.lo = 0;
            a.hi = nax - 1;
        } else {
            a.lo = -K;
            a.hi = K;
        }
    } else {
        a.lo = (-K > -a.c0) ? -K : -a.c0;
        a.hi = (K < nax - 1 - a.c0) ? K : nax - 1 - a.c0;
    }
    return a;
}

// lower bound of the distance along one axis from the target to the cell at
// offset o, reduced by the rounding margin
__device__ __forceinline__ double axis_gap(const AxisWalk& a, int o)
{
    if (a.all || a.empty || o == 0) return 0.0;
    double d = (o > 0) ? (double)o * a.ce - a.f : a.f - (double)(o + 1) * a.ce;
    d -= kCullMargin * a.ce;
    return d > 0.0 ? d : 0.0;
}

__device__ __forceinline__ int axis_cell(const AxisWalk& a, int o, int nax)
{
    if (a.all || a.empty) return o;
    int c = a.c0 + o;
    if (c < 0) c += nax;
    else if (c >= nax) c -= nax;
    return c;
}

// Visit every particle of every cell whose box may hold a point closer than R
// to `pos` and that `want(cell, gap2)` accepts.
template <class Want, class Body>
__device__ __forceinline__ void walk_cells(const Params& P, const Domain& D,
                                           const int32_t* __restrict__ cs,
                                           const int32_t* __restrict__ ce, double xa, double ya,
                                           double za, double R, Want&& want, Body&& body)
{
    const int nax = D.ncell_axis;
    AxisWalk wx = axis_walk(P, D, 0, xa, R);
    AxisWalk wy = axis_walk(P, D, 1, ya, R);
    AxisWalk wz = axis_walk(P, D, 2, za, R);
    const double R2 = R * R;
    for (int oz = wz.lo; oz <= wz.hi; ++oz) {
        double gz = axis_gap(wz, oz);
        double gz2 = gz * gz;
        if (gz2 >= R2) continue;
        uint64_t mz = spread3((uint64_t)axis_cell(wz, oz, nax));
        for (int oy = wy.lo; oy <= wy.hi; ++oy) {
            double gy = axis_gap(wy, oy);
            double gzy2 = gz2 + gy * gy;
            if (gzy2 >= R2) continue;
            uint64_t mzy = mz | (spread3((uint64_t)axis_cell(wy, oy, nax)) << 1);
            for (int ox = wx.lo; ox <= wx.hi; ++ox) {
                double gx = axis_gap(wx, ox);
                double g2 = gzy2 + gx * gx;
                if (g2 >= R2) continue;
                uint64_t cid = mzy | (spread3((uint64_t)axis_cell(wx, ox, nax)) << 2);
                if (!want(cid, g2)) continue;
                int32_t b0 = cs[cid], b1 = ce[cid];
                for (int32_t b = b0; b < b1; ++b) body(b);
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_update_h(Params P, const Domain* __restrict__ dom,
                                                     const int32_t* __restrict__ cs,
                                                     const int32_t* __restrict__ ce,
                                                     const double* __restrict__ x,
                                                     const double* __restrict__ y,
                                                     const double* __restrict__ z,
                                                     double* __restrict__ h)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    const int64_t a = lb * kBlock + threadIdx.x;
    if (a >= P.n) return;
    const Domain D = *dom;
    const double xa = x[a], ya = y[a], za = z[a];
    const double h0 = h[a];
    const double k3 = (32.0 * kPi / 3.0) * P.bn;
    const double kap = P.kappa;
    double hc = h0;
    for (int it = 0; it < P.newton_iters; ++it) {
        const double h2 = 2.0 * hc;
        const double R2 = h2 * h2;
        const double tsc = kPiHalfSq / (hc * hc);
        double sS = 0.0, sV = 0.0;
        walk_cells(P, D, cs, ce, xa, ya, za, h2, [](uint64_t, double) { return true; },
                   [&](int32_t b) {
                       double dx, dy, dz;
                       double r2 = disp(P, xa, ya, za, x[b], y[b], z[b], dx, dy, dz);
                       if (r2 < R2) {
                           double S, vdS;
                           sinc_terms(r2 * tsc, P.sinc_n, S, vdS);
                           sS += S;
                           sV += vdS;
                       }
                   });
        double F = k3 * sS - P.n_target;
        double Fp = -(k3 / hc) * sV;
        double hn = (Fp > 0.0) ? hc - F / Fp : kap * h0;
        if (hn < h0 / kap) hn = h0 / kap;
        if (hn > kap * h0) hn = kap * h0;
        hc = hn;
    }
    h[a] = hc;
}

__global__ void k_hmax_begin(Domain* d) { d->hmax_new_bits = ord_bits(0.0); }

// largest h per cell (for the symmetric search) and overall
__global__ __launch_bounds__(kBlock) void k_cells_hmax(Params P, Domain* __restrict__ dom,
                                                       const int32_t* __restrict__ cs,
                                                       const int32_t* __restrict__ ce,
                                                       const double* __restrict__ h,
                                                       double* __restrict__ chmax, int64_t cap)
{
    int64_t c = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    int64_t ncell = int64_t(1) << (3 * dom->level);
    double hm = 0.0;
    if (c < ncell && c < cap) {
        for (int32_t b = cs[c]; b < ce[c]; ++b) hm = fmax(hm, h[b]);
        chmax[c] = hm;
    }
    for (int o = 32; o > 0; o >>= 1) hm = fmax(hm, __shfl_xor(hm, o, 64));
    if ((threadIdx.x & 63) == 0) {
        atomicMax((unsigned long long*)&dom->hmax_new_bits, (unsigned long long)ord_bits(hm));
        bool bad = false;
        for (int k = 0; k < 3; ++k)
            if (P.periodic[k] && !(4.0 * hm < P.L[k])) bad = true;
        if (bad && hm > 0.0) set_err(dom, SPH_ERRBIT_CELL_RANGE);
    }
}

// symmetric neighbour lists: gather members of N(a) from the front of the
// column, members of N_s(a) \ N(a) from the back
__global__ __launch_bounds__(kBlock) void k_find_neighbors(Params P, Domain* __restrict__ dom,
                                                           const int32_t* __restrict__ cs,
                                                           const int32_t* __restrict__ ce,
                                                           const double* __restrict__ chmax,
                                                           const double* __restrict__ x,
                                                           const double* __restrict__ y,
                                                           const double* __restrict__ z,
                                                           const double* __restrict__ h,
                                                           int32_t* __restrict__ nc,
                                                           int32_t* __restrict__ ns,
                                                           int32_t* __restrict__ list)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    const int64_t a = lb * kBlock + threadIdx.x;
    if (a >= P.n) return;
    const Domain D = *dom;
    const double xa = x[a], ya = y[a], za = z[a], ha = h[a];
    const double hnew = ord_value(D.hmax_new_bits);
    const double ha2 = 2.0 * ha;
    const double Ra2 = ha2 * ha2;
    const int ng = P.ng_max;
    const int64_t st = P.stride;
    int cg = 0, co = 0;
    walk_cells(
        P, D, cs, ce, xa, ya, za, 2.0 * fmax(ha, hnew),
        [&](uint64_t cid, double g2) {
            double hc = 2.0 * fmax(ha, chmax[cid]);
            return g2 < hc * hc;
        },
        [&](int32_t b) {
            if (b == a) return;
            double dx, dy, dz;
            double r2 = disp(P, xa, ya, za, x[b], y[b], z[b], dx, dy, dz);
            if (r2 < Ra2) {
                if (cg < ng) list[(int64_t)cg * st + a] = b;
                ++cg;
            } else {
                double hb2 = 2.0 * fmax(ha, h[b]);
                if (r2 < hb2 * hb2) {
                    if (co < ng) list[(int64_t)(ng - 1 - co) * st + a] = b;
                    ++co;
                }
            }
        });
    nc[a] = cg;
    ns[a] = cg + co;
    if (cg + co > ng) set_err(dom, SPH_ERRBIT_NEIGHBOR_OVERFLOW);
}

}  // namespace

hipError_t launch_update_h(const Params& P, const Layout& L, const Ws& W, sph_particles* p,
                           hipStream_t s)
{
    if (P.newton_iters == 0) return hipSuccess;
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    k_update_h<<<grid_xcd(nb), kBlock, 0, s>>>(P, W.dom, W.cstart, W.cend, p->x, p->y, p->z,
                                               p->h);
    return hipGetLastError();
}

hipError_t launch_find_neighbors(const Params& P, const Layout& L, const Ws& W,
                                 const sph_particles* p, hipStream_t s)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    k_hmax_begin<<<1, 1, 0, s>>>(W.dom);
    int64_t cb = (L.ncells_cap + kBlock - 1) / kBlock;
    k_cells_hmax<<<cb, kBlock, 0, s>>>(P, W.dom, W.cstart, W.cend, p->h, W.chmax, L.ncells_cap);
    k_find_neighbors<<<grid_xcd(nb), kBlock, 0, s>>>(P, W.dom, W.cstart, W.cend, W.chmax, p->x,
                                                     p->y, p->z, p->h, W.nc, W.ns, W.list);
    return hipGetLastError();
}

}  // namespace sph
