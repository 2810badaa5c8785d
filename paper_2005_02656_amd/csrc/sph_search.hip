// sph_search.hip -- smoothing-length Newton update and neighbour search.
//
// Cell walk: one thread per target slot; consecutive slots are Morton-
// consecutive, so the lanes of a wavefront sit in a few neighbouring cells and
// walk mostly the same candidate cells (same-address loads across lanes, served
// from L1/L2).  Cells are smaller than the kernel reach (edge >= h_max/2); each
// target walks its own stencil and skips cells whose box is out of reach, with a
// margin covering the rounding of the key quantisation.  Candidate positions and
// h come from the packed 32-byte records.
//
// Two compositions use these kernels:
//  * the stage entry points: Newton by cell walks (any kappa, any iteration
//    count) and the neighbour lists by one more walk;
//  * the fused step: ONE walk collects candidates within 2 kappa max(h0_a, h0_b)
//    (a superset of every set the step needs, since the Newton clamp keeps
//    h <= kappa h0), the Newton iterations sum over the candidate list, and a
//    filter pass writes the exact lists from the candidates with the final h.
//    The neighbour sets are identical; only the visiting order differs.
#include <cmath>

#include "sph_common.h"

namespace sph {
namespace {

constexpr double kCullMargin = 1e-9;  // relative to the cell edge

// particle records of one cell loaded together by the cell walk (a batch may
// read up to kCellBatch - 1 records past the cell's end: the record arrays keep
// kWalkPad spare entries), and cell
// records of one row (along z) loaded together
#ifndef SPH_CELL_BATCH
#define SPH_CELL_BATCH 2
#endif
static_assert(SPH_CELL_BATCH - 1 <= kWalkPad, "cell-walk batch overruns the record padding");
#ifndef SPH_CELL_ROW
#define SPH_CELL_ROW 2
#endif

// spread the low 10 bits of v to every third bit (cell coordinates, level <= 9)
__device__ __forceinline__ uint32_t spread10(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

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

__device__ __forceinline__ uint32_t axis_cell(const AxisWalk& a, int o, int nax)
{
    if (a.all || a.empty) return (uint32_t)o;
    int c = a.c0 + o;
    if (c < 0) c += nax;
    else if (c >= nax) c -= nax;
    return (uint32_t)c;
}

// Visit every particle of every cell whose box may hold a point closer than R
// to the target and that `want(cell, gap2)` accepts; body(b, record_of_b).
// Row by row, x outermost and rows along z: z takes the lowest bit of each
// coordinate triple of the Morton code, so the cells of a row pair are
// adjacent in the table and in particle order, and the lists the walk writes
// follow the particle order closely; the 64 lanes of a wavefront, whose
// targets are neighbours, then read the same records at about the same time in
// every later pass over the lists.  (Rows along x, the same walk with z
// outermost, made every list pass 5-15% slower at 64 M particles, and a walk
// block by block in Morton order made the walk itself 25% slower.)  The cell
// records of one row (up to kRow cells) are loaded together, then each cell's
// particle records in batches: independent loads in flight instead of one
// dependent load per candidate.
template <class Rec, class Want, class Body>
__device__ __forceinline__ void walk_cells(const Params& P, const Domain& D,
                                           const CellRange* __restrict__ cells,
                                           const Rec* __restrict__ recs, double xa, double ya,
                                           double za, double R, Want&& want, Body&& body)
{
    constexpr int kRow = SPH_CELL_ROW;
    constexpr int kCellBatch = SPH_CELL_BATCH;
    const int nax = D.ncell_axis;
    AxisWalk wx = axis_walk(P, D, 0, xa, R);
    AxisWalk wy = axis_walk(P, D, 1, ya, R);
    AxisWalk wz = axis_walk(P, D, 2, za, R);
    const AxisWalk& wo = wx;   // outer axis and its Morton bit offset
    const AxisWalk& wi = wz;   // row axis
    constexpr int so = 2, si = 0;
    const double R2 = R * R;
    for (int oo = wo.lo; oo <= wo.hi; ++oo) {
        double go = axis_gap(wo, oo);
        double go2 = go * go;
        if (go2 >= R2) continue;
        uint32_t mo = spread10(axis_cell(wo, oo, nax)) << so;
        for (int oy = wy.lo; oy <= wy.hi; ++oy) {
            double gy = axis_gap(wy, oy);
            double goy2 = go2 + gy * gy;
            if (goy2 >= R2) continue;
            uint32_t moy = mo | (spread10(axis_cell(wy, oy, nax)) << 1);
            for (int oi0 = wi.lo; oi0 <= wi.hi; oi0 += kRow) {
                uint32_t cid[kRow];
                double g2[kRow];
                bool in[kRow];
#pragma unroll
                for (int i = 0; i < kRow; ++i) {
                    const int oi = oi0 + i;
                    double gi = (oi <= wi.hi) ? axis_gap(wi, oi) : 0.0;
                    g2[i] = goy2 + gi * gi;
                    in[i] = (oi <= wi.hi) && g2[i] < R2;
                    cid[i] = in[i] ? (moy | (spread10(axis_cell(wi, oi, nax)) << si)) : 0u;
                }
                CellRange cr[kRow];
#pragma unroll
                for (int i = 0; i < kRow; ++i) cr[i] = cells[cid[i]];
#pragma unroll
                for (int i = 0; i < kRow; ++i) {
                    if (!in[i] || !want(cr[i], g2[i])) continue;
                    const int32_t e = cr[i].e;
                    for (int32_t b0 = cr[i].s; b0 < e; b0 += kCellBatch) {
                        Rec q[kCellBatch];
#pragma unroll
                        for (int u = 0; u < kCellBatch; ++u) q[u] = recs[b0 + u];
#pragma unroll
                        for (int u = 0; u < kCellBatch; ++u)
                            if (b0 + u < e) body(b0 + u, q[u]);
                    }
                }
            }
        }
    }
}


__device__ __forceinline__ double newton_step(const Params& P, double hc, double h0, double sS,
                                              double sV)
{
    const double k3 = (32.0 * kPi / 3.0) * P.bn;
    const double kap = P.kappa;
    double F = k3 * sS - P.n_target;
    double Fp = -(k3 / hc) * sV;
    double hn = (Fp > 0.0) ? hc - F / Fp : kap * h0;
    if (hn < h0 / kap) hn = h0 / kap;
    if (hn > kap * h0) hn = kap * h0;
    return hn;
}

__device__ __forceinline__ void check_cell_range(const Params& P, Domain* dom, double h)
{
    for (int k = 0; k < 3; ++k)
        if (P.periodic[k] && !(4.0 * h < P.L[k])) set_err(dom, SPH_ERRBIT_CELL_RANGE);
}

// ---------------------------------------------------------------- cell-walk forms
__global__ __launch_bounds__(kBlock) void k_update_h(Params P, const Domain* __restrict__ dom,
                                                     const CellRange* __restrict__ cells,
                                                     const Pos4* __restrict__ p4,
                                                     double* __restrict__ h)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    const int64_t a = lb * kBlock + threadIdx.x;
    if (a >= P.n) return;
    const Domain D = *dom;
    const Pos4 pa = p4[a];
    const double xa = pa.x, ya = pa.y, za = pa.z;
    const double h0 = h[a];
    double hc = h0;
    for (int it = 0; it < P.newton_iters; ++it) {
        const double h2 = 2.0 * hc;
        const double R2 = h2 * h2;
        const double tsc = kPiHalfSq / (hc * hc);
        double sS = 0.0, sV = 0.0;
        walk_cells(P, D, cells, p4, xa, ya, za, h2,
                   [](const CellRange&, double) { return true; },
                   [&](int32_t b, const Pos4& q) {
                       double dx, dy, dz;
                       double r2 = disp(P, xa, ya, za, q.x, q.y, q.z, dx, dy, dz);
                       if (r2 < R2) {
                           double S, vdS;
                           kern_terms(P, r2 * tsc, S, vdS);
                           sS += S;
                           sV += vdS;
                       }
                   });
        hc = newton_step(P, hc, h0, sS, sV);
    }
    h[a] = hc;
}

__global__ void k_hmax_begin(Domain* d)
{
    d->hmax_new_bits = ord_bits(0.0);
    d->refit = 0u;
}

// largest h per cell (for the symmetric search) and overall
// (h is read from the slot-ordered array: consecutive cells read consecutive
// runs of it)
__global__ __launch_bounds__(kBlock) void k_cells_hmax(Params P, Domain* __restrict__ dom,
                                                       CellRange* __restrict__ cells,
                                                       const double* __restrict__ h, int64_t cap)
{
    int64_t c = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    int64_t ncell = int64_t(1) << (3 * dom->level);
    double hm = 0.0;
    if (c < ncell && c < cap) {
        const CellRange cr = cells[c];
        for (int32_t b = cr.s; b < cr.e; ++b) hm = fmax(hm, h[b]);
        cells[c].hmax = hm;
    }
    for (int o = 32; o > 0; o >>= 1) hm = fmax(hm, __shfl_xor(hm, o, 64));
    if ((threadIdx.x & 63) == 0) {
        ord_max_to(&dom->hmax_new_bits, hm);
        if (hm > 0.0) check_cell_range(P, dom, hm);
    }
}

// ---------------------------------------------------------------- walk reach
// The fused walk's stencil must hold every b within 2 kap max(h_a, h_b) of its
// target.  With one global bound (the largest h) the free surfaces and the
// thin outskirts of a cluster size every target's stencil.  Instead: blocks of
// the Morton octree at a level lc whose edge E exceeds 2 kappa h_max (plus the
// rounding of the keys and of the walk's FP32 test) bound h_b by the largest h
// of the target's block and its 26 neighbours (periodic axes wrap).  A b
// outside those blocks is at least one block edge away, E > 2 kap max(h_a, h_b),
// so it can be no candidate; a b inside has h_b at most that bound.  Each walk
// then reaches 2 kap max(h_a, H(block of a)).

// offset of level l in the table of block maxima (levels 0 .. finest-1)
__host__ __device__ inline int64_t reach_level_offset(int l)
{
    int64_t o = 0;
    for (int k = 0; k < l; ++k) o += int64_t(1) << (3 * k);
    return o;
}

// the block level: the finest level below the cells whose block edge on every
// axis with extent exceeds the bound (level 0, one block, when none does)
__global__ void k_reach_level(Params P, Domain* d)
{
    const double need = 2.0 * P.kappa * ord_value(d->hmax_new_bits);
    double emin = INFINITY, emax = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double e = d->hi[k] - d->lo[k];
        if (e > 0.0) {
            emin = fmin(emin, e);
            emax = fmax(emax, e);
        }
    }
    // four key units and the walk's slack (2^-20 of the extent) cover the
    // quantised block boundaries and the FP32 test's widened reach
    const double margin = 4.0 * emax * 0x1p-21 + 2.0 * emax * 0x1p-20;
    int lc = 0;
    for (int l = d->level - 1; l > 0; --l) {
        if ((emin / (double)(1 << l)) * (1.0 - 1e-9) >= need * (1.0 + 0x1p-18) + margin) {
            lc = l;
            break;
        }
    }
    d->reach_level = lc;
}

// block maxima of level l from level l + 1 (the cells when l + 1 is the finest)
__global__ __launch_bounds__(kBlock) void k_reach_up(const Domain* __restrict__ d,
                                                     const CellRange* __restrict__ cells,
                                                     double* __restrict__ tab, int l)
{
    const int64_t c = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (l >= d->level || l < d->reach_level || c >= (int64_t(1) << (3 * l))) return;
    double m = 0.0;
    for (int k = 0; k < 8; ++k) {
        const int64_t ch = 8 * c + k;
        m = fmax(m, (l + 1 == d->level) ? cells[ch].hmax : tab[reach_level_offset(l + 1) + ch]);
    }
    tab[reach_level_offset(l) + c] = m;
}

__device__ __forceinline__ uint32_t compact10(uint32_t v)
{
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030c30c3u;
    v = (v | (v >> 4)) & 0x0300f00fu;
    v = (v | (v >> 8)) & 0x030000ffu;
    v = (v | (v >> 16)) & 0x3ffu;
    return v;
}

// the bound of each block at the block level: the largest h of it and its 26
// neighbours (wrapped on periodic axes, clipped on open ones)
__global__ __launch_bounds__(kBlock) void k_reach_bound(Params P, const Domain* __restrict__ d,
                                                        const CellRange* __restrict__ cells,
                                                        const double* __restrict__ tab,
                                                        double* __restrict__ bound)
{
    const int lc = d->reach_level;
    const int64_t c = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (c >= (int64_t(1) << (3 * lc))) return;
    const int nb = 1 << lc;
    const int b[3] = {(int)compact10((uint32_t)c >> 2), (int)compact10((uint32_t)c >> 1),
                      (int)compact10((uint32_t)c)};
    const double* lev = tab + reach_level_offset(lc);
    double m = 0.0;
    for (int ox = -1; ox <= 1; ++ox) {
        for (int oy = -1; oy <= 1; ++oy) {
            for (int oz = -1; oz <= 1; ++oz) {
                int q[3] = {b[0] + ox, b[1] + oy, b[2] + oz};
                bool in = true;
                for (int k = 0; k < 3; ++k) {
                    if (q[k] < 0 || q[k] >= nb) {
                        if (P.periodic[k]) q[k] = (q[k] + nb) % nb;
                        else in = false;
                    }
                }
                if (!in) continue;
                const uint32_t cc = (spread10((uint32_t)q[0]) << 2) |
                                    (spread10((uint32_t)q[1]) << 1) | spread10((uint32_t)q[2]);
                // (a single cell, level 0, is its own block)
                m = fmax(m, lc == d->level ? cells[cc].hmax : lev[cc]);
            }
        }
    }
    bound[c] = m;
}

// symmetric neighbour lists: gather members of N(a) from the front of the
// tile row, members of N_s(a) \ N(a) from the back
__global__ __launch_bounds__(kBlock) void k_find_neighbors(Params P, Domain* __restrict__ dom,
                                                           const CellRange* __restrict__ cells,
                                                           const Pos4* __restrict__ p4,
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
    const Pos4 pa = p4[a];
    const double xa = pa.x, ya = pa.y, za = pa.z, ha = pa.h;
    const double hnew = ord_value(D.hmax_new_bits);
    const double ha2 = 2.0 * ha;
    const double Ra2 = ha2 * ha2;
    const int ng = P.ng_max;
    int cg = 0, co = 0;
    walk_cells(
        P, D, cells, p4, xa, ya, za, 2.0 * fmax(ha, hnew),
        [&](const CellRange& cr, double g2) {
            double hc = 2.0 * fmax(ha, cr.hmax);
            return g2 < hc * hc;
        },
        [&](int32_t b, const Pos4& q) {
            if (b == a) return;
            double dx, dy, dz;
            double r2 = disp(P, xa, ya, za, q.x, q.y, q.z, dx, dy, dz);
            if (r2 < Ra2) {
                if (cg < ng) list[lpos(a, cg, ng)] = b;
                ++cg;
            } else {
                double hb2 = 2.0 * fmax(ha, q.h);
                if (r2 < hb2 * hb2) {
                    if (co < ng) list[lpos(a, ng - 1 - co, ng)] = b;
                    ++co;
                }
            }
        });
    nc[a] = cg;
    ns[a] = cg + co;
    if (cg + co > ng) set_err(dom, SPH_ERRBIT_NEIGHBOR_OVERFLOW);
}

// ---------------------------------------------------------------- fused step
// Candidates: every b != a with r^2 < (2 kap max(h0_a, h0_b))^2 (kap: the reach
// factor of this pass), by the same per-target cell walk over 16-byte FP32
// records.  The test runs in FP32 on offsets from the domain's low corner, with
// the reach widened by a bound on their rounding (the cell build stores each
// particle's widened squared reach in its record): each offset is within
// 2^-24 ext of its FP64 value (ext: the largest extent of the key domain); the
// difference, the FP32 box length and the shift by it each add at most as much
// again, and where d/L rounds across +-1/2 the other image is taken, at most
// 2^-24 L farther.  Every displacement component is then within 6 * 2^-24 ext
// and the distance within sqrt(3) times that, below the slack 2^-20 ext added
// to the reach; the factor 1 + 2^-18 on the squared reach covers the FP32
// rounding of r^2 and of the reach itself.  The extras are at most a relative 1e-4 beyond the reach at
// the benchmark sizes, and the passes after this one test every candidate in
// FP64.  (A wavefront walking the union of its 64 targets' stencils, with
// scalar or LDS-staged particle loads, tested 2.4x more pairs and ran 1.6-2.1x
// slower at 64 M particles.)
// kMode: 0 the short-reach pass over every target; at full reach, 1 the
// targets whose h left the short reach (flag 2), marking every candidate not
// so flagged (flag 1), then 2 the marked targets (flag 1)
template <int kPer, int kMode>   // bit k of kPer set: axis k periodic
__device__ __forceinline__ void candidates(const Params& P, Domain* __restrict__ dom,
                                           const CellRange* __restrict__ cells,
                                           const Pos4* __restrict__ p4,
                                           const Pos4f* __restrict__ pf, int32_t* __restrict__ nk,
                                           int32_t* __restrict__ cand, double kap, float sc,
                                           uint8_t* __restrict__ flag,
                                           const uint64_t* __restrict__ keys,
                                           const double* __restrict__ reach)
{
    constexpr bool kFull = kMode != 0;
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    const int64_t a = lb * kBlock + threadIdx.x;
    if (a >= P.n) return;
    if (kMode == 1 && flag[a] != 2) return;
    if (kMode == 2 && flag[a] != 1) return;
    const Domain D = *dom;
    const Pos4 pa = p4[a];
    const Pos4f fa = pf[a];
    const uint32_t far2 = __float_as_uint(kFull ? fa.r2 * sc : fa.r2);
    // the largest h the target's candidates can have (its block's bound)
    const double hreach = reach[keys[a] >> (3 * (kKeyBits - D.reach_level))];
    const int cap = P.cand_cap;
    // candidates are staged in LDS, column per lane, and written out in
    // whole chunks of 8 (two 16-byte stores per lane)
    __shared__ int32_t stage[8][kBlock];
    const int t = threadIdx.x;
    const int32_t self = (int32_t)a;
    int k = 0;
    walk_cells(
        P, D, cells, pf, pa.x, pa.y, pa.z, 2.0 * kap * fmax(pa.h, hreach),
        [&](const CellRange& cr, double g2) {
            double hc = 2.0 * kap * fmax(pa.h, cr.hmax);
            return g2 < hc * hc;
        },
        [&](int32_t b, const Pos4f& q) {
            // r^2 may fuse multiply-adds: the widening factor of the reach
            // covers its FP32 rounding either way
#pragma clang fp contract(fast)
            // minimum image without branches: the shift is 0 on open axes
            float d[3] = {q.x - fa.x, q.y - fa.y, q.z - fa.z};
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if (kPer & (1 << c)) d[c] = fmaf(-P.wrapL[c], rintf(d[c] * P.wrapInvL[c]), d[c]);
            const float r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            // r < 2 kap max(h_a, h_b) (+ slack): r^2 below either widened
            // squared reach (the full pass scales the short ones up by sc).
            // All three are non-negative floats, whose order is that of their
            // bit patterns as unsigned integers: one integer max and one
            // compare (a float max quiets NaNs first, one more instruction).
            const float qr2 = kFull ? q.r2 * sc : q.r2;
            const bool near = __float_as_uint(r2) < max(far2, __float_as_uint(qr2));
            if (near & (b != self)) {
                // a neighbour of a grown h redoes its own walk at full reach
                if (kMode == 1 && flag[b] == 0) flag[b] = 1;
                if (k < cap) {
                    stage[k & 7][t] = b;
                    if ((k & 7) == 7) {
                        int4* dst = (int4*)(cand + lpos8(a, k & ~7, cap));
                        dst[0] = make_int4(stage[0][t], stage[1][t], stage[2][t], stage[3][t]);
                        dst[1] = make_int4(stage[4][t], stage[5][t], stage[6][t], stage[7][t]);
                    }
                }
                ++k;
            }
        });
    if (k < cap && (k & 7) != 0) {   // the partial last chunk
        int4* dst = (int4*)(cand + lpos8(a, k & ~7, cap));
        dst[0] = make_int4(stage[0][t], stage[1][t], stage[2][t], stage[3][t]);
        dst[1] = make_int4(stage[4][t], stage[5][t], stage[6][t], stage[7][t]);
    }
    nk[a] = k;
    if (k > cap) set_err(dom, SPH_ERRBIT_NEIGHBOR_OVERFLOW);
}

// the short-reach pass, and the full-reach pass that runs only if flagged
template <int kPer>
__global__ __launch_bounds__(kBlock) SPH_WAVES_CAND_ATTR void k_candidates(
    Params P, Domain* __restrict__ dom, const CellRange* __restrict__ cells,
    const Pos4* __restrict__ p4, const Pos4f* __restrict__ pf, int32_t* __restrict__ nk,
    int32_t* __restrict__ cand, double kap, float sc, uint8_t* __restrict__ flag,
    const uint64_t* __restrict__ keys, const double* __restrict__ reach)
{
    candidates<kPer, 0>(P, dom, cells, p4, pf, nk, cand, kap, sc, flag, keys, reach);
}
template <int kPer, int kMode>
__global__ __launch_bounds__(kBlock) SPH_WAVES_CAND_ATTR void k_candidates_full(
    Params P, Domain* __restrict__ dom, const CellRange* __restrict__ cells,
    const Pos4* __restrict__ p4, const Pos4f* __restrict__ pf, int32_t* __restrict__ nk,
    int32_t* __restrict__ cand, double kap, float sc, uint8_t* __restrict__ flag,
    const uint64_t* __restrict__ keys, const double* __restrict__ reach)
{
    if (dom->refit == 0u) return;
    candidates<kPer, kMode>(P, dom, cells, p4, pf, nk, cand, kap, sc, flag, keys, reach);
}

// the candidate pass for the periodic axes of P: mode 0 short reach, 1 and 2
// the full-reach refits (see candidates())
static void launch_candidates(int mode, const Params& P, const Ws& W, double kap, hipStream_t s)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    // the per-block bounds of the walk's reach follow the block maxima of
    // every level below the finest
    const double* bound = W.reach + reach_level_offset(P.lcap);
    // the records hold the squared short reach; the full pass scales it by
    // at least (kap / lambda)^2 (the slack scales with it, which only widens)
    const double lam = fmin(kFusedReach, P.kappa);
    const double q = (kap / lam) * (kap / lam) * (1.0 + 0x1p-20);
    float sc = (float)q;
    if ((double)sc < q) sc = nextafterf(sc, INFINITY);
    with_periodic(P, [&](auto per) {
        constexpr int kPer = decltype(per)::value;
        if (mode == 1)
            k_candidates_full<kPer, 1><<<grid_xcd(nb), kBlock, 0, s>>>(
                P, W.dom, W.cells, W.p4, W.pf, W.nk, W.cand, kap, sc, W.flag, W.keys0, bound);
        else if (mode == 2)
            k_candidates_full<kPer, 2><<<grid_xcd(nb), kBlock, 0, s>>>(
                P, W.dom, W.cells, W.p4, W.pf, W.nk, W.cand, kap, sc, W.flag, W.keys0, bound);
        else
            k_candidates<kPer><<<grid_xcd(nb), kBlock, 0, s>>>(P, W.dom, W.cells, W.p4, W.pf,
                                                               W.nk, W.cand, kap, sc, W.flag, W.keys0, bound);
    });
}

// one chunk of 8 candidates of slot a (entries at or past cnt read as a itself)
__device__ __forceinline__ void load_chunk(const int32_t* __restrict__ cand, int64_t a, int j0,
                                           int cap, int cnt, int32_t bb[8])
{
    const int4* src = (const int4*)(cand + lpos8(a, j0, cap));
    const int4 lo = src[0], hi = src[1];
    const int32_t v[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
    for (int u = 0; u < 8; ++u) bb[u] = (j0 + u < cnt) ? v[u] : (int32_t)a;
}

// the chunk at j0, or the target itself in every entry when j0 >= cnt
__device__ __forceinline__ void load_chunk_or_self(const int32_t* __restrict__ cand, int64_t a,
                                                   int j0, int cap, int cnt, int32_t bb[8])
{
    if (j0 < cnt) {
        load_chunk(cand, a, j0, cap, cnt, bb);
    } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) bb[u] = (int32_t)a;
    }
}

// Newton iterations summing over the candidate list (self term added: S(0) = 1)
// x, y, z of candidate b of this lane, gathered by the two lanes of a pair
// together: one 16-byte load per lane fetches the even lane's record (x, y to
// the even lane, z, h to the odd one) and a second the odd lane's, so the two
// loads of a pair touch one line each instead of two per lane; a swap then
// completes each lane's own position.  Both lanes of the pair must be active.
// kNarrow (the records span under 4 GiB): the byte offsets fit 32 bits, so
// each address is one shift-or on a scalar base instead of a 64-bit
// sign-extend, shift and add (Newton 27.0 -> 26.0 ms at 64 M particles; the
// same form in the list filter made it slower, 21.9 -> 29.0 ms).
template <bool kNarrow>
__device__ __forceinline__ void pair_gather_xyz(const Pos4* __restrict__ p4, int32_t b, int odd,
                                                double& x, double& y, double& z)
{
    const int32_t o = pair_swap(b);
    const int32_t rA = odd ? o : b;   // the even lane's candidate
    const int32_t rB = odd ? b : o;   // the odd lane's candidate
    double2 A, B;
    if constexpr (kNarrow) {
        const char* base = (const char*)p4;
        A = *(const double2*)(base + (((uint32_t)rA << 5) | (uint32_t)(odd << 4)));
        B = *(const double2*)(base + (((uint32_t)rB << 5) | (uint32_t)(odd << 4)));
    } else {
        const double2* half = (const double2*)p4;
        A = half[2 * (int64_t)rA + odd];
        B = half[2 * (int64_t)rB + odd];
    }
    // even lane: A = (x, y) of its own record, B = (x, y) of the odd lane's;
    // odd lane: A = (z, h) of the even lane's record, B = (z, h) of its own
    const double r0 = pair_swap(odd ? A.x : B.x);
    const double r1 = pair_swap(B.y);
    x = odd ? r0 : A.x;
    y = odd ? r1 : A.y;
    z = odd ? B.x : r0;
}

template <int kPer, bool kTab>
__device__ __forceinline__ void update_h_list(const Params& P, Domain* __restrict__ dom,
                                              const int32_t* __restrict__ nk,
                                              const int32_t* __restrict__ cand,
                                              const Pos4* __restrict__ p4, double* __restrict__ h,
                                              double lam, uint8_t* __restrict__ flag, bool full)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    // lanes past the end shadow the last particle with no candidates, so that
    // both lanes of every pair run the gathers together; in the full-reach pass
    // only the targets whose h left the short reach (flag 2) are live
    const int64_t a0 = lb * kBlock + threadIdx.x;
    const int64_t a = a0 < P.n ? a0 : P.n - 1;
    const bool live = a0 < P.n && (!full || flag[a] == 2);
    const int odd = threadIdx.x & 1;
    const Pos4 pa = p4[a];
    const double xa = pa.x, ya = pa.y, za = pa.z;
    const double h0 = pa.h;
    const int cap = P.cand_cap;
    const int cnt = live ? min(nk[a], cap) : 0;
    const int cntp = max(cnt, pair_swap(cnt));   // the pair's trip count
    // the candidates reach 2 lam max(h0_a, h0_b): exact as long as every
    // iterate stays at or below lam h0 (2 (lam h0) == (2 lam) h0 in FP64)
    const double hlim = lam * h0;
    bool over = false;
    double hc = h0;
    auto iterate = [&](auto narrow) {
        constexpr bool kNarrow = decltype(narrow)::value;
        for (int it = 0; it < P.newton_iters; ++it) {
            const double h2 = 2.0 * hc;
            const double R2 = h2 * h2;
            const double tsc = kPiHalfSq / (hc * hc);
            double sS = 1.0, sV = 0.0;
            for (int j0 = 0; j0 < cntp; j0 += 8) {
                int32_t bb[8];
                load_chunk_or_self(cand, a, j0, cap, cnt, bb);
                double qx[8], qy[8], qz[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    pair_gather_xyz<kNarrow>(p4, bb[u], odd, qx[u], qy[u], qz[u]);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    double dx, dy, dz;
                    double r2 = disp_p<kPer>(P, xa, ya, za, qx[u], qy[u], qz[u], dx, dy, dz);
                    if (j0 + u < cnt && r2 < R2) {
                        double S, vdS;
                        kern_terms_t<kTab>(P, r2 * tsc, S, vdS);
                        sS += S;
                        sV += vdS;
                    }
                }
            }
            hc = newton_step(P, hc, h0, sS, sV);
            over = over || hc > hlim;
        }
    };
    if ((uint64_t)P.n * sizeof(Pos4) <= 0xffffffffull) iterate(std::true_type{});
    else iterate(std::false_type{});
    if (!live) return;
    h[a] = hc;
    // the short pass flags the targets whose h may have missed candidates
    // (2) and clears the others (0); the full-reach pass recomputes the former
    if (!full) flag[a] = over ? 2 : 0;
    if (over) {
        flag_or(&dom->refit, 1u);
    } else {
        check_cell_range(P, dom, hc);
    }
}

template <int kPer, bool kTab>
__global__ __launch_bounds__(kBlock) SPH_NEWTON_ATTR void k_update_h_list(
    Params P, Domain* __restrict__ dom, const int32_t* __restrict__ nk,
    const int32_t* __restrict__ cand, const Pos4* __restrict__ p4, double* __restrict__ h,
    double lam, uint8_t* __restrict__ flag)
{
    update_h_list<kPer, kTab>(P, dom, nk, cand, p4, h, lam, flag, false);
}
template <int kPer, bool kTab>
__global__ __launch_bounds__(kBlock) SPH_NEWTON_ATTR void k_update_h_list_full(
    Params P, Domain* __restrict__ dom, const int32_t* __restrict__ nk,
    const int32_t* __restrict__ cand, const Pos4* __restrict__ p4, double* __restrict__ h,
    double lam, uint8_t* __restrict__ flag)
{
    if (dom->refit == 0u) return;
    update_h_list<kPer, kTab>(P, dom, nk, cand, p4, h, lam, flag, true);
}

// exact lists from the candidates with the final h (same layout as k_find_neighbors)
// kDens: also the density sums over the gather members (the same order as the
// density pass over the gather list), then rho, Omega and the EOS
template <bool kDens, int kPer, bool kTab>
__global__ __launch_bounds__(kBlock) SPH_FILTER_ATTR void k_filter(Params P, Domain* __restrict__ dom,
                                                   const int32_t* __restrict__ nk,
                                                   const int32_t* __restrict__ cand,
                                                   const Pos4* __restrict__ p4,
                                                   int32_t* __restrict__ nc,
                                                   int32_t* __restrict__ ns,
                                                   int32_t* __restrict__ list, DensOut O)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    // lanes past the end shadow the last particle with no candidates, so that
    // both lanes of every pair run the gathers together
    const int64_t a0 = lb * kBlock + threadIdx.x;
    const bool live = a0 < P.n;
    const int64_t a = live ? a0 : P.n - 1;
    const int odd = threadIdx.x & 1;
    const Pos4 pa = p4[a];
    const double xa = pa.x, ya = pa.y, za = pa.z, ha = pa.h;
    const double ha2 = 2.0 * ha;
    const double Ra2 = ha2 * ha2;
    const int cap = P.cand_cap;
    const int cnt = live ? min(nk[a], cap) : 0;
    const int cntl = max(cnt, pair_swap(cnt));   // the pair's trip count
    const int ng = P.ng_max;
    const double tsc = kPiHalfSq / (ha * ha);
    double sS = 0.0, sD = 0.0;
    if (kDens) {
        sS = O.m[a];          // self term: S = 1, v dS/dv = 0
        sD = 3.0 * O.m[a];
    }
    // with equal masses (flagged by the cell build) the mass of every
    // neighbour is slot 0's: no gather
    const bool mvar = !kDens || dom->mass_varies != 0u;
    const double m0 = kDens ? O.m[0] : 0.0;
    int cg = 0, co = 0;
    for (int j0 = 0; j0 < cntl; j0 += 8) {
        int32_t bb[8];
        load_chunk_or_self(cand, a, j0, cap, cnt, bb);
        Pos4 q[8];
        double mb[8];
        // one straight run of loads per case (a test per load would split the
        // batch into blocks and serialise its gathers)
        if (mvar) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                q[u] = pair_gather32(p4, bb[u], odd);
                if (kDens) mb[u] = O.m[bb[u]];
            }
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                q[u] = pair_gather32(p4, bb[u], odd);
                mb[u] = m0;
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (j0 + u >= cnt) continue;
            const int32_t b = bb[u];
            double dx, dy, dz;
            double r2 = disp_p<kPer>(P, xa, ya, za, q[u].x, q[u].y, q[u].z, dx, dy, dz);
            if (r2 < Ra2) {
                if (cg < ng) {
                    list[lpos(a, cg, ng)] = b;
                    if (kDens) {
                        double S, vdS;
                        kern_terms_t<kTab>(P, r2 * tsc, S, vdS);
                        sS += mb[u] * S;
                        sD += mb[u] * (3.0 * S + vdS);
                    }
                }
                ++cg;
            } else {
                double hb2 = 2.0 * fmax(ha, q[u].h);
                if (r2 < hb2 * hb2) {
                    if (co < ng) list[lpos(a, ng - 1 - co, ng)] = b;
                    ++co;
                }
            }
        }
    }
    if (!live) return;
    nc[a] = cg;
    ns[a] = cg + co;
    if (cg + co > ng) set_err(dom, SPH_ERRBIT_NEIGHBOR_OVERFLOW);
    if (kDens) finish_density(P, dom, O, a, ha, sS, sD);
}

}  // namespace

int candidate_capacity(int ng_max)
{
    // the candidate reach is at most kFusedKappaMax times the list reach:
    // kFusedKappaMax^3 times the volume, with 25% headroom
    double c = ng_max * kFusedKappaMax * kFusedKappaMax * kFusedKappaMax * 1.25;
    int cap = ((int)ceil(c) + 7) & ~7;   // whole chunks of 8
    return cap > 8192 ? 8192 : cap;
}

hipError_t launch_update_h(const Params& P, const Layout& L, const Ws& W, sph_particles* p,
                           hipStream_t s, bool pack)
{
    if (P.newton_iters == 0) return hipSuccess;
    if (pack) {
        hipError_t e = launch_pack_p4(P, W, p, s);
        if (e != hipSuccess) return e;
    }
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    k_update_h<<<grid_xcd(nb), kBlock, 0, s>>>(P, W.dom, W.cells, W.p4, p->h);
    return hipGetLastError();
}

// always repacks: h may have changed since the cell build
hipError_t launch_find_neighbors(const Params& P, const Layout& L, const Ws& W,
                                 const sph_particles* p, hipStream_t s)
{
    hipError_t e = launch_pack_p4(P, W, p, s);
    if (e != hipSuccess) return e;
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    k_hmax_begin<<<1, 1, 0, s>>>(W.dom);
    int64_t cb = (L.ncells_cap + kBlock - 1) / kBlock;
    k_cells_hmax<<<cb, kBlock, 0, s>>>(P, W.dom, W.cells, p->h, L.ncells_cap);
    k_find_neighbors<<<grid_xcd(nb), kBlock, 0, s>>>(P, W.dom, W.cells, W.p4, W.nc, W.ns,
                                                     W.list);
    return hipGetLastError();
}


// fused: candidates at h0, Newton over candidates, exact lists at the new h.
// Expects the packed positions and walk records of the cell build (h0 in them).
hipError_t launch_fused_h_lists(const Params& P, const Layout& L, const Ws& W, sph_particles* p,
                                hipStream_t s, const Marks& mk, bool with_density)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    k_hmax_begin<<<1, 1, 0, s>>>(W.dom);
    int64_t cb = (L.ncells_cap + kBlock - 1) / kBlock;
    k_cells_hmax<<<cb, kBlock, 0, s>>>(P, W.dom, W.cells, p->h, L.ncells_cap);
    // the walk's reach bounds: the block level, the block maxima of the levels
    // from the finest down to it, then each block's bound
    k_reach_level<<<1, 1, 0, s>>>(P, W.dom);
    for (int l = L.lcap - 1; l >= 0; --l) {
        const int64_t nl = int64_t(1) << (3 * l);
        k_reach_up<<<(nl + kBlock - 1) / kBlock, kBlock, 0, s>>>(W.dom, W.cells, W.reach, l);
    }
    {
        const int64_t nl = L.lcap > 0 ? int64_t(1) << (3 * (L.lcap - 1)) : 1;
        k_reach_bound<<<(nl + kBlock - 1) / kBlock, kBlock, 0, s>>>(
            P, W.dom, W.cells, W.reach, W.reach + reach_level_offset(L.lcap));
    }
    mk.at(0, s);
    // short reach first; the full-reach pair runs only if an h left it (the
    // kernels read the device flag and return at once when it is clear)
    const double lam = fmin(kFusedReach, P.kappa);
    launch_candidates(0, P, W, lam, s);
    mk.at(1, s);
    if (P.newton_iters > 0) {
        with_periodic(P, [&](auto per) {
            with_table(P, [&](auto tab) {
                constexpr int kPer = decltype(per)::value;
                constexpr bool kTab = decltype(tab)::value;
                k_update_h_list<kPer, kTab><<<grid_xcd(nb), kBlock, 0, s>>>(
                    P, W.dom, W.nk, W.cand, W.p4, p->h, lam, W.flag);
            });
        });
        if (lam < P.kappa) {
            // targets whose h left the short reach walk again at full reach
            // and mark their candidates, whose symmetric sets may now hold
            // them; the marked targets walk again too (their own h stands),
            // then the grown ones redo Newton over their full candidates
            launch_candidates(1, P, W, P.kappa, s);
            launch_candidates(2, P, W, P.kappa, s);
            with_periodic(P, [&](auto per) {
                with_table(P, [&](auto tab) {
                    constexpr int kPer = decltype(per)::value;
                    constexpr bool kTab = decltype(tab)::value;
                    k_update_h_list_full<kPer, kTab><<<grid_xcd(nb), kBlock, 0, s>>>(
                        P, W.dom, W.nk, W.cand, W.p4, p->h, P.kappa, W.flag);
                });
            });
        }
    }
    mk.at(2, s);
    hipError_t e = launch_pack_p4(P, W, p, s);
    if (e != hipSuccess) return e;
    const DensOut O{p->m, p->u, p->p_ref, p->rho_ref, p->rho, p->omega, p->p, p->c};
    with_periodic(P, [&](auto per) {
        with_table(P, [&](auto tab) {
            constexpr int kPer = decltype(per)::value;
            constexpr bool kTab = decltype(tab)::value;
            if (with_density)
                k_filter<true, kPer, kTab><<<grid_xcd(nb), kBlock, 0, s>>>(
                    P, W.dom, W.nk, W.cand, W.p4, W.nc, W.ns, W.list, O);
            else
                k_filter<false, kPer, kTab><<<grid_xcd(nb), kBlock, 0, s>>>(
                    P, W.dom, W.nk, W.cand, W.p4, W.nc, W.ns, W.list, O);
        });
    });
    return hipGetLastError();
}

}  // namespace sph
