// sph_mixed.hip -- mixed-precision pair passes (precision SPH_MIXED).
//
// The paper keeps FP64 throughout and names a mixed-precision approach as
// future work (section 4.2).  This form evaluates every pair term of the
// density, IAD and momentum/energy passes in FP32 and accumulates the
// per-particle sums in FP64.  Positions are 32-bit fixed-point coordinates
// over the key domain, so a pair displacement is an exact integer difference
// (modulo 2^32 on periodic axes: the minimum image) converted to FP32 and
// scaled (fix_disp, sph_mixed_geom.h).  The neighbour test that builds the
// lists, the Newton update of h, the EOS, the 3x3 inversion, the integrator
// and the global sums stay in FP64.
//
// Gathered bytes per neighbour: 16 (position and FP32 mass, or volume) in the
// density and IAD passes, one 80-byte record in the momentum
// pass, or one 64-byte record, staged through LDS by the wavefront, with
// equal masses and sound speeds (FP64: 32 + 8, 32, and 144 or 112).
#include "sph_common.h"
#include "sph_mixed_geom.h"

namespace sph {
namespace {


struct alignas(16) PosM {
    uint32_t qx, qy, qz;  // fixed-point coordinates (fix_coord)
    float w;              // the mass (packed), then the volume m/rho (IAD pass)
};
// a neighbour's momentum/energy record: its position as in PosM, then the
// folded factors of the FP64 record (K = (m/rho) C, q = P/(Omega rho)).  Five
// 16-byte columns: an odd stride puts the same field of the records that the
// lanes of a wavefront load in different columns of their cache lines.
struct alignas(16) RecM {
    uint32_t qx, qy, qz;
    uint32_t pad;
    float k11, k12, k13, k22, k23, k33;
    float q, c, m, ih;
    float vx, vy, vz;
    float spare[3];
};

// the same factors when every mass and sound speed is equal (m and c from
// slot 0): four columns, which the wavefront stages through LDS together
struct alignas(16) RecMU {
    uint32_t qx, qy, qz;
    uint32_t pad;
    float k11, k12, k13, k22, k23, k33;
    float q, ih;
    float vx, vy, vz;
    float spare;
};

// the FP32 unit length of each axis
struct FixGeom {
    float unit[3];
};

__device__ __forceinline__ FixGeom fix_geom(const Params& P, const Domain& D)
{
    FixGeom g;
    const double emax = fix_emax(D.lo, D.hi);
    for (int k = 0; k < 3; ++k) {
        double origin, units;
        fix_axis(D.lo[k], D.hi[k], P.periodic[k] != 0, emax, origin, units, g.unit[k]);
    }
    return g;
}

// displacement b - a and its square, all FP32
__device__ __forceinline__ float disp_m(const FixGeom& g, const PosM& a, const PosM& b, float& dx,
                                        float& dy, float& dz)
{
    dx = fix_disp(a.qx, b.qx, g.unit[0]);
    dy = fix_disp(a.qy, b.qy, g.unit[1]);
    dz = fix_disp(a.qz, b.qz, g.unit[2]);
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

template <int K>
__device__ __forceinline__ float horner_f(const float (&c)[K], float t)
{
    float s = c[K - 1];
#pragma unroll
    for (int k = K - 2; k >= 0; --k) s = fmaf(s, t, c[k]);
    return s;
}

// FP32 S_n and v dS_n/dv from the FP32 fits of sinc and x sinc'(x) / t
__device__ __forceinline__ void sinc_terms_f(float t, int n, float& S, float& vdS)
{
    const float s = horner_f(kSincS32, t);
    const float q = horner_f(kSincQ32, t) * t;
    const float p = pow_nm1(s, n);
    S = p * s;
    vdS = (float)n * p * q;
}

__device__ __forceinline__ float sinc_S_f(float t, int n)
{
    const float s = horner_f(kSincS32, t);
    return pow_nm1(s, n) * s;
}

// the FP32 fits, or (kTab) the FP32 copies of the kernel tables (section 4.5)
template <bool kTab>
__device__ __forceinline__ void kern_terms_f_t(const Params& P, float t, float& S, float& vdS)
{
    if (kTab) {
        const float v = sqrtf(t) * (float)(2.0 / kPi);
        int i;
        float f;
        tab_index(v, (float)P.tab_inv_dv, P.tab_n, i, f);
        const float2 e = P.tabSf[i], d = P.tabDf[i];
        S = (1.0f - f) * e.x + f * e.y;
        vdS = v * ((1.0f - f) * d.x + f * d.y);
    } else {
        sinc_terms_f(t, P.sinc_n, S, vdS);
    }
}

template <bool kTab>
__device__ __forceinline__ float kern_S_f_t(const Params& P, float t)
{
    if (kTab) {
        const float v = sqrtf(t) * (float)(2.0 / kPi);
        int i;
        float f;
        tab_index(v, (float)P.tab_inv_dv, P.tab_n, i, f);
        const float2 e = P.tabSf[i];
        return (1.0f - f) * e.x + f * e.y;
    }
    return sinc_S_f(t, P.sinc_n);
}

__device__ __forceinline__ void kern_terms_f(const Params& P, float t, float& S, float& vdS)
{
    if (P.tab_n > 0) kern_terms_f_t<true>(P, t, S, vdS);
    else kern_terms_f_t<false>(P, t, S, vdS);
}

// fixed-point positions and FP32 masses
__global__ __launch_bounds__(kBlock) void k_pack_posm(Params P, const Domain* __restrict__ dom,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      const double* __restrict__ z,
                                                      const double* __restrict__ m,
                                                      PosM* __restrict__ pm)
{
    int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= P.n) return;
    const Domain& D = *dom;
    const double pos[3] = {x[i], y[i], z[i]};
    const double emax = fix_emax(D.lo, D.hi);
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) {
        const bool per = P.periodic[k] != 0;
        double origin, units;
        float unit;
        fix_axis(D.lo[k], D.hi[k], per, emax, origin, units, unit);
        q[k] = fix_coord(pos[k], origin, units, per);
    }
    pm[i] = PosM{q[0], q[1], q[2], (float)m[i]};
}

__global__ __launch_bounds__(kBlock) SPH_WAVES_CAP(SPH_WAVES_MIXED) void k_density_m(Params P, Domain* __restrict__ dom,
                                                      const int32_t* __restrict__ nc,
                                                      const int32_t* __restrict__ list,
                                                      const PosM* __restrict__ pm,
                                                      const double* __restrict__ h,
                                                      const double* __restrict__ m,
                                                      const double* __restrict__ u,
                                                      const double* __restrict__ p_ref,
                                                      const double* __restrict__ rho_ref,
                                                      double* __restrict__ rho,
                                                      double* __restrict__ omega,
                                                      double* __restrict__ pr,
                                                      double* __restrict__ cs)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    const int64_t a = lb * kBlock + threadIdx.x;
    if (a >= P.n) return;
    const FixGeom g = fix_geom(P, *dom);
    const PosM pa = pm[a];
    const double ha = h[a];
    const float tsc = (float)(kPiHalfSq / (ha * ha));
    const int cnt = min(nc[a], P.ng_max);
    double sS = m[a], sD = 3.0 * m[a];
    for (int j0 = 0; j0 < cnt; j0 += kBatch) {
        int32_t bb[kBatch];
        bool ok[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int32_t b = (j0 + u < cnt) ? list[lpos(a, j0 + u, P.ng_max)] : -1;
            ok[u] = (uint32_t)b < (uint32_t)P.n;
            bb[u] = ok[u] ? b : (int32_t)a;
        }
        PosM q[kBatch];
        float mb[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            q[u] = pm[bb[u]];
            mb[u] = q[u].w;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            if (!ok[u]) continue;
            float dx, dy, dz;
            const float r2 = disp_m(g, pa, q[u], dx, dy, dz);
            float S, vdS;
            kern_terms_f(P, r2 * tsc, S, vdS);
            sS += (double)(mb[u] * S);
            sD += (double)(mb[u] * (3.0f * S + vdS));
        }
    }
    const double w0 = P.bn / (ha * ha * ha);
    const double r = w0 * sS;
    const double om = 1.0 - w0 * sD / (3.0 * r);
    double p, c;
    if (P.eos == SPH_EOS_IDEAL) {
        p = (P.gamma - 1.0) * r * u[a];
        c = sqrt(P.gamma * (P.gamma - 1.0) * u[a]);
    } else {
        p = p_ref[a] + P.c0 * P.c0 * (r - rho_ref[a]);
        c = P.c0;
    }
    rho[a] = r;
    omega[a] = om;
    pr[a] = p;
    cs[a] = c;
    if (!isfinite(r) || !isfinite(om) || !isfinite(p) || !isfinite(c))
        set_err(dom, SPH_ERRBIT_NONFINITE);
}

// the volume m/rho in the position records' spare lane, once the densities
// that read the masses there are done: the IAD pass gathers one record per
// neighbour
__global__ __launch_bounds__(kBlock) void k_volume_m(int64_t n, const double* __restrict__ m,
                                                     const double* __restrict__ rho,
                                                     PosM* __restrict__ pm)
{
    int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i < n) pm[i].w = (float)(m[i] / rho[i]);
}

struct RecSrcM {
    const double *m, *rho, *omega, *p, *c, *vx, *vy, *vz, *h;
};

__device__ __forceinline__ RecM make_recm(const RecSrcM& R, int64_t a, const PosM& pa,
                                          double c11, double c12, double c13, double c22,
                                          double c23, double c33)
{
    RecM q;
    q.qx = pa.qx; q.qy = pa.qy; q.qz = pa.qz; q.pad = 0u;
    const double r = R.rho[a], m = R.m[a];
    const double v = m / r;
    q.k11 = (float)(v * c11); q.k12 = (float)(v * c12); q.k13 = (float)(v * c13);
    q.k22 = (float)(v * c22); q.k23 = (float)(v * c23); q.k33 = (float)(v * c33);
    q.q = (float)(R.p[a] / (R.omega[a] * r));
    q.c = (float)R.c[a];
    q.m = (float)m;
    q.ih = (float)(1.0 / R.h[a]);
    q.vx = (float)R.vx[a]; q.vy = (float)R.vy[a]; q.vz = (float)R.vz[a];
    q.spare[0] = q.spare[1] = q.spare[2] = 0.0f;
    return q;
}

__device__ __forceinline__ RecMU make_recmu(const RecM& f)
{
    RecMU q;
    q.qx = f.qx; q.qy = f.qy; q.qz = f.qz; q.pad = 0u;
    q.k11 = f.k11; q.k12 = f.k12; q.k13 = f.k13; q.k22 = f.k22; q.k23 = f.k23; q.k33 = f.k33;
    q.q = f.q; q.ih = f.ih;
    q.vx = f.vx; q.vy = f.vy; q.vz = f.vz;
    q.spare = 0.0f;
    return q;
}

// the record of slot a in the layout the uniformity flag selects
__device__ __forceinline__ void put_recm(const Domain* dom, void* rec, const RecSrcM& R,
                                         int64_t a, const PosM& pa, double c11, double c12,
                                         double c13, double c22, double c23, double c33)
{
    const RecM f = make_recm(R, a, pa, c11, c12, c13, c22, c23, c33);
    if (dom->nonuniform) ((RecM*)rec)[a] = f;
    else ((RecMU*)rec)[a] = make_recmu(f);
}

template <bool kTab>
__global__ __launch_bounds__(kBlock) SPH_WAVES_CAP(SPH_WAVES_MIXED) void k_iad_m(Params P, Domain* __restrict__ dom,
                                                  const int32_t* __restrict__ nc,
                                                  const int32_t* __restrict__ list,
                                                  const PosM* __restrict__ pm,
                                                  const double* __restrict__ h,
                                                  double* __restrict__ c11, double* __restrict__ c12,
                                                  double* __restrict__ c13, double* __restrict__ c22,
                                                  double* __restrict__ c23, double* __restrict__ c33,
                                                  RecSrcM R, void* __restrict__ rec)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    const int64_t a = lb * kBlock + threadIdx.x;
    if (a >= P.n) return;
    const FixGeom g = fix_geom(P, *dom);
    const PosM pa = pm[a];
    const double ha = h[a];
    const float tsc = (float)(kPiHalfSq / (ha * ha));
    const float w0 = (float)(P.bn / (ha * ha * ha));
    const int cnt = min(nc[a], P.ng_max);
    double t11 = 0, t12 = 0, t13 = 0, t22 = 0, t23 = 0, t33 = 0;
    // the next batch's list entries are fetched while this batch computes
    int32_t nx[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) nx[u] = (u < cnt) ? list[lpos(a, u, P.ng_max)] : -1;
    for (int j0 = 0; j0 < cnt; j0 += kBatch) {
        bool ok[kBatch];
        PosM q[kBatch];
        float vb[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            ok[u] = (uint32_t)nx[u] < (uint32_t)P.n;
            const int32_t b = ok[u] ? nx[u] : (int32_t)a;
            q[u] = pm[b];
            vb[u] = q[u].w;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int j = j0 + kBatch + u;
            nx[u] = (j < cnt) ? list[lpos(a, j, P.ng_max)] : -1;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
#pragma clang fp contract(fast)
            if (!ok[u]) continue;
            float dx, dy, dz;
            const float r2 = disp_m(g, pa, q[u], dx, dy, dz);
            const float sw = vb[u] * (w0 * kern_S_f_t<kTab>(P, r2 * tsc));
            const float sx = sw * dx, sy = sw * dy, sz = sw * dz;
            t11 += (double)(sx * dx);
            t12 += (double)(sx * dy);
            t13 += (double)(sx * dz);
            t22 += (double)(sy * dy);
            t23 += (double)(sy * dz);
            t33 += (double)(sz * dz);
        }
    }
    // 3x3 inversion in FP64
    double a11 = t22 * t33 - t23 * t23;
    double a12 = t13 * t23 - t12 * t33;
    double a13 = t12 * t23 - t13 * t22;
    double a22 = t11 * t33 - t13 * t13;
    double a23 = t12 * t13 - t11 * t23;
    double a33 = t11 * t22 - t12 * t12;
    double det = t11 * a11 + t12 * a12 + t13 * a13;
    if (det > 0.0) {
        double id = 1.0 / det;
        a11 *= id; a12 *= id; a13 *= id; a22 *= id; a23 *= id; a33 *= id;
    } else {
        a11 = a12 = a13 = a22 = a23 = a33 = 0.0;
        set_err(dom, SPH_ERRBIT_SINGULAR_TAU);
    }
    c11[a] = a11; c12[a] = a12; c13[a] = a13;
    c22[a] = a22; c23[a] = a23; c33[a] = a33;
    if (rec) put_recm(dom, rec, R, a, pa, a11, a12, a13, a22, a23, a33);
}

__global__ __launch_bounds__(kBlock) void k_pack_recm(int64_t n, const Domain* __restrict__ dom,
                                                      RecSrcM R,
                                                      const PosM* __restrict__ pm,
                                                      const double* __restrict__ c11,
                                                      const double* __restrict__ c12,
                                                      const double* __restrict__ c13,
                                                      const double* __restrict__ c22,
                                                      const double* __restrict__ c23,
                                                      const double* __restrict__ c33,
                                                      void* __restrict__ rec)
{
    int64_t a = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (a < n) put_recm(dom, rec, R, a, pm[a], c11[a], c12[a], c13[a], c22[a], c23[a], c33[a]);
}

struct MomOutM {
    double *ax, *ay, *az, *du;
};

__global__ void k_dtmin_begin_m(Domain* d) { d->dtmin_bits = ord_bits(INFINITY); }

// what the target reads of itself beside its record (FP64 arrays)
struct MomSelfM {
    const double *h, *c, *c11, *c12, *c13, *c22, *c23, *c33, *rho, *omega, *p, *m;
};

template <class Rec>
__device__ __forceinline__ PosM rec_pos(const Rec& r) { return PosM{r.qx, r.qy, r.qz, 0.0f}; }

// a neighbour's record (its position in the first column): 80 bytes, or 64
// with equal masses and sound speeds
struct NbrM {
    const RecM* rec;
    const RecMU* recu;
};
SPH_DEV const RecM* nbr_recs(const NbrM& N, const RecM&) { return N.rec; }
SPH_DEV const RecMU* nbr_recs(const NbrM& N, const RecMU&) { return N.recu; }
SPH_DEV float nbr_m(const RecM& r, float) { return r.m; }
SPH_DEV float nbr_c(const RecM& r, float) { return r.c; }
SPH_DEV float nbr_m(const RecMU&, float m0) { return m0; }
SPH_DEV float nbr_c(const RecMU&, float c0) { return c0; }

// the LDS staging of the momentum pass: batches of SPH_MOM_M_U_BATCH records
// per wavefront at a stride of kMixPad columns (both record layouts)
constexpr int kMixPad = 5;
constexpr int kMixStage = (kBlock / 64) * SPH_MOM_M_U_BATCH * 64 * kMixPad;

template <class Rec, bool kTab>
__device__ __forceinline__ void momentum_energy_m(const Params& P, Domain* __restrict__ dom,
                                                  const int32_t* __restrict__ nc,
                                                  const int32_t* __restrict__ ns,
                                                  const int32_t* __restrict__ list,
                                                  const NbrM& N, const MomSelfM& T,
                                                  const double* __restrict__ u,
                                                  const MomOutM& O, int64_t a_lane,
                                                  int4* __restrict__ stage)
{
    // lanes past the end shadow the last slot with an empty list (every lane
    // of a wavefront takes part in the staged gathers)
    const bool live = a_lane < P.n;
    const int64_t a = live ? a_lane : P.n - 1;
    double dtc = INFINITY;
    {
        const FixGeom g = fix_geom(P, *dom);
        const Rec* __restrict__ recs = nbr_recs(N, Rec{});
        const Rec ra = recs[a];
        const PosM pa = rec_pos(ra);
        const float m0 = (float)T.m[0], c0 = (float)T.c[0];   // the uniform record's m, c
        const double ha = T.h[a];
        const float tsa = (float)(kPiHalfSq / (ha * ha));
        const float w0a = (float)(P.bn / (ha * ha * ha));
        const float bn = (float)P.bn;
        const float al = (float)P.alpha;
        const double rho_a = T.rho[a];
        const float pa_ = (float)(T.p[a] / (T.omega[a] * rho_a * rho_a));   // P/(Omega rho^2)
        const float ira = (float)(1.0 / rho_a), ca = nbr_c(ra, c0);
        const float ca11 = (float)T.c11[a], ca12 = (float)T.c12[a], ca13 = (float)T.c13[a];
        const float ca22 = (float)T.c22[a], ca23 = (float)T.c23[a], ca33 = (float)T.c33[a];
        const int ng = P.ng_max;
        const int cg = live ? min(nc[a], ng) : 0;
        const int co = live ? min(ns[a] - nc[a], ng) : 0;
        double axs = 0.0, ays = 0.0, azs = 0.0, e1 = 0.0, e2 = 0.0;
        const int total = cg + co;
        constexpr int kB = SPH_MOM_M_U_BATCH;
        // list entries of the batch starting at k0 (-1 past the end); the next
        // batch's are fetched while this batch computes
        auto entries = [&](int k0, int32_t (&e)[kB]) {
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int k = k0 + u;
                const int j = (k < cg) ? k : ng - 1 - (k - cg);
                e[u] = (k < total) ? list[lpos(a, j, ng)] : -1;
            }
        };
        auto pair = [&](bool gather, const Rec& rb) {
#pragma clang fp contract(fast)
            float dx, dy, dz;
            const float r2 = disp_m(g, pa, rec_pos(rb), dx, dy, dz);
            float Wa = 0.0f;
            if (gather) Wa = w0a * kern_S_f_t<kTab>(P, r2 * tsa);
            // support of W(h_b): v_b < 2, i.e. t_b < pi^2
            const float ih2 = rb.ih * rb.ih;
            const float tb = r2 * ((float)kPiHalfSq * ih2);
            float Wb = 0.0f;
            if (tb < (float)(4.0 * kPiHalfSq)) Wb = bn * (ih2 * rb.ih) * kern_S_f_t<kTab>(P, tb);
            const float Aax = (ca11 * dx + ca12 * dy + ca13 * dz) * Wa;
            const float Aay = (ca12 * dx + ca22 * dy + ca23 * dz) * Wa;
            const float Aaz = (ca13 * dx + ca23 * dy + ca33 * dz) * Wa;
            const float Kx = rb.k11 * dx + rb.k12 * dy + rb.k13 * dz;
            const float Ky = rb.k12 * dx + rb.k22 * dy + rb.k23 * dz;
            const float Kz = rb.k13 * dx + rb.k23 * dy + rb.k33 * dz;
            const float vx = ra.vx - rb.vx, vy = ra.vy - rb.vy, vz = ra.vz - rb.vz;
            const float xv = -(vx * dx + vy * dy + vz * dz);
            float hPi = 0.0f;   // Pi_ab / 2
            if (xv < 0.0f) {
                const float w = xv * __builtin_amdgcn_rsqf(r2);
                const float vsig = ca + nbr_c(rb, c0) - 3.0f * w;
                hPi = -0.25f * al * vsig * w;
            }
            const float mb = nbr_m(rb, m0);
            const float sa = mb * (pa_ + hPi * ira);
            const float sb = (rb.q + hPi) * Wb;
            axs += (double)(-(sa * Aax + sb * Kx));
            ays += (double)(-(sa * Aay + sb * Ky));
            azs += (double)(-(sa * Aaz + sb * Kz));
            const float va = vx * Aax + vy * Aay + vz * Aaz;
            const float vk = vx * Kx + vy * Ky + vz * Kz;
            e1 += (double)(mb * va);
            e2 += (double)(hPi * (mb * ira * va + Wb * vk));
        };
        int32_t nx[kB];
        entries(0, nx);
        {
            // Staged gathers: in load i lane L takes column (64 i + L) mod C of
            // record (64 i + L) / C (C = 4 columns with equal masses and sound
            // speeds, else 5), so that C lanes read one whole record and a
            // load covers 64 / C; the columns go to LDS at a stride of five
            // columns per record (20 dwords: the lanes' 16-byte reads of their
            // own records then hit distinct banks).  Dword-wide reads at that
            // stride conflict four ways: a layout whose used fields let the
            // compiler pair dwords across column boundaries (7 ds_read2_b32
            // per record instead of 16-byte reads) made this pass 26.5 ->
            // 30.9 ms at 64 M particles, hence lds_record.  C3 (unequal sound
            // speeds): 7.66 -> 7.40 ms against per-lane gathers.
            constexpr int kCols = (int)(sizeof(Rec) / 16);
            static_assert(sizeof(Rec) % 16 == 0, "records of whole 16-byte columns");
            static_assert(kCols <= kMixPad, "the staging stride holds a record");
            const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
            int4* const mine = stage + wv * (kB * 64 * kMixPad);
            int tmax = total;   // the wavefront runs to its longest list
            for (int o = 32; o > 0; o >>= 1) tmax = max(tmax, __shfl_xor(tmax, o, 64));
            const int4* col = (const int4*)recs;
            for (int k0 = 0; k0 < tmax; k0 += kB) {
                bool ok[kB];
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    ok[u] = (uint32_t)nx[u] < (uint32_t)P.n;
                    const int32_t src = ok[u] ? nx[u] : (int32_t)a;
#pragma unroll
                    for (int i = 0; i < kCols; ++i) {
                        const int q = 64 * i + lane;
                        const int r = q / kCols, c = q % kCols;
                        const int32_t b = __shfl(src, r, 64);
                        mine[(u * 64 + r) * kMixPad + c] = col[(int64_t)b * kCols + c];
                    }
                }
                entries(k0 + kB, nx);
                // LDS operations of one wavefront complete in order; the fences
                // keep the compiler from moving the reads above the writes or
                // the next batch's writes above this batch's reads
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    const Rec rb = lds_record<Rec>(&mine[(u * 64 + lane) * kMixPad]);
                    if (ok[u]) pair(k0 + u < cg, rb);
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
        }
        if (live) {
            // the energy rate is assembled in FP64
            const double du = (double)pa_ * e1 + 0.5 * e2;
            O.ax[a] = axs;
            O.ay[a] = ays;
            O.az[a] = azs;
            O.du[a] = du;
            if (!isfinite(axs) || !isfinite(ays) || !isfinite(azs) || !isfinite(du))
                set_err(dom, SPH_ERRBIT_NONFINITE);
            const double cA = T.c[a];
            dtc = P.courant * (ha / cA);
            if (P.acc_dt > 0.0) {
                double am = sqrt((axs * axs + ays * ays) + azs * azs);
                double qa = P.acc_dt * sqrt(ha / am);
                if (qa < dtc) dtc = qa;
            }
            if (P.energy_dt > 0.0) {
                double qu = P.energy_dt * (fabs(u[a]) / fabs(du));
                if (qu < dtc) dtc = qu;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) dtc = fmin(dtc, __shfl_xor(dtc, o, 64));
    if ((threadIdx.x & 63) == 0 && dtc < INFINITY)
        ord_min_to(&dom->dtmin_bits, dtc);
}

// the record layout the uniformity flag selected when the records were written
template <bool kTab>
__global__ __launch_bounds__(kBlock) SPH_WAVES_CAP(SPH_WAVES_MIXED) void k_momentum_energy_m(Params P, Domain* __restrict__ dom,
                                                              const int32_t* __restrict__ nc,
                                                              const int32_t* __restrict__ ns,
                                                              const int32_t* __restrict__ list,
                                                              NbrM N, MomSelfM T,
                                                              const double* __restrict__ u,
                                                              MomOutM O)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    const int64_t a = lb * kBlock + threadIdx.x;
    // one staging buffer for both layouts (two would both be allocated)
    __shared__ int4 stage[kMixStage];
    if (dom->nonuniform)
        momentum_energy_m<RecM, kTab>(P, dom, nc, ns, list, N, T, u, O, a, stage);
    else
        momentum_energy_m<RecMU, kTab>(P, dom, nc, ns, list, N, T, u, O, a, stage);
}

RecSrcM recm_src(const sph_particles* p)
{
    return RecSrcM{p->m, p->rho, p->omega, p->p, p->c, p->vx, p->vy, p->vz, p->h};
}

}  // namespace

static_assert(sizeof(PosM) == 16, "PosM layout");
static_assert(sizeof(RecM) == 80, "RecM layout");
static_assert(sizeof(RecM) <= sizeof(MomRec), "RecM records alias the MomRec area");
static_assert(sizeof(RecMU) == 64, "RecMU layout: four 16-byte columns");
size_t mixed_posm_bytes() { return sizeof(PosM); }
size_t mixed_rec_bytes() { return sizeof(RecM); }

hipError_t launch_pack_posm(const Params& P, const Ws& W, const sph_particles* p, hipStream_t s)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    k_pack_posm<<<nb, kBlock, 0, s>>>(P, W.dom, p->x, p->y, p->z, p->m, (PosM*)W.posm);
    return hipGetLastError();
}

hipError_t launch_density_mixed(const Params& P, const Layout& L, const Ws& W, sph_particles* p,
                                hipStream_t s, bool pack)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    PosM* pm = (PosM*)W.posm;
    if (pack) k_pack_posm<<<nb, kBlock, 0, s>>>(P, W.dom, p->x, p->y, p->z, p->m, pm);
    // The weakly compressible EOS P = p_ref + c0^2 (rho - rho_ref) multiplies a
    // relative density error by c0^2 rho / |P| (about 340 on the rotating square
    // patch), so its density pair terms stay FP64; IAD and momentum stay mixed.
    if (P.eos == SPH_EOS_WEAKLY_COMPRESSIBLE) return launch_density(P, L, W, p, s, pack);
    k_density_m<<<grid_xcd(nb), kBlock, 0, s>>>(P, W.dom, W.nc, W.list, pm, p->h, p->m,
                                                p->u, p->p_ref, p->rho_ref, p->rho, p->omega,
                                                p->p, p->c);
    return hipGetLastError();
}

hipError_t launch_iad_mixed(const Params& P, const Layout& L, const Ws& W, sph_particles* p,
                            hipStream_t s, bool pack, bool write_rec)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    PosM* pm = (PosM*)W.posm;
    if (pack) k_pack_posm<<<nb, kBlock, 0, s>>>(P, W.dom, p->x, p->y, p->z, p->m, pm);
    if (write_rec) launch_uniform_check(P, W, p, s);
    k_volume_m<<<nb, kBlock, 0, s>>>(P.n, p->m, p->rho, pm);
    with_table(P, [&](auto tab) {
        k_iad_m<decltype(tab)::value><<<grid_xcd(nb), kBlock, 0, s>>>(
            P, W.dom, W.nc, W.list, pm, p->h, p->c11, p->c12, p->c13, p->c22, p->c23,
            p->c33, recm_src(p), write_rec ? W.recm : nullptr);
    });
    return hipGetLastError();
}

hipError_t launch_momentum_energy_mixed(const Params& P, const Layout& L, const Ws& W,
                                        sph_particles* p, hipStream_t s, bool pack)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    PosM* pm = (PosM*)W.posm;
    if (pack) {
        k_pack_posm<<<nb, kBlock, 0, s>>>(P, W.dom, p->x, p->y, p->z, p->m, pm);
        launch_uniform_check(P, W, p, s);
        k_pack_recm<<<nb, kBlock, 0, s>>>(P.n, W.dom, recm_src(p), pm, p->c11, p->c12, p->c13,
                                          p->c22, p->c23, p->c33, W.recm);
    }
    MomOutM O{p->ax, p->ay, p->az, p->du};
    MomSelfM T{p->h, p->c, p->c11, p->c12, p->c13, p->c22, p->c23, p->c33, p->rho, p->omega, p->p,
               p->m};
    NbrM N{(const RecM*)W.recm, (const RecMU*)W.recm};
    k_dtmin_begin_m<<<1, 1, 0, s>>>(W.dom);
    with_table(P, [&](auto tab) {
        k_momentum_energy_m<decltype(tab)::value><<<grid_xcd(nb), kBlock, 0, s>>>(
            P, W.dom, W.nc, W.ns, W.list, N, T, p->u, O);
    });
    return hipGetLastError();
}

}  // namespace sph
