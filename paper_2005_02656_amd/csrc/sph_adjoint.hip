// sph_adjoint.hip -- reverse mode of one SPH step with a frozen structure.
//
// Frozen: h of every particle, the time steps dt and dt_m1, the neighbour sets
// (they follow from the fixed h) and the artificial-viscosity branches.  What
// is differentiated is the step map of section 4.1 as the forward kernels
// evaluate it: density and grad-h term (eq. 1), EOS, IAD matrix tau and its
// inverse C, momentum/energy rates (eqs. 2-5, with AV) and the kick-drift /
// Adams-Bashforth integrator.
//
// Every pass is in gather form: the symmetric list N_s(i) holds every j for
// which i takes part in a pair term (i in N_s(j) iff j in N_s(i)), so the
// thread of particle i adds the contributions of the pair (i, j) -- i the
// target -- and of the pair (j, i) -- i the neighbour -- to i's own adjoint.
// There are no floating-point atomics; results are bitwise reproducible.
//
// Passes (reverse order of the forward):
//   integrate^T -> momentum/energy^T (+ EOS^T, tau_bar = -C Cbar C)
//   -> IAD^T (+ rho/Omega -> density-sum seeds) -> density^T -> unpermute.
#include "sph_common.h"

// neighbours whose records are loaded before computing on them, per pass
#ifndef SPH_ADJ_MOM_BATCH
#define SPH_ADJ_MOM_BATCH 1
#endif
#ifndef SPH_ADJ_DENS_BATCH
#define SPH_ADJ_DENS_BATCH 4
#endif

namespace sph {

// ---------------------------------------------------------------- adjoint workspace
// Packed per-slot records gathered by the neighbour loops of later passes.
struct alignas(16) RateBar {   // adjoints of the rates of one slot
    double ax, ay, az, du;
};
struct alignas(16) TauBar {    // symmetric tau adjoint and the volume m/rho
    double t11, t12, t13, t22, t23, t33, vol, pad;
};
struct alignas(16) SumBar {    // adjoints of the two density sums, and the mass
    double sS, sD, m, pad;
};

struct AdjLayout {
    size_t rate, tau, sum, xb, yb, zb, vxb, vyb, vzb, rhob, omb, ub, vhxb, vhyb, vhzb, dum1b;
    size_t total;
};

static size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

static AdjLayout adj_layout(int64_t n)
{
    AdjLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = a256(o + bytes); return at; };
    L.rate = take(sizeof(RateBar) * n);
    L.tau = take(sizeof(TauBar) * n);
    L.sum = take(sizeof(SumBar) * n);
    size_t* soa[] = {&L.xb, &L.yb, &L.zb, &L.vxb, &L.vyb, &L.vzb, &L.rhob, &L.omb, &L.ub,
                     &L.vhxb, &L.vhyb, &L.vhzb, &L.dum1b};
    for (size_t* f : soa) *f = take(sizeof(double) * n);
    L.total = o;
    return L;
}

size_t adjoint_workspace_bytes(int64_t n) { return adj_layout(n).total; }

namespace {

struct Adj {
    RateBar* rate;
    TauBar* tau;
    SumBar* sum;
    double *xb, *yb, *zb, *vxb, *vyb, *vzb, *rhob, *omb, *ub, *vhxb, *vhyb, *vhzb, *dum1b;
};

Adj carve_adj(void* base, int64_t n)
{
    const AdjLayout L = adj_layout(n);
    char* b = (char*)base;
    Adj J;
    J.rate = (RateBar*)(b + L.rate);
    J.tau = (TauBar*)(b + L.tau);
    J.sum = (SumBar*)(b + L.sum);
    J.xb = (double*)(b + L.xb);
    J.yb = (double*)(b + L.yb);
    J.zb = (double*)(b + L.zb);
    J.vxb = (double*)(b + L.vxb);
    J.vyb = (double*)(b + L.vyb);
    J.vzb = (double*)(b + L.vzb);
    J.rhob = (double*)(b + L.rhob);
    J.omb = (double*)(b + L.omb);
    J.ub = (double*)(b + L.ub);
    J.vhxb = (double*)(b + L.vhxb);
    J.vhyb = (double*)(b + L.vhyb);
    J.vhzb = (double*)(b + L.vhzb);
    J.dum1b = (double*)(b + L.dum1b);
    return J;
}

// ---------------------------------------------------------------- kernel derivatives
// value and t-derivative of a polynomial in t (Horner on both)
template <int K>
SPH_DEV void horner_d(const double (&c)[K], double t, double& p, double& dp)
{
    p = c[K - 1];
    dp = 0.0;
#pragma unroll
    for (int k = K - 2; k >= 0; --k) {
        dp = fma(dp, t, p);
        p = fma_sc(p, t, c[k]);
    }
}

// S = sinc^n and dS/dt at t = (pi/2)^2 v^2 (the forward's polynomial for sinc)
SPH_DEV void sinc_dt(double t, int n, double& S, double& dS)
{
    double s, ds;
    horner_d(kSincS64, t, s, ds);
    const double p = pow_nm1(s, n);   // s^(n-1)
    S = p * s;
    dS = (double)n * p * ds;
}

// dS/dt and dQ/dt, with Q = v dS/dv = n s^(n-1) q and q = x sinc'(x) = t qt(t)
SPH_DEV void sinc_dt2(double t, int n, double& dS, double& dQ)
{
    double s, ds, qt, dqt;
    horner_d(kSincS64, t, s, ds);
    horner_d(kSincQ64, t, qt, dqt);
    const double q = qt * t;
    const double dq = qt + t * dqt;
    double p2 = 1.0;   // s^(n-2)
    for (int i = 2; i < n; ++i) p2 = p2 * s;
    const double p1 = p2 * s;   // s^(n-1)
    dS = (double)n * p1 * ds;
    dQ = (double)n * ((double)(n - 1) * p2 * ds * q + p1 * dq);
}

// W(r, h) and dW/d(r^2), or zeros outside the support r < 2h
SPH_DEV void kernel_w(const Params& P, double r2, double h, double& W, double& dW)
{
    const double h2 = 2.0 * h;
    if (r2 < h2 * h2) {
        const double ts = kPiHalfSq / (h * h);
        const double w0 = P.bn / (h * h * h);
        double S, dS;
        sinc_dt(r2 * ts, P.sinc_n, S, dS);
        W = w0 * S;
        dW = w0 * dS * ts;
    } else {
        W = 0.0;
        dW = 0.0;
    }
}

SPH_DEV void cmul(const MomRec& R, const double d[3], double o[3])
{
    o[0] = R.c11 * d[0] + R.c12 * d[1] + R.c13 * d[2];
    o[1] = R.c12 * d[0] + R.c22 * d[1] + R.c23 * d[2];
    o[2] = R.c13 * d[0] + R.c23 * d[1] + R.c33 * d[2];
}

// what one particle receives from the momentum/energy reverse pass
struct MomAcc {
    double x[3], v[3];
    double irho, pb, c;
    double C[6];   // symmetric part of the C adjoint, packed 11 12 13 22 23 33
    double e1;     // sum_b m_b v_ab . A_ab(h_a) of the target (for d du / d pb)
};

// Reverse mode of the momentum/energy term of target a with neighbour b
// (d = x_b - x_a, Wa = W(r, h_a) if b in N(a) else 0, Wb = W(r, h_b) if
// r < 2 h_b else 0, dWa, dWb their r^2 derivatives), given the target's rate
// adjoints rb.  Adds to the adjoint of side a (kToA) or side b.
template <bool kToA>
SPH_DEV void mom_pair_bwd(const Params& P, const double d[3], double r2, double Wa, double dWa,
                          double Wb, double dWb, const MomRec& A, const MomRec& B,
                          const RateBar& rb, MomAcc& acc)
{
    double Ua[3], Ub[3];
    cmul(A, d, Ua);
    cmul(B, d, Ub);
    const double Aa[3] = {Ua[0] * Wa, Ua[1] * Wa, Ua[2] * Wa};
    const double Ab[3] = {Ub[0] * Wb, Ub[1] * Wb, Ub[2] * Wb};
    const double vab[3] = {A.vx - B.vx, A.vy - B.vy, A.vz - B.vz};
    const double xv = -(vab[0] * d[0] + vab[1] * d[1] + vab[2] * d[2]);
    const bool av = xv < 0.0;
    double Pi = 0.0, w = 0.0, ir = 1.0;   // ir = 1/r
    if (av) {
        ir = rsqrt_nr(r2);
        w = xv * ir;
        Pi = -0.5 * P.alpha * (A.c + B.c - 3.0 * w) * w;
    }
    const double mb = B.m;
    const double gk = 0.5 * mb * Pi;
    // forward: f = mb (pb_a Aa + pb_b Ab), g = gk (Aa/rho_a + Ab/rho_b),
    //          a -= f + g, e1 += mb vab.Aa, e2 += vab.g, du = pb_a e1 + e2/2
    const double abar[3] = {rb.ax, rb.ay, rb.az};
    const double e1b = rb.du * A.pb, e2b = 0.5 * rb.du;
    double gb[3], Abar_a[3], Abar_b[3], vabb[3];
    double fA = 0.0, fB = 0.0, gA = 0.0, gB = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        gb[k] = -abar[k] + e2b * vab[k];
        const double g = gk * (Aa[k] * A.irho + Ab[k] * B.irho);
        Abar_a[k] = -mb * A.pb * abar[k] + gk * A.irho * gb[k] + e1b * mb * vab[k];
        Abar_b[k] = -mb * B.pb * abar[k] + gk * B.irho * gb[k];
        vabb[k] = e1b * mb * Aa[k] + e2b * g;
        fA += abar[k] * Aa[k];
        fB += abar[k] * Ab[k];
        gA += gb[k] * Aa[k];
        gB += gb[k] * Ab[k];
    }
    double db[3];
    double Ca[3], Cb[3];
    cmul(A, Abar_a, Ca);
    cmul(B, Abar_b, Cb);
    const double Wab = Abar_a[0] * Ua[0] + Abar_a[1] * Ua[1] + Abar_a[2] * Ua[2];
    const double Wbb = Abar_b[0] * Ub[0] + Abar_b[1] * Ub[1] + Abar_b[2] * Ub[2];
    const double r2b = Wab * dWa + Wbb * dWb;
#pragma unroll
    for (int k = 0; k < 3; ++k) db[k] = Wa * Ca[k] + Wb * Cb[k] + 2.0 * r2b * d[k];
    double cbar = 0.0;
    if (av) {
        const double Pib = 0.5 * mb * (A.irho * gA + B.irho * gB);
        cbar = Pib * (-0.5 * P.alpha * w);
        const double wb = Pib * (-0.5 * P.alpha) * (A.c + B.c - 6.0 * w);
        const double xvb = wb * ir;          // w = xv / r
        const double rbar = -wb * xv * (ir * ir);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            vabb[k] -= xvb * d[k];          // xv = -vab . d
            db[k] += -xvb * vab[k] + rbar * d[k] * ir;
        }
    }
    if (kToA) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            acc.x[k] -= db[k];
            acc.v[k] += vabb[k];
        }
        acc.irho += gk * gA;
        acc.pb += -mb * fA;
        acc.c += cbar;
        const double s = Wa;
        acc.C[0] += s * Abar_a[0] * d[0];
        acc.C[1] += s * 0.5 * (Abar_a[0] * d[1] + Abar_a[1] * d[0]);
        acc.C[2] += s * 0.5 * (Abar_a[0] * d[2] + Abar_a[2] * d[0]);
        acc.C[3] += s * Abar_a[1] * d[1];
        acc.C[4] += s * 0.5 * (Abar_a[1] * d[2] + Abar_a[2] * d[1]);
        acc.C[5] += s * Abar_a[2] * d[2];
        acc.e1 += mb * (vab[0] * Aa[0] + vab[1] * Aa[1] + vab[2] * Aa[2]);
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            acc.x[k] += db[k];
            acc.v[k] -= vabb[k];
        }
        acc.irho += gk * gB;
        acc.pb += -mb * fB;
        acc.c += cbar;
        const double s = Wb;
        acc.C[0] += s * Abar_b[0] * d[0];
        acc.C[1] += s * 0.5 * (Abar_b[0] * d[1] + Abar_b[1] * d[0]);
        acc.C[2] += s * 0.5 * (Abar_b[0] * d[2] + Abar_b[2] * d[0]);
        acc.C[3] += s * Abar_b[1] * d[1];
        acc.C[4] += s * 0.5 * (Abar_b[1] * d[2] + Abar_b[2] * d[1]);
        acc.C[5] += s * Abar_b[2] * d[2];
    }
}

// ---------------------------------------------------------------- integrate^T
struct GradIO {
    const double *x, *y, *z, *vx, *vy, *vz, *vhx, *vhy, *vhz, *u, *du_m1;
};

// x' = x + vh' dt (wrap: a constant shift), vh' = vh + a kick, v' = vh' + a dt/2,
// u' = u + dt((1+q) du - q du_m1) (q = dt / (2 dt_m1); first step: u + dt du),
// du_m1' = du.
__global__ __launch_bounds__(kBlock) void k_adj_integrate(Params P, const sph_globals* __restrict__ g,
                                                          GradIO go, Adj J)
{
    const int64_t a = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (a >= P.n) return;
    const double dt = g->dt, lam = g->dt_m1;
    const double kick = 0.5 * (lam + dt), half = 0.5 * dt;
    const bool ab2 = lam > 0.0;
    const double q = ab2 ? dt / (2.0 * lam) : 0.0;
    const double xo[3] = {go.x[a], go.y[a], go.z[a]};
    const double vo[3] = {go.vx[a], go.vy[a], go.vz[a]};
    const double vho[3] = {go.vhx[a], go.vhy[a], go.vhz[a]};
    double vhb[3], ab[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        vhb[k] = vho[k] + vo[k] + xo[k] * dt;
        ab[k] = vo[k] * half + vhb[k] * kick;
    }
    const double uo = go.u[a];
    RateBar r;
    r.ax = ab[0];
    r.ay = ab[1];
    r.az = ab[2];
    r.du = go.du_m1[a] + uo * dt * (ab2 ? 1.0 + q : 1.0);
    J.rate[a] = r;
    J.xb[a] = xo[0];
    J.yb[a] = xo[1];
    J.zb[a] = xo[2];
    J.ub[a] = uo;
    J.vhxb[a] = vhb[0];
    J.vhyb[a] = vhb[1];
    J.vhzb[a] = vhb[2];
    J.dum1b[a] = ab2 ? -uo * dt * q : 0.0;
}

// ---------------------------------------------------------------- momentum/energy^T
struct MomFwd {
    const Pos4* p4;
    const MomRec* rec;
    const double *rho, *omega, *c, *u, *vol;
};

// two wavefronts per SIMD: the pair's reverse terms fit 256 registers without
// spills, and at one wavefront the gathers' latency went unhidden
#ifndef SPH_ADJ_MOM_ATTR
#define SPH_ADJ_MOM_ATTR SPH_WAVES_EXACT(2)
#endif
__global__ __launch_bounds__(kBlock) SPH_ADJ_MOM_ATTR void k_adj_momentum(Params P, const int32_t* __restrict__ nc,
                                                         const int32_t* __restrict__ ns,
                                                         const int32_t* __restrict__ list,
                                                         MomFwd F, Adj J)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    const int64_t i = lb * kBlock + threadIdx.x;
    if (i >= P.n) return;
    const MomRec ri = F.rec[i];   // the record holds the position and h
    const RateBar bi = J.rate[i];
    MomAcc acc = {};
    const int ng = P.ng_max;
    const int cg = min(nc[i], ng);
    const int total = cg + min(ns[i] - nc[i], ng);
    constexpr int kB = SPH_ADJ_MOM_BATCH;
    for (int k0 = 0; k0 < total; k0 += kB) {
        int32_t jj[kB];
        bool ok[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int k = k0 + u;
            const int slot = k < cg ? k : ng - 1 - (k - cg);
            const int32_t j = k < total ? list[lpos(i, slot, ng)] : -1;
            ok[u] = (uint32_t)j < (uint32_t)P.n;
            jj[u] = ok[u] ? j : (int32_t)i;
        }
        MomRec rj[kB];
        RateBar bj[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            rj[u] = F.rec[jj[u]];
            bj[u] = J.rate[jj[u]];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            if (!ok[u]) continue;
            double d[3];
            const double r2 = disp(P, ri.x, ri.y, ri.z, rj[u].x, rj[u].y, rj[u].z, d[0], d[1], d[2]);
            double Wi, dWi, Wj, dWj;
            kernel_w(P, r2, ri.h, Wi, dWi);   // nonzero iff j in N(i)
            kernel_w(P, r2, rj[u].h, Wj, dWj);
            // pair (i, j): i the target
            mom_pair_bwd<true>(P, d, r2, Wi, dWi, Wj, dWj, ri, rj[u], bi, acc);
            // pair (j, i): i the neighbour, displacement x_i - x_j
            const double dn[3] = {-d[0], -d[1], -d[2]};
            mom_pair_bwd<false>(P, dn, r2, Wj, dWj, Wi, dWi, rj[u], ri, bj[u], acc);
        }
    }
    // pb = P / (Omega rho^2) also enters du through pb_a e1
    const double rho = F.rho[i], om = F.omega[i];
    const double pbb = acc.pb + bi.du * acc.e1;
    const double pb = ri.pb;
    const double Pbar = pbb / (om * rho * rho);
    const double ombar = -pbb * pb / om;
    double rhobar = -2.0 * pbb * pb / rho - acc.irho * (ri.irho * ri.irho);
    double ubar = J.ub[i];
    // EOS
    if (P.eos == SPH_EOS_IDEAL) {
        const double u = F.u[i];
        rhobar += Pbar * (P.gamma - 1.0) * u;
        ubar += Pbar * (P.gamma - 1.0) * rho;
        const double c = F.c[i];
        if (c > 0.0) ubar += acc.c * P.gamma * (P.gamma - 1.0) / (2.0 * c);
    } else {
        rhobar += Pbar * P.c0 * P.c0;
    }
    // tau = C^-1: tau_bar = -C Cbar C (Cbar symmetric, C symmetric)
    const double Cm[9] = {ri.c11, ri.c12, ri.c13, ri.c12, ri.c22, ri.c23, ri.c13, ri.c23, ri.c33};
    const double G[9] = {acc.C[0], acc.C[1], acc.C[2], acc.C[1], acc.C[3], acc.C[4],
                         acc.C[2], acc.C[4], acc.C[5]};
    double M[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            M[3 * r + c] = G[3 * r] * Cm[c] + G[3 * r + 1] * Cm[3 + c] + G[3 * r + 2] * Cm[6 + c];
    auto T = [&](int r, int c) {
        return -(Cm[3 * r] * M[c] + Cm[3 * r + 1] * M[3 + c] + Cm[3 * r + 2] * M[6 + c]);
    };
    TauBar tb;
    tb.t11 = T(0, 0);
    tb.t12 = 0.5 * (T(0, 1) + T(1, 0));
    tb.t13 = 0.5 * (T(0, 2) + T(2, 0));
    tb.t22 = T(1, 1);
    tb.t23 = 0.5 * (T(1, 2) + T(2, 1));
    tb.t33 = T(2, 2);
    tb.vol = F.vol[i];
    tb.pad = 0.0;
    J.tau[i] = tb;
    J.xb[i] += acc.x[0];
    J.yb[i] += acc.x[1];
    J.zb[i] += acc.x[2];
    J.vxb[i] = acc.v[0];
    J.vyb[i] = acc.v[1];
    J.vzb[i] = acc.v[2];
    J.rhob[i] = rhobar;
    J.omb[i] = ombar;
    J.ub[i] = ubar;
}

// ---------------------------------------------------------------- IAD^T
// gradient with respect to d of V W(r, h) d^T T d (T symmetric), and d^T T d
SPH_DEV void tau_term_bwd(const TauBar& T, const double d[3], double W, double dW, double V,
                          double g[3], double& q)
{
    const double Td0 = T.t11 * d[0] + T.t12 * d[1] + T.t13 * d[2];
    const double Td1 = T.t12 * d[0] + T.t22 * d[1] + T.t23 * d[2];
    const double Td2 = T.t13 * d[0] + T.t23 * d[1] + T.t33 * d[2];
    q = Td0 * d[0] + Td1 * d[1] + Td2 * d[2];
    const double a = 2.0 * V * W, b = 2.0 * V * dW * q;
    g[0] = a * Td0 + b * d[0];
    g[1] = a * Td1 + b * d[1];
    g[2] = a * Td2 + b * d[2];
}

__global__ __launch_bounds__(kBlock) void k_adj_iad(Params P, const int32_t* __restrict__ nc,
                                                    const int32_t* __restrict__ ns,
                                                    const int32_t* __restrict__ list,
                                                    const Pos4* __restrict__ p4,
                                                    const double* __restrict__ m,
                                                    const double* __restrict__ rho,
                                                    const double* __restrict__ omega, Adj J)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    const int64_t i = lb * kBlock + threadIdx.x;
    if (i >= P.n) return;
    const Pos4 qi = p4[i];
    const TauBar ti = J.tau[i];
    const double hi2 = 2.0 * qi.h;
    double xb[3] = {0.0, 0.0, 0.0};
    double volb = 0.0;
    const int ng = P.ng_max;
    const int cg = min(nc[i], ng);
    const int total = cg + min(ns[i] - nc[i], ng);
    constexpr int kB = 4;
    for (int k0 = 0; k0 < total; k0 += kB) {
        int32_t jj[kB];
        bool ok[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int k = k0 + u;
            const int slot = k < cg ? k : ng - 1 - (k - cg);
            const int32_t j = k < total ? list[lpos(i, slot, ng)] : -1;
            ok[u] = (uint32_t)j < (uint32_t)P.n;
            jj[u] = ok[u] ? j : (int32_t)i;
        }
        Pos4 qj[kB];
        TauBar tj[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            qj[u] = p4[jj[u]];
            tj[u] = J.tau[jj[u]];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            if (!ok[u]) continue;
            double d[3];
            const double r2 = disp(P, qi.x, qi.y, qi.z, qj[u].x, qj[u].y, qj[u].z, d[0], d[1], d[2]);
            double W, dW, g[3], q;
            // tau_i holds V_j W(r, h_i) d d^T (d = x_j - x_i): x_i enters as -d
            if (r2 < hi2 * hi2) {
                kernel_w(P, r2, qi.h, W, dW);
                tau_term_bwd(ti, d, W, dW, tj[u].vol, g, q);
                xb[0] -= g[0];
                xb[1] -= g[1];
                xb[2] -= g[2];
            }
            // tau_j holds V_i W(r, h_j) d' d'^T with d' = x_i - x_j = -d; the
            // gradient is odd in d, so the one with respect to d' is -g
            const double hj2 = 2.0 * qj[u].h;
            if (r2 < hj2 * hj2) {
                kernel_w(P, r2, qj[u].h, W, dW);
                tau_term_bwd(tj[u], d, W, dW, ti.vol, g, q);
                xb[0] -= g[0];
                xb[1] -= g[1];
                xb[2] -= g[2];
                volb += W * q;
            }
        }
    }
    J.xb[i] += xb[0];
    J.yb[i] += xb[1];
    J.zb[i] += xb[2];
    // V_i = m_i / rho_i
    const double r = rho[i];
    const double rb = J.rhob[i] - volb * ti.vol / r;
    // rho = w0 sS and Omega = 1 - sD / (3 sS) with w0 = B_n / h^3
    const double w0 = P.bn / (qi.h * qi.h * qi.h);
    const double sS = r / w0;
    const double ob = J.omb[i];
    SumBar s;
    s.sS = rb * w0 + ob * (1.0 - omega[i]) / sS;
    s.sD = -ob / (3.0 * sS);
    s.m = m[i];
    s.pad = 0.0;
    J.sum[i] = s;
}

// ---------------------------------------------------------------- density^T
// sS_a = m_a + sum_b m_b S(t_ab), sD_a = 3 m_a + sum_b m_b (3 S + Q)(t_ab),
// t_ab = (pi/2)^2 r_ab^2 / h_a^2; returns the r^2 adjoint of one term
SPH_DEV double sum_term_bwd(const Params& P, double r2, double h, double mb, const SumBar& s)
{
    const double ts = kPiHalfSq / (h * h);
    double dS, dQ;
    sinc_dt2(r2 * ts, P.sinc_n, dS, dQ);
    return mb * ts * (s.sS * dS + s.sD * (3.0 * dS + dQ));
}

__global__ __launch_bounds__(kBlock) void k_adj_density(Params P, const int32_t* __restrict__ nc,
                                                        const int32_t* __restrict__ ns,
                                                        const int32_t* __restrict__ list,
                                                        const Pos4* __restrict__ p4, Adj J)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    const int64_t i = lb * kBlock + threadIdx.x;
    if (i >= P.n) return;
    const Pos4 qi = p4[i];
    const SumBar si = J.sum[i];
    const double hi2 = 2.0 * qi.h;
    double xb[3] = {0.0, 0.0, 0.0};
    const int ng = P.ng_max;
    const int cg = min(nc[i], ng);
    const int total = cg + min(ns[i] - nc[i], ng);
    constexpr int kB = SPH_ADJ_DENS_BATCH;
    for (int k0 = 0; k0 < total; k0 += kB) {
        int32_t jj[kB];
        bool ok[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int k = k0 + u;
            const int slot = k < cg ? k : ng - 1 - (k - cg);
            const int32_t j = k < total ? list[lpos(i, slot, ng)] : -1;
            ok[u] = (uint32_t)j < (uint32_t)P.n;
            jj[u] = ok[u] ? j : (int32_t)i;
        }
        Pos4 qj[kB];
        SumBar sj[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            qj[u] = p4[jj[u]];
            sj[u] = J.sum[jj[u]];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            if (!ok[u]) continue;
            double d[3];
            const double r2 = disp(P, qi.x, qi.y, qi.z, qj[u].x, qj[u].y, qj[u].z, d[0], d[1], d[2]);
            double r2b = 0.0;
            if (r2 < hi2 * hi2) r2b += sum_term_bwd(P, r2, qi.h, sj[u].m, si);
            const double hj2 = 2.0 * qj[u].h;
            if (r2 < hj2 * hj2) r2b += sum_term_bwd(P, r2, qj[u].h, si.m, sj[u]);
            // r^2 = |x_j - x_i|^2: d r^2 / d x_i = -2 d
            xb[0] -= 2.0 * r2b * d[0];
            xb[1] -= 2.0 * r2b * d[1];
            xb[2] -= 2.0 * r2b * d[2];
        }
    }
    J.xb[i] += xb[0];
    J.yb[i] += xb[1];
    J.zb[i] += xb[2];
}

// density-only reverse pass (a loss on rho): sS_bar = rho_bar w0, sD_bar = 0
__global__ __launch_bounds__(kBlock) void k_adj_density_seed(Params P, const double* __restrict__ rhob,
                                                             const Pos4* __restrict__ p4,
                                                             const double* __restrict__ m, Adj J)
{
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= P.n) return;
    const double h = p4[i].h;
    SumBar s;
    s.sS = rhob[i] * (P.bn / (h * h * h));
    s.sD = 0.0;
    s.m = m[i];
    s.pad = 0.0;
    J.sum[i] = s;
    J.xb[i] = 0.0;
    J.yb[i] = 0.0;
    J.zb[i] = 0.0;
}

// ---------------------------------------------------------------- unpermute
struct GradOut {
    double *x, *y, *z, *vx, *vy, *vz, *vhx, *vhy, *vhz, *u, *du_m1;
};

// gradients from the slot order of the step back to the order before its sort
__global__ __launch_bounds__(kBlock) void k_adj_unpermute(int64_t n, const uint32_t* __restrict__ perm,
                                                          Adj J, GradOut gi, int full)
{
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t o = perm[i];
    gi.x[o] = J.xb[i];
    gi.y[o] = J.yb[i];
    gi.z[o] = J.zb[i];
    if (!full) return;
    gi.vx[o] = J.vxb[i];
    gi.vy[o] = J.vyb[i];
    gi.vz[o] = J.vzb[i];
    gi.vhx[o] = J.vhxb[i];
    gi.vhy[o] = J.vhyb[i];
    gi.vhz[o] = J.vhzb[i];
    gi.u[o] = J.ub[i];
    gi.du_m1[o] = J.dum1b[i];
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_step_backward(const Params& P, const Ws& W, const sph_particles* p,
                                const sph_globals* g, const sph_grads* gout, sph_grads* gin,
                                void* adj_ws, hipStream_t s)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    Adj J = carve_adj(adj_ws, P.n);
    GradIO go{gout->x, gout->y, gout->z, gout->vx, gout->vy, gout->vz, gout->vhx, gout->vhy,
              gout->vhz, gout->u, gout->du_m1};
    GradOut gi{gin->x, gin->y, gin->z, gin->vx, gin->vy, gin->vz, gin->vhx, gin->vhy, gin->vhz,
               gin->u, gin->du_m1};
    MomFwd F{W.p4, W.rec, p->rho, p->omega, p->c, p->u, W.vol};
    hipError_t e = launch_pack_rec(P, W, p, s);
    if (e != hipSuccess) return e;
    k_adj_integrate<<<nb, kBlock, 0, s>>>(P, g, go, J);
    k_adj_momentum<<<grid_xcd(nb), kBlock, 0, s>>>(P, W.nc, W.ns, W.list, F, J);
    k_adj_iad<<<grid_xcd(nb), kBlock, 0, s>>>(P, W.nc, W.ns, W.list, W.p4, p->m, p->rho, p->omega,
                                             J);
    k_adj_density<<<grid_xcd(nb), kBlock, 0, s>>>(P, W.nc, W.ns, W.list, W.p4, J);
    k_adj_unpermute<<<nb, kBlock, 0, s>>>(P.n, W.idx0, J, gi, 1);
    return hipGetLastError();
}

hipError_t launch_density_backward(const Params& P, const Ws& W, const sph_particles* p,
                                   const double* rho_bar, double* xb, double* yb, double* zb,
                                   void* adj_ws, hipStream_t s)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    Adj J = carve_adj(adj_ws, P.n);
    GradOut gi{xb, yb, zb, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    k_adj_density_seed<<<nb, kBlock, 0, s>>>(P, rho_bar, W.p4, p->m, J);
    k_adj_density<<<grid_xcd(nb), kBlock, 0, s>>>(P, W.nc, W.ns, W.list, W.p4, J);
    k_adj_unpermute<<<nb, kBlock, 0, s>>>(P.n, W.idx0, J, gi, 0);
    return hipGetLastError();
}

}  // namespace sph
