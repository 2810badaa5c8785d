// sph_pairs.hip -- the three pair passes over the neighbour lists (section 4.1):
// density + grad-h + EOS (eq. 1), IAD matrix and its inverse, and the
// momentum/energy rates with artificial viscosity (eqs. 2-5); plus the global
// minimum time step (section 4.2).
//
// One thread per target slot, wavefronts mapped XCD-contiguously; list column j
// of 64 consecutive targets is one 256-byte coalesced load.  Neighbour data is
// gathered as packed records (32-byte positions, 128-byte momentum records) from
// Morton-local slots (L1/L2 resident).  Sums are FP64 in list order; no atomics
// on floating-point values.
#include "sph_common.h"

namespace sph {
namespace {

// 1: the IAD and momentum pair terms may fuse multiply-adds
#ifndef SPH_PAIR_CONTRACT
#define SPH_PAIR_CONTRACT 1
#endif


__global__ __launch_bounds__(kBlock) SPH_WAVES_CAP(SPH_WAVES_PAIR) void k_density(Params P, Domain* __restrict__ dom,
                                                    const int32_t* __restrict__ nc,
                                                    const int32_t* __restrict__ list,
                                                    const Pos4* __restrict__ p4,
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
    const Pos4 pa = p4[a];
    const double xa = pa.x, ya = pa.y, za = pa.z, ha = pa.h;
    const double tsc = kPiHalfSq / (ha * ha);
    const int cnt = min(nc[a], P.ng_max);
    // self term: S = 1, v dS/dv = 0
    double sS = m[a], sD = 3.0 * m[a];
    for (int j0 = 0; j0 < cnt; j0 += kBatch) {
        int32_t bb[kBatch];
        bool ok[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            int32_t b = (j0 + u < cnt) ? list[lpos(a, j0 + u, P.ng_max)] : -1;
            ok[u] = (uint32_t)b < (uint32_t)P.n;   // also rejects lists not built for this ws
            bb[u] = ok[u] ? b : (int32_t)a;
        }
        double qx[kBatch], qy[kBatch], qz[kBatch], mb[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const Pos4* q = p4 + bb[u];
            qx[u] = q->x; qy[u] = q->y; qz[u] = q->z;
            mb[u] = m[bb[u]];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            if (!ok[u]) continue;
            double dx, dy, dz;
            double r2 = disp(P, xa, ya, za, qx[u], qy[u], qz[u], dx, dy, dz);
            double S, vdS;
            kern_terms(P, r2 * tsc, S, vdS);
            sS += mb[u] * S;
            sD += mb[u] * (3.0 * S + vdS);
        }
    }
    finish_density(P, dom, DensOut{m, u, p_ref, rho_ref, rho, omega, pr, cs}, a, ha, sS, sD);
}

// volume m/rho of every particle (one division per particle instead of per pair)
__global__ __launch_bounds__(kBlock) void k_volume(int64_t n, const double* __restrict__ m,
                                                   const double* __restrict__ rho,
                                                   const Pos4* __restrict__ p4,
                                                   double* __restrict__ vol,
                                                   PosV* __restrict__ pv)
{
    int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= n) return;
    const double v = m[i] / rho[i];
    const Pos4 q = p4[i];
    vol[i] = v;
    pv[i] = PosV{q.x, q.y, q.z, v};
}

struct RecSrc {
    const double *m, *rho, *omega, *p, *c, *vx, *vy, *vz, *h, *x, *y, *z;
};

__device__ __forceinline__ MomNbr make_nbr(const RecSrc& R, int64_t a, const Pos4& pa,
                                           double c11, double c12, double c13, double c22,
                                           double c23, double c33)
{
    MomNbr q;
    q.x = pa.x; q.y = pa.y; q.z = pa.z; q.h = pa.h;
    q.ih = 1.0 / pa.h;
    const double r = R.rho[a], m = R.m[a];
    const double v = m / r;
    q.k11 = v * c11; q.k12 = v * c12; q.k13 = v * c13;
    q.k22 = v * c22; q.k23 = v * c23; q.k33 = v * c33;
    q.q = R.p[a] / (R.omega[a] * r);
    q.c = R.c[a];
    q.m = m;
    q.vx = R.vx[a]; q.vy = R.vy[a]; q.vz = R.vz[a];
    q.spare = 0.0;
    return q;
}

__device__ __forceinline__ MomNbrU make_nbr_u(const RecSrc& R, int64_t a, const Pos4& pa,
                                              double c11, double c12, double c13, double c22,
                                              double c23, double c33)
{
    const MomNbr f = make_nbr(R, a, pa, c11, c12, c13, c22, c23, c33);
    MomNbrU q;
    q.x = f.x; q.y = f.y; q.z = f.z; q.ih = f.ih;
    q.k11 = f.k11; q.k12 = f.k12; q.k13 = f.k13; q.k22 = f.k22; q.k23 = f.k23; q.k33 = f.k33;
    q.q = f.q;
    q.vx = f.vx; q.vy = f.vy; q.vz = f.vz;
    return q;
}

// the record of slot a in the layout the uniformity flag selects
__device__ __forceinline__ void put_nbr(const Domain* dom, void* rec, const RecSrc& R, int64_t a,
                                        const Pos4& pa, double c11, double c12, double c13,
                                        double c22, double c23, double c33)
{
    if (dom->nonuniform)
        ((MomNbr*)rec)[a] = make_nbr(R, a, pa, c11, c12, c13, c22, c23, c33);
    else
        ((MomNbrU*)rec)[a] = make_nbr_u(R, a, pa, c11, c12, c13, c22, c23, c33);
}

__global__ void k_uniform_begin(Domain* d) { d->nonuniform = 0u; }

// flags the step if any mass or sound speed differs from slot 0's
__global__ __launch_bounds__(kBlock) void k_uniform_check(int64_t n, const double* __restrict__ m,
                                                          const double* __restrict__ c,
                                                          Domain* __restrict__ dom)
{
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    const bool diff = i < n && (m[i] != m[0] || c[i] != c[0]);
    if (__ballot(diff) && (threadIdx.x & 63) == 0) flag_or(&dom->nonuniform, 1u);
}

template <int kPer, bool kTab>
__global__ __launch_bounds__(kBlock) SPH_WAVES_CAP(SPH_WAVES_IAD) void k_iad(Params P, Domain* __restrict__ dom,
                                                const int32_t* __restrict__ nc,
                                                const int32_t* __restrict__ list,
                                                const Pos4* __restrict__ p4,
                                                const PosV* __restrict__ pv,
                                                double* __restrict__ c11, double* __restrict__ c12,
                                                double* __restrict__ c13, double* __restrict__ c22,
                                                double* __restrict__ c23, double* __restrict__ c33,
                                                RecSrc R, void* __restrict__ rec)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    const int64_t a = lb * kBlock + threadIdx.x;
    if (a >= P.n) return;
    const Pos4 pa = p4[a];
    const double xa = pa.x, ya = pa.y, za = pa.z, ha = pa.h;
    const double tsc = kPiHalfSq / (ha * ha);
    const double w0 = P.bn / (ha * ha * ha);
    const int cnt = min(nc[a], P.ng_max);
    double t11 = 0, t12 = 0, t13 = 0, t22 = 0, t23 = 0, t33 = 0;
    // the next batch's list entries are fetched while this batch computes
    int32_t nx[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) nx[u] = (u < cnt) ? list[lpos(a, u, P.ng_max)] : -1;
    for (int j0 = 0; j0 < cnt; j0 += kBatch) {
        bool ok[kBatch];
        PosV q[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            ok[u] = (uint32_t)nx[u] < (uint32_t)P.n;
            q[u] = pv[ok[u] ? nx[u] : (int32_t)a];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int j = j0 + kBatch + u;
            nx[u] = (j < cnt) ? list[lpos(a, j, P.ng_max)] : -1;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
#if SPH_PAIR_CONTRACT
#pragma clang fp contract(fast)
#endif
            if (!ok[u]) continue;
            double dx, dy, dz;
            double r2 = disp_p<kPer>(P, xa, ya, za, q[u].x, q[u].y, q[u].z, dx, dy, dz);
            double s = q[u].v * (w0 * kern_S_t<kTab>(P, r2 * tsc));
            t11 += s * dx * dx;
            t12 += s * dx * dy;
            t13 += s * dx * dz;
            t22 += s * dy * dy;
            t23 += s * dy * dz;
            t33 += s * dz * dz;
        }
    }
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
    if (rec) put_nbr(dom, rec, R, a, pa, a11, a12, a13, a22, a23, a33);
}

__global__ __launch_bounds__(kBlock) void k_pack_nbr(int64_t n, const Domain* __restrict__ dom,
                                                     RecSrc R,
                                                     const double* __restrict__ c11,
                                                     const double* __restrict__ c12,
                                                     const double* __restrict__ c13,
                                                     const double* __restrict__ c22,
                                                     const double* __restrict__ c23,
                                                     const double* __restrict__ c33,
                                                     void* __restrict__ rec)
{
    int64_t a = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (a < n)
        put_nbr(dom, rec, R, a, Pos4{R.x[a], R.y[a], R.z[a], R.h[a]}, c11[a], c12[a], c13[a],
                c22[a], c23[a], c33[a]);
}

// the reverse pass's unfolded records, from the positions the IAD pass read
__global__ __launch_bounds__(kBlock) void k_pack_rec(int64_t n, RecSrc R,
                                                     const Pos4* __restrict__ p4,
                                                     const double* __restrict__ c11,
                                                     const double* __restrict__ c12,
                                                     const double* __restrict__ c13,
                                                     const double* __restrict__ c22,
                                                     const double* __restrict__ c23,
                                                     const double* __restrict__ c33,
                                                     MomRec* __restrict__ rec)
{
    const int64_t a = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (a >= n) return;
    const Pos4 pa = p4[a];
    MomRec q;
    q.x = pa.x; q.y = pa.y; q.z = pa.z; q.h = pa.h;
    q.c11 = c11[a]; q.c12 = c12[a]; q.c13 = c13[a];
    q.c22 = c22[a]; q.c23 = c23[a]; q.c33 = c33[a];
    const double r = R.rho[a];
    q.irho = 1.0 / r;
    q.c = R.c[a];
    q.pb = R.p[a] / (R.omega[a] * r * r);
    q.m = R.m[a];
    q.vx = R.vx[a]; q.vy = R.vy[a]; q.vz = R.vz[a];
    q.invh = 1.0 / pa.h;
    rec[a] = q;
}

struct MomOut {
    double *ax, *ay, *az, *du;
};

__global__ void k_dtmin_begin(Domain* d) { d->dtmin_bits = ord_bits(INFINITY); }

// what the target reads of itself beside its record: the unfolded factors,
// and h, m and c (the uniform record holds none of them)
struct MomSelf {
    const double *c11, *c12, *c13, *c22, *c23, *c33, *rho, *omega, *p, *h, *m, *c;
};

// mass and sound speed of a neighbour: its own, or slot 0's in the uniform record
SPH_DEV double nbr_m(const MomNbr& r, double) { return r.m; }
SPH_DEV double nbr_c(const MomNbr& r, double) { return r.c; }
SPH_DEV double nbr_m(const MomNbrU&, double m0) { return m0; }
SPH_DEV double nbr_c(const MomNbrU&, double c0) { return c0; }
template <class Rec, int kMomBatch, int kPer, bool kTab>
__device__ __forceinline__ void momentum_energy(const Params& P, Domain* __restrict__ dom,
                                                const int32_t* __restrict__ nc,
                                                const int32_t* __restrict__ ns,
                                                const int32_t* __restrict__ list,
                                                const Rec* __restrict__ rec, const MomSelf& T,
                                                const double* __restrict__ u, const MomOut& O,
                                                int64_t a_lane)
{
    // lanes past the end shadow the last slot with an empty list (every lane
    // of a wavefront takes part in the staged gathers)
    const bool live = a_lane < P.n;
    const int64_t a = live ? a_lane : P.n - 1;
    double dtc = INFINITY;
    {
        const Rec ra = rec[a];
        const double m0 = T.m[0], c0 = T.c[0];
        const double xa = ra.x, ya = ra.y, za = ra.z, ha = T.h[a];
        const double vxa = ra.vx, vya = ra.vy, vza = ra.vz;
        const double ca11 = T.c11[a], ca12 = T.c12[a], ca13 = T.c13[a];
        const double ca22 = T.c22[a], ca23 = T.c23[a], ca33 = T.c33[a];
        const double rho_a = T.rho[a];
        const double ca = nbr_c(ra, c0), ira = 1.0 / rho_a;
        const double pa_ = T.p[a] / (T.omega[a] * rho_a * rho_a);   // P/(Omega rho^2)
        const double tsa = kPiHalfSq / (ha * ha);
        const double w0a = P.bn / (ha * ha * ha);
        const double al = P.alpha;
        const int ng = P.ng_max;
        const int cg = live ? min(nc[a], ng) : 0;
        const int co = live ? min(ns[a] - nc[a], ng) : 0;
        double axs = 0.0, ays = 0.0, azs = 0.0, e1 = 0.0, e2 = 0.0;
        const int total = cg + co;
        // list entries of the batch starting at k0 (-1 past the end)
        auto entries = [&](int k0, int32_t (&e)[kMomBatch]) {
#pragma unroll
            for (int u = 0; u < kMomBatch; ++u) {
                const int k = k0 + u;
                const int j = (k < cg) ? k : ng - 1 - (k - cg);
                e[u] = (k < total) ? list[lpos(a, j, ng)] : -1;
            }
        };
        auto pair = [&](bool gather, const Rec& rb) {
#if SPH_PAIR_CONTRACT
            // the pair terms may fuse multiply-adds (rounding-level changes
            // only); r^2 itself comes from disp(), which never contracts
#pragma clang fp contract(fast)
#endif
            double dx, dy, dz;
            double r2 = disp_p<kPer>(P, xa, ya, za, rb.x, rb.y, rb.z, dx, dy, dz);
            double Wa = 0.0;
            if (gather) Wa = w0a * kern_S_t<kTab>(P, r2 * tsa);
            // W(r, h_b) on its support t_b < pi^2 (v_b < 2)
            double Wb = 0.0;
            const double ih = rb.ih, ih2 = ih * ih;
            const double tb = r2 * (kPiHalfSq * ih2);
            if (tb < 4.0 * kPiHalfSq) Wb = P.bn * (ih2 * ih) * kern_S_t<kTab>(P, tb);
            // A_ab(h_a) = C_a d W_a and K_b d with d = x_b - x_a
            const double Aax = (ca11 * dx + ca12 * dy + ca13 * dz) * Wa;
            const double Aay = (ca12 * dx + ca22 * dy + ca23 * dz) * Wa;
            const double Aaz = (ca13 * dx + ca23 * dy + ca33 * dz) * Wa;
            const double Kx = rb.k11 * dx + rb.k12 * dy + rb.k13 * dz;
            const double Ky = rb.k12 * dx + rb.k22 * dy + rb.k23 * dz;
            const double Kz = rb.k13 * dx + rb.k23 * dy + rb.k33 * dz;
            const double vx = vxa - rb.vx, vy = vya - rb.vy, vz = vza - rb.vz;
            // x_ab . v_ab with x_ab = -d
            const double xv = -(vx * dx + vy * dy + vz * dz);
            double hPi = 0.0;   // Pi_ab / 2
            if (xv < 0.0) {
                const double w = xv * rsqrt_nr(r2);
                const double vsig = ca + nbr_c(rb, c0) - 3.0 * w;
                hPi = -0.25 * al * vsig * w;
            }
            // a_a -= m_b (pb_a + Pi/(2 rho_a)) A_ab(h_a) + (q_b + Pi/2) W_b K_b d
            const double mb = nbr_m(rb, m0);
            const double sa = mb * (pa_ + hPi * ira);
            const double sb = (rb.q + hPi) * Wb;
            axs -= sa * Aax + sb * Kx;
            ays -= sa * Aay + sb * Ky;
            azs -= sa * Aaz + sb * Kz;
            // e1 += m_b v_ab . A_ab(h_a); e2 += v_ab . (Pi/2)(m_b A_ab(h_a)/rho_a + W_b K_b d)
            const double va = vx * Aax + vy * Aay + vz * Aaz;
            const double vk = vx * Kx + vy * Ky + vz * Kz;
            e1 += mb * va;
            e2 += hPi * (mb * ira * va + Wb * vk);
        };
        // the records of a batch are gathered, then the next batch's list
        // entries fetched while this batch computes (entries past the end read
        // the target itself and are skipped)
        int32_t nx[kMomBatch];
        entries(0, nx);
        if constexpr (sizeof(Rec) == sizeof(MomNbrU)) {
            // Staged gathers (the 112-byte records): each lane's loads of its
            // own neighbour's record fetch seven columns from seven places.
            // Instead the wavefront loads the 64 records of a batch step
            // together, lane L taking column (64 i + L) mod 7 of record
            // (64 i + L) / 7 in load i, so that each load covers nine whole
            // records; the columns go to LDS in record order and every lane
            // then reads its own record (a stride of 28 dwords: no bank
            // conflicts).  C4: 52.4 -> 48.9 ms.
            constexpr int kCols = (int)(sizeof(Rec) / 16);
            static_assert(sizeof(Rec) % 16 == 0, "records of whole 16-byte columns");
            __shared__ int4 stage[kBlock / 64][kMomBatch][64 * kCols];
            const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
            int tmax = total;   // the wavefront runs to its longest list
            for (int o = 32; o > 0; o >>= 1) tmax = max(tmax, __shfl_xor(tmax, o, 64));
            const int4* col = (const int4*)rec;
            for (int k0 = 0; k0 < tmax; k0 += kMomBatch) {
                bool ok[kMomBatch];
#pragma unroll
                for (int u = 0; u < kMomBatch; ++u) {
                    ok[u] = (uint32_t)nx[u] < (uint32_t)P.n;
                    const int32_t src = ok[u] ? nx[u] : (int32_t)a;
#pragma unroll
                    for (int i = 0; i < kCols; ++i) {
                        const int q = 64 * i + lane;
                        const int r = q / kCols;
                        const int32_t b = __shfl(src, r, 64);
                        stage[wv][u][q] = col[(int64_t)b * kCols + (q - r * kCols)];
                    }
                }
                entries(k0 + kMomBatch, nx);
                // LDS operations of one wavefront complete in order; the fences
                // keep the compiler from moving the reads above the writes or
                // the next batch's writes above this batch's reads
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
                for (int u = 0; u < kMomBatch; ++u) {
                    const Rec rb = lds_record<Rec>(&stage[wv][u][lane * kCols]);
                    if (ok[u]) pair(k0 + u < cg, rb);
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
        } else {
            for (int k0 = 0; k0 < total; k0 += kMomBatch) {
                bool ok[kMomBatch];
                Rec rb[kMomBatch];
#pragma unroll
                for (int u = 0; u < kMomBatch; ++u) {
                    ok[u] = (uint32_t)nx[u] < (uint32_t)P.n;
                    rb[u] = rec[ok[u] ? nx[u] : (int32_t)a];
                }
                entries(k0 + kMomBatch, nx);
#pragma unroll
                for (int u = 0; u < kMomBatch; ++u)
                    if (ok[u]) pair(k0 + u < cg, rb[u]);
            }
        }
        const double du = pa_ * e1 + 0.5 * e2;
        if (live) {
            O.ax[a] = axs;
            O.ay[a] = ays;
            O.az[a] = azs;
            O.du[a] = du;
            if (!isfinite(axs) || !isfinite(ays) || !isfinite(azs) || !isfinite(du))
                set_err(dom, SPH_ERRBIT_NONFINITE);
            // time-step candidate: Courant, acceleration and energy criteria
            dtc = P.courant * (ha / ca);
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
    // wavefront minimum of the candidates, then the global one
    for (int o = 32; o > 0; o >>= 1) dtc = fmin(dtc, __shfl_xor(dtc, o, 64));
    if ((threadIdx.x & 63) == 0 && dtc < INFINITY)
        ord_min_to(&dom->dtmin_bits, dtc);
}

// One kernel for both record layouts, the uniformity flag choosing the path:
// the 144-byte records gather per lane in batches of 4, the 112-byte records
// are staged through LDS in batches of 2, both at two wavefronts per SIMD (the
// 144-byte path spills at three; the staging's LDS allows two).  At 64 M
// particles the staged path takes 47.5 ms; per-lane gathers took 52.4 ms at
// three wavefronts and batches of 3, 54.9 at two and batches of 4.  (Two
// kernels, one returning at once, cost the unselected launch 2.6 ms at 8 M
// particles: its LDS held the workgroups of the empty launch to two per CU.)
template <int kPer, bool kTab>
__global__ __launch_bounds__(kBlock) SPH_MOM_ATTR void k_momentum_energy(Params P, Domain* __restrict__ dom,
                                                            const int32_t* __restrict__ nc,
                                                            const int32_t* __restrict__ ns,
                                                            const int32_t* __restrict__ list,
                                                            const void* __restrict__ rec,
                                                            MomSelf T,
                                                            const double* __restrict__ u,
                                                            MomOut O)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    const int64_t a = lb * kBlock + threadIdx.x;
    if (dom->nonuniform != 0u)
        momentum_energy<MomNbr, SPH_MOM_BATCH, kPer, kTab>(P, dom, nc, ns, list,
                                                           (const MomNbr*)rec, T, u, O, a);
    else
        momentum_energy<MomNbrU, SPH_MOM_U_BATCH, kPer, kTab>(P, dom, nc, ns, list,
                                                              (const MomNbrU*)rec, T, u, O, a);
}

__global__ void k_timestep(Params P, const Domain* __restrict__ dom, sph_globals* g)
{
    double dt = ord_value(dom->dtmin_bits);
    double prev = g->dt_m1;
    if (prev > 0.0) {
        double lim = P.growth * prev;
        if (lim < dt) dt = lim;
    }
    g->dt = dt;
}

RecSrc rec_src(const sph_particles* p)
{
    return RecSrc{p->m, p->rho, p->omega, p->p, p->c, p->vx, p->vy, p->vz, p->h,
                  p->x, p->y, p->z};
}

}  // namespace

hipError_t launch_density(const Params& P, const Layout& L, const Ws& W, sph_particles* p,
                          hipStream_t s, bool pack)
{
    if (pack) {
        hipError_t e = launch_pack_p4(P, W, p, s);
        if (e != hipSuccess) return e;
    }
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    k_density<<<grid_xcd(nb), kBlock, 0, s>>>(P, W.dom, W.nc, W.list, W.p4, p->m, p->u, p->p_ref,
                                              p->rho_ref, p->rho, p->omega, p->p, p->c);
    return hipGetLastError();
}

hipError_t launch_iad(const Params& P, const Layout& L, const Ws& W, sph_particles* p,
                      hipStream_t s, bool pack, bool write_rec)
{
    if (pack) {
        hipError_t e = launch_pack_p4(P, W, p, s);
        if (e != hipSuccess) return e;
    }
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    k_volume<<<nb, kBlock, 0, s>>>(P.n, p->m, p->rho, W.p4, W.vol, W.pv);
    if (write_rec) launch_uniform_check(P, W, p, s);
    with_periodic(P, [&](auto per) {
        with_table(P, [&](auto tab) {
            k_iad<decltype(per)::value, decltype(tab)::value><<<grid_xcd(nb), kBlock, 0, s>>>(
                P, W.dom, W.nc, W.list, W.p4, W.pv, p->c11, p->c12, p->c13, p->c22, p->c23,
                p->c33, rec_src(p), write_rec ? (void*)W.rec : nullptr);
        });
    });
    return hipGetLastError();
}

hipError_t launch_uniform_check(const Params& P, const Ws& W, const sph_particles* p,
                                hipStream_t s)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    k_uniform_begin<<<1, 1, 0, s>>>(W.dom);
    k_uniform_check<<<nb, kBlock, 0, s>>>(P.n, p->m, p->c, W.dom);
    return hipGetLastError();
}

hipError_t launch_pack_rec(const Params& P, const Ws& W, const sph_particles* p, hipStream_t s)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    k_pack_rec<<<nb, kBlock, 0, s>>>(P.n, rec_src(p), W.p4, p->c11, p->c12, p->c13, p->c22,
                                     p->c23, p->c33, W.rec);
    return hipGetLastError();
}

hipError_t launch_momentum_energy(const Params& P, const Layout& L, const Ws& W,
                                  sph_particles* p, hipStream_t s, bool pack)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    if (pack) {
        hipError_t e = launch_pack_p4(P, W, p, s);
        if (e != hipSuccess) return e;
        launch_uniform_check(P, W, p, s);
        k_pack_nbr<<<nb, kBlock, 0, s>>>(P.n, W.dom, rec_src(p), p->c11, p->c12, p->c13,
                                         p->c22, p->c23, p->c33, (void*)W.rec);
    }
    MomOut O{p->ax, p->ay, p->az, p->du};
    MomSelf T{p->c11, p->c12, p->c13, p->c22, p->c23, p->c33, p->rho, p->omega, p->p,
              p->h, p->m, p->c};
    k_dtmin_begin<<<1, 1, 0, s>>>(W.dom);
    with_periodic(P, [&](auto per) {
        with_table(P, [&](auto tab) {
            constexpr int kPer = decltype(per)::value;
            constexpr bool kTab = decltype(tab)::value;
            k_momentum_energy<kPer, kTab><<<grid_xcd(nb), kBlock, 0, s>>>(
                P, W.dom, W.nc, W.ns, W.list, (const void*)W.rec, T, p->u, O);
        });
    });
    return hipGetLastError();
}

hipError_t launch_timestep(const Params& P, const Ws& W, sph_globals* g, hipStream_t s)
{
    k_timestep<<<1, 1, 0, s>>>(P, W.dom, g);
    return hipGetLastError();
}

}  // namespace sph
