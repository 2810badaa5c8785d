// sph_pairs.hip -- the three pair passes over the neighbour lists (section 4.1):
// density + grad-h + EOS (eq. 1), IAD matrix and its inverse, and the
// momentum/energy rates with artificial viscosity (eqs. 2-5); plus the global
// minimum time step (section 4.2).
//
// One thread per target slot, wavefronts mapped XCD-contiguously; list column j
// of 64 consecutive targets is one 256-byte coalesced load; neighbour fields
// are gathers from Morton-local slots (L1/L2 resident).  Sums are in FP64 in
// list order; no atomics on floating point values.
#include "sph_common.h"

namespace sph {
namespace {

__global__ __launch_bounds__(kBlock) void k_density(Params P, Domain* __restrict__ dom,
                                                    const int32_t* __restrict__ nc,
                                                    const int32_t* __restrict__ list,
                                                    const double* __restrict__ x,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ z,
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
    const double xa = x[a], ya = y[a], za = z[a], ha = h[a];
    const double tsc = kPiHalfSq / (ha * ha);
    const int cnt = min(nc[a], P.ng_max);
    // self term: S = 1, v dS/dv = 0
    double sS = m[a], sD = 3.0 * m[a];
    for (int j = 0; j < cnt; ++j) {
        int32_t b = list[(int64_t)j * P.stride + a];
        if ((uint64_t)(uint32_t)b >= (uint64_t)P.n) continue;  // lists not built for this ws
        double dx, dy, dz;
        double r2 = disp(P, xa, ya, za, x[b], y[b], z[b], dx, dy, dz);
        double S, vdS;
        sinc_terms(r2 * tsc, P.sinc_n, S, vdS);
        double mb = m[b];
        sS += mb * S;
        sD += mb * (3.0 * S + vdS);
    }
    const double w0 = P.bn / (ha * ha * ha);
    const double r = w0 * sS;
    // Omega = 1 + h/(3 rho) sum m dW/dh, dW/dh = -(B/h^4)(3S + v dS/dv)
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

__global__ __launch_bounds__(kBlock) void k_iad(Params P, Domain* __restrict__ dom,
                                                const int32_t* __restrict__ nc,
                                                const int32_t* __restrict__ list,
                                                const double* __restrict__ x,
                                                const double* __restrict__ y,
                                                const double* __restrict__ z,
                                                const double* __restrict__ h,
                                                const double* __restrict__ m,
                                                const double* __restrict__ rho,
                                                double* __restrict__ c11, double* __restrict__ c12,
                                                double* __restrict__ c13, double* __restrict__ c22,
                                                double* __restrict__ c23, double* __restrict__ c33)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    const int64_t a = lb * kBlock + threadIdx.x;
    if (a >= P.n) return;
    const double xa = x[a], ya = y[a], za = z[a], ha = h[a];
    const double tsc = kPiHalfSq / (ha * ha);
    const double w0 = P.bn / (ha * ha * ha);
    const int cnt = min(nc[a], P.ng_max);
    double t11 = 0, t12 = 0, t13 = 0, t22 = 0, t23 = 0, t33 = 0;
    for (int j = 0; j < cnt; ++j) {
        int32_t b = list[(int64_t)j * P.stride + a];
        if ((uint64_t)(uint32_t)b >= (uint64_t)P.n) continue;
        double dx, dy, dz;
        double r2 = disp(P, xa, ya, za, x[b], y[b], z[b], dx, dy, dz);
        double s = m[b] / rho[b] * (w0 * sinc_S(r2 * tsc, P.sinc_n));
        t11 += s * dx * dx;
        t12 += s * dx * dy;
        t13 += s * dx * dz;
        t22 += s * dy * dy;
        t23 += s * dy * dz;
        t33 += s * dz * dz;
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
        c11[a] = a11 * id; c12[a] = a12 * id; c13[a] = a13 * id;
        c22[a] = a22 * id; c23[a] = a23 * id; c33[a] = a33 * id;
    } else {
        c11[a] = 0.0; c12[a] = 0.0; c13[a] = 0.0;
        c22[a] = 0.0; c23[a] = 0.0; c33[a] = 0.0;
        set_err(dom, SPH_ERRBIT_SINGULAR_TAU);
    }
}

struct MomIn {
    const double *x, *y, *z, *vx, *vy, *vz, *h, *m, *u, *rho, *omega, *p, *c;
    const double *c11, *c12, *c13, *c22, *c23, *c33;
};
struct MomOut {
    double *ax, *ay, *az, *du;
};

__global__ void k_dtmin_begin(Domain* d) { d->dtmin_bits = ord_bits(INFINITY); }

__global__ __launch_bounds__(kBlock) void k_momentum_energy(Params P, Domain* __restrict__ dom,
                                                            const int32_t* __restrict__ nc,
                                                            const int32_t* __restrict__ ns,
                                                            const int32_t* __restrict__ list,
                                                            MomIn I, MomOut O)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    const int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    const int64_t a = lb * kBlock + threadIdx.x;
    double dtc = INFINITY;
    if (a < P.n) {
        const double xa = I.x[a], ya = I.y[a], za = I.z[a];
        const double vxa = I.vx[a], vya = I.vy[a], vza = I.vz[a];
        const double ha = I.h[a], ra = I.rho[a], ca = I.c[a];
        const double C11 = I.c11[a], C12 = I.c12[a], C13 = I.c13[a];
        const double C22 = I.c22[a], C23 = I.c23[a], C33 = I.c33[a];
        const double pa = I.p[a] / (I.omega[a] * ra * ra);
        const double tsa = kPiHalfSq / (ha * ha);
        const double w0a = P.bn / (ha * ha * ha);
        const double al = P.alpha;
        const int ng = P.ng_max;
        const int cg = min(nc[a], ng);
        const int co = min(ns[a] - nc[a], ng);
        double axs = 0.0, ays = 0.0, azs = 0.0, e1 = 0.0, e2 = 0.0;
        const int total = cg + co;
        for (int k = 0; k < total; ++k) {
            const bool gather = k < cg;
            const int j = gather ? k : ng - 1 - (k - cg);
            const int32_t b = list[(int64_t)j * P.stride + a];
            if ((uint64_t)(uint32_t)b >= (uint64_t)P.n) continue;
            double dx, dy, dz;
            double r2 = disp(P, xa, ya, za, I.x[b], I.y[b], I.z[b], dx, dy, dz);
            const double hb = I.h[b];
            double Wa = 0.0;
            if (gather) Wa = w0a * sinc_S(r2 * tsa, P.sinc_n);
            double Wb = 0.0;
            const double hb2 = 2.0 * hb;
            if (r2 < hb2 * hb2) Wb = P.bn / (hb * hb * hb) * sinc_S(r2 * (kPiHalfSq / (hb * hb)), P.sinc_n);
            // A_ab(h_a) = C_a d W_a, A_ab(h_b) = C_b d W_b, d = x_b - x_a
            const double Aax = (C11 * dx + C12 * dy + C13 * dz) * Wa;
            const double Aay = (C12 * dx + C22 * dy + C23 * dz) * Wa;
            const double Aaz = (C13 * dx + C23 * dy + C33 * dz) * Wa;
            const double D11 = I.c11[b], D12 = I.c12[b], D13 = I.c13[b];
            const double D22 = I.c22[b], D23 = I.c23[b], D33 = I.c33[b];
            const double Abx = (D11 * dx + D12 * dy + D13 * dz) * Wb;
            const double Aby = (D12 * dx + D22 * dy + D23 * dz) * Wb;
            const double Abz = (D13 * dx + D23 * dy + D33 * dz) * Wb;
            const double vx = vxa - I.vx[b], vy = vya - I.vy[b], vz = vza - I.vz[b];
            // x_ab . v_ab with x_ab = -d
            const double xv = -(vx * dx + vy * dy + vz * dz);
            const double rb = I.rho[b];
            double Pi = 0.0;
            if (xv < 0.0) {
                const double w = xv / sqrt(r2);
                const double vsig = ca + I.c[b] - 3.0 * w;
                Pi = -0.5 * al * vsig * w;
            }
            const double mb = I.m[b];
            const double pb = I.p[b] / (I.omega[b] * rb * rb);
            const double gk = 0.5 * mb * Pi;
            const double ira = 1.0 / ra, irb = 1.0 / rb;
            const double gx = gk * (Aax * ira + Abx * irb);
            const double gy = gk * (Aay * ira + Aby * irb);
            const double gz = gk * (Aaz * ira + Abz * irb);
            axs += -(mb * (pa * Aax + pb * Abx)) - gx;
            ays += -(mb * (pa * Aay + pb * Aby)) - gy;
            azs += -(mb * (pa * Aaz + pb * Abz)) - gz;
            e1 += mb * (vx * Aax + vy * Aay + vz * Aaz);
            e2 += vx * gx + vy * gy + vz * gz;
        }
        const double du = pa * e1 + 0.5 * e2;
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
            double qu = P.energy_dt * (fabs(I.u[a]) / fabs(du));
            if (qu < dtc) dtc = qu;
        }
    }
    // block minimum of the Courant candidates, one atomic per wavefront
    for (int o = 32; o > 0; o >>= 1) dtc = fmin(dtc, __shfl_xor(dtc, o, 64));
    if ((threadIdx.x & 63) == 0 && dtc < INFINITY)
        atomicMin((unsigned long long*)&dom->dtmin_bits, (unsigned long long)ord_bits(dtc));
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

}  // namespace

hipError_t launch_density(const Params& P, const Layout& L, const Ws& W, sph_particles* p,
                          hipStream_t s)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    k_density<<<grid_xcd(nb), kBlock, 0, s>>>(P, W.dom, W.nc, W.list, p->x, p->y, p->z, p->h,
                                              p->m, p->u, p->p_ref, p->rho_ref, p->rho, p->omega,
                                              p->p, p->c);
    return hipGetLastError();
}

hipError_t launch_iad(const Params& P, const Layout& L, const Ws& W, sph_particles* p,
                      hipStream_t s)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    k_iad<<<grid_xcd(nb), kBlock, 0, s>>>(P, W.dom, W.nc, W.list, p->x, p->y, p->z, p->h, p->m,
                                          p->rho, p->c11, p->c12, p->c13, p->c22, p->c23, p->c33);
    return hipGetLastError();
}

hipError_t launch_momentum_energy(const Params& P, const Layout& L, const Ws& W,
                                  sph_particles* p, hipStream_t s)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    MomIn I{p->x, p->y, p->z, p->vx, p->vy, p->vz, p->h, p->m, p->u, p->rho, p->omega, p->p, p->c,
            p->c11, p->c12, p->c13, p->c22, p->c23, p->c33};
    MomOut O{p->ax, p->ay, p->az, p->du};
    k_dtmin_begin<<<1, 1, 0, s>>>(W.dom);
    k_momentum_energy<<<grid_xcd(nb), kBlock, 0, s>>>(P, W.dom, W.nc, W.ns, W.list, I, O);
    return hipGetLastError();
}

hipError_t launch_timestep(const Params& P, const Ws& W, sph_globals* g, hipStream_t s)
{
    k_timestep<<<1, 1, 0, s>>>(P, W.dom, g);
    return hipGetLastError();
}

}  // namespace sph
