/*
 * sph_oracle.c -- plain, slow, brute-force FP64 CPU oracle of one SPH time step
 * as described in Cavelan, Cabezon, Grabarczyk and Ciorba, "A Smoothed Particle
 * Hydrodynamics Mini-App for Exascale" (arXiv 2005.02656), section 4.1.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the HIP implementation.
 *
 * Style: every pair sum runs over ALL particles b in ascending index order
 * (O(N^2) per pass).  The compact support of the kernel appears only as the
 * literal test r^2 < (2h)^2.  There is no sorting, no cell structure, no
 * blocking and no fusion.  Targets a may be restricted to an index list so the
 * same definitions can be evaluated at a few sampled particles of a large input.
 * Compiled with -ffp-contract=off; uses libm sin, cos, sqrt.
 *
 * Notation (paper section 4.1): x_ab = x_a - x_b, v_ab = v_a - v_b; here
 * d_ab = x_b - x_a (minimum image) is the displacement used by the IAD terms.
 *
 * Readings of points the paper leaves open are the ones listed in the design
 * notes; each function names the ones it takes.  Parity of every function is
 * pinned by the CPU tests (closed forms, lattice values, conservation
 * identities, invariances, brute-force counts), except where a header comment
 * says "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_PI 3.14159265358979323846

typedef struct {
    double  box_lo[3], box_hi[3];
    int32_t periodic[3];
    double  sinc_n;        /* exponent n of S_n = sinc^n (eq. 6) */
    double  n_target;      /* target effective neighbour number N_t */
    int32_t newton_iters;  /* fixed number of Newton iterations on h */
    double  h_ratio_max;   /* kappa_h: h stays in [h0/kappa, kappa*h0] */
    int32_t eos;           /* 0 ideal gas, 1 weakly compressible */
    double  gamma, c0;
    double  alpha_av;      /* alpha of the artificial viscosity (eq. 5) */
    double  courant, dt_growth;
    double  acc_dt;        /* coefficient of the acceleration criterion, 0 = off */
    double  energy_dt;     /* coefficient of the energy criterion, 0 = off */
    int32_t kernel_table;  /* 0: S_n exact; N > 1: the N-value lookup table (section 4.5) */
} ora_config;

/* ------------------------------------------------------------------------ */
/* Geometry: minimum-image displacement and squared distance.               */
/* Periodic axis of length L: d -> d - L if d > L/2, d -> d + L if d <= -L/2 */
/* (half-open interval (-L/2, L/2]).  r^2 = (dx*dx + dy*dy) + dz*dz.        */
/* ------------------------------------------------------------------------ */
static void ora_min_image(const ora_config* cf, double d[3])
{
    for (int k = 0; k < 3; ++k) {
        if (!cf->periodic[k]) continue;
        double L = cf->box_hi[k] - cf->box_lo[k];
        double half = 0.5 * L;
        if (d[k] > half) d[k] -= L;
        else if (d[k] <= -half) d[k] += L;
    }
}

/* d = x_b - x_a with minimum image; returns r^2 */
static double ora_disp(const ora_config* cf, const double* x, const double* y,
                       const double* z, int64_t a, int64_t b, double d[3])
{
    d[0] = x[b] - x[a];
    d[1] = y[b] - y[a];
    d[2] = z[b] - z[a];
    ora_min_image(cf, d);
    double r2 = d[0] * d[0];
    r2 = r2 + d[1] * d[1];
    r2 = r2 + d[2] * d[2];
    return r2;
}

/* ------------------------------------------------------------------------ */
/* Sinc kernel family, eq. (6): W = B_n/h^3 S_n(pi v / 2), v = r/h, v <= 2.  */
/* ------------------------------------------------------------------------ */
static double ora_pow_n(double s, double n)
{
    /* integer exponents by repeated multiplication (section 4.5), real ones by pow */
    if (n == floor(n) && n >= 0.0 && n <= 16.0) {
        double r = 1.0;
        for (int i = 0; i < (int)n; ++i) r = r * s;
        return r;
    }
    return pow(s, n);
}

static double ora_sinc(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

/* derivative of sin(x)/x; the closed form cancels badly for small x, where
 * the Taylor series of the derivative is used instead */
static double ora_dsinc(double x)
{
    if (fabs(x) < 0.1) {
        double x2 = x * x;
        return x * (-1.0 / 3.0 + x2 * (1.0 / 30.0 + x2 * (-1.0 / 840.0 + x2 * (1.0 / 45360.0))));
    }
    return (x * cos(x) - sin(x)) / (x * x);
}

/* S_n(pi v/2) */
double ora_S(double v, double n) { return ora_pow_n(ora_sinc(0.5 * ORA_PI * v), n); }

/* d S_n(pi v/2) / dv */
double ora_dSdv(double v, double n)
{
    double x = 0.5 * ORA_PI * v;
    if (n == 0.0) return 0.0;
    return n * ora_pow_n(ora_sinc(x), n - 1.0) * ora_dsinc(x) * (0.5 * ORA_PI);
}

/* Gauss-Legendre nodes/weights on [-1,1] by Newton iteration on P_m */
static void ora_gauss_legendre(int m, double* t, double* w)
{
    for (int i = 0; i < m; ++i) {
        double z = cos(ORA_PI * (i + 0.75) / (m + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= m; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = m * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        t[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Normalisation of eq. (6) in three dimensions:
 * B_n = 1 / (4 pi int_0^2 S_n(pi v/2) v^2 dv), 96-point Gauss-Legendre. */
double ora_bn(double n)
{
    enum { M = 96 };
    double t[M], w[M];
    ora_gauss_legendre(M, t, w);
    double s = 0.0;
    for (int i = 0; i < M; ++i) {
        double v = 1.0 + t[i]; /* map [-1,1] -> [0,2] */
        s += w[i] * ora_S(v, n) * v * v;
    }
    return 1.0 / (4.0 * ORA_PI * s);
}

/* Kernel lookup table (section 4.5): with N = kernel_table > 1 values at the
 * nodes v_i = 2i/(N-1), S_n(v) and dS_n/dv are interpolated linearly in v
 * between the exact values at the two nodes around v, (1 - f) y_i + f y_{i+1}
 * with i = floor(v (N-1)/2) (clamped to the last interval) and f the fraction
 * past node i.  With N = 0 they are evaluated exactly. */
static double ora_table_lerp(const ora_config* cf, double v, int deriv)
{
    const int64_t N = cf->kernel_table;
    const double s = v * (0.5 * (double)(N - 1));
    int64_t i = (int64_t)s;
    if (i > N - 2) i = N - 2;
    const double f = s - (double)i;
    const double v0 = 2.0 * (double)i / (double)(N - 1);
    const double v1 = 2.0 * (double)(i + 1) / (double)(N - 1);
    const double y0 = deriv ? ora_dSdv(v0, cf->sinc_n) : ora_S(v0, cf->sinc_n);
    const double y1 = deriv ? ora_dSdv(v1, cf->sinc_n) : ora_S(v1, cf->sinc_n);
    return (1.0 - f) * y0 + f * y1;
}

static double ora_Sk(const ora_config* cf, double v)
{
    return cf->kernel_table > 1 ? ora_table_lerp(cf, v, 0) : ora_S(v, cf->sinc_n);
}

static double ora_dSk(const ora_config* cf, double v)
{
    return cf->kernel_table > 1 ? ora_table_lerp(cf, v, 1) : ora_dSdv(v, cf->sinc_n);
}

/* S_n and dS_n/dv as the configuration evaluates them, at one v (pins) */
double ora_S_cfg(const ora_config* cf, double v) { return ora_Sk(cf, v); }
double ora_dSdv_cfg(const ora_config* cf, double v) { return ora_dSk(cf, v); }

/* W and dW/dh through the configured kernel evaluation */
static double ora_Wc(const ora_config* cf, double r2, double h, double bn)
{
    double h2 = 2.0 * h;
    if (!(r2 < h2 * h2)) return 0.0;
    double v = sqrt(r2) / h;
    return bn / (h * h * h) * ora_Sk(cf, v);
}

static double ora_dWdhc(const ora_config* cf, double r2, double h, double bn)
{
    double h2 = 2.0 * h;
    if (!(r2 < h2 * h2)) return 0.0;
    double v = sqrt(r2) / h;
    return -bn / (h * h * h * h) * (3.0 * ora_Sk(cf, v) + v * ora_dSk(cf, v));
}

/* W(r, h) with support r^2 < (2h)^2; r2 is the squared distance */
double ora_W(double r2, double h, double n, double bn)
{
    double h2 = 2.0 * h;
    if (!(r2 < h2 * h2)) return 0.0;
    double v = sqrt(r2) / h;
    return bn / (h * h * h) * ora_S(v, n);
}

/* dW/dh at fixed r:  -(B_n/h^4) (3 S_n + v dS_n/dv) */
double ora_dWdh(double r2, double h, double n, double bn)
{
    double h2 = 2.0 * h;
    if (!(r2 < h2 * h2)) return 0.0;
    double v = sqrt(r2) / h;
    return -bn / (h * h * h * h) * (3.0 * ora_S(v, n) + v * ora_dSdv(v, n));
}

/* ------------------------------------------------------------------------ */
/* Target list helper                                                        */
/* ------------------------------------------------------------------------ */
static inline int64_t ora_tgt(const int64_t* targets, int64_t t) { return targets ? targets[t] : t; }

/* ------------------------------------------------------------------------ */
/* Smoothing length (reading of the "local spatial resolution" update,      */
/* section 4.1 and the neighbour count of section 4.3): fixed number of     */
/* Newton steps on the effective neighbour number                           */
/*   F(h) = (32 pi/3) B_n sum_{b, r<2h} S_n(pi r/2h) - N_t  (self included)  */
/*   F'(h) = -(32 pi/3)(B_n/h) sum_b v dS_n/dv                               */
/* h <- h - F/F', clamped to [h0/kappa, kappa h0]; F' = 0 gives kappa h0.    */
/* ------------------------------------------------------------------------ */
void ora_update_h(const ora_config* cf, int64_t n, const double* x, const double* y,
                  const double* z, const double* h_in, double* h_out,
                  int64_t nt, const int64_t* targets)
{
    const double bn = ora_bn(cf->sinc_n);
    const double k3 = 32.0 * ORA_PI / 3.0;
    const double kap = cf->h_ratio_max;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = ora_tgt(targets, t);
        double h0 = h_in[a], h = h0;
        for (int it = 0; it < cf->newton_iters; ++it) {
            double sS = 0.0, sV = 0.0;
            double h2 = 2.0 * h;
            double R2 = h2 * h2;
            for (int64_t b = 0; b < n; ++b) {
                double d[3];
                double r2 = ora_disp(cf, x, y, z, a, b, d);
                if (r2 < R2) {
                    double v = sqrt(r2) / h;
                    sS += ora_Sk(cf, v);
                    sV += v * ora_dSk(cf, v);
                }
            }
            double F = k3 * bn * sS - cf->n_target;
            double Fp = -k3 * (bn / h) * sV;
            double hn = (Fp > 0.0) ? h - F / Fp : kap * h0;
            if (hn < h0 / kap) hn = h0 / kap;
            if (hn > kap * h0) hn = kap * h0;
            h = hn;
        }
        h_out[a] = h;
    }
}

/* The two Newton sums at a given h (for the Newton identity pin). */
void ora_newton_terms(const ora_config* cf, int64_t n, const double* x, const double* y,
                      const double* z, const double* h, int64_t nt, const int64_t* targets,
                      double* F, double* Fp)
{
    const double bn = ora_bn(cf->sinc_n);
    const double k3 = 32.0 * ORA_PI / 3.0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = ora_tgt(targets, t);
        double ha = h[a], sS = 0.0, sV = 0.0;
        double h2 = 2.0 * ha;
        for (int64_t b = 0; b < n; ++b) {
            double d[3];
            double r2 = ora_disp(cf, x, y, z, a, b, d);
            if (r2 < h2 * h2) {
                double v = sqrt(r2) / ha;
                sS += ora_Sk(cf, v);
                sV += v * ora_dSk(cf, v);
            }
        }
        F[a] = k3 * bn * sS - cf->n_target;
        Fp[a] = -k3 * (bn / ha) * sV;
    }
}

/* ------------------------------------------------------------------------ */
/* Neighbour sets (section 4.3: stored as integer index lists).             */
/*   N(a)   = { b != a : r^2 < (2 h_a)^2 }                 (gather set)      */
/*   N_s(a) = { b != a : r^2 < (2 max(h_a,h_b))^2 }        (symmetric set)   */
/* Output per target slot t: nc[t] = |N(a)|, ns[t] = |N_s(a)|, and the first */
/* min(ns, cap) members of N_s(a) in ascending index in ids[t*cap + j], with  */
/* gather[t*cap + j] = 1 when the member is also in N(a).                    */
/* ------------------------------------------------------------------------ */
void ora_neighbors(const ora_config* cf, int64_t n, const double* x, const double* y,
                   const double* z, const double* h, int64_t nt, const int64_t* targets,
                   int32_t* nc, int32_t* ns, int64_t cap, int64_t* ids, uint8_t* gather)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = ora_tgt(targets, t);
        int32_t cg = 0, cs = 0;
        double ha2 = 2.0 * h[a];
        for (int64_t b = 0; b < n; ++b) {
            if (b == a) continue;
            double d[3];
            double r2 = ora_disp(cf, x, y, z, a, b, d);
            double hm = h[a] > h[b] ? h[a] : h[b];
            double hm2 = 2.0 * hm;
            int in_g = r2 < ha2 * ha2;
            int in_s = r2 < hm2 * hm2;
            if (in_s) {
                if (ids && cs < cap) {
                    ids[t * cap + cs] = b;
                    gather[t * cap + cs] = (uint8_t)in_g;
                }
                ++cs;
            }
            if (in_g) ++cg;
        }
        nc[t] = cg;
        ns[t] = cs;
    }
}

/* ------------------------------------------------------------------------ */
/* Density, eq. (1), self term included; grad-h term Omega (section 4.1):   */
/*   Omega_a = 1 + h_a/(3 rho_a) sum_b m_b dW/dh(r_ab, h_a)                  */
/* Equation of state (not printed in the paper; reading): ideal gas          */
/*   P = (gamma-1) rho u, c = sqrt(gamma (gamma-1) u);                       */
/* weakly compressible P = p_ref + c0^2 (rho - rho_ref), c = c0.             */
/* ------------------------------------------------------------------------ */
void ora_density(const ora_config* cf, int64_t n, const double* x, const double* y,
                 const double* z, const double* h, const double* m, const double* u,
                 const double* p_ref, const double* rho_ref, int64_t nt,
                 const int64_t* targets, double* rho, double* omega, double* p, double* c)
{
    const double bn = ora_bn(cf->sinc_n);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = ora_tgt(targets, t);
        double ha = h[a], sr = 0.0, sw = 0.0;
        for (int64_t b = 0; b < n; ++b) {
            double d[3];
            double r2 = ora_disp(cf, x, y, z, a, b, d);
            sr += m[b] * ora_Wc(cf, r2, ha, bn);
            sw += m[b] * ora_dWdhc(cf, r2, ha, bn);
        }
        rho[a] = sr;
        omega[a] = 1.0 + ha / (3.0 * sr) * sw;
        if (cf->eos == 0) {
            p[a] = (cf->gamma - 1.0) * sr * u[a];
            c[a] = sqrt(cf->gamma * (cf->gamma - 1.0) * u[a]);
        } else {
            p[a] = p_ref[a] + cf->c0 * cf->c0 * (sr - rho_ref[a]);
            c[a] = cf->c0;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* IAD (section 4.1, the integral approach to derivatives; formula not      */
/* printed, reading): tau_a = sum_{b in N(a)} (m_b/rho_b) W(r_ab,h_a) d d^T,  */
/* C_a = tau_a^{-1} by adjugate over determinant.  det <= 0 gives C = 0 and  */
/* sets *singular.  Output order of the six entries: 11 12 13 22 23 33.      */
/* ------------------------------------------------------------------------ */
void ora_iad(const ora_config* cf, int64_t n, const double* x, const double* y,
             const double* z, const double* h, const double* m, const double* rho,
             int64_t nt, const int64_t* targets, double* c11, double* c12, double* c13,
             double* c22, double* c23, double* c33, int32_t* singular)
{
    const double bn = ora_bn(cf->sinc_n);
    int32_t sing = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : sing)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = ora_tgt(targets, t);
        double ha = h[a];
        double t11 = 0, t12 = 0, t13 = 0, t22 = 0, t23 = 0, t33 = 0;
        for (int64_t b = 0; b < n; ++b) {
            if (b == a) continue;
            double d[3];
            double r2 = ora_disp(cf, x, y, z, a, b, d);
            double w = ora_Wc(cf, r2, ha, bn);
            if (w == 0.0) continue;
            double s = m[b] / rho[b] * w;
            t11 += s * d[0] * d[0];
            t12 += s * d[0] * d[1];
            t13 += s * d[0] * d[2];
            t22 += s * d[1] * d[1];
            t23 += s * d[1] * d[2];
            t33 += s * d[2] * d[2];
        }
        /* adjugate of the symmetric tau */
        double a11 = t22 * t33 - t23 * t23;
        double a12 = t13 * t23 - t12 * t33;
        double a13 = t12 * t23 - t13 * t22;
        double a22 = t11 * t33 - t13 * t13;
        double a23 = t12 * t13 - t11 * t23;
        double a33 = t11 * t22 - t12 * t12;
        double det = t11 * a11 + t12 * a12 + t13 * a13;
        if (det > 0.0) {
            c11[a] = a11 / det; c12[a] = a12 / det; c13[a] = a13 / det;
            c22[a] = a22 / det; c23[a] = a23 / det; c33[a] = a33 / det;
        } else {
            c11[a] = c12[a] = c13[a] = c22[a] = c23[a] = c33[a] = 0.0;
            sing = 1;
        }
    }
    if (singular) *singular = sing;
}

/* ------------------------------------------------------------------------ */
/* Momentum and energy, eqs. (2)-(5), with the readings: the AV acceleration */
/* is subtracted (dissipative sign), the energy prefactor is                 */
/* P_a/(Omega_a rho_a^2), the AV energy term uses the per-pair AV force, the */
/* pair set is the symmetric N_s(a), and                                     */
/*   A_ab(h_a) = C_a d_ab W(r_ab, h_a),  A_ab(h_b) = C_b d_ab W(r_ab, h_b).   */
/* Outputs per target: acceleration, du/dt, Courant candidate h_a/c_a and   */
/* the per-particle magnitude sums of the pair terms (tolerance scales).    */
/* ------------------------------------------------------------------------ */
static void ora_cmul(const double* C, const double d[3], double w, double out[3])
{
    /* C packed as 11 12 13 22 23 33 */
    out[0] = (C[0] * d[0] + C[1] * d[1] + C[2] * d[2]) * w;
    out[1] = (C[1] * d[0] + C[3] * d[1] + C[4] * d[2]) * w;
    out[2] = (C[2] * d[0] + C[4] * d[1] + C[5] * d[2]) * w;
}

void ora_momentum_energy(const ora_config* cf, int64_t n, const double* x, const double* y,
                         const double* z, const double* vx, const double* vy,
                         const double* vz, const double* h, const double* m,
                         const double* rho, const double* omega, const double* p,
                         const double* c, const double* c11, const double* c12,
                         const double* c13, const double* c22, const double* c23,
                         const double* c33, int64_t nt, const int64_t* targets, double* ax,
                         double* ay, double* az, double* du, double* dt_cand,
                         double* scale_a, double* scale_du)
{
    const double bn = ora_bn(cf->sinc_n);
    const double al = cf->alpha_av;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = ora_tgt(targets, t);
        double Ca[6] = {c11[a], c12[a], c13[a], c22[a], c23[a], c33[a]};
        double pa = p[a] / (omega[a] * rho[a] * rho[a]);
        double acc[3] = {0, 0, 0}, e1 = 0.0, e2 = 0.0, sa = 0.0, se = 0.0;
        for (int64_t b = 0; b < n; ++b) {
            if (b == a) continue;
            double d[3];
            double r2 = ora_disp(cf, x, y, z, a, b, d);
            double hm = h[a] > h[b] ? h[a] : h[b];
            double hm2 = 2.0 * hm;
            if (!(r2 < hm2 * hm2)) continue;
            double r = sqrt(r2);
            double wa = ora_Wc(cf, r2, h[a], bn);
            double wb = ora_Wc(cf, r2, h[b], bn);
            double Cb[6] = {c11[b], c12[b], c13[b], c22[b], c23[b], c33[b]};
            double Aa[3], Ab[3];
            ora_cmul(Ca, d, wa, Aa);
            ora_cmul(Cb, d, wb, Ab);
            double vab[3] = {vx[a] - vx[b], vy[a] - vy[b], vz[a] - vz[b]};
            /* x_ab = -d */
            double xv = -(vab[0] * d[0] + vab[1] * d[1] + vab[2] * d[2]);
            double Pi = 0.0;
            if (xv < 0.0) {
                double w = xv / r;
                double vsig = c[a] + c[b] - 3.0 * w;
                Pi = -0.5 * al * vsig * w;
            }
            double pb = p[b] / (omega[b] * rho[b] * rho[b]);
            double g[3], f[3];
            for (int k = 0; k < 3; ++k) {
                g[k] = 0.5 * m[b] * Pi * (Aa[k] / rho[a] + Ab[k] / rho[b]);
                f[k] = m[b] * (pa * Aa[k] + pb * Ab[k]);
                acc[k] += -f[k] - g[k];
            }
            double vA = vab[0] * Aa[0] + vab[1] * Aa[1] + vab[2] * Aa[2];
            double vg = vab[0] * g[0] + vab[1] * g[1] + vab[2] * g[2];
            e1 += m[b] * vA;
            e2 += vg;
            /* error scales: sums of the norms of the terms; for du the dot
               products are bounded by the products of the norms, since they
               cancel (to rounding) whenever v_ab is orthogonal to x_ab */
            double nf = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
            double ng = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
            double nv = sqrt(vab[0] * vab[0] + vab[1] * vab[1] + vab[2] * vab[2]);
            double nA = sqrt(Aa[0] * Aa[0] + Aa[1] * Aa[1] + Aa[2] * Aa[2]);
            sa += nf + ng;
            se += fabs(pa) * m[b] * nv * nA + 0.5 * nv * ng;
        }
        ax[a] = acc[0];
        ay[a] = acc[1];
        az[a] = acc[2];
        du[a] = pa * e1 + 0.5 * e2;
        if (dt_cand) dt_cand[a] = h[a] / c[a];
        if (scale_a) scale_a[a] = sa;
        if (scale_du) scale_du[a] = se;
    }
}

/* ------------------------------------------------------------------------ */
/* Global minimum time step (section 4.2, second global reduction; the rule is */
/* not printed, reading): the minimum over particles of                      */
/*   courant * (h/c),  acc_dt * sqrt(h/|a|),  energy_dt * (|u|/|du|)          */
/* (a zero coefficient switches a criterion off), limited to dt_growth times */
/* the previous step when there is one.                                      */
/* ------------------------------------------------------------------------ */
double ora_dt_candidate(const ora_config* cf, double h, double c, double u, double ax,
                        double ay, double az, double du)
{
    double q = cf->courant * (h / c);
    if (cf->acc_dt > 0.0) {
        double a = sqrt((ax * ax + ay * ay) + az * az);
        double qa = cf->acc_dt * sqrt(h / a);
        if (qa < q) q = qa;
    }
    if (cf->energy_dt > 0.0) {
        double qu = cf->energy_dt * (fabs(u) / fabs(du));
        if (qu < q) q = qu;
    }
    return q;
}

double ora_timestep(const ora_config* cf, int64_t n, const double* h, const double* c,
                    const double* u, const double* ax, const double* ay, const double* az,
                    const double* du, double dt_m1)
{
    double dt = INFINITY;
    for (int64_t a = 0; a < n; ++a) {
        double q = ora_dt_candidate(cf, h[a], c[a], u[a], ax[a], ay[a], az[a], du[a]);
        if (q < dt) dt = q;
    }
    if (dt_m1 > 0.0) {
        double g = cf->dt_growth * dt_m1;
        if (g < dt) dt = g;
    }
    return dt;
}

/* ------------------------------------------------------------------------ */
/* Integrator (section 4.1: second-order Press method for x, v and second-  */
/* order Adams-Bashforth for u; reading): variable-step kick-drift leapfrog  */
/* with lambda = previous dt (0 on the first step):                          */
/*   vh += a (lambda+dt)/2 ; x += vh dt (wrapped) ; v = vh + a dt/2          */
/*   u += dt [(1 + dt/2lambda) du - (dt/2lambda) du_m1]  (Euler if lambda=0) */
/*   du_m1 = du                                                              */
/* ------------------------------------------------------------------------ */
void ora_integrate(const ora_config* cf, int64_t n, double* x, double* y, double* z,
                   double* vx, double* vy, double* vz, double* vhx, double* vhy,
                   double* vhz, double* u, double* du_m1, const double* ax,
                   const double* ay, const double* az, const double* du, double dt,
                   double dt_m1)
{
    double* X[3] = {x, y, z};
    double* V[3] = {vx, vy, vz};
    double* VH[3] = {vhx, vhy, vhz};
    const double* A[3] = {ax, ay, az};
    double kick = 0.5 * (dt_m1 + dt);
    double half = 0.5 * dt;
    for (int64_t a = 0; a < n; ++a) {
        for (int k = 0; k < 3; ++k) {
            double vh = VH[k][a] + A[k][a] * kick;
            double xn = X[k][a] + vh * dt;
            if (cf->periodic[k]) {
                double L = cf->box_hi[k] - cf->box_lo[k];
                if (xn >= cf->box_hi[k]) xn -= L;
                else if (xn < cf->box_lo[k]) xn += L;
            }
            VH[k][a] = vh;
            X[k][a] = xn;
            V[k][a] = vh + A[k][a] * half;
        }
        if (dt_m1 > 0.0) {
            double q = dt / (2.0 * dt_m1);
            u[a] = u[a] + dt * ((1.0 + q) * du[a] - q * du_m1[a]);
        } else {
            u[a] = u[a] + dt * du[a];
        }
        du_m1[a] = du[a];
    }
}

/* ------------------------------------------------------------------------ */
/* Conservation sums (section 4.2, third global reduction): out = [M,        */
/* Px, Py, Pz, Lx, Ly, Lz, E_kin, E_int] with L = sum m x cross v.           */
/* ------------------------------------------------------------------------ */
void ora_sums(int64_t n, const double* m, const double* x, const double* y,
              const double* z, const double* vx, const double* vy, const double* vz,
              const double* u, double* out)
{
    double s[9] = {0};
    for (int64_t a = 0; a < n; ++a) {
        s[0] += m[a];
        s[1] += m[a] * vx[a];
        s[2] += m[a] * vy[a];
        s[3] += m[a] * vz[a];
        s[4] += m[a] * (y[a] * vz[a] - z[a] * vy[a]);
        s[5] += m[a] * (z[a] * vx[a] - x[a] * vz[a]);
        s[6] += m[a] * (x[a] * vy[a] - y[a] * vx[a]);
        s[7] += 0.5 * m[a] * (vx[a] * vx[a] + vy[a] * vy[a] + vz[a] * vz[a]);
        s[8] += m[a] * u[a];
    }
    memcpy(out, s, sizeof s);
}

/* ------------------------------------------------------------------------ */
/* Depth-first (Morton-like) particle order, section 4.3.  Reading: per axis */
/* 21-bit cell coordinate q = min(2^21-1, floor((x-lo) * (2^21/D))), clamped  */
/* below at 0, q = 0 when D = 0; the key interleaves the bits with x highest */
/* in each triplet.  lo/hi are the box on periodic axes and the particle     */
/* bounding box on open axes.                                                */
/* ------------------------------------------------------------------------ */
static uint64_t ora_quant(double xk, double lo, double hi)
{
    double D = hi - lo;
    if (!(D > 0.0)) return 0;
    double s = 2097152.0 / D;
    double t = xk - lo;
    double q = floor(t * s);
    if (!(q >= 0.0)) return 0;
    if (q > 2097151.0) return 2097151;
    return (uint64_t)q;
}

void ora_morton_keys(int64_t n, const double* x, const double* y, const double* z,
                     const double* lo, const double* hi, uint64_t* keys)
{
    for (int64_t a = 0; a < n; ++a) {
        uint64_t qx = ora_quant(x[a], lo[0], hi[0]);
        uint64_t qy = ora_quant(y[a], lo[1], hi[1]);
        uint64_t qz = ora_quant(z[a], lo[2], hi[2]);
        uint64_t key = 0;
        for (int i = 0; i < 21; ++i) {
            key |= ((qx >> i) & 1ull) << (3 * i + 2);
            key |= ((qy >> i) & 1ull) << (3 * i + 1);
            key |= ((qz >> i) & 1ull) << (3 * i);
        }
        keys[a] = key;
    }
}

/* bounding box and largest h: out = [xmin,ymin,zmin,xmax,ymax,zmax,hmax] */
void ora_bbox(int64_t n, const double* x, const double* y, const double* z,
              const double* h, double* out)
{
    double o[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t a = 0; a < n; ++a) {
        if (x[a] < o[0]) o[0] = x[a];
        if (y[a] < o[1]) o[1] = y[a];
        if (z[a] < o[2]) o[2] = z[a];
        if (x[a] > o[3]) o[3] = x[a];
        if (y[a] > o[4]) o[4] = y[a];
        if (z[a] > o[5]) o[5] = z[a];
        if (h[a] > o[6]) o[6] = h[a];
    }
    memcpy(out, o, sizeof o);
}

/* stable ordering of keys: perm[i] = index of the i-th smallest key, ties by
 * index.  Only the key's prefix above bit g_sort_shift is compared: the depth
 * first order of the octree down to a given level, particles in one cell of
 * that level keeping the order they came in (section 4.3 orders the particles
 * by the tree; it leaves the order inside the finest cells open). */
static const uint64_t* g_sort_keys;
static int g_sort_shift;
static int ora_key_cmp(const void* pa, const void* pb)
{
    int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
    uint64_t ka = g_sort_keys[a] >> g_sort_shift, kb = g_sort_keys[b] >> g_sort_shift;
    if (ka != kb) return ka < kb ? -1 : 1;
    return (a > b) - (a < b);
}

static void ora_sort_by(int64_t n, const uint64_t* keys, int shift, int64_t* perm)
{
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    g_sort_keys = keys;
    g_sort_shift = shift;
    qsort(perm, (size_t)n, sizeof(int64_t), ora_key_cmp);
    g_sort_keys = NULL;
}

/* the whole 63-bit key */
void ora_sort_keys(int64_t n, const uint64_t* keys, int64_t* perm)
{
    ora_sort_by(n, keys, 0, perm);
}

/* the prefix of L levels (3L bits) */
void ora_sort_keys_level(int64_t n, const uint64_t* keys, int L, int64_t* perm)
{
    ora_sort_by(n, keys, 3 * (21 - L), perm);
}

/* ------------------------------------------------------------------------ */
/* Self-gravity (section 4.1: a multipole expansion evaluated on the same    */
/* octree that finds the neighbours; order, opening rule and softening not   */
/* printed, readings):                                                       */
/*   g_a = -G sum_{b != a} m_b (x_a - x_b) / (|x_a - x_b|^2 + eps^2)^(3/2)    */
/* (Plummer softening eps), approximated on the octree of the particle keys. */
/* ------------------------------------------------------------------------ */

/* The exact definition by direct summation over all b in ascending index. */
void ora_gravity_direct(int64_t n, const double* x, const double* y, const double* z,
                        const double* m, double G, double eps, int64_t nt,
                        const int64_t* targets, double* gx, double* gy, double* gz,
                        double* scale)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = ora_tgt(targets, t);
        double acc[3] = {0, 0, 0}, sc = 0.0;
        for (int64_t b = 0; b < n; ++b) {
            if (b == a) continue;
            double d[3] = {x[a] - x[b], y[a] - y[b], z[a] - z[b]};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps * eps;
            double f = G * m[b] / (r2 * sqrt(r2));
            for (int k = 0; k < 3; ++k) acc[k] -= f * d[k];
            sc += f * sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        }
        gx[a] = acc[0];
        gy[a] = acc[1];
        gz[a] = acc[2];
        if (scale) scale[a] = sc;
    }
}

/* Monopole and quadrupole moments of a set of particles (indices idx[0..k)):
 * M, the centre of mass c and the traceless quadrupole
 *   Q_ij = sum m (3 d_i d_j - |d|^2 delta_ij),  d = x_b - c,
 * packed as [M, cx, cy, cz, Q11, Q12, Q13, Q22, Q23, Q33].  The sums over a
 * node run in extended precision (long double): a node can hold millions of
 * particles, and a running double sum of that length would lose more than the
 * 1e-12 the accelerations are compared at; the terms themselves are doubles. */
void ora_moments(int64_t k, const int64_t* idx, const double* x, const double* y,
                 const double* z, const double* m, double* out)
{
    long double M = 0.0L, sx = 0.0L, sy = 0.0L, sz = 0.0L;
    for (int64_t i = 0; i < k; ++i) {
        int64_t b = idx[i];
        M += m[b];
        sx += m[b] * x[b];
        sy += m[b] * y[b];
        sz += m[b] * z[b];
    }
    double c[3] = {0, 0, 0};
    if (M > 0.0L) { c[0] = (double)(sx / M); c[1] = (double)(sy / M); c[2] = (double)(sz / M); }
    long double Q[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; i < k; ++i) {
        int64_t b = idx[i];
        double d[3] = {x[b] - c[0], y[b] - c[1], z[b] - c[2]};
        double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        Q[0] += m[b] * (3.0 * d[0] * d[0] - d2);
        Q[1] += m[b] * (3.0 * d[0] * d[1]);
        Q[2] += m[b] * (3.0 * d[0] * d[2]);
        Q[3] += m[b] * (3.0 * d[1] * d[1] - d2);
        Q[4] += m[b] * (3.0 * d[1] * d[2]);
        Q[5] += m[b] * (3.0 * d[2] * d[2] - d2);
    }
    out[0] = (double)M; out[1] = c[0]; out[2] = c[1]; out[3] = c[2];
    for (int j = 0; j < 6; ++j) out[4 + j] = (double)Q[j];
}

/* Acceleration at x of the expansion (mo as ora_moments packs it) to second
 * order, with the Plummer-softened distance rho^2 = |r|^2 + eps^2, r = x - c:
 *   g = -G M r / rho^3 + G (Q r / rho^5 - (5/2) (r.Q.r) r / rho^7). */
void ora_multipole_accel(const double* mo, const double* x, double G, double eps,
                         double* g)
{
    double r[3] = {x[0] - mo[1], x[1] - mo[2], x[2] - mo[3]};
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps * eps;
    double ir = 1.0 / sqrt(r2);
    double ir2 = ir * ir;
    double ir3 = ir * ir2, ir5 = ir3 * ir2, ir7 = ir5 * ir2;
    const double* Q = mo + 4;
    double Qr[3] = {Q[0] * r[0] + Q[1] * r[1] + Q[2] * r[2],
                    Q[1] * r[0] + Q[3] * r[1] + Q[4] * r[2],
                    Q[2] * r[0] + Q[4] * r[1] + Q[5] * r[2]};
    double rQr = r[0] * Qr[0] + r[1] * Qr[1] + r[2] * Qr[2];
    for (int k = 0; k < 3; ++k)
        g[k] = -G * mo[0] * r[k] * ir3 + G * (Qr[k] * ir5 - 2.5 * rQr * r[k] * ir7);
}

/* The tree: the particles in the stable order of their keys' prefix of L
 * levels (key domain lo/hi as ora_morton_keys); the node of level l (0..L) with prefix P holds the
 * particles whose key shifted right by 3(21-l) equals P; its size is the
 * largest extent of the key domain over 2^l.  Walk per target, depth first
 * from the root, children in ascending prefix:
 *   - a node holding the target's own key prefix is opened;
 *   - otherwise a node whose size s and distance d = |x_a - c| satisfy
 *     s < theta d (tested as s^2 < theta^2 d^2) contributes its expansion;
 *   - an opened node of level L contributes its particles b != a directly
 *     (in key order), an opened node above L its children.
 * theta = 0 opens every node and so sums every pair directly. */
typedef struct {
    int64_t start, end;   /* range in the sorted order */
    uint64_t prefix;
    double mo[10];
} ora_gnode;

typedef struct {
    int L;
    int64_t count[10];
    ora_gnode* lev[10];
    const int64_t* order;     /* sorted position -> particle */
    const uint64_t* skeys;    /* keys in sorted order */
    double size[10];
} ora_gtree;

static void ora_gwalk(const ora_gtree* T, int l, int64_t node, int64_t a, uint64_t ka,
                      const double* x, const double* y, const double* z, const double* m,
                      double G, double eps, double theta, double acc[3], double* sc)
{
    const ora_gnode* nd = &T->lev[l][node];
    const int sh = 3 * (21 - l);
    const double xa[3] = {x[a], y[a], z[a]};
    int open = (ka >> sh) == nd->prefix;
    if (!open) {
        double d[3] = {xa[0] - nd->mo[1], xa[1] - nd->mo[2], xa[2] - nd->mo[3]};
        double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (T->size[l] * T->size[l] < theta * theta * d2) {
            double g[3];
            ora_multipole_accel(nd->mo, xa, G, eps, g);
            for (int k = 0; k < 3; ++k) acc[k] += g[k];
            *sc += sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
            return;
        }
    }
    if (l == T->L) {
        for (int64_t i = nd->start; i < nd->end; ++i) {
            int64_t b = T->order[i];
            if (b == a) continue;
            double d[3] = {xa[0] - x[b], xa[1] - y[b], xa[2] - z[b]};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps * eps;
            double f = G * m[b] / (r2 * sqrt(r2));
            for (int k = 0; k < 3; ++k) acc[k] -= f * d[k];
            *sc += f * sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        }
        return;
    }
    /* children: the nodes of level l+1 with prefixes 8P .. 8P+7 */
    const ora_gnode* ch = T->lev[l + 1];
    int64_t lo = 0, hi = T->count[l + 1];
    while (lo < hi) {   /* first child with prefix >= 8P */
        int64_t mid = (lo + hi) / 2;
        if (ch[mid].prefix < nd->prefix * 8) lo = mid + 1; else hi = mid;
    }
    for (int64_t c = lo; c < T->count[l + 1] && ch[c].prefix < nd->prefix * 8 + 8; ++c)
        ora_gwalk(T, l + 1, c, a, ka, x, y, z, m, G, eps, theta, acc, sc);
}

void ora_gravity_tree(int64_t n, const double* x, const double* y, const double* z,
                      const double* m, const double* lo, const double* hi, int L, double G,
                      double eps, double theta, int64_t nt, const int64_t* targets,
                      double* gx, double* gy, double* gz, double* scale)
{
    if (L < 0 || L > 9) return;
    uint64_t* keys = malloc(sizeof(uint64_t) * n);
    int64_t* order = malloc(sizeof(int64_t) * n);
    uint64_t* skeys = malloc(sizeof(uint64_t) * n);
    ora_morton_keys(n, x, y, z, lo, hi, keys);
    ora_sort_keys_level(n, keys, L, order);
    for (int64_t i = 0; i < n; ++i) skeys[i] = keys[order[i]];
    ora_gtree T;
    T.L = L;
    T.order = order;
    T.skeys = skeys;
    double ext = 0.0;
    for (int k = 0; k < 3; ++k)
        if (hi[k] - lo[k] > ext) ext = hi[k] - lo[k];
    for (int l = 0; l <= L; ++l) {
        T.size[l] = ext / (double)(1 << l);
        const int sh = 3 * (21 - l);
        /* the nodes of level l: runs of equal prefix in the sorted keys */
        int64_t cnt = 0;
        for (int64_t i = 0; i < n; ++i)
            if (i == 0 || (skeys[i] >> sh) != (skeys[i - 1] >> sh)) ++cnt;
        T.count[l] = cnt;
        T.lev[l] = malloc(sizeof(ora_gnode) * (cnt > 0 ? cnt : 1));
        int64_t j = -1;
        for (int64_t i = 0; i < n; ++i) {
            if (i == 0 || (skeys[i] >> sh) != (skeys[i - 1] >> sh)) {
                ++j;
                T.lev[l][j].start = i;
                T.lev[l][j].prefix = skeys[i] >> sh;
            }
            T.lev[l][j].end = i + 1;
        }
        for (int64_t c = 0; c < cnt; ++c) {
            ora_gnode* nd = &T.lev[l][c];
            ora_moments(nd->end - nd->start, order + nd->start, x, y, z, m, nd->mo);
        }
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = ora_tgt(targets, t);
        double acc[3] = {0, 0, 0}, sc = 0.0;
        if (T.count[0] > 0)
            ora_gwalk(&T, 0, 0, a, keys[a], x, y, z, m, G, eps, theta, acc, &sc);
        gx[a] = acc[0];
        gy[a] = acc[1];
        gz[a] = acc[2];
        if (scale) scale[a] = sc;
    }
    for (int l = 0; l <= L; ++l) free(T.lev[l]);
    free(keys);
    free(order);
    free(skeys);
}

/* threads the OpenMP loops above run on */
#ifdef _OPENMP
#include <omp.h>
int ora_num_threads(void) { return omp_get_max_threads(); }
void ora_set_num_threads(int k) { omp_set_num_threads(k > 0 ? k : 1); }
#else
int ora_num_threads(void) { return 1; }
void ora_set_num_threads(int k) { (void)k; }
#endif
