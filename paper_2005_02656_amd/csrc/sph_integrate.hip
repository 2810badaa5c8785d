// sph_integrate.hip -- kick-drift leapfrog for x and v, variable-step
// Adams-Bashforth for u (section 4.1), periodic wrap, and the conservation sums
// of the third global reduction (section 4.2).  The sums use a fixed grid and a
// fixed reduction tree, so they are bitwise reproducible.
#include "sph_common.h"

namespace sph {
namespace {

constexpr int kNSum = 9;  // mass, mom[3], ang[3], e_kin, e_int

struct IntState {
    double *x, *y, *z, *vx, *vy, *vz, *vhx, *vhy, *vhz, *u, *du_m1;
    const double *m, *ax, *ay, *az, *du;
};

__device__ __forceinline__ double block_sum(double v, double* lds)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < kBlock / 64; ++i) s += lds[i];
    return s;
}

__global__ __launch_bounds__(kBlock) void k_integrate(Params P, const sph_globals* __restrict__ g,
                                                      IntState S, double* __restrict__ part)
{
    const double dt = g->dt, lam = g->dt_m1;
    const double kick = 0.5 * (lam + dt), half = 0.5 * dt;
    const bool ab2 = lam > 0.0;
    const double q = ab2 ? dt / (2.0 * lam) : 0.0;
    double acc[kNSum] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t a = blockIdx.x * (int64_t)kBlock + threadIdx.x; a < P.n;
         a += (int64_t)gridDim.x * kBlock) {
        double X[3] = {S.x[a], S.y[a], S.z[a]};
        double VH[3] = {S.vhx[a], S.vhy[a], S.vhz[a]};
        const double A[3] = {S.ax[a], S.ay[a], S.az[a]};
        double V[3];
        for (int k = 0; k < 3; ++k) {
            double vh = VH[k] + A[k] * kick;
            double xn = X[k] + vh * dt;
            if (P.periodic[k]) {
                if (xn >= P.box_hi[k]) xn -= P.L[k];
                else if (xn < P.box_lo[k]) xn += P.L[k];
            }
            VH[k] = vh;
            X[k] = xn;
            V[k] = vh + A[k] * half;
        }
        const double du = S.du[a];
        double un = ab2 ? S.u[a] + dt * ((1.0 + q) * du - q * S.du_m1[a]) : S.u[a] + dt * du;
        S.x[a] = X[0]; S.y[a] = X[1]; S.z[a] = X[2];
        S.vhx[a] = VH[0]; S.vhy[a] = VH[1]; S.vhz[a] = VH[2];
        S.vx[a] = V[0]; S.vy[a] = V[1]; S.vz[a] = V[2];
        S.u[a] = un;
        S.du_m1[a] = du;
        const double m = S.m[a];
        acc[0] += m;
        acc[1] += m * V[0];
        acc[2] += m * V[1];
        acc[3] += m * V[2];
        acc[4] += m * (X[1] * V[2] - X[2] * V[1]);
        acc[5] += m * (X[2] * V[0] - X[0] * V[2]);
        acc[6] += m * (X[0] * V[1] - X[1] * V[0]);
        acc[7] += 0.5 * m * (V[0] * V[0] + V[1] * V[1] + V[2] * V[2]);
        acc[8] += m * un;
    }
    __shared__ double lds[kBlock / 64];
    for (int k = 0; k < kNSum; ++k) {
        double s = block_sum(acc[k], lds);
        if (threadIdx.x == 0) part[blockIdx.x * 10 + k] = s;
    }
}

__global__ __launch_bounds__(kBlock) void k_sums_finish(const double* __restrict__ part, int nblk,
                                                        sph_globals* g)
{
    __shared__ double lds[kBlock / 64];
    double out[kNSum];
    for (int k = 0; k < kNSum; ++k) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kBlock) v += part[b * 10 + k];
        out[k] = block_sum(v, lds);
    }
    if (threadIdx.x == 0) {
        g->mass = out[0];
        g->mom[0] = out[1]; g->mom[1] = out[2]; g->mom[2] = out[3];
        g->ang[0] = out[4]; g->ang[1] = out[5]; g->ang[2] = out[6];
        g->e_kin = out[7];
        g->e_int = out[8];
        g->t = g->t + g->dt;
        g->dt_m1 = g->dt;
    }
}

}  // namespace

hipError_t launch_integrate(const Params& P, const Ws& W, sph_particles* p, sph_globals* g,
                            hipStream_t s)
{
    IntState S{p->x, p->y, p->z, p->vx, p->vy, p->vz, p->vhx, p->vhy, p->vhz, p->u, p->du_m1,
               p->m, p->ax, p->ay, p->az, p->du};
    int64_t nb = (P.n + kBlock - 1) / kBlock;
    int grid = nb < kSumBlocks ? (int)nb : kSumBlocks;
    k_integrate<<<grid, kBlock, 0, s>>>(P, g, S, W.sums);
    k_sums_finish<<<1, kBlock, 0, s>>>(W.sums, grid, g);
    return hipGetLastError();
}

}  // namespace sph
