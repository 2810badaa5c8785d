// sph_common.h -- internal declarations shared by the libsph HIP sources.
//
// Data layout in HBM (all caller-owned, see include/sph.h):
//   * particle fields are structure-of-arrays FP64, one array per field, so a
//     wavefront of 64 consecutive slots reads 512 contiguous bytes per field;
//   * neighbour lists are int32 in tiles of 64 slots (see lpos), so the 64 lanes
//     of a wavefront reading entry j of their own targets hit 256 contiguous
//     bytes and one wavefront's rows are contiguous;
//   * the workspace holds the device-resident domain record, sort buffers, the
//     dense cell table (start/end/max-h per Morton cell) and the lists.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "sph.h"

namespace sph {

constexpr int kBlock = 256;          // threads per workgroup (4 wavefronts)
constexpr int kMaxLevel = 9;         // cell table holds at most 8^9 cells
constexpr int kKeyBits = 21;         // bits per axis in the 63-bit key
constexpr int kSumBlocks = 1024;     // fixed partition of the conservation sums
constexpr int kMaxPermFields = 16;
constexpr int kWalkPad = 8;          // spare records after the last slot (cell-walk batches)

// ---------------------------------------------------------------- run parameters
// POD copied by value into every kernel.
struct Params {
    int64_t n;
    double box_lo[3], box_hi[3], L[3], halfL[3];
    int periodic[3];
    int sinc_n;
    double bn;             // B_n normalisation of the sinc kernel
    double n_target;
    int ng_max;
    int newton_iters;
    double kappa;
    int eos;
    double gamma, c0, alpha;
    double courant, growth, acc_dt, energy_dt;
    int lcap;              // largest admissible cell level (8^lcap <= table size)
    int precision;
    int cand_cap;          // candidate-list capacity of the fused step (0: off)
    double wrapLd[3], wrapInvLd[3];  // L and 1/L on periodic axes, 0 on open ones
    float wrapL[3], wrapInvL[3];     // the same in FP32 (the fused step's candidate walk)
    // kernel tables (section 4.5): tab_n values of S_n and dS_n/dv at v_i = i dv,
    // dv = 2/(tab_n - 1), entry i holding the values at nodes i and i+1; 0 = off
    int tab_n;
    double tab_inv_dv;
    const double2* tabS;
    const double2* tabD;
    const float2* tabSf;
    const float2* tabDf;
};

// ---------------------------------------------------------------- device domain
// Written on the device by sph_build_cells (and find_neighbors for hmax_new);
// read by every later kernel, never by the host in the hot path.
struct Domain {
    double lo[3], hi[3];       // key domain: the box on periodic axes, bbox on open ones
    double scale[3];           // 2^21 / (hi - lo), 0 on a zero-extent axis
    double cell[3];            // cell edge (hi - lo) / 2^level
    double hmax;               // largest h at build time
    uint64_t hmax_new_bits;    // largest h after update_h (order-preserving bits)
    uint64_t ord_min[3];       // order-preserving bits for the bbox reduction
    uint64_t ord_max[3];
    uint64_t ord_hmax;
    uint64_t dtmin_bits;       // min_a h_a/c_a (bits of a positive double)
    int32_t level, shift, ncell_axis;
    uint32_t err;              // sticky SPH_ERRBIT_* word
    uint32_t refit;            // fused step: an h left the short candidate reach
    uint32_t nonuniform;       // some m or c differs from slot 0's (full momentum records)
    uint32_t mass_varies;      // some m differs from slot 0's (set by the cell build)
    int32_t reach_level;       // fused step: level of the blocks that bound each walk's reach
    float walk_slack;          // 2^-20 x the largest extent (FP32 candidate walk)
    int64_t built_n;
};

// ---------------------------------------------------------------- packed records
// Gathered per neighbour; one record is a few 16-byte loads instead of one
// load per structure-of-arrays field.
struct alignas(32) Pos4 {
    double x, y, z, h;
};
// the candidate walk's record (fused step): FP32 offsets of the position from
// the key domain's low corner and the particle's squared short reach, widened
// to cover the rounding of the FP32 test ((2 lambda h + slack)^2 (1 + 2^-18),
// h rounded up), so the walk's candidates are a superset of the exact ones
struct alignas(16) Pos4f {
    float x, y, z, r2;
};
constexpr float kWalkGrow = 1.0f + 0x1p-18f;
// what the IAD pass needs of a neighbour: position and volume m/rho
struct alignas(32) PosV {
    double x, y, z, v;
};
// everything the momentum/energy pass needs of a neighbour.  With d = x_b - x_a
// the b-side terms of a_a are
//   m_b P_b/(Omega_b rho_b^2) C_b d W_b = q_b W_b K_b d   (pressure)
//   (m_b/rho_b) C_b d W_b               = W_b K_b d       (viscosity),
// so C_b, 1/rho_b, P_b/(Omega_b rho_b^2) and m_b fold into K_b = (m_b/rho_b) C_b
// and q_b = P_b/(Omega_b rho_b); m_b stays for the a-side terms.
// A neighbour's fields fill the first eight 16-byte columns; the ninth holds h,
// which only the target reads.  The stride of nine columns, an odd number,
// matters: the lanes of a wavefront load the same field of different records,
// and an odd stride puts those fields in different columns of their cache
// lines.  (At 64 M particles the pass took 63 ms so, 82 ms with 128-byte
// records, where they all share one column, and 70 ms with a neighbour field
// in the ninth column, one more load per neighbour.)
struct alignas(16) MomNbr {
    double x, y, z, ih;                    // position and 1/h
    double k11, k12, k13, k22, k23, k33;   // K = (m/rho) C, C = tau^-1
    double q, c, m;                        // P/(Omega rho), sound speed, mass
    double vx, vy, vz;
    double h, spare;                       // smoothing length (the target's own)
};
static_assert(sizeof(MomNbr) == 144, "an odd number of 16-byte columns");
// The same record when every particle has the same mass and sound speed (the
// weakly compressible EOS sets c = c0): m and c come from slot 0, and the
// fourteen doubles fill seven columns, again an odd number (112 B).
struct alignas(16) MomNbrU {
    double x, y, z, ih;
    double k11, k12, k13, k22, k23, k33;
    double q;
    double vx, vy, vz;
};
static_assert(sizeof(MomNbrU) == 112, "an odd number of 16-byte columns");
// the reverse pass reads the factors unfolded (144 B)
struct alignas(16) MomRec {
    double x, y, z, h;                     // position and smoothing length
    double c11, c12, c13, c22, c23, c33;   // IAD matrix C = tau^-1
    double irho, c, pb, m;                 // 1/rho, sound speed, P/(Omega rho^2), mass
    double vx, vy, vz, invh;
};
static_assert(sizeof(MomNbr) <= sizeof(MomRec), "MomNbr records alias the MomRec area");
struct alignas(16) CellRange {
    int32_t s, e;   // particle slots [s, e) of one Morton cell
    double hmax;    // largest h in the cell (set before the symmetric searches)
};

// ---------------------------------------------------------------- neighbour lists
// Lists are stored in tiles of 64 consecutive slots (one wavefront): entry j of
// slot a lives at ((a/64)*cap + j)*64 + a%64.  Lanes reading or writing entry j
// of their own targets touch one 256-byte row, and one wavefront's rows are
// contiguous (a global column-major layout would put them n*4 bytes apart).
__host__ __device__ inline int64_t lpos(int64_t a, int j, int cap)
{
    return ((a >> 6) * (int64_t)cap + j) * 64 + (a & 63);
}

// Candidate lists (fused step) are stored in chunks of 8 entries per slot: the
// 8 entries j..j+7 (j a multiple of 8) of slot a are 32 contiguous bytes, and
// the 64 slots of a wavefront tile keep their chunks side by side.  The walk
// appends into registers and writes whole chunks (the writes are not lane-
// synchronous, so one 4-byte write per entry left lines partly written); the
// readers load one chunk per batch of 8.  cap is a multiple of 8.
__host__ __device__ inline int64_t lpos8(int64_t a, int j, int cap)
{
    return (((a >> 6) * (int64_t)(cap >> 3) + (j >> 3)) * 64 + (a & 63)) * 8 + (j & 7);
}

// The fused step walks the cells once for a candidate list with reach
// 2 kappa max(h0_a, h0_b): the Newton clamp keeps h <= kappa h0, so every set
// the step needs is a subset.  Used when kappa <= kFusedKappaMax; the
// workspace layout depends on (n, ng_max) only, never on per-call parameters.
constexpr double kFusedKappaMax = 1.25;
// The fused step first collects candidates within 2 lambda max(h0_a, h0_b),
// lambda = kFusedReach (1.09x the list volume instead of kappa^3 = 1.95x), and
// runs Newton on them; if any iterate h leaves [0, lambda h0] it repeats both
// with the full reach kappa.  Either way the sets are exact.
constexpr double kFusedReach = SPH_SHORT_REACH;

// 2 kap in FP32, rounded up (host side)
inline float reach_f32(double kap)
{
    float f = (float)(2.0 * kap);
    return ((double)f < 2.0 * kap) ? nextafterf(f, INFINITY) : f;
}
// the same for the fused step's short reach lambda = min(kFusedReach, kappa)
inline float short_reach_f32(double kappa)
{
    return reach_f32(kappa < kFusedReach ? kappa : kFusedReach);
}
int candidate_capacity(int ng_max);

// ---------------------------------------------------------------- workspace layout
struct Layout {
    size_t domain, sums, keys0, keys1, idx0, idx1, hist, scanpart;
    size_t cells, nc, ns, nk, p4, pf, rec, vol, pv, list, cand, posm;
    size_t tabS, tabD, tabSf, tabDf;
    size_t flag, reach;
    size_t total;
    int64_t n, nsort_blocks, hist_len, scan_blocks, ncells_cap;
    int lcap, cand_cap;
};
Layout make_layout(int64_t n, int ng_max);

// device pointers carved out of ws
struct Ws {
    Domain* dom;
    double* sums;
    uint64_t *keys0, *keys1;
    uint32_t *idx0, *idx1;
    uint32_t* hist;
    uint32_t* scanpart;
    CellRange* cells;
    int32_t *nc, *ns, *list;
    int32_t *nk, *cand;        // candidate counts and lists of the fused step
    Pos4* p4;
    MomRec* rec;               // the reverse pass's records; the step's MomNbr alias them
    double* vol;               // m/rho per particle (IAD pass)
    PosV* pv;                  // position and m/rho (IAD neighbour records)
    Pos4f* pf;                 // FP32 walk records of the fused candidate pass
    void* posm;                // mixed precision: fixed-point position + FP32 mass or volume (16 B)
    void* recm;                // mixed precision: FP32 momentum records (aliases rec)
    double* tmp;               // permute scratch (aliases the list area)
    double2 *tabS, *tabD;      // kernel tables (kernel_table > 0), FP64 and FP32
    float2 *tabSf, *tabDf;
    uint8_t* flag;             // fused step: 2 h left the short reach, 1 a neighbour of one
    double* reach;             // fused step: per-block h bounds of the walk (levels, then reach)
};
Ws carve(void* ws, const Layout& L);

// ---------------------------------------------------------------- device helpers
#define SPH_DEV __device__ __forceinline__
#define SPH_HD __host__ __device__ __forceinline__

// map a double to uint64 bits whose unsigned order is the numeric order
SPH_HD uint64_t ord_bits(double v)
{
    uint64_t b = __builtin_bit_cast(uint64_t, v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
SPH_HD double ord_value(uint64_t o)
{
    uint64_t b = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
    return __builtin_bit_cast(double, b);
}

// Sets bits of a flag word that only gains bits: a wavefront that reads them
// already set skips the atomic (one atomic per wavefront on one address
// serialises: 125 K of them made the 8 M-particle uniformity check take 1 ms).
SPH_DEV void flag_or(uint32_t* p, uint32_t bits)
{
    if ((__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bits) != bits)
        atomicOr(p, bits);
}

SPH_DEV void set_err(Domain* d, uint32_t bit) { flag_or(&d->err, bit); }

// Global minimum / maximum of order-preserving bits.  The held value only moves
// one way, so a wavefront whose value is no better than one it reads cannot
// change it and skips the atomic (a stale read costs an atomic, never an
// update).  With one atomic per wavefront on one address these serialise:
// 262 K of them made the 16.7 M-cell h_max pass take 3 ms.
SPH_DEV void ord_min_to(uint64_t* p, double v)
{
    const uint64_t b = ord_bits(v);
    if (b < __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMin((unsigned long long*)p, (unsigned long long)b);
}
SPH_DEV void ord_max_to(uint64_t* p, double v)
{
    const uint64_t b = ord_bits(v);
    if (b > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax((unsigned long long*)p, (unsigned long long)b);
}

// spread the low 21 bits of v to every third bit (bit i -> bit 3i)
SPH_HD uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x001f00000000ffffull;
    v = (v | (v << 16)) & 0x001f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}
SPH_HD uint64_t morton3(uint64_t qx, uint64_t qy, uint64_t qz)
{
    return (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
}

// per-axis 21-bit coordinate (floor((x-lo)*scale), clamped to [0, 2^21-1])
SPH_DEV uint32_t quantize(double x, double lo, double scale)
{
    if (!(scale > 0.0)) return 0u;
    double t = x - lo;
    double q = floor(t * scale);
    if (!(q >= 0.0)) return 0u;
    if (q > 2097151.0) return 2097151u;
    return (uint32_t)q;
}

// displacement b - a with the minimum image, and r^2 in the fixed association
// (dx*dx + dy*dy) + dz*dz (no contraction: the library is built with
// -ffp-contract=off, so the neighbour test rounds the same everywhere)
SPH_DEV double disp(const Params& P, double xa, double ya, double za, double xb, double yb,
                    double zb, double& dx, double& dy, double& dz)
{
    // minimum image: d - L rint(d/L), a single rounding like d -= L, and no
    // shift on open axes (L = 0 there).  It picks the image of the half-open
    // (-L/2, L/2] everywhere except within rounding of |d| = L/2, where no
    // pair is within reach (the step flags 4h >= L as an error).
    dx = xb - xa;
    dy = yb - ya;
    dz = zb - za;
    dx = fma(-P.wrapLd[0], rint(dx * P.wrapInvLd[0]), dx);
    dy = fma(-P.wrapLd[1], rint(dy * P.wrapInvLd[1]), dy);
    dz = fma(-P.wrapLd[2], rint(dz * P.wrapInvLd[2]), dz);
    double r2 = dx * dx;
    r2 = r2 + dy * dy;
    r2 = r2 + dz * dz;
    return r2;
}

// disp() with the minimum image applied on the axes of kPer only (bit k: axis
// k periodic); on the others it is the identity there too, so the results are
// the same bits as disp()'s
template <int kPer>
SPH_DEV double disp_p(const Params& P, double xa, double ya, double za, double xb, double yb,
                      double zb, double& dx, double& dy, double& dz)
{
    dx = xb - xa;
    dy = yb - ya;
    dz = zb - za;
    if (kPer & 1) dx = fma(-P.wrapLd[0], rint(dx * P.wrapInvLd[0]), dx);
    if (kPer & 2) dy = fma(-P.wrapLd[1], rint(dy * P.wrapInvLd[1]), dy);
    if (kPer & 4) dz = fma(-P.wrapLd[2], rint(dz * P.wrapInvLd[2]), dz);
    double r2 = dx * dx;
    r2 = r2 + dy * dy;
    r2 = r2 + dz * dz;
    return r2;
}

// A record staged in LDS, read back as whole 16-byte columns.  Staged records
// sit at strides (20 or 28 dwords) where 16-byte reads by the lanes of a
// wavefront hit distinct banks but narrower ones conflict two to four ways;
// read as a structure, the compiler may split the record into 8-byte or
// dword pairs, so the columns are read as 4-dword vectors first.
template <class Rec>
SPH_DEV Rec lds_record(const int4* col)
{
    static_assert(sizeof(Rec) % 16 == 0, "records of whole 16-byte columns");
    typedef int v4i __attribute__((ext_vector_type(4)));
    constexpr int kCols = (int)(sizeof(Rec) / 16);
    const v4i* src = (const v4i*)col;
    v4i cw[kCols];
#pragma unroll
    for (int i = 0; i < kCols; ++i) cw[i] = src[i];
    Rec r;
    __builtin_memcpy(&r, cw, sizeof(Rec));
    return r;
}

// The two lanes of a pair (2q, 2q+1) swap a 32-bit value (quad permute 1 0 3 2).
SPH_DEV int32_t pair_swap(int32_t v)
{
    return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
}
SPH_DEV double pair_swap(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)pair_swap((int32_t)(uint32_t)u);
    const uint32_t hi = (uint32_t)pair_swap((int32_t)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Record b (four doubles, 32 bytes) of this lane, gathered by the two lanes of
// a pair together: one 16-byte load per lane fetches the even lane's record
// (first half to the even lane, second to the odd one) and a second the odd
// lane's, so each load touches one line per pair instead of one per lane; a
// swap then completes each lane's own record.  Both lanes must be active.
template <class T>
SPH_DEV T pair_gather32(const T* __restrict__ base, int32_t b, int odd)
{
    static_assert(sizeof(T) == 32, "a record of four doubles");
    const int32_t o = pair_swap(b);
    const int32_t rA = odd ? o : b;   // the even lane's record
    const int32_t rB = odd ? b : o;   // the odd lane's record
    const double2* half = (const double2*)base;
    const double2 A = half[2 * (int64_t)rA + odd];
    const double2 B = half[2 * (int64_t)rB + odd];
    // even lane: A = first half of its own record, B = first half of the odd
    // lane's; odd lane: A = second half of the even lane's, B = its own
    const double r0 = pair_swap(odd ? A.x : B.x);
    const double r1 = pair_swap(odd ? A.y : B.y);
    return odd ? T{r0, r1, B.x, B.y} : T{A.x, A.y, r0, r1};
}

// calls f(std::integral_constant<int, kPer>) for the periodic axes of P
template <class F>
inline void with_periodic(const Params& P, F&& f)
{
    const int per = (P.periodic[0] ? 1 : 0) | (P.periodic[1] ? 2 : 0) | (P.periodic[2] ? 4 : 0);
    switch (per) {
    case 0: f(std::integral_constant<int, 0>{}); break;
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    default: f(std::integral_constant<int, 7>{}); break;
    }
}

// ------------------------------------------------------------- sinc kernel
// With x = (pi/2) v and t = x^2 the kernel needs only even functions of x,
// i.e. functions of t on 0 <= t <= pi^2:
//   sinc(x)      ~ kSincS64 polynomial in t (11 terms)
//   x sinc'(x)   ~ t * kSincQ64 polynomial in t (10 terms)
// (fits on the support, accurate to the rounding of their Horner evaluation,
// generated by gen_sinc_poly.py).  No sin, sqrt or division per pair.
}  // namespace sph
#include "sph_sinc_poly.h"
namespace sph {

constexpr double kPi = 3.14159265358979323846;
constexpr double kPiHalfSq = (kPi * kPi) / 4.0;

// s t + c as one v_fma_f64 that takes the coefficient c from a scalar register
// pair.  Written out because, left to itself, the compiler keeps polynomial
// coefficients in vector registers and issues a copy before each step
// (v_mov_b64 + v_fmac_f64), twice the vector instructions of the polynomial.
SPH_DEV double fma_sc(double s, double t, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(s), "v"(t), "s"(c));
    return r;
}

// 1/sqrt(x) for normal x > 0: the hardware estimate (relative error about
// 2^-23) refined by two Newton steps on f(y) = 1/y^2 - x, each
// y <- y + (y/2)(1 - x y^2), to within a few ulp.
SPH_DEV double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double e = fma(-(x * y), y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

template <int K>
SPH_DEV double horner(const double (&c)[K], double t)
{
    double s = c[K - 1];
#pragma unroll
    for (int k = K - 2; k >= 0; --k) s = fma_sc(s, t, c[k]);
    return s;
}

// s^(n-1) for the integer exponent n (n is uniform across the launch; the usual
// n = 6 takes three multiplications)
template <class T>
SPH_DEV T pow_nm1(T s, int n)
{
    if (n == 6) {
        T s2 = s * s;
        return s2 * s2 * s;
    }
    T p = T(1);
    for (int i = 1; i < n; ++i) p = p * s;
    return p;
}

// S_n and v dS_n/dv at t = (pi/2)^2 v^2, integer n >= 1
SPH_DEV void sinc_terms(double t, int n, double& S, double& vdS)
{
    const double s = horner(kSincS64, t);
    const double q = horner(kSincQ64, t) * t;   // x sinc'(x)
    const double p = pow_nm1(s, n);             // s^(n-1)
    S = p * s;
    vdS = (double)n * p * q;
}

SPH_DEV double sinc_S(double t, int n)
{
    const double s = horner(kSincS64, t);
    return pow_nm1(s, n) * s;
}

// Kernel lookup table (section 4.5): S_n at v = r/h by linear interpolation
// between the two nodes around v, (1 - f) S_i + f S_{i+1}; likewise dS_n/dv.
// The index is clamped to the last interval (v reaches 2 only to rounding).
template <class T>
SPH_DEV void tab_index(T v, T inv_dv, int n, int& i, T& f)
{
    const T s = v * inv_dv;
    i = (int)s;
    if (i > n - 2) i = n - 2;
    f = s - (T)i;
}

// S_n and v dS_n/dv at t = (pi/2)^2 v^2: the fitted polynomials, or (kTab)
// the tables; the hot kernels are compiled once per choice
template <bool kTab>
SPH_DEV void kern_terms_t(const Params& P, double t, double& S, double& vdS)
{
    if (kTab) {
        const double v = sqrt(t) * (2.0 / kPi);
        int i;
        double f;
        tab_index(v, P.tab_inv_dv, P.tab_n, i, f);
        const double2 e = P.tabS[i], d = P.tabD[i];
        S = (1.0 - f) * e.x + f * e.y;
        vdS = v * ((1.0 - f) * d.x + f * d.y);
    } else {
        sinc_terms(t, P.sinc_n, S, vdS);
    }
}

template <bool kTab>
SPH_DEV double kern_S_t(const Params& P, double t)
{
    if (kTab) {
        const double v = sqrt(t) * (2.0 / kPi);
        int i;
        double f;
        tab_index(v, P.tab_inv_dv, P.tab_n, i, f);
        const double2 e = P.tabS[i];
        return (1.0 - f) * e.x + f * e.y;
    }
    return sinc_S(t, P.sinc_n);
}

// the same chosen at run time (the stage kernels)
SPH_DEV void kern_terms(const Params& P, double t, double& S, double& vdS)
{
    if (P.tab_n > 0) kern_terms_t<true>(P, t, S, vdS);
    else kern_terms_t<false>(P, t, S, vdS);
}

SPH_DEV double kern_S(const Params& P, double t)
{
    return P.tab_n > 0 ? kern_S_t<true>(P, t) : kern_S_t<false>(P, t);
}

// calls f(std::integral_constant<bool, kTab>) for the kernel evaluation of P
template <class F>
inline void with_table(const Params& P, F&& f)
{
    if (P.tab_n > 0) f(std::integral_constant<bool, true>{});
    else f(std::integral_constant<bool, false>{});
}

// Largest number of wavefronts per SIMD for the neighbour-loop kernels (0: as
// many as the registers allow).  These kernels gather neighbour records that
// the wavefronts of a compute unit do not share, so past a point more resident
// wavefronts only evict each other's records from the caches.
#define SPH_WAVES_CAP(n) __attribute__((amdgpu_waves_per_eu(1, n)))
#ifndef SPH_WAVES_MOM
#define SPH_WAVES_MOM 2
#endif
#ifndef SPH_WAVES_PAIR
#define SPH_WAVES_PAIR 2
#endif
#ifndef SPH_WAVES_IAD
#define SPH_WAVES_IAD 3
#endif
#ifndef SPH_WAVES_SEARCH
#define SPH_WAVES_SEARCH 3
#endif
// exactly n wavefronts per SIMD (the compiler holds the registers to fit)
#define SPH_WAVES_EXACT(n) __attribute__((amdgpu_waves_per_eu(n, n)))
#ifndef SPH_WAVES_NEWTON
#define SPH_WAVES_NEWTON 4
#endif
#ifndef SPH_NEWTON_ATTR
#define SPH_NEWTON_ATTR SPH_WAVES_EXACT(SPH_WAVES_NEWTON)
#endif
#ifndef SPH_FILTER_ATTR
#define SPH_FILTER_ATTR SPH_WAVES_CAP(SPH_WAVES_SEARCH)
#endif
#ifndef SPH_MOM_ATTR
#define SPH_MOM_ATTR SPH_WAVES_CAP(SPH_WAVES_MOM)
#endif
#ifndef SPH_WAVES_CAND
#define SPH_WAVES_CAND 7
#endif
// the candidate walk runs best with exactly this many (registers held to fit):
// its dependent cell-record -> particle-record round trips need resident
// wavefronts more than batches in flight
#ifndef SPH_WAVES_CAND_EXACT
#define SPH_WAVES_CAND_EXACT 1
#endif
#if SPH_WAVES_CAND_EXACT
#define SPH_WAVES_CAND_ATTR __attribute__((amdgpu_waves_per_eu(SPH_WAVES_CAND, SPH_WAVES_CAND)))
#else
#define SPH_WAVES_CAND_ATTR SPH_WAVES_CAP(SPH_WAVES_CAND)
#endif
#ifndef SPH_WAVES_MIXED
#define SPH_WAVES_MIXED 3
#endif

// Density, grad-h term and EOS of slot a from its two density sums
// sS = sum m_b S, sD = sum m_b (3 S + v dS/dv) over N(a) and a itself (eq. 1;
// Omega = 1 + h/(3 rho) sum m dW/dh with dW/dh = -(B/h^4)(3 S + v dS/dv)).
struct DensOut {
    const double *m, *u, *p_ref, *rho_ref;
    double *rho, *omega, *p, *c;
};
SPH_DEV void finish_density(const Params& P, Domain* dom, const DensOut& O, int64_t a, double ha,
                            double sS, double sD)
{
    const double w0 = P.bn / (ha * ha * ha);
    const double r = w0 * sS;
    const double om = 1.0 - w0 * sD / (3.0 * r);
    double pr, c;
    if (P.eos == SPH_EOS_IDEAL) {
        pr = (P.gamma - 1.0) * r * O.u[a];
        c = sqrt(P.gamma * (P.gamma - 1.0) * O.u[a]);
    } else {
        pr = O.p_ref[a] + P.c0 * P.c0 * (r - O.rho_ref[a]);
        c = P.c0;
    }
    O.rho[a] = r;
    O.omega[a] = om;
    O.p[a] = pr;
    O.c[a] = c;
    if (!isfinite(r) || !isfinite(om) || !isfinite(pr) || !isfinite(c))
        set_err(dom, SPH_ERRBIT_NONFINITE);
}

// neighbours whose records the momentum/energy loops load before computing
#ifndef SPH_MOM_BATCH
#define SPH_MOM_BATCH 4
#endif
// the momentum pass over 112-byte records, staged through LDS: batches of 2
// at two wavefronts (57 KB of LDS per workgroup)
#ifndef SPH_MOM_U_BATCH
#define SPH_MOM_U_BATCH 2
#endif
// the mixed-precision momentum pass over 64-byte records, staged the same way
// (20 KB of LDS per batch and workgroup)
#ifndef SPH_MOM_M_U_BATCH
#define SPH_MOM_M_U_BATCH 2
#endif

// neighbour loops load this many neighbours' records before computing on them
// (independent gathers in flight per wavefront)
#ifndef SPH_GATHER_BATCH
#define SPH_GATHER_BATCH 8
#endif
constexpr int kBatch = SPH_GATHER_BATCH;

// ------------------------------------------------------------- launch helpers
// The hardware hands workgroup i to XCD (i mod 8); remap so that each XCD
// works on one contiguous range of slots (spatially close particles share the
// XCD's L2).  Launch grid_xcd(nb) groups; returns -1 for padding groups.
constexpr int kXcds = 8;
inline int64_t grid_xcd(int64_t nb) { return (nb + kXcds - 1) / kXcds * kXcds; }
SPH_DEV int64_t xcd_block(int64_t nb)
{
    int64_t bid = blockIdx.x;
    int64_t per = (nb + kXcds - 1) / kXcds;
    int64_t lb = (bid % kXcds) * per + bid / kXcds;
    return lb < nb ? lb : -1;
}

// ------------------------------------------------------------- host launchers
Params make_params(const sph_config* cfg, double bn, int lcap, int cand_cap);   // cand_cap 0: fused path off
double sinc_bn(int n);   // host: B_n normalisation

hipError_t launch_build_cells(const Params& P, const Layout& L, const Ws& W,
                              const sph_particles* p, hipStream_t s);
// `pack` refreshes the packed positions from the caller's x, y, z, h first (the
// stage entry points do; sph_step packs once after the cell build)
hipError_t launch_pack_p4(const Params& P, const Ws& W, const sph_particles* p, hipStream_t s);
hipError_t launch_update_h(const Params& P, const Layout& L, const Ws& W, sph_particles* p,
                           hipStream_t s, bool pack);
hipError_t launch_find_neighbors(const Params& P, const Layout& L, const Ws& W,
                                 const sph_particles* p, hipStream_t s);
hipError_t launch_density(const Params& P, const Layout& L, const Ws& W, sph_particles* p,
                          hipStream_t s, bool pack);
// write_rec: also fill the momentum records (sph_step), else momentum packs them
hipError_t launch_iad(const Params& P, const Layout& L, const Ws& W, sph_particles* p,
                      hipStream_t s, bool pack, bool write_rec);
// sets Domain::nonuniform if any m or c differs from slot 0's (before the
// momentum records are written: it selects their layout)
hipError_t launch_uniform_check(const Params& P, const Ws& W, const sph_particles* p,
                                hipStream_t s);
// the unfolded 144-byte records the reverse pass reads (over the step's MomNbr)
hipError_t launch_pack_rec(const Params& P, const Ws& W, const sph_particles* p, hipStream_t s);
hipError_t launch_momentum_energy(const Params& P, const Layout& L, const Ws& W,
                                  sph_particles* p, hipStream_t s, bool pack);
// mixed-precision forms of the three pair passes (precision SPH_MIXED)
size_t mixed_posm_bytes();
size_t mixed_rec_bytes();
hipError_t launch_density_mixed(const Params& P, const Layout& L, const Ws& W, sph_particles* p,
                                hipStream_t s, bool pack);
hipError_t launch_iad_mixed(const Params& P, const Layout& L, const Ws& W, sph_particles* p,
                            hipStream_t s, bool pack, bool write_rec);
hipError_t launch_momentum_energy_mixed(const Params& P, const Layout& L, const Ws& W,
                                        sph_particles* p, hipStream_t s, bool pack);
// Optional phase markers: event k is recorded on the stream once phase k's
// launches are enqueued (sph_step_marked); no-ops without events.
struct Marks {
    hipEvent_t* ev = nullptr;
    int n = 0;
    void at(int k, hipStream_t s) const
    {
        if (ev && k < n) (void)hipEventRecord(ev[k], s);
    }
};
// with_density: the list filter also forms rho, Omega, P and c (the gather test
// it makes is the density's support test, with the final h)
hipError_t launch_fused_h_lists(const Params& P, const Layout& L, const Ws& W, sph_particles* p,
                                hipStream_t s, const Marks& mk = Marks(),
                                bool with_density = false);
hipError_t launch_pack_posm(const Params& P, const Ws& W, const sph_particles* p, hipStream_t s);
hipError_t launch_timestep(const Params& P, const Ws& W, sph_globals* g, hipStream_t s);
hipError_t launch_integrate(const Params& P, const Ws& W, sph_particles* p, sph_globals* g,
                            hipStream_t s);
hipError_t launch_clear_domain(const Ws& W, hipStream_t s);
// reverse mode (frozen structure): the forward stages of the step must have run
// on W and p (lists, packed positions and records, stage outputs, g->dt)
size_t adjoint_workspace_bytes(int64_t n);
size_t gravity_workspace_bytes(int L);
hipError_t launch_gravity(const Params& P, const Ws& W, const sph_particles* p, void* gws,
                          double G, double eps, double theta, double* gx, double* gy,
                          double* gz, hipStream_t s);
hipError_t launch_step_backward(const Params& P, const Ws& W, const sph_particles* p,
                                const sph_globals* g, const sph_grads* gout, sph_grads* gin,
                                void* adj_ws, hipStream_t s);
hipError_t launch_density_backward(const Params& P, const Ws& W, const sph_particles* p,
                                   const double* rho_bar, double* xb, double* yb, double* zb,
                                   void* adj_ws, hipStream_t s);

}  // namespace sph
