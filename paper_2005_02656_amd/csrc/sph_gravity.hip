// sph_gravity.hip -- self-gravity by a multipole expansion evaluated on the
// particle octree (section 4.1: gravity uses the tree that finds the
// neighbours).  Plummer-softened Newtonian gravity
//   g_a = -G sum_{b != a} m_b (x_a - x_b) / (|x_a - x_b|^2 + eps^2)^(3/2),
// approximated on the octree of the Morton keys: the node of level l
// (0 <= l <= L, L the deepest dense cell level of the layout) holds the slots
// whose key shifted right by 3(21 - l) equals its index, so each level is a
// dense table indexed by key prefix over the sorted slots.  Nodes carry the
// mass, the centre of mass and the traceless quadrupole about it; leaves from
// their particles, parents from their eight children (parallel-axis rule).
// Each target walks the tree depth first from the root, children in ascending
// prefix: a node holding the target's own key prefix is opened; another node of
// size s (the key domain's largest extent over 2^l) at distance d from its
// centre of mass contributes its expansion when s < theta d; an opened leaf
// contributes its particles directly, in slot order.
#include "sph_common.h"

namespace sph {
namespace {

constexpr int kGravBlock = 256;
constexpr int kGravStack = 7 * kMaxLevel + 1;   // deepest depth-first stack

struct alignas(16) GNode {
    double M, cx, cy, cz;
    double q11, q12, q13, q22, q23, q33;
    int32_t s, e;   // slot range (s == e: empty)
};

struct GLevels {
    GNode* lev[kMaxLevel + 1];
    int L;
};

size_t level_offset(int l)
{
    size_t o = 0;
    for (int k = 0; k < l; ++k) o += size_t(1) << (3 * k);
    return o;
}

GLevels carve_gravity(void* gws, int L)
{
    GLevels G{};
    G.L = L;
    for (int l = 0; l <= L; ++l) G.lev[l] = (GNode*)gws + level_offset(l);
    return G;
}

__global__ __launch_bounds__(kBlock) void k_gleaf_clear(GNode* __restrict__ leaf, int64_t nl)
{
    const int64_t c = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (c < nl) {
        leaf[c].s = 0;
        leaf[c].e = 0;
    }
}

// slot ranges of the leaves from the sorted keys
__global__ __launch_bounds__(kBlock) void k_gleaf_ranges(const uint64_t* __restrict__ keys,
                                                         int64_t n, int shift,
                                                         GNode* __restrict__ leaf)
{
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= n) return;
    const uint64_t c = keys[i] >> shift;
    if (i == 0 || (keys[i - 1] >> shift) != c) leaf[c].s = (int32_t)i;
    if (i == n - 1 || (keys[i + 1] >> shift) != c) leaf[c].e = (int32_t)(i + 1);
}

// leaf moments from their particles: M, the centre of mass, then the traceless
// quadrupole sum m (3 d d^T - |d|^2 I) about it
__global__ __launch_bounds__(kBlock) void k_gleaf_moments(const double* __restrict__ x,
                                                          const double* __restrict__ y,
                                                          const double* __restrict__ z,
                                                          const double* __restrict__ m,
                                                          GNode* __restrict__ leaf, int64_t nl)
{
    const int64_t c = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (c >= nl) return;
    GNode nd = leaf[c];
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    for (int32_t b = nd.s; b < nd.e; ++b) {
        M += m[b];
        sx += m[b] * x[b];
        sy += m[b] * y[b];
        sz += m[b] * z[b];
    }
    double cx = 0.0, cy = 0.0, cz = 0.0;
    if (M > 0.0) {
        cx = sx / M;
        cy = sy / M;
        cz = sz / M;
    }
    double q11 = 0, q12 = 0, q13 = 0, q22 = 0, q23 = 0, q33 = 0;
    for (int32_t b = nd.s; b < nd.e; ++b) {
        const double dx = x[b] - cx, dy = y[b] - cy, dz = z[b] - cz;
        const double d2 = dx * dx + dy * dy + dz * dz;
        q11 += m[b] * (3.0 * dx * dx - d2);
        q12 += m[b] * (3.0 * dx * dy);
        q13 += m[b] * (3.0 * dx * dz);
        q22 += m[b] * (3.0 * dy * dy - d2);
        q23 += m[b] * (3.0 * dy * dz);
        q33 += m[b] * (3.0 * dz * dz - d2);
    }
    nd.M = M;
    nd.cx = cx; nd.cy = cy; nd.cz = cz;
    nd.q11 = q11; nd.q12 = q12; nd.q13 = q13; nd.q22 = q22; nd.q23 = q23; nd.q33 = q33;
    leaf[c] = nd;
}

// a parent from its eight children: masses add, the centre of mass is their
// mass-weighted mean, and each child's quadrupole moves to the parent's centre
// by adding M_c (3 d d^T - |d|^2 I), d = c_child - c_parent
__global__ __launch_bounds__(kBlock) void k_gnode_up(const GNode* __restrict__ child,
                                                     GNode* __restrict__ node, int64_t nn)
{
    const int64_t c = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (c >= nn) return;
    const GNode* ch = child + 8 * c;
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    int32_t s = 0, e = 0;
    bool any = false;
    for (int k = 0; k < 8; ++k) {
        const GNode q = ch[k];
        if (q.e <= q.s) continue;
        if (!any) s = q.s;
        e = q.e;
        any = true;
        M += q.M;
        sx += q.M * q.cx;
        sy += q.M * q.cy;
        sz += q.M * q.cz;
    }
    GNode nd{};
    nd.s = s;
    nd.e = e;
    if (any && M > 0.0) {
        nd.M = M;
        nd.cx = sx / M;
        nd.cy = sy / M;
        nd.cz = sz / M;
        for (int k = 0; k < 8; ++k) {
            const GNode q = ch[k];
            if (q.e <= q.s) continue;
            const double dx = q.cx - nd.cx, dy = q.cy - nd.cy, dz = q.cz - nd.cz;
            const double d2 = dx * dx + dy * dy + dz * dz;
            nd.q11 += q.q11 + q.M * (3.0 * dx * dx - d2);
            nd.q12 += q.q12 + q.M * (3.0 * dx * dy);
            nd.q13 += q.q13 + q.M * (3.0 * dx * dz);
            nd.q22 += q.q22 + q.M * (3.0 * dy * dy - d2);
            nd.q23 += q.q23 + q.M * (3.0 * dy * dz);
            nd.q33 += q.q33 + q.M * (3.0 * dz * dz - d2);
        }
    }
    node[c] = nd;
}

struct GravOut {
    double *gx, *gy, *gz;
};

// The walk.  Each lane takes one target, and the 64 lanes of a wavefront walk
// the tree together: a node is loaded once for the wavefront (its address is
// uniform), every lane still live at it applies its own opening test, the
// lanes that accept it add its expansion, and the node is opened for the lanes
// that do not (children pushed with that lane set).  A lane's terms are thus
// the nodes and particles its own depth-first walk would visit, in the same
// order: the result is that of one walk per target, bit for bit, while the
// traversal and its loads are shared.  The stack (level << 27 | index, and the
// 64-bit set of lanes still live below the entry) is uniform and lives in LDS.
__global__ __launch_bounds__(kGravBlock) void k_gravity(GLevels T, const Domain* __restrict__ dom,
                                                        const uint64_t* __restrict__ keys,
                                                        const double* __restrict__ x,
                                                        const double* __restrict__ y,
                                                        const double* __restrict__ z,
                                                        const double* __restrict__ m, int64_t n,
                                                        double G, double eps, double theta,
                                                        GravOut O)
{
    constexpr int kWaves = kGravBlock / 64;
    __shared__ uint32_t st_node[kWaves][kGravStack];
    __shared__ uint64_t st_live[kWaves][kGravStack];
    const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
    const int64_t a0 = blockIdx.x * (int64_t)kGravBlock + threadIdx.x;
    const bool live0 = a0 < n;
    const int64_t a = live0 ? a0 : n - 1;   // lanes past the end shadow the last target
    const double xa = x[a], ya = y[a], za = z[a];
    const uint64_t ka = keys[a];
    double ext = 0.0;
    for (int k = 0; k < 3; ++k) ext = fmax(ext, dom->hi[k] - dom->lo[k]);
    const double eps2 = eps * eps, th2 = theta * theta;
    double gx = 0.0, gy = 0.0, gz = 0.0;
    int sp = 0;
    const uint64_t all = __ballot(live0);
    if (lane == 0) {
        st_node[wv][0] = 0u;   // the root
        st_live[wv][0] = all;
    }
    sp = 1;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    while (sp > 0) {
        --sp;
        // (the builtin reads and returns int: each half goes back through
        // uint32_t, so that the low half is not sign-extended)
        const uint32_t top = (uint32_t)__builtin_amdgcn_readfirstlane((int)st_node[wv][sp]);
        const uint64_t lv = st_live[wv][sp];
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(lv >> 32));
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)lv);
        const uint64_t lmask = ((uint64_t)hi << 32) | (uint64_t)lo;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int l = (int)(top >> 27);
        const uint32_t idx = top & ((1u << 27) - 1u);
        const GNode nd = T.lev[l][idx];
        if (nd.e <= nd.s) continue;
        const bool mine = (lmask >> lane) & 1u;
        const bool own = (ka >> (3 * (kKeyBits - l))) == (uint64_t)idx;
        bool open = mine;
        if (mine && !own) {
            const double dx = xa - nd.cx, dy = ya - nd.cy, dz = za - nd.cz;
            const double d2 = dx * dx + dy * dy + dz * dz;
            const double sz = ext / (double)(1 << l);
            if (sz * sz < th2 * d2) {
                // the expansion with rho^2 = |r|^2 + eps^2, r = x_a - c
                const double r2 = d2 + eps2;
                const double ir = 1.0 / sqrt(r2);
                const double ir2 = ir * ir;
                const double ir3 = ir * ir2, ir5 = ir3 * ir2, ir7 = ir5 * ir2;
                const double Qx = nd.q11 * dx + nd.q12 * dy + nd.q13 * dz;
                const double Qy = nd.q12 * dx + nd.q22 * dy + nd.q23 * dz;
                const double Qz = nd.q13 * dx + nd.q23 * dy + nd.q33 * dz;
                const double rQr = dx * Qx + dy * Qy + dz * Qz;
                gx += -G * nd.M * dx * ir3 + G * (Qx * ir5 - 2.5 * rQr * dx * ir7);
                gy += -G * nd.M * dy * ir3 + G * (Qy * ir5 - 2.5 * rQr * dy * ir7);
                gz += -G * nd.M * dz * ir3 + G * (Qz * ir5 - 2.5 * rQr * dz * ir7);
                open = false;
            }
        }
        const uint64_t omask = __ballot(open);
        if (omask == 0) continue;
        if (l == T.L) {
            // an opened leaf: its particles directly, in slot order (four
            // particles' loads issued together)
            auto direct = [&](int32_t b, double xb, double yb, double zb, double mb) {
                if (!open || b == (int32_t)a) return;
                const double dx = xa - xb, dy = ya - yb, dz = za - zb;
                const double r2 = dx * dx + dy * dy + dz * dz + eps2;
                const double f = G * mb / (r2 * sqrt(r2));
                gx -= f * dx;
                gy -= f * dy;
                gz -= f * dz;
            };
            int32_t b = nd.s;
            for (; b + 4 <= nd.e; b += 4) {
                double xb[4], yb[4], zb[4], mb[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    xb[u] = x[b + u];
                    yb[u] = y[b + u];
                    zb[u] = z[b + u];
                    mb[u] = m[b + u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) direct(b + u, xb[u], yb[u], zb[u], mb[u]);
            }
            for (; b < nd.e; ++b) direct(b, x[b], y[b], z[b], m[b]);
            continue;
        }
        // children, last first, so that the walk visits them in ascending prefix
        const uint32_t base = (uint32_t)(l + 1) << 27;
        if (lane == 0) {
            for (int k = 7; k >= 0; --k) {
                st_node[wv][sp + 7 - k] = base | (idx * 8u + (uint32_t)k);
                st_live[wv][sp + 7 - k] = omask;
            }
        }
        sp += 8;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    if (!live0) return;
    O.gx[a] = gx;
    O.gy[a] = gy;
    O.gz[a] = gz;
}

}  // namespace

size_t gravity_workspace_bytes(int L) { return level_offset(L + 1) * sizeof(GNode); }

hipError_t launch_gravity(const Params& P, const Ws& W, const sph_particles* p, void* gws,
                          double G, double eps, double theta, double* gx, double* gy,
                          double* gz, hipStream_t s)
{
    const int L = P.lcap;
    GLevels T = carve_gravity(gws, L);
    const int64_t n = P.n;
    const int64_t nl = int64_t(1) << (3 * L);
    k_gleaf_clear<<<(nl + kBlock - 1) / kBlock, kBlock, 0, s>>>(T.lev[L], nl);
    k_gleaf_ranges<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(W.keys0, n, 3 * (kKeyBits - L),
                                                                T.lev[L]);
    k_gleaf_moments<<<(nl + kBlock - 1) / kBlock, kBlock, 0, s>>>(p->x, p->y, p->z, p->m,
                                                                  T.lev[L], nl);
    for (int l = L - 1; l >= 0; --l) {
        const int64_t nn = int64_t(1) << (3 * l);
        k_gnode_up<<<(nn + kBlock - 1) / kBlock, kBlock, 0, s>>>(T.lev[l + 1], T.lev[l], nn);
    }
    GravOut O{gx, gy, gz};
    k_gravity<<<(n + kGravBlock - 1) / kGravBlock, kGravBlock, 0, s>>>(
        T, W.dom, W.keys0, p->x, p->y, p->z, p->m, n, G, eps, theta, O);
    return hipGetLastError();
}

}  // namespace sph
