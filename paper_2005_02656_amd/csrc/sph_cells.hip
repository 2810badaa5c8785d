// sph_cells.hip -- sph_build_cells: keep particles in the depth-first (Morton)
// order of the octree (section 4.3).
//
//   1. bounding box of the open axes and largest h (block reduction + one
//      order-preserving 64-bit atomic per block; min/max are exact and
//      order-free, so the result is deterministic);
//   2. domain record: key domain, 2^21 scale per axis, cell level;
//   3. 63-bit keys (21 bits per axis, x highest in each bit triplet) + iota;
//   4. stable LSD radix sort of (key, slot), 8 passes of 8 bits.  Per pass:
//      LDS tile histogram -> exclusive scan of the digit-major counts ->
//      stable LDS-local ranking (wave ballots) -> tile reordered in LDS and
//      written digit run by digit run (coalesced);
//   5. dense cell table (start/end per Morton cell at the chosen level);
//   6. every state array gathered through the permutation into workspace
//      scratch and copied back.
#include "sph_common.h"

namespace sph {
namespace {

constexpr int kSortItems = 16;                      // keys per thread per tile
constexpr int kSortTile = kBlock * kSortItems;      // 4096
constexpr int kWaves = kBlock / 64;
constexpr int kWaveItems = kSortTile / kWaves;      // 1024 consecutive keys per wave
constexpr int kRedGrid = 1024;                      // bbox reduction blocks
#ifndef SPH_CELL_FACTOR
#define SPH_CELL_FACTOR 0.5
#endif
// cell edge >= kCellFactor * hmax: cells smaller than the kernel reach, walked
// with a per-target stencil and per-cell distance culling
constexpr double kCellFactor = SPH_CELL_FACTOR;

__global__ void k_clear_domain(Domain* d)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        Domain z = {};
        *d = z;
    }
}

__global__ void k_domain_begin(Domain* d)
{
    for (int k = 0; k < 3; ++k) {
        d->ord_min[k] = ~0ull;
        d->ord_max[k] = 0ull;
    }
    d->ord_hmax = 0ull;
    d->mass_varies = 0u;
}

__device__ __forceinline__ double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__global__ __launch_bounds__(kBlock) void k_bbox(const double* __restrict__ x,
                                                 const double* __restrict__ y,
                                                 const double* __restrict__ z,
                                                 const double* __restrict__ h,
                                                 const double* __restrict__ m, int64_t n,
                                                 Domain* d)
{
    double mn[3] = {INFINITY, INFINITY, INFINITY};
    double mx[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
    // whether every mass equals slot 0's (the density sums then skip the
    // mass gather); the order of the slots does not matter
    const double m0 = m[0];
    bool mv = false;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        double px = x[i], py = y[i], pz = z[i], ph = h[i];
        mv |= m[i] != m0;
        mn[0] = fmin(mn[0], px); mx[0] = fmax(mx[0], px);
        mn[1] = fmin(mn[1], py); mx[1] = fmax(mx[1], py);
        mn[2] = fmin(mn[2], pz); mx[2] = fmax(mx[2], pz);
        mx[3] = fmax(mx[3], ph);
    }
    __shared__ double s[kWaves][7];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (__ballot(mv) && lane == 0) flag_or(&d->mass_varies, 1u);
    double r[7];
    for (int k = 0; k < 3; ++k) r[k] = wave_min(mn[k]);
    for (int k = 0; k < 4; ++k) r[3 + k] = wave_max(mx[k]);
    if (lane == 0)
        for (int k = 0; k < 7; ++k) s[w][k] = r[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int ww = 1; ww < kWaves; ++ww) {
            for (int k = 0; k < 3; ++k) r[k] = fmin(r[k], s[ww][k]);
            for (int k = 3; k < 7; ++k) r[k] = fmax(r[k], s[ww][k]);
        }
        for (int k = 0; k < 3; ++k) {
            atomicMin((unsigned long long*)&d->ord_min[k], (unsigned long long)ord_bits(r[k]));
            atomicMax((unsigned long long*)&d->ord_max[k], (unsigned long long)ord_bits(r[3 + k]));
        }
        atomicMax((unsigned long long*)&d->ord_hmax, (unsigned long long)ord_bits(r[6]));
    }
}

__global__ void k_domain_end(Params P, Domain* d)
{
    double hm = ord_value(d->ord_hmax);
    if (!(hm > 0.0)) hm = 0.0;
    double D[3], ext = 0.0;
    for (int k = 0; k < 3; ++k) {
        double lo = P.periodic[k] ? P.box_lo[k] : ord_value(d->ord_min[k]);
        double hi = P.periodic[k] ? P.box_hi[k] : ord_value(d->ord_max[k]);
        d->lo[k] = lo;
        d->hi[k] = hi;
        D[k] = hi - lo;
        d->scale[k] = (D[k] > 0.0) ? 2097152.0 / D[k] : 0.0;
        ext = fmax(ext, D[k]);
    }
    d->walk_slack = (float)(ext * 0x1p-20);
    int level = 0;
    for (int l = P.lcap; l >= 0; --l) {
        bool ok = true;
        for (int k = 0; k < 3; ++k)
            if (D[k] > 0.0 && D[k] / (double)(1 << l) < kCellFactor * hm) ok = false;
        if (ok) { level = l; break; }
    }
    d->level = level;
    d->shift = 3 * (kKeyBits - level);
    d->ncell_axis = 1 << level;
    for (int k = 0; k < 3; ++k) d->cell[k] = (D[k] > 0.0) ? D[k] / (double)(1 << level) : 0.0;
    d->hmax = hm;
    d->built_n = P.n;
}

__global__ __launch_bounds__(kBlock) void k_keys(const double* __restrict__ x,
                                                 const double* __restrict__ y,
                                                 const double* __restrict__ z, int64_t n,
                                                 const Domain* __restrict__ d,
                                                 uint64_t* __restrict__ keys,
                                                 uint32_t* __restrict__ idx)
{
    int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= n) return;
    uint32_t qx = quantize(x[i], d->lo[0], d->scale[0]);
    uint32_t qy = quantize(y[i], d->lo[1], d->scale[1]);
    uint32_t qz = quantize(z[i], d->lo[2], d->scale[2]);
    keys[i] = morton3(qx, qy, qz);
    idx[i] = (uint32_t)i;
}

// ------------------------------------------------------------------ radix sort
__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint64_t* __restrict__ keys,
                                                       int64_t n, int shift,
                                                       uint32_t* __restrict__ hist, int64_t nb)
{
    __shared__ uint32_t hh[256];
    hh[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = blockIdx.x * (int64_t)kSortTile;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        int64_t g = base + i * kBlock + threadIdx.x;
        if (g < n) atomicAdd(&hh[(uint32_t)(keys[g] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = hh[threadIdx.x];
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// exclusive scan over the block (kBlock threads); lds needs kWaves+1 entries
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lds, uint32_t& total)
{
    uint32_t inc = wave_incl_scan(v);
    int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int i = 0; i < kWaves; ++i) {
            uint32_t t = lds[i];
            lds[i] = acc;
            acc += t;
        }
        lds[kWaves] = acc;
    }
    __syncthreads();
    uint32_t r = lds[w] + inc - v;
    total = lds[kWaves];
    __syncthreads();
    return r;
}

// sums of consecutive chunks of kSortTile entries
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* __restrict__ a,
                                                        int64_t len, uint32_t* __restrict__ part)
{
    __shared__ uint32_t lds[kWaves + 1];
    int64_t base = blockIdx.x * (int64_t)kSortTile + threadIdx.x * kSortItems;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i)
        if (base + i < len) s += a[base + i];
    uint32_t total;
    block_excl_scan(s, lds, total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// exclusive scan of the chunk sums, one block, chunks of kBlock with a carry
__global__ __launch_bounds__(kBlock) void k_scan_top(uint32_t* part, int64_t np)
{
    __shared__ uint32_t lds[kWaves + 1];
    uint32_t carry = 0;
    for (int64_t base = 0; base < np; base += kBlock) {
        int64_t i = base + threadIdx.x;
        uint32_t v = i < np ? part[i] : 0u;
        uint32_t total;
        uint32_t ex = block_excl_scan(v, lds, total);
        if (i < np) part[i] = carry + ex;
        carry += total;
    }
}

// exclusive scan of each chunk, offset by the chunk's prefix, in place
__global__ __launch_bounds__(kBlock) void k_scan_down(uint32_t* __restrict__ a, int64_t len,
                                                      const uint32_t* __restrict__ part)
{
    __shared__ uint32_t lds[kWaves + 1];
    int64_t base = blockIdx.x * (int64_t)kSortTile + threadIdx.x * kSortItems;
    uint32_t v[kSortItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        v[i] = (base + i < len) ? a[base + i] : 0u;
        s += v[i];
    }
    uint32_t total;
    uint32_t ex = block_excl_scan(s, lds, total) + part[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        if (base + i < len) a[base + i] = ex;
        ex += v[i];
    }
}

// stable scatter of one tile by the digit at `shift`
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ iin,
    uint64_t* __restrict__ kout, uint32_t* __restrict__ iout, int64_t n, int shift,
    const uint32_t* __restrict__ offs, int64_t nb)
{
    __shared__ uint32_t wcount[kWaves][256];   // running digit counts per wave
    __shared__ uint32_t bstart[256];           // digit start in the reordered tile
    __shared__ uint32_t gofs[256];             // global start of the digit for this tile
    __shared__ uint32_t lds[kWaves + 1];
    __shared__ uint64_t skey[kSortTile];
    __shared__ uint32_t sidx[kSortTile];

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int ww = 0; ww < kWaves; ++ww) wcount[ww][t] = 0;
    gofs[t] = offs[(int64_t)t * nb + blockIdx.x];
    __syncthreads();

    const int64_t tile = blockIdx.x * (int64_t)kSortTile;
    const int64_t base = tile + (int64_t)w * kWaveItems;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t k[kSortItems];
    uint32_t v[kSortItems], r[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        int64_t g = base + (int64_t)i * 64 + lane;
        bool ok = g < n;
        uint64_t key = ok ? kin[g] : 0ull;
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t rank = __popcll(peers & below);
        uint32_t before = wcount[w][d];
        // lanes of one wavefront run in lockstep: every peer has read `before`
        // when the lowest peer stores the advanced count
        if (ok && (peers & below) == 0) wcount[w][d] = before + (uint32_t)__popcll(peers);
        k[i] = key;
        v[i] = ok ? iin[g] : 0u;
        r[i] = ok ? before + rank : 0xffffffffu;
    }
    __syncthreads();
    {
        uint32_t c[kWaves], tot = 0;
        for (int ww = 0; ww < kWaves; ++ww) {
            c[ww] = wcount[ww][t];
            wcount[ww][t] = tot;
            tot += c[ww];
        }
        uint32_t total;
        bstart[t] = block_excl_scan(tot, lds, total);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        if (r[i] != 0xffffffffu) {
            uint32_t d = (uint32_t)(k[i] >> shift) & 255u;
            uint32_t pos = bstart[d] + wcount[w][d] + r[i];
            skey[pos] = k[i];
            sidx[pos] = v[i];
        }
    }
    __syncthreads();
    int64_t rem = n - tile;
    int cnt = rem < kSortTile ? (int)rem : kSortTile;
    for (int p = t; p < cnt; p += kBlock) {
        uint64_t key = skey[p];
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        int64_t dst = (int64_t)gofs[d] + (p - (int64_t)bstart[d]);
        kout[dst] = key;
        iout[dst] = sidx[p];
    }
}

// ------------------------------------------------------------------ cell table
__global__ __launch_bounds__(kBlock) void k_cells_clear(const Domain* __restrict__ d,
                                                        CellRange* __restrict__ cells,
                                                        int64_t cap)
{
    int64_t c = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    int64_t ncell = int64_t(1) << (3 * d->level);
    if (c < ncell && c < cap) cells[c] = CellRange{0, 0};
}

__global__ __launch_bounds__(kBlock) void k_cells_fill(const Domain* __restrict__ d,
                                                       const uint64_t* __restrict__ keys,
                                                       int64_t n,
                                                       CellRange* __restrict__ cells)
{
    int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= n) return;
    int sh = d->shift;
    uint64_t c = (sh >= 64) ? 0ull : (keys[i] >> sh);
    uint64_t cp = (i > 0) ? ((sh >= 64) ? 0ull : (keys[i - 1] >> sh)) : ~0ull;
    uint64_t cn = (i + 1 < n) ? ((sh >= 64) ? 0ull : (keys[i + 1] >> sh)) : ~0ull;
    if (cp != c) cells[c].s = (int32_t)i;
    if (cn != c) cells[c].e = (int32_t)(i + 1);
}

// ------------------------------------------------------------------ permutation
struct PermSet {
    uint64_t* f[kMaxPermFields];
    int nf;
};

__global__ __launch_bounds__(kBlock) void k_gather(PermSet S, const uint32_t* __restrict__ perm,
                                                   uint64_t* __restrict__ tmp, int64_t n)
{
    int64_t nb = (n + kBlock - 1) / kBlock;
    int64_t lb = xcd_block(nb);
    if (lb < 0) return;
    int64_t i = lb * kBlock + threadIdx.x;
    if (i >= n) return;
    uint32_t src = perm[i];
    for (int f = 0; f < S.nf; ++f) tmp[(int64_t)f * n + i] = S.f[f][src];
}

// smallest float >= v, for v > 0
__device__ __forceinline__ float float_up(double v)
{
    float f = (float)v;
    if ((double)f < v) f = __uint_as_float(__float_as_uint(f) + 1u);
    return f;
}

// copy back, and pack positions and h (fields 0, 1, 2 and 9 of the set); with
// pf, also the FP32 walk records of the fused candidate pass
__global__ __launch_bounds__(kBlock) void k_scatter_back(PermSet S,
                                                         const uint64_t* __restrict__ tmp,
                                                         int64_t n, const Domain* __restrict__ dom,
                                                         Pos4* __restrict__ p4,
                                                         Pos4f* __restrict__ pf, float k2s)
{
    int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= n) return;
    for (int f = 0; f < S.nf; ++f) S.f[f][i] = tmp[(int64_t)f * n + i];
    Pos4 q;
    q.x = __builtin_bit_cast(double, tmp[i]);
    q.y = __builtin_bit_cast(double, tmp[n + i]);
    q.z = __builtin_bit_cast(double, tmp[2 * n + i]);
    q.h = __builtin_bit_cast(double, tmp[9 * n + i]);
    p4[i] = q;
    if (pf) {
        const float R = fmaf(k2s, float_up(q.h), dom->walk_slack);
        pf[i] = Pos4f{(float)(q.x - dom->lo[0]), (float)(q.y - dom->lo[1]),
                      (float)(q.z - dom->lo[2]), (R * R) * kWalkGrow};
    }
}

__global__ __launch_bounds__(kBlock) void k_pack_p4(const double* __restrict__ x,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ z,
                                                    const double* __restrict__ h, int64_t n,
                                                    Pos4* __restrict__ p4)
{
    int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= n) return;
    p4[i] = Pos4{x[i], y[i], z[i], h[i]};
}

}  // namespace

// The kernel tables (section 4.5): entry i holds the values at nodes i and
// i+1 of v_i = 2i/(N-1), from the same fitted polynomials as the direct
// evaluation; dS_n/dv = (v dS_n/dv) / v, 0 at v = 0 (S_n is even in v).
__global__ __launch_bounds__(kBlock) void k_fill_tables(Params P, double2* __restrict__ tS,
                                                        double2* __restrict__ tD,
                                                        float2* __restrict__ tSf,
                                                        float2* __restrict__ tDf)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= P.tab_n - 1) return;
    double S[2], D[2];
    for (int k = 0; k < 2; ++k) {
        const double v = (double)(i + k) / P.tab_inv_dv;
        double vdS;
        sinc_terms(kPiHalfSq * v * v, P.sinc_n, S[k], vdS);
        D[k] = v > 0.0 ? vdS / v : 0.0;
    }
    tS[i] = make_double2(S[0], S[1]);
    tD[i] = make_double2(D[0], D[1]);
    tSf[i] = make_float2((float)S[0], (float)S[1]);
    tDf[i] = make_float2((float)D[0], (float)D[1]);
}

__global__ __launch_bounds__(kBlock) void k_copy_sorted(const uint64_t* __restrict__ kin,
                                                        const uint32_t* __restrict__ iin,
                                                        uint64_t* __restrict__ kout,
                                                        uint32_t* __restrict__ iout, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i < n) {
        kout[i] = kin[i];
        iout[i] = iin[i];
    }
}

hipError_t launch_clear_domain(const Ws& W, hipStream_t s)
{
    k_clear_domain<<<1, 64, 0, s>>>(W.dom);
    return hipGetLastError();
}

hipError_t launch_build_cells(const Params& P, const Layout& L, const Ws& W,
                              const sph_particles* p, hipStream_t s)
{
    const int64_t n = P.n;
    const int64_t nb = (n + kBlock - 1) / kBlock;
    if (P.tab_n > 0)
        k_fill_tables<<<(P.tab_n + kBlock - 1) / kBlock, kBlock, 0, s>>>(P, W.tabS, W.tabD,
                                                                          W.tabSf, W.tabDf);
    k_domain_begin<<<1, 1, 0, s>>>(W.dom);
    int64_t rg = nb < kRedGrid ? nb : kRedGrid;
    k_bbox<<<rg, kBlock, 0, s>>>(p->x, p->y, p->z, p->h, p->m, n, W.dom);
    k_domain_end<<<1, 1, 0, s>>>(P, W.dom);
    k_keys<<<nb, kBlock, 0, s>>>(p->x, p->y, p->z, n, W.dom, W.keys0, W.idx0);

    // Stable LSD radix sort by the key's prefix of lcap levels (3 lcap bits, 8
    // bits a pass): the depth-first order of the octree down to its finest
    // cells (section 4.3), every cell level the step uses being at most lcap.
    // Inside a finest cell the particles keep the order they came in, so the
    // order is updated, not rebuilt: only particles that changed cells move.
    const int s0 = 3 * (kKeyBits - L.lcap);
    const int passes = (3 * L.lcap + 7) / 8;
    uint64_t* kin = W.keys0;
    uint64_t* kout = W.keys1;
    uint32_t* iin = W.idx0;
    uint32_t* iout = W.idx1;
    for (int pass = 0; pass < passes; ++pass) {
        int shift = s0 + 8 * pass;
        k_radix_hist<<<L.nsort_blocks, kBlock, 0, s>>>(kin, n, shift, W.hist, L.nsort_blocks);
        k_scan_reduce<<<L.scan_blocks, kBlock, 0, s>>>(W.hist, L.hist_len, W.scanpart);
        k_scan_top<<<1, kBlock, 0, s>>>(W.scanpart, L.scan_blocks);
        k_scan_down<<<L.scan_blocks, kBlock, 0, s>>>(W.hist, L.hist_len, W.scanpart);
        k_radix_scatter<<<L.nsort_blocks, kBlock, 0, s>>>(kin, iin, kout, iout, n, shift, W.hist,
                                                         L.nsort_blocks);
        uint64_t* tk = kin; kin = kout; kout = tk;
        uint32_t* ti = iin; iin = iout; iout = ti;
    }
    // the sorted keys and order end in keys0/idx0
    if (kin != W.keys0) k_copy_sorted<<<nb, kBlock, 0, s>>>(kin, iin, W.keys0, W.idx0, n);

    int64_t cb = (L.ncells_cap + kBlock - 1) / kBlock;
    k_cells_clear<<<cb, kBlock, 0, s>>>(W.dom, W.cells, L.ncells_cap);
    k_cells_fill<<<nb, kBlock, 0, s>>>(W.dom, W.keys0, n, W.cells);

    PermSet S{};
    uint64_t* fields[] = {(uint64_t*)p->x, (uint64_t*)p->y, (uint64_t*)p->z,
                          (uint64_t*)p->vx, (uint64_t*)p->vy, (uint64_t*)p->vz,
                          (uint64_t*)p->vhx, (uint64_t*)p->vhy, (uint64_t*)p->vhz,
                          (uint64_t*)p->h, (uint64_t*)p->m, (uint64_t*)p->u,
                          (uint64_t*)p->du_m1, (uint64_t*)p->id,
                          (uint64_t*)p->p_ref, (uint64_t*)p->rho_ref};
    for (uint64_t* f : fields)
        if (f) S.f[S.nf++] = f;
    k_gather<<<grid_xcd(nb), kBlock, 0, s>>>(S, W.idx0, (uint64_t*)W.tmp, n);
    k_scatter_back<<<nb, kBlock, 0, s>>>(S, (const uint64_t*)W.tmp, n, W.dom, W.p4,
                                         P.cand_cap > 0 ? W.pf : nullptr,
                                         short_reach_f32(P.kappa));
    return hipGetLastError();
}

hipError_t launch_pack_p4(const Params& P, const Ws& W, const sph_particles* p, hipStream_t s)
{
    const int64_t nb = (P.n + kBlock - 1) / kBlock;
    k_pack_p4<<<nb, kBlock, 0, s>>>(p->x, p->y, p->z, p->h, P.n, W.p4);
    return hipGetLastError();
}

}  // namespace sph
