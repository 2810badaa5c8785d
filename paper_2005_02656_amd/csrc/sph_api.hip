// sph_api.hip -- the C ABI of libsph: argument validation, workspace carve-up and
// launch sequencing on the caller's stream.  No allocation; the only global
// state is the fixed device scratch of sph_step_static and its per-device
// address.
#include <math.h>
#include <string.h>

#include <mutex>

#include <new>

#include "sph_common.h"

namespace sph {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(int64_t n, int ng_max)
{
    Layout L{};
    L.n = n;
    // largest level whose dense table has no more cells than particles
    int lcap = 0;
    while (lcap < kMaxLevel && (int64_t(1) << (3 * (lcap + 1))) <= (n > 1 ? n : 1)) ++lcap;
    L.lcap = lcap;
    L.ncells_cap = int64_t(1) << (3 * lcap);
    L.nsort_blocks = (n + 4095) / 4096;
    L.hist_len = 256 * L.nsort_blocks;
    L.scan_blocks = (L.hist_len + 4095) / 4096;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    L.domain = take(sizeof(Domain));
    L.sums = take(sizeof(double) * kSumBlocks * 10);
    L.keys0 = take(sizeof(uint64_t) * n);
    L.keys1 = take(sizeof(uint64_t) * n);
    L.idx0 = take(sizeof(uint32_t) * n);
    L.idx1 = take(sizeof(uint32_t) * n);
    L.hist = take(sizeof(uint32_t) * L.hist_len);
    L.scanpart = take(sizeof(uint32_t) * (L.scan_blocks + 1));
    L.cells = take(sizeof(CellRange) * L.ncells_cap);
    L.nc = take(sizeof(int32_t) * n);
    L.ns = take(sizeof(int32_t) * n);
    L.nk = take(sizeof(int32_t) * n);
    // the cell walk loads whole batches past the end of a cell: both record
    // arrays the walks read have kWalkPad spare entries after the last slot
    L.p4 = take(sizeof(Pos4) * (n + kWalkPad));
    L.pf = take(sizeof(Pos4f) * (n + kWalkPad));
    L.rec = take(sizeof(MomRec) * n);
    L.vol = take(sizeof(double) * n);
    L.pv = take(sizeof(PosV) * n);
    const size_t padded = (size_t)((n + 63) / 64) * 64;   // lists are tiled by 64 slots
    size_t lst = sizeof(int32_t) * (size_t)ng_max * padded;
    size_t tmp = sizeof(double) * kMaxPermFields * n;
    L.list = take(lst > tmp ? lst : tmp);
    L.cand_cap = candidate_capacity(ng_max);
    L.cand = take(sizeof(int32_t) * (size_t)L.cand_cap * padded);
    L.posm = take(mixed_posm_bytes() * n);
    // kernel tables, sized for the largest kernel_table whatever the config
    L.tabS = take(sizeof(double2) * SPH_KERNEL_TABLE_MAX);
    L.tabD = take(sizeof(double2) * SPH_KERNEL_TABLE_MAX);
    L.tabSf = take(sizeof(float2) * SPH_KERNEL_TABLE_MAX);
    L.tabDf = take(sizeof(float2) * SPH_KERNEL_TABLE_MAX);
    L.flag = take(sizeof(uint8_t) * n);
    // the walk's reach bounds: the block maxima of every level below the
    // finest (1 + 8 + ... + 8^(lcap-1)), then the bound of each block
    size_t levels = 0;
    for (int l = 0; l < lcap; ++l) levels += size_t(1) << (3 * l);
    L.reach = take(sizeof(double) * (levels + (size_t)L.ncells_cap));
    L.total = o;
    return L;
}

Ws carve(void* ws, const Layout& L)
{
    char* b = (char*)ws;
    Ws W;
    W.dom = (Domain*)(b + L.domain);
    W.sums = (double*)(b + L.sums);
    W.keys0 = (uint64_t*)(b + L.keys0);
    W.keys1 = (uint64_t*)(b + L.keys1);
    W.idx0 = (uint32_t*)(b + L.idx0);
    W.idx1 = (uint32_t*)(b + L.idx1);
    W.hist = (uint32_t*)(b + L.hist);
    W.scanpart = (uint32_t*)(b + L.scanpart);
    W.cells = (CellRange*)(b + L.cells);
    W.nc = (int32_t*)(b + L.nc);
    W.ns = (int32_t*)(b + L.ns);
    W.nk = (int32_t*)(b + L.nk);
    W.cand = (int32_t*)(b + L.cand);
    W.posm = (void*)(b + L.posm);
    W.recm = (void*)(b + L.rec);   // FP32 records use the first half of the FP64 record area
    W.p4 = (Pos4*)(b + L.p4);
    W.pf = (Pos4f*)(b + L.pf);
    W.rec = (MomRec*)(b + L.rec);
    W.vol = (double*)(b + L.vol);
    W.pv = (PosV*)(b + L.pv);
    W.list = (int32_t*)(b + L.list);
    W.tmp = (double*)(b + L.list);
    W.tabS = (double2*)(b + L.tabS);
    W.tabD = (double2*)(b + L.tabD);
    W.tabSf = (float2*)(b + L.tabSf);
    W.tabDf = (float2*)(b + L.tabDf);
    W.flag = (uint8_t*)(b + L.flag);
    W.reach = (double*)(b + L.reach);
    return W;
}

// B_n = 1 / (4 pi int_0^2 S_n(pi v/2) v^2 dv): composite Simpson on 2^13 and
// 2^14 panels combined by one Richardson step (error O(h^6), far below 1e-16
// relative), evaluated once per exponent when the library is loaded.
static double simpson_bn(int n, int panels)
{
    const double hstep = 2.0 / panels;
    double acc = 0.0;
    for (int i = 0; i <= panels; ++i) {
        double v = i * hstep;
        double x = 0.5 * kPi * v;
        double s = (i == 0) ? 1.0 : sin(x) / x;
        double f = 1.0;
        for (int k = 0; k < n; ++k) f *= s;
        f *= v * v;
        double w = (i == 0 || i == panels) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
        acc += w * f;
    }
    return acc * hstep / 3.0;
}

namespace {
struct BnTable {
    double v[10];
    BnTable()
    {
        for (int n = 0; n < 10; ++n) {
            if (n < 3) { v[n] = 0.0; continue; }
            double coarse = simpson_bn(n, 1 << 13), fine = simpson_bn(n, 1 << 14);
            double integral = fine + (fine - coarse) / 15.0;
            v[n] = 1.0 / (4.0 * kPi * integral);
        }
    }
};
const BnTable kBn;  // constant after load
}  // namespace

double sinc_bn(int n) { return (n >= 3 && n <= 9) ? kBn.v[n] : 0.0; }

Params make_params(const sph_config* cfg, double bn, int lcap, int cand_cap)
{
    Params P{};
    P.n = cfg->n;
    for (int k = 0; k < 3; ++k) {
        P.box_lo[k] = cfg->box_lo[k];
        P.box_hi[k] = cfg->box_hi[k];
        P.L[k] = cfg->box_hi[k] - cfg->box_lo[k];
        P.halfL[k] = 0.5 * P.L[k];
        P.periodic[k] = cfg->periodic[k] ? 1 : 0;
        P.wrapLd[k] = P.periodic[k] ? P.L[k] : 0.0;
        P.wrapInvLd[k] = P.periodic[k] ? 1.0 / P.L[k] : 0.0;
        P.wrapL[k] = P.periodic[k] ? (float)P.L[k] : 0.0f;
        P.wrapInvL[k] = P.periodic[k] ? (float)(1.0 / P.L[k]) : 0.0f;
    }
    P.sinc_n = (int)cfg->sinc_n;
    P.bn = bn;
    P.n_target = cfg->n_target;
    P.ng_max = cfg->ng_max;
    P.newton_iters = cfg->newton_iters;
    P.kappa = cfg->h_ratio_max;
    P.eos = cfg->eos;
    P.gamma = cfg->gamma;
    P.c0 = cfg->c0;
    P.alpha = cfg->alpha_av;
    P.courant = cfg->courant;
    P.growth = cfg->dt_growth;
    P.acc_dt = cfg->acc_dt;
    P.energy_dt = cfg->energy_dt;
    P.lcap = lcap;
    P.cand_cap = cand_cap;
    P.precision = cfg->precision;
    P.tab_n = cfg->kernel_table;
    P.tab_inv_dv = cfg->kernel_table > 1 ? 0.5 * (double)(cfg->kernel_table - 1) : 0.0;
    return P;
}

}  // namespace sph

using namespace sph;

namespace {

bool config_ok(const sph_config* c)
{
    if (!c) return false;
    if (c->n < 1 || c->n > (int64_t(1) << 31) - 1) return false;
    if (c->ng_max < 1 || c->ng_max > 4096) return false;
    if (c->newton_iters < 0 || c->newton_iters > 64) return false;
    if (!(c->h_ratio_max > 1.0)) return false;
    if (c->sinc_n != floor(c->sinc_n) || c->sinc_n < 3 || c->sinc_n > 9) return false;
    if (c->eos != SPH_EOS_IDEAL && c->eos != SPH_EOS_WEAKLY_COMPRESSIBLE) return false;
    if (c->precision != SPH_FP64 && c->precision != SPH_MIXED) return false;
    if (c->kernel_table != 0 && (c->kernel_table < 2 || c->kernel_table > SPH_KERNEL_TABLE_MAX))
        return false;
    if (!(c->n_target > 0.0) || !(c->courant > 0.0) || !(c->dt_growth > 0.0)) return false;
    if (!(c->alpha_av >= 0.0)) return false;
    if (!(c->acc_dt >= 0.0) || !(c->energy_dt >= 0.0)) return false;
    if (c->eos == SPH_EOS_IDEAL && !(c->gamma > 1.0)) return false;
    if (c->eos == SPH_EOS_WEAKLY_COMPRESSIBLE && !(c->c0 > 0.0)) return false;
    for (int k = 0; k < 3; ++k) {
        if (c->periodic[k] != 0 && c->periodic[k] != 1) return false;
        if (c->periodic[k] && !(c->box_hi[k] > c->box_lo[k])) return false;
    }
    return true;
}

bool state_ok(const sph_config* c, const sph_particles* p)
{
    if (!p) return false;
    const void* req[] = {p->x, p->y, p->z, p->vx, p->vy, p->vz, p->vhx, p->vhy, p->vhz,
                         p->h, p->m, p->u, p->du_m1, p->id};
    for (const void* q : req)
        if (!q) return false;
    if (c->eos == SPH_EOS_WEAKLY_COMPRESSIBLE && (!p->p_ref || !p->rho_ref)) return false;
    return true;
}

struct Ctx {
    Params P;
    Layout L;
    Ws W;
    hipStream_t s;
};

sph_status prepare(const sph_config* cfg, void* ws, sph_stream stream, Ctx& c)
{
    if (!config_ok(cfg)) return SPH_E_ARG;
    if (!ws || ((uintptr_t)ws & 255)) return SPH_E_WORKSPACE;
    c.L = make_layout(cfg->n, cfg->ng_max);
    c.W = carve(ws, c.L);
    const bool fused = cfg->h_ratio_max <= kFusedKappaMax;
    c.P = make_params(cfg, sinc_bn((int)cfg->sinc_n), c.L.lcap, fused ? c.L.cand_cap : 0);
    c.P.tabS = c.W.tabS;
    c.P.tabD = c.W.tabD;
    c.P.tabSf = c.W.tabSf;
    c.P.tabDf = c.W.tabDf;
    c.s = (hipStream_t)stream;
    return SPH_OK;
}

sph_status hip_status(hipError_t e) { return e == hipSuccess ? SPH_OK : SPH_E_HIP; }

}  // namespace

extern "C" {

size_t sph_workspace_bytes(const sph_config* cfg)
{
    if (!config_ok(cfg)) return 0;
    return make_layout(cfg->n, cfg->ng_max).total;
}

sph_status sph_workspace_init(const sph_config* cfg, void* ws, sph_stream stream)
{
    Ctx c;
    sph_status st = prepare(cfg, ws, stream, c);
    if (st) return st;
    return hip_status(launch_clear_domain(c.W, c.s));
}

sph_status sph_build_cells(const sph_config* cfg, sph_particles* p, void* ws, sph_stream stream)
{
    Ctx c;
    sph_status st = prepare(cfg, ws, stream, c);
    if (st) return st;
    if (!state_ok(cfg, p)) return SPH_E_ARG;
    return hip_status(launch_build_cells(c.P, c.L, c.W, p, c.s));
}

sph_status sph_update_h(const sph_config* cfg, sph_particles* p, void* ws, sph_stream stream)
{
    Ctx c;
    sph_status st = prepare(cfg, ws, stream, c);
    if (st) return st;
    if (!p || !p->x || !p->y || !p->z || !p->h) return SPH_E_ARG;
    return hip_status(launch_update_h(c.P, c.L, c.W, p, c.s, true));
}

sph_status sph_find_neighbors(const sph_config* cfg, const sph_particles* p, void* ws,
                              sph_stream stream)
{
    Ctx c;
    sph_status st = prepare(cfg, ws, stream, c);
    if (st) return st;
    if (!p || !p->x || !p->y || !p->z || !p->h) return SPH_E_ARG;
    return hip_status(launch_find_neighbors(c.P, c.L, c.W, p, c.s));
}

sph_status sph_density(const sph_config* cfg, sph_particles* p, void* ws, sph_stream stream)
{
    Ctx c;
    sph_status st = prepare(cfg, ws, stream, c);
    if (st) return st;
    if (!p || !p->x || !p->y || !p->z || !p->h || !p->m || !p->u || !p->rho || !p->omega ||
        !p->p || !p->c)
        return SPH_E_ARG;
    if (cfg->eos == SPH_EOS_WEAKLY_COMPRESSIBLE && (!p->p_ref || !p->rho_ref)) return SPH_E_ARG;
    if (c.P.precision == SPH_MIXED)
        return hip_status(launch_density_mixed(c.P, c.L, c.W, p, c.s, true));
    return hip_status(launch_density(c.P, c.L, c.W, p, c.s, true));
}

sph_status sph_iad(const sph_config* cfg, sph_particles* p, void* ws, sph_stream stream)
{
    Ctx c;
    sph_status st = prepare(cfg, ws, stream, c);
    if (st) return st;
    if (!p || !p->x || !p->y || !p->z || !p->h || !p->m || !p->rho || !p->c11 || !p->c12 ||
        !p->c13 || !p->c22 || !p->c23 || !p->c33)
        return SPH_E_ARG;
    if (c.P.precision == SPH_MIXED)
        return hip_status(launch_iad_mixed(c.P, c.L, c.W, p, c.s, true, false));
    return hip_status(launch_iad(c.P, c.L, c.W, p, c.s, true, false));
}

sph_status sph_momentum_energy(const sph_config* cfg, sph_particles* p, void* ws,
                               sph_stream stream)
{
    Ctx c;
    sph_status st = prepare(cfg, ws, stream, c);
    if (st) return st;
    if (!p || !p->x || !p->y || !p->z || !p->vx || !p->vy || !p->vz || !p->h || !p->m ||
        !p->u || !p->rho || !p->omega || !p->p || !p->c || !p->c11 || !p->c12 || !p->c13 || !p->c22 ||
        !p->c23 || !p->c33 || !p->ax || !p->ay || !p->az || !p->du)
        return SPH_E_ARG;
    if (c.P.precision == SPH_MIXED)
        return hip_status(launch_momentum_energy_mixed(c.P, c.L, c.W, p, c.s, true));
    return hip_status(launch_momentum_energy(c.P, c.L, c.W, p, c.s, true));
}

sph_status sph_timestep(const sph_config* cfg, sph_globals* g, void* ws, sph_stream stream)
{
    Ctx c;
    sph_status st = prepare(cfg, ws, stream, c);
    if (st) return st;
    if (!g) return SPH_E_ARG;
    return hip_status(launch_timestep(c.P, c.W, g, c.s));
}

sph_status sph_integrate(const sph_config* cfg, sph_particles* p, sph_globals* g, void* ws,
                         sph_stream stream)
{
    Ctx c;
    sph_status st = prepare(cfg, ws, stream, c);
    if (st) return st;
    if (!g || !state_ok(cfg, p) || !p->ax || !p->ay || !p->az || !p->du) return SPH_E_ARG;
    return hip_status(launch_integrate(c.P, c.W, p, g, c.s));
}

}  // extern "C"

namespace {

bool step_args_ok(const sph_config* cfg, const sph_particles* p, const sph_globals* g)
{
    return g && state_ok(cfg, p) && p->rho && p->omega && p->p && p->c && p->c11 && p->c12 &&
           p->c13 && p->c22 && p->c23 && p->c33 && p->ax && p->ay && p->az && p->du;
}

// every stage of the step up to and including the time step (not the integration);
// mk marks the phases: 1 cell build, 2 candidates, 3 Newton h, 4 lists, 5 density,
// 6 IAD, 7 momentum/energy and time step (the walk-based path marks 2-4 after
// update_h, update_h and find_neighbors)
sph_status step_rates(Ctx& c, sph_particles* p, sph_globals* g, const Marks& mk = Marks())
{
    hipError_t e;
    if ((e = launch_build_cells(c.P, c.L, c.W, p, c.s))) return SPH_E_HIP;
    mk.at(1, c.s);
    // the cell build packs positions; with a small clamp ratio one cell walk
    // feeds both the Newton iterations and the lists (fused), else the walks of
    // the stage entry points run; the IAD pass writes the momentum records
    const bool fused = c.P.cand_cap > 0;
    if (fused) {
        // the fused launcher re-records event 1 after its cell h_max pass, so
        // that phase 2 holds the candidate walk alone; its list filter also
        // forms the density (FP64 in both precisions)
        Marks sub;
        if (mk.ev && mk.n > 1) sub = Marks{mk.ev + 1, mk.n - 1};
        if ((e = launch_fused_h_lists(c.P, c.L, c.W, p, c.s, sub, true))) return SPH_E_HIP;
    } else {
        if ((e = launch_update_h(c.P, c.L, c.W, p, c.s, false))) return SPH_E_HIP;
        mk.at(2, c.s);
        mk.at(3, c.s);
        if ((e = launch_find_neighbors(c.P, c.L, c.W, p, c.s))) return SPH_E_HIP;
    }
    mk.at(4, c.s);
    if (c.P.precision == SPH_MIXED) {
        if (fused) e = launch_pack_posm(c.P, c.W, p, c.s);
        else e = launch_density_mixed(c.P, c.L, c.W, p, c.s, true);
        if (e) return SPH_E_HIP;
        mk.at(5, c.s);
        if ((e = launch_iad_mixed(c.P, c.L, c.W, p, c.s, false, true))) return SPH_E_HIP;
        mk.at(6, c.s);
        if ((e = launch_momentum_energy_mixed(c.P, c.L, c.W, p, c.s, false))) return SPH_E_HIP;
    } else {
        if (!fused && (e = launch_density(c.P, c.L, c.W, p, c.s, false))) return SPH_E_HIP;
        mk.at(5, c.s);
        if ((e = launch_iad(c.P, c.L, c.W, p, c.s, false, true))) return SPH_E_HIP;
        mk.at(6, c.s);
        if ((e = launch_momentum_energy(c.P, c.L, c.W, p, c.s, false))) return SPH_E_HIP;
    }
    if ((e = launch_timestep(c.P, c.W, g, c.s))) return SPH_E_HIP;
    mk.at(7, c.s);
    return SPH_OK;
}

bool grads_ok(const sph_grads* q)
{
    if (!q) return false;
    const void* f[] = {q->x, q->y, q->z, q->vx, q->vy, q->vz, q->vhx, q->vhy, q->vhz, q->u,
                       q->du_m1};
    for (const void* v : f)
        if (!v) return false;
    return true;
}

}  // namespace

extern "C" {

sph_status sph_step(const sph_config* cfg, sph_particles* p, sph_globals* g, void* ws,
                    sph_stream stream)
{
    Ctx c;
    sph_status st = prepare(cfg, ws, stream, c);
    if (st) return st;
    if (!step_args_ok(cfg, p, g)) return SPH_E_ARG;
    if ((st = step_rates(c, p, g))) return st;
    return hip_status(launch_integrate(c.P, c.W, p, g, c.s));
}

sph_status sph_step_marked(const sph_config* cfg, sph_particles* p, sph_globals* g, void* ws,
                           sph_stream stream, void* const* events, int32_t nevents)
{
    Ctx c;
    sph_status st = prepare(cfg, ws, stream, c);
    if (st) return st;
    if (!step_args_ok(cfg, p, g) || !events || nevents != SPH_STEP_PHASES + 1) return SPH_E_ARG;
    for (int k = 0; k < nevents; ++k)
        if (!events[k]) return SPH_E_ARG;
    Marks mk{(hipEvent_t*)events, nevents};
    mk.at(0, c.s);
    if ((st = step_rates(c, p, g, mk))) return st;
    hipError_t e = launch_integrate(c.P, c.W, p, g, c.s);
    mk.at(8, c.s);
    return hip_status(e);
}

}  // extern "C"

// ---------------------------------------------------------------- step graphs
struct sph_step_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" {

sph_status sph_step_graph_create(const sph_config* cfg, sph_particles* p, sph_globals* g,
                                 void* ws, int32_t steps, sph_step_graph* graph)
{
    if (!graph) return SPH_E_ARG;
    *graph = nullptr;
    if (steps < 1 || steps > SPH_GRAPH_MAX_STEPS) return SPH_E_ARG;
    Ctx c;
    sph_status st = prepare(cfg, ws, nullptr, c);
    if (st) return st;
    if (!step_args_ok(cfg, p, g)) return SPH_E_ARG;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return SPH_E_HIP;
    c.s = cs;
    hipGraph_t gr = nullptr;
    st = SPH_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        st = SPH_E_HIP;
    } else {
        for (int32_t k = 0; k < steps && st == SPH_OK; ++k) {
            st = step_rates(c, p, g);
            if (st == SPH_OK) st = hip_status(launch_integrate(c.P, c.W, p, g, c.s));
        }
        // the capture is always ended, whatever the steps returned
        if (hipStreamEndCapture(cs, &gr) != hipSuccess && st == SPH_OK) st = SPH_E_HIP;
    }
    hipGraphExec_t ex = nullptr;
    if (st == SPH_OK && hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) != hipSuccess)
        st = SPH_E_HIP;
    (void)hipStreamDestroy(cs);
    sph_step_graph_s* h = nullptr;
    if (st == SPH_OK) {
        h = new (std::nothrow) sph_step_graph_s{gr, ex};
        if (!h) st = SPH_E_HIP;
    }
    if (st != SPH_OK) {
        if (ex) (void)hipGraphExecDestroy(ex);
        if (gr) (void)hipGraphDestroy(gr);
        return st;
    }
    *graph = h;
    return SPH_OK;
}

sph_status sph_step_graph_launch(sph_step_graph graph, sph_stream stream)
{
    if (!graph) return SPH_E_ARG;
    return hip_status(hipGraphLaunch(graph->exec, (hipStream_t)stream));
}

void sph_step_graph_destroy(sph_step_graph graph)
{
    if (!graph) return;
    (void)hipGraphExecDestroy(graph->exec);
    (void)hipGraphDestroy(graph->graph);
    delete graph;
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free step
// sph_step_static runs sph_step with its workspace in this fixed device array
// (each GPU the library runs on holds its own copy until the process ends).
// In host code `scratch` names a host-side stand-in, not device memory: every
// host use goes through the address hipGetSymbolAddress returns for the
// current device, taken once per device on the first call there.
namespace {

static_assert(SPH_STATIC_SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");
__device__ __align__(256) unsigned char scratch[SPH_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

// device address of this device's scratch, or nullptr
void* static_scratch()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::call_once(g_scratch_once[dev], [dev] {
        void* ptr = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = ptr;
    });
    return g_scratch_err[dev] == hipSuccess ? g_scratch_ptr[dev] : nullptr;
}

__global__ void k_copy_err(const Domain* __restrict__ dom, uint32_t* __restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = dom->err;
}

}  // namespace

extern "C" {

sph_status sph_step_static(const sph_config* cfg, sph_particles* p, sph_globals* g,
                           uint32_t* err_out, sph_stream stream)
{
    if (!config_ok(cfg)) return SPH_E_ARG;
    if (make_layout(cfg->n, cfg->ng_max).total > (size_t)SPH_STATIC_SCRATCH_BYTES)
        return SPH_E_WORKSPACE;
    if (!step_args_ok(cfg, p, g)) return SPH_E_ARG;
    void* ws = static_scratch();
    if (!ws) return SPH_E_HIP;
    Ctx c;
    sph_status st = prepare(cfg, ws, stream, c);
    if (st) return st;
    // the array keeps the last call's contents: the header record (error word,
    // flags, cached domain) starts from zero; everything else a step reads it
    // writes first
    if (launch_clear_domain(c.W, c.s) != hipSuccess) return SPH_E_HIP;
    if ((st = step_rates(c, p, g))) return st;
    if (launch_integrate(c.P, c.W, p, g, c.s) != hipSuccess) return SPH_E_HIP;
    if (err_out) k_copy_err<<<1, 64, 0, c.s>>>(c.W.dom, err_out);
    return hip_status(hipGetLastError());
}

size_t sph_adjoint_workspace_bytes(const sph_config* cfg)
{
    if (!config_ok(cfg)) return 0;
    return adjoint_workspace_bytes(cfg->n);
}

sph_status sph_step_backward(const sph_config* cfg, sph_particles* p, sph_globals* g, void* ws,
                             void* adj_ws, const sph_grads* gout, sph_grads* gin,
                             sph_stream stream)
{
    Ctx c;
    sph_status st = prepare(cfg, ws, stream, c);
    if (st) return st;
    if (cfg->precision != SPH_FP64 || cfg->kernel_table != 0) return SPH_E_ARG;
    if (!adj_ws || ((uintptr_t)adj_ws & 255)) return SPH_E_WORKSPACE;
    if (!step_args_ok(cfg, p, g) || !grads_ok(gout) || !grads_ok(gin)) return SPH_E_ARG;
    if ((st = step_rates(c, p, g))) return st;
    return hip_status(launch_step_backward(c.P, c.W, p, g, gout, gin, adj_ws, c.s));
}

sph_status sph_density_backward(const sph_config* cfg, const sph_particles* p, void* ws,
                                void* adj_ws, const double* rho_bar, double* x_bar,
                                double* y_bar, double* z_bar, sph_stream stream)
{
    Ctx c;
    sph_status st = prepare(cfg, ws, stream, c);
    if (st) return st;
    if (!adj_ws || ((uintptr_t)adj_ws & 255)) return SPH_E_WORKSPACE;
    if (cfg->kernel_table != 0) return SPH_E_ARG;
    if (!p || !p->m || !rho_bar || !x_bar || !y_bar || !z_bar) return SPH_E_ARG;
    return hip_status(launch_density_backward(c.P, c.W, p, rho_bar, x_bar, y_bar, z_bar, adj_ws,
                                              c.s));
}

size_t sph_gravity_workspace_bytes(const sph_config* cfg)
{
    if (!config_ok(cfg)) return 0;
    return gravity_workspace_bytes(make_layout(cfg->n, cfg->ng_max).lcap);
}

sph_status sph_gravity(const sph_config* cfg, const sph_particles* p,
                       const sph_gravity_params* gp, void* ws, void* gws, double* gx,
                       double* gy, double* gz, sph_stream stream)
{
    Ctx c;
    sph_status st = prepare(cfg, ws, stream, c);
    if (st) return st;
    if (!gws || ((uintptr_t)gws & 255)) return SPH_E_WORKSPACE;
    if (!p || !p->x || !p->y || !p->z || !p->m || !gx || !gy || !gz || !gp) return SPH_E_ARG;
    if (cfg->periodic[0] || cfg->periodic[1] || cfg->periodic[2]) return SPH_E_ARG;
    if (!(gp->G >= 0.0) || !(gp->eps >= 0.0) || !(gp->theta >= 0.0) || !isfinite(gp->G) ||
        !isfinite(gp->eps) || !isfinite(gp->theta))
        return SPH_E_ARG;
    return hip_status(launch_gravity(c.P, c.W, p, gws, gp->G, gp->eps, gp->theta, gx, gy, gz,
                                     c.s));
}

sph_status sph_neighbors_view(const sph_config* cfg, void* ws, const int32_t** nc,
                              const int32_t** ns, const int32_t** list, int32_t* capacity)
{
    if (!config_ok(cfg)) return SPH_E_ARG;
    if (!ws || ((uintptr_t)ws & 255)) return SPH_E_WORKSPACE;
    Layout L = make_layout(cfg->n, cfg->ng_max);
    Ws W = carve(ws, L);
    if (nc) *nc = W.nc;
    if (ns) *ns = W.ns;
    if (list) *list = W.list;
    if (capacity) *capacity = cfg->ng_max;
    return SPH_OK;
}

sph_status sph_candidates_view(const sph_config* cfg, void* ws, const int32_t** nk,
                               int32_t* capacity)
{
    if (!config_ok(cfg)) return SPH_E_ARG;
    if (!ws || ((uintptr_t)ws & 255)) return SPH_E_WORKSPACE;
    Layout L = make_layout(cfg->n, cfg->ng_max);
    Ws W = carve(ws, L);
    if (nk) *nk = W.nk;
    if (capacity) *capacity = L.cand_cap;
    return SPH_OK;
}

sph_status sph_order_view(const sph_config* cfg, void* ws, const uint64_t** keys,
                          const uint32_t** perm)
{
    if (!config_ok(cfg)) return SPH_E_ARG;
    if (!ws || ((uintptr_t)ws & 255)) return SPH_E_WORKSPACE;
    Layout L = make_layout(cfg->n, cfg->ng_max);
    Ws W = carve(ws, L);
    if (keys) *keys = W.keys0;
    if (perm) *perm = W.idx0;
    return SPH_OK;
}

sph_status sph_status_sync(void* ws, sph_stream stream, uint32_t* bits)
{
    if (!ws || ((uintptr_t)ws & 255)) return SPH_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Domain* dom = (Domain*)ws;  // the domain record sits at offset 0
    uint32_t word = 0;
    if (hipMemcpyAsync(&word, &dom->err, sizeof word, hipMemcpyDeviceToHost, s) != hipSuccess)
        return SPH_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return SPH_E_HIP;
    uint32_t zero = 0;
    if (hipMemcpyAsync(&dom->err, &zero, sizeof zero, hipMemcpyHostToDevice, s) != hipSuccess)
        return SPH_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return SPH_E_HIP;
    if (bits) *bits = word;
    if (word & SPH_ERRBIT_NONFINITE) return SPH_E_NONFINITE;
    if (word & SPH_ERRBIT_SINGULAR_TAU) return SPH_E_SINGULAR_TAU;
    if (word & SPH_ERRBIT_NEIGHBOR_OVERFLOW) return SPH_E_NEIGHBOR_OVERFLOW;
    if (word & SPH_ERRBIT_CELL_RANGE) return SPH_E_CELL_RANGE;
    return SPH_OK;
}

const char* sph_status_string(sph_status s)
{
    switch (s) {
    case SPH_OK: return "SPH_OK";
    case SPH_E_ARG: return "SPH_E_ARG: invalid argument";
    case SPH_E_HIP: return "SPH_E_HIP: HIP launch or query failed";
    case SPH_E_WORKSPACE: return "SPH_E_WORKSPACE: workspace NULL or not 256-byte aligned";
    case SPH_E_NEIGHBOR_OVERFLOW: return "SPH_E_NEIGHBOR_OVERFLOW: a neighbour count exceeded ng_max";
    case SPH_E_CELL_RANGE: return "SPH_E_CELL_RANGE: 4h reached the box length on a periodic axis";
    case SPH_E_NONFINITE: return "SPH_E_NONFINITE: non-finite density or rate";
    case SPH_E_SINGULAR_TAU: return "SPH_E_SINGULAR_TAU: IAD matrix not positive definite";
    }
    return "unknown sph_status";
}

}  // extern "C"
