/*
 * sph.h -- C ABI of libsph, an MI355X (gfx950) implementation of the smoothed
 * particle hydrodynamics time step of Cavelan, Cabezon, Grabarczyk and Ciorba,
 * "A Smoothed Particle Hydrodynamics Mini-App for Exascale" (arXiv 2005.02656).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers are DEVICE pointers unless a comment says (host).  Every array is
 *   caller-owned, length cfg->n, stride 1, FP64 unless stated (structure of
 *   arrays).  The library allocates nothing and frees nothing; all scratch
 *   lives in the caller's workspace `ws`, except for sph_step_static, whose
 *   scratch is a fixed device array of the library (the only global state),
 *   and the step graphs, whose HIP graph objects live from
 *   sph_step_graph_create to sph_step_graph_destroy.
 * - `stream` is a hipStream_t (NULL = the legacy default stream).  Every call
 *   only enqueues work on it and returns; results are ready when the stream is.
 *   Two workspaces may be used concurrently on two streams.
 * - Argument errors (NULL pointers, n <= 0, unknown enums, a periodic box that
 *   is not larger than the smoothing kernel's reach) are returned synchronously
 *   as SPH_E_ARG before anything is enqueued.  A failed HIP launch returns
 *   SPH_E_HIP.  Conditions found on the device (list overflow, non-finite
 *   values, singular IAD matrix, h beyond the minimum-image limit) set bits of
 *   a sticky error word in `ws`; read and clear it with sph_status_sync.
 *   Nothing aborts and nothing throws across this ABI.
 * - Particle order: sph_build_cells permutes every state array in place into
 *   the depth-first (Morton) order of section 4.3.  All later outputs are per
 *   slot of that order; `id` carries each slot's original particle number.
 *
 * The stage entry points must be called in step order on one workspace:
 *   build_cells -> update_h -> find_neighbors -> density -> iad ->
 *   momentum_energy -> timestep -> integrate
 * (sph_step does exactly that).  Each stage reads the arrays its comment names
 * as inputs, so a caller may overwrite an input field between stages (the
 * tests do, to feed identical inputs to an independent implementation).
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* sph_stream;  /* hipStream_t */

typedef enum {
    SPH_OK = 0,
    SPH_E_ARG = 1,               /* bad argument, detected on the host */
    SPH_E_HIP = 2,               /* a HIP launch or query failed */
    SPH_E_WORKSPACE = 3,         /* workspace NULL, misaligned or built for another n */
    SPH_E_NEIGHBOR_OVERFLOW = 4, /* a neighbour count exceeded ng_max (lists truncated) */
    SPH_E_CELL_RANGE = 5,        /* 4h >= box length on a periodic axis */
    SPH_E_NONFINITE = 6,         /* NaN/Inf in density or rates */
    SPH_E_SINGULAR_TAU = 7       /* det(tau) <= 0 in the IAD pass */
} sph_status;

/* bits of the device error word (sph_status_sync) */
#define SPH_ERRBIT_NEIGHBOR_OVERFLOW (1u << 0)
#define SPH_ERRBIT_CELL_RANGE (1u << 1)
#define SPH_ERRBIT_NONFINITE (1u << 2)
#define SPH_ERRBIT_SINGULAR_TAU (1u << 3)

typedef enum { SPH_FP64 = 0, SPH_MIXED = 1 } sph_precision;
typedef enum { SPH_EOS_IDEAL = 0, SPH_EOS_WEAKLY_COMPRESSIBLE = 1 } sph_eos;

/* (host) Plain-old-data run configuration, read at every call. */
typedef struct {
    int64_t n;              /* number of particles, >= 1 */
    double  box_lo[3];      /* box; used on periodic axes (open axes use the   */
    double  box_hi[3];      /*   particles' bounding box, recomputed per call) */
    int32_t periodic[3];    /* 1 = periodic axis, 0 = open */
    int32_t eos;            /* sph_eos */
    double  sinc_n;         /* exponent n of the sinc kernel S_n (eq. 6); integer 3..9 */
    double  n_target;       /* target effective neighbour number of the h update */
    int32_t ng_max;         /* neighbour-list capacity per particle, 1..4096 */
    int32_t newton_iters;   /* Newton iterations per sph_update_h call, 0..64 */
    double  h_ratio_max;    /* kappa: h stays in [h0/kappa, kappa*h0] per call, > 1 */
    double  gamma;          /* ideal-gas adiabatic index (EOS_IDEAL) */
    double  c0;             /* sound speed (EOS_WEAKLY_COMPRESSIBLE) */
    double  alpha_av;       /* artificial-viscosity alpha (eq. 5) */
    double  courant;        /* Courant criterion: courant * h/c */
    double  dt_growth;      /* dt <= dt_growth * previous dt */
    double  acc_dt;         /* acceleration criterion acc_dt * sqrt(h/|a|); 0 = off */
    double  energy_dt;      /* energy criterion energy_dt * |u|/|du|; 0 = off */
    int32_t precision;      /* sph_precision */
    int32_t kernel_table;   /* 0: S_n evaluated directly (fitted even polynomials in
                             *    v^2, FP64 to 1e-15); N in 2..SPH_KERNEL_TABLE_MAX:
                             *    S_n and dS_n/dv read from tables of N values at
                             *    v_i = 2i/(N-1) and interpolated linearly in v
                             *    (section 4.5 uses N = 20,000).  Applies to every
                             *    kernel evaluation of the forward step, in both
                             *    precisions; the reverse mode needs 0. */
} sph_config;

/* largest kernel_table; the tables live in the workspace, which always
 * reserves room for the largest (48 bytes per entry, 3 MiB) */
#define SPH_KERNEL_TABLE_MAX 65536

/* Particle arrays (device, caller-owned).  State arrays are permuted in place by
 * sph_build_cells; output arrays are written by the stage that names them. */
typedef struct {
    /* state: x^n, v^n (integer time), v^{n-1/2} (leapfrog half-step velocity) */
    double  *x, *y, *z;
    double  *vx, *vy, *vz;
    double  *vhx, *vhy, *vhz;
    double  *h;             /* smoothing length */
    double  *m;             /* mass */
    double  *u;             /* specific internal energy */
    double  *du_m1;         /* du/dt of the previous step (Adams-Bashforth) */
    double  *p_ref;         /* EOS_WEAKLY_COMPRESSIBLE only, else NULL */
    double  *rho_ref;       /* EOS_WEAKLY_COMPRESSIBLE only, else NULL */
    int64_t *id;            /* original particle number, permuted with the state */
    /* outputs */
    double  *rho, *omega, *p, *c;                 /* sph_density */
    double  *c11, *c12, *c13, *c22, *c23, *c33;   /* sph_iad: C = tau^-1 */
    double  *ax, *ay, *az, *du;                   /* sph_momentum_energy */
} sph_particles;

/* Global scalars (DEVICE memory, caller-owned, 14 doubles). */
typedef struct {
    double dt;       /* step being taken (written by sph_timestep) */
    double dt_m1;    /* previous step, 0 before the first step */
    double t;        /* simulated time */
    double mass, mom[3], ang[3], e_kin, e_int;   /* conservation sums after the step */
} sph_globals;

/* (host) Bytes of workspace needed for cfg (pure function of n and ng_max).
 * Returns 0 if cfg is invalid. */
size_t sph_workspace_bytes(const sph_config* cfg);

/* Clears the workspace header (error word, cached domain).  Call once after
 * allocating ws; a zero-filled ws is already initialised. */
sph_status sph_workspace_init(const sph_config* cfg, void* ws, sph_stream stream);

/* Bounding box, largest h, 63-bit Morton keys, stable radix sort, permutation
 * of every state array into key order, and the cell table (section 4.3: the
 * particles are kept in the depth-first order of the octree; the domain size
 * is the bounding box after particles moved).
 * In: x y z h (and every other state array, permuted along).
 * Out: state arrays permuted; ws holds keys, permutation and cell table. */
sph_status sph_build_cells(const sph_config* cfg, sph_particles* p, void* ws, sph_stream stream);

/* Smoothing-length update (section 4.1 "local spatial resolution"; the rule is
 * not printed, the reading used is a fixed number `newton_iters` of Newton
 * steps on the effective neighbour number (32 pi/3) B_n sum_b S_n(pi r/2h) =
 * n_target, clamped to [h0/kappa, kappa h0]).
 * In: x y z h (slot order of the last sph_build_cells).  Out: h in place. */
sph_status sph_update_h(const sph_config* cfg, sph_particles* p, void* ws, sph_stream stream);

/* Neighbour search within 2h (section 4.1, neighbours found with the tree of
 * section 4.3, stored as integer lists as in section 4.3).
 *   N(a)   = {b != a : r^2 < (2 h_a)^2}            gather set, nc[a] = |N(a)|
 *   N_s(a) = {b != a : r^2 < (2 max(h_a,h_b))^2}   symmetric set, ns[a] = |N_s(a)|
 * Lists are written to ws (sph_neighbors_view).  In: x y z h. */
sph_status sph_find_neighbors(const sph_config* cfg, const sph_particles* p, void* ws,
                              sph_stream stream);

/* Density (eq. 1, self term included), grad-h term Omega (section 4.1) and the
 * equation of state.  In: lists, x y z h m u (p_ref rho_ref).  Out: rho omega p c. */
sph_status sph_density(const sph_config* cfg, sph_particles* p, void* ws, sph_stream stream);

/* IAD matrix (section 4.1, integral approach to derivatives):
 * tau_a = sum_{b in N(a)} (m_b/rho_b) W(r_ab,h_a) d_ab d_ab^T, C_a = tau_a^-1.
 * det(tau) <= 0 writes C = 0 and sets SPH_ERRBIT_SINGULAR_TAU.
 * In: lists, x y z h m rho.  Out: c11 c12 c13 c22 c23 c33. */
sph_status sph_iad(const sph_config* cfg, sph_particles* p, void* ws, sph_stream stream);

/* Momentum and energy rates with artificial viscosity (eqs. 2-5), summed over
 * N_s(a), with A_ab(h_k) = C_k (x_b - x_a) W(r_ab, h_k), the AV acceleration
 * subtracted and the energy prefactor P_a/(Omega_a rho_a^2).  Also reduces the
 * per-particle time-step candidates (see sph_timestep) into ws.
 * In: lists, x y z vx vy vz h m u rho omega p c c11..c33.  Out: ax ay az du. */
sph_status sph_momentum_energy(const sph_config* cfg, sph_particles* p, void* ws,
                               sph_stream stream);

/* Global minimum time step (section 4.2, second global reduction; the rule is
 * not printed, the reading used): g->dt = min over particles of
 *   courant * (h/c),  acc_dt * sqrt(h/|a|),  energy_dt * (|u|/|du|)
 * (zero coefficients switch the last two off), at most dt_growth * g->dt_m1 if
 * g->dt_m1 > 0.
 * In: the candidates of the last sph_momentum_energy.  Out: g->dt (device). */
sph_status sph_timestep(const sph_config* cfg, sph_globals* g, void* ws, sph_stream stream);

/* Integrator (section 4.1: second-order Press method for x and v, second-order
 * Adams-Bashforth for u), read as kick-drift leapfrog with lambda = g->dt_m1:
 * vh += a (lambda+dt)/2; x += vh dt (wrapped on periodic axes); v = vh + a dt/2;
 * u += dt[(1+q) du - q du_m1], q = dt/(2 lambda) (Euler when lambda = 0);
 * du_m1 = du.  Then the conservation sums (section 4.2, third reduction) into g
 * and g->dt_m1 = g->dt, g->t += g->dt.
 * In: state, ax ay az du, g->dt, g->dt_m1.  Out: state, g. */
sph_status sph_integrate(const sph_config* cfg, sph_particles* p, sph_globals* g, void* ws,
                         sph_stream stream);

/* One full time step: build_cells, update_h, find_neighbors, density, iad,
 * momentum_energy, timestep, integrate (the step order follows the three halo
 * refreshes of section 4.4 and the global reductions of section 4.2).
 * With h_ratio_max <= 1.25 the h update and the neighbour search share one cell
 * walk: it collects candidates within 2*h_ratio_max*max(h_a, h_b) (every pair
 * the clamped Newton steps and the lists can need), the Newton sums run over
 * the candidates and the lists are filtered from them; the results are the
 * ones of the separate stages (same sets, other summation order).  The
 * workspace holds ceil(1.25^4 * ng_max) candidate slots
 * per particle; a candidate overflow sets SPH_ERRBIT_NEIGHBOR_OVERFLOW. */
sph_status sph_step(const sph_config* cfg, sph_particles* p, sph_globals* g, void* ws,
                    sph_stream stream);

/* sph_step with phase markers, for timing the step's kernels on its own stream.
 * Enqueues exactly the launches of sph_step and records events[k] (hipEvent_t
 * handles created by the caller, (host) array of SPH_STEP_PHASES + 1) after
 * phase k: 0 start; 1 cell build (and the per-cell h_max pass of the fused
 * path); 2 candidate walk (walk path: the h update); 3 Newton h update (walk
 * path: empty); 4 neighbour lists;
 * 5 density; 6 IAD; 7 momentum/energy and the time step; 8 integration and
 * sums.  Returns SPH_E_ARG if nevents differs or a handle is NULL. */
#define SPH_STEP_PHASES 8
sph_status sph_step_marked(const sph_config* cfg, sph_particles* p, sph_globals* g, void* ws,
                           sph_stream stream, void* const* events, int32_t nevents);

/* (host) A HIP graph of `steps` consecutive sph_step calls (section 4.1: the
 * whole time step, `steps` times) on these particles, globals and workspace,
 * replayed by one launch.  Small problems are bound by the launch cost of the
 * step's ~40 kernels; a graph hands the device the whole sequence at once.
 * The step is captured on a stream of the library's own (the caller's stream
 * may be the legacy default stream, which cannot be captured) and nothing is
 * run at creation; every sph_step_graph_launch then enqueues the steps on
 * `stream` with exactly sph_step's kernels and arguments, so the results are
 * bit-identical to `steps` calls of sph_step.  The graph keeps the pointers
 * and the configuration it was created with: the arrays, globals and ws must
 * stay allocated and be used by nothing else while a launch runs.  Device
 * conditions accumulate in ws's error word as for sph_step (read them with
 * sph_status_sync).
 * Errors: SPH_E_ARG for an invalid config, NULL arguments or steps outside
 * 1..SPH_GRAPH_MAX_STEPS; SPH_E_WORKSPACE for a NULL or misaligned ws;
 * SPH_E_HIP if capture or instantiation fails (*graph is then NULL). */
#define SPH_GRAPH_MAX_STEPS 1024
typedef struct sph_step_graph_s* sph_step_graph;
sph_status sph_step_graph_create(const sph_config* cfg, sph_particles* p, sph_globals* g,
                                 void* ws, int32_t steps, sph_step_graph* graph);
/* Enqueues the graph's steps on `stream`.  SPH_E_ARG for a NULL graph. */
sph_status sph_step_graph_launch(sph_step_graph graph, sph_stream stream);
/* Frees the graph (NULL is a no-op).  No launch of it may still be running. */
void sph_step_graph_destroy(sph_step_graph graph);

/* ------------------------------------------------------------------------
 * Self-gravity (section 4.1: a multipole expansion evaluated on the same
 * octree that finds the neighbours).  Plummer-softened Newtonian gravity
 *   g_a = -G sum_{b != a} m_b (x_a - x_b) / (|x_a - x_b|^2 + eps^2)^(3/2),
 * evaluated on the octree of the Morton keys of the last sph_build_cells: the
 * node of level l (0 .. L, L the deepest level with 8^L <= n, at most 9) holds
 * the particles whose key prefix of 3l bits is its index.  Each node carries
 * its mass, centre of mass c and traceless quadrupole
 * Q = sum m (3 d d^T - |d|^2 I), d = x - c.  A target walks the tree depth first
 * from the root, children in ascending prefix: the node holding the target is
 * opened; another node of size s (the key domain's largest extent over 2^l) at
 * distance d = |x_a - c| contributes, when s < theta d, its expansion
 *   -G M r / rho^3 + G (Q r / rho^5 - (5/2)(r.Q.r) r / rho^7),
 *   r = x_a - c, rho^2 = |r|^2 + eps^2;
 * an opened leaf contributes its particles b != a directly.  theta = 0 gives
 * the direct sum.  Open boundaries only (no periodic images).
 * In: x y z m in the slot order of the last sph_build_cells on ws (call it
 * first).  Out: gx gy gz per slot (device, caller-owned, length n).
 * gws: caller-owned gravity workspace of sph_gravity_workspace_bytes(cfg)
 * bytes, 256-byte aligned, used only by this call.
 * Errors: SPH_E_ARG for a periodic axis, NULL arrays, negative or non-finite
 * G, eps or theta; SPH_E_WORKSPACE for a NULL or misaligned ws or gws. */
typedef struct {
    double G;       /* gravitational constant */
    double eps;     /* Plummer softening length, >= 0 */
    double theta;   /* opening angle: a node is expanded when size < theta * distance */
} sph_gravity_params;

size_t sph_gravity_workspace_bytes(const sph_config* cfg);
sph_status sph_gravity(const sph_config* cfg, const sph_particles* p,
                       const sph_gravity_params* gp, void* ws, void* gws, double* gx,
                       double* gy, double* gz, sph_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sph_step
 * without a caller workspace.  Its scratch is a fixed device array of
 * SPH_STATIC_SCRATCH_BYTES held by the library on each GPU it runs on until
 * the process ends; the call allocates nothing and frees nothing.  The caller
 * still passes the particles and globals as for sph_step, on the current
 * device (the stream must belong to it).
 * Limit: configurations whose sph_workspace_bytes exceeds
 * SPH_STATIC_SCRATCH_BYTES return SPH_E_WORKSPACE before anything is enqueued
 * (64 MiB: 25,536 particles at ng_max = 160).
 * err_out: device pointer to one uint32 that receives this call's device error
 * word (SPH_ERRBIT_* bits) when the stream reaches the end of the step, or
 * NULL.  Each call starts from a cleared word.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (two streams, two threads) race and give undefined results. */
#define SPH_STATIC_SCRATCH_BYTES (64u << 20)
sph_status sph_step_static(const sph_config* cfg, sph_particles* p, sph_globals* g,
                           uint32_t* err_out, sph_stream stream);

/* ------------------------------------------------------------------------
 * Reverse mode (adjoint) of one step.  The map differentiated is the step of
 * section 4.1 with its STRUCTURE FROZEN: the smoothing lengths h, the time
 * steps dt and dt_m1, the neighbour sets and the artificial-viscosity branches
 * (v_ab . x_ab < 0) are those of the forward step and are not differentiated
 * (the set indicators and the clamp have zero derivative almost everywhere).
 * The masses are constants.  FP64 only (precision must be SPH_FP64).
 * ---------------------------------------------------------------------- */

/* Gradient arrays (device, caller-owned, FP64, length n) of the fields one
 * step maps: x^n, v^n, v^{n-1/2}, u, du_m1 (the others are constants of the
 * frozen step). */
typedef struct {
    double *x, *y, *z;
    double *vx, *vy, *vz;
    double *vhx, *vhy, *vhz;
    double *u, *du_m1;
} sph_grads;

/* (host) Bytes of the adjoint workspace for cfg (224 B per particle plus
 * alignment; a pure function of n).  Returns 0 if cfg is invalid. */
size_t sph_adjoint_workspace_bytes(const sph_config* cfg);

/* Vector-Jacobian product of one sph_step.
 * In:  p, g and ws exactly as they were when the forward sph_step was called
 *      (the step's input state, e.g. restored from a checkpoint, with g->dt_m1
 *      of that step); gout: adjoints of the step's outputs x, v, vh, u, du_m1,
 *      per slot of the order the forward step left the particles in.
 * Out: gin: adjoints of the step's inputs, per slot of the order p has on
 *      entry (the permutation of the cell build is undone: it is linear and its
 *      adjoint is its inverse).  gin may alias gout.
 * The call first re-runs the forward stages of the step (cell build, h update,
 * lists, density, IAD, momentum/energy, time step; not the integration), so
 * on return p is in the step's slot order with every stage output filled and
 * g->dt set, as after those stages of sph_step; the other fields of g are
 * unchanged.  Then, in gather form over the symmetric lists (no atomics,
 * bitwise reproducible): integrate^T, momentum/energy^T with the EOS^T and
 * tau_bar = -C Cbar C, IAD^T, density^T (eq. 1 with the grad-h term).
 * adj_ws: sph_adjoint_workspace_bytes, 256-byte aligned, no initialisation. */
sph_status sph_step_backward(const sph_config* cfg, sph_particles* p, sph_globals* g, void* ws,
                             void* adj_ws, const sph_grads* gout, sph_grads* gin,
                             sph_stream stream);

/* Vector-Jacobian product of the density (eq. 1) with respect to positions,
 * h frozen: x_bar = (d rho / d x)^T rho_bar, for a loss on the density.
 * In:  the state of a completed sph_build_cells -> (update_h) -> find_neighbors
 *      -> sph_density sequence on ws and p; rho_bar per slot of the current order.
 * Out: x_bar, y_bar, z_bar per slot of the order before that sph_build_cells
 *      (the cell build's permutation is undone).  They must not alias rho_bar. */
sph_status sph_density_backward(const sph_config* cfg, const sph_particles* p, void* ws,
                                void* adj_ws, const double* rho_bar, double* x_bar,
                                double* y_bar, double* z_bar, sph_stream stream);

/* (host) Device pointers into ws after sph_find_neighbors or sph_step: nc, ns
 * (int32[n]) and the list (int32, tiled by 64 slots so that a wavefront's
 * entries are contiguous: entry j of slot a is at
 *     list[((a/64)*capacity + j)*64 + a%64],   capacity = ng_max).
 * Slot a's gather neighbours are at j = 0..nc[a]-1; its symmetric-only
 * neighbours (in N_s(a) but not N(a)) are at j = ng_max-(ns[a]-nc[a]) .. ng_max-1.
 * Entries are slot indices.  Counts are true counts even when they exceed
 * ng_max (then SPH_ERRBIT_NEIGHBOR_OVERFLOW is set and the lists truncated). */
sph_status sph_neighbors_view(const sph_config* cfg, void* ws, const int32_t** nc,
                              const int32_t** ns, const int32_t** list, int32_t* capacity);

/* Short candidate reach of the fused step (h_ratio_max <= 1.25): the step
 * collects candidates within 2*lambda*max(h0_a, h0_b), lambda =
 * min(SPH_SHORT_REACH, h_ratio_max), and repeats the walk and the Newton
 * iterations at the full reach h_ratio_max only if an iterate h leaves
 * lambda*h0.  The lists are exact either way; the constant trades the walk's
 * volume (lambda^3) against how often h grows past it in one step. */
#define SPH_SHORT_REACH 1.03

/* (host) Device pointers into ws after sph_step with h_ratio_max <= 1.25 (the
 * fused path): nk (int32[n]), each slot's candidate count, and the candidate
 * capacity per slot.  The candidates of a slot are every b != a within
 * 2*lambda*max(h0_a, h0_b) (lambda = min(SPH_SHORT_REACH, h_ratio_max), or h_ratio_max
 * when the full-reach pass ran), plus any pairs the FP32 prefilter's rounding
 * margin admits beyond that reach (within a relative 2^-20 of the box extent
 * and 2^-18 of the squared reach). */
sph_status sph_candidates_view(const sph_config* cfg, void* ws, const int32_t** nk,
                               int32_t* capacity);

/* (host) Device pointers into ws after sph_build_cells: the sorted keys
 * (uint64[n]) and the permutation perm (uint32[n], slot -> slot before the call). */
sph_status sph_order_view(const sph_config* cfg, void* ws, const uint64_t** keys,
                          const uint32_t** perm);

/* Synchronises the stream, returns the most severe pending device condition
 * (NONFINITE > SINGULAR_TAU > NEIGHBOR_OVERFLOW > CELL_RANGE) or SPH_OK, stores
 * the raw bits in *bits (host, may be NULL) and clears the word. */
sph_status sph_status_sync(void* ws, sph_stream stream, uint32_t* bits);

/* (host) Static string naming a status. */
const char* sph_status_string(sph_status s);

#ifdef __cplusplus
}
#endif
#endif /* SPH_H */
