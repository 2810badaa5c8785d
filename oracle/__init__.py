"""FP64 CPU oracle of the SPH time step (arXiv 2005.02656, section 4.1).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  The product path never imports this
package.  It shares no code with the HIP implementation; the arithmetic lives in
``sph_oracle.c`` (plain C, brute force O(N^2), -ffp-contract=off), and this module
only marshals numpy arrays through ctypes and composes the documented steps:

    smoothing-length Newton -> neighbour sets -> density, Omega, EOS -> IAD ->
    momentum/energy/AV -> global dt -> integrator -> conservation sums

(the step order follows the three halo exchanges per step, section 4.4, and the
three global reductions, section 4.2).  Parity status of every function is
pinned by ``tests/test_oracle_*.py``; the square-patch angular-momentum value of
section 4.6 is "parity unpinned" (it needs the parent codes).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


@dataclasses.dataclass
class Config:
    box_lo: tuple = (0.0, 0.0, 0.0)
    box_hi: tuple = (1.0, 1.0, 1.0)
    periodic: tuple = (1, 1, 1)
    sinc_n: float = 6.0
    n_target: float = 100.0
    newton_iters: int = 2
    h_ratio_max: float = 1.25
    eos: int = 0  # 0 ideal gas, 1 weakly compressible
    gamma: float = 5.0 / 3.0
    c0: float = 0.0
    alpha_av: float = 1.0
    courant: float = 0.2
    dt_growth: float = 1.1
    acc_dt: float = 0.2
    energy_dt: float = 0.2
    kernel_table: int = 0  # 0: exact S_n; N > 1: the N-value table of section 4.5

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


class _CConfig(C.Structure):
    _fields_ = [
        ("box_lo", C.c_double * 3),
        ("box_hi", C.c_double * 3),
        ("periodic", C.c_int32 * 3),
        ("sinc_n", C.c_double),
        ("n_target", C.c_double),
        ("newton_iters", C.c_int32),
        ("h_ratio_max", C.c_double),
        ("eos", C.c_int32),
        ("gamma", C.c_double),
        ("c0", C.c_double),
        ("alpha_av", C.c_double),
        ("courant", C.c_double),
        ("dt_growth", C.c_double),
        ("acc_dt", C.c_double),
        ("energy_dt", C.c_double),
        ("kernel_table", C.c_int32),
    ]


def _cc(cfg: Config) -> _CConfig:
    c = _CConfig()
    c.box_lo[:] = [float(v) for v in cfg.box_lo]
    c.box_hi[:] = [float(v) for v in cfg.box_hi]
    c.periodic[:] = [int(v) for v in cfg.periodic]
    c.sinc_n = cfg.sinc_n
    c.n_target = cfg.n_target
    c.newton_iters = cfg.newton_iters
    c.h_ratio_max = cfg.h_ratio_max
    c.eos = cfg.eos
    c.gamma = cfg.gamma
    c.c0 = cfg.c0
    c.alpha_av = cfg.alpha_av
    c.courant = cfg.courant
    c.dt_growth = cfg.dt_growth
    c.acc_dt = cfg.acc_dt
    c.energy_dt = cfg.energy_dt
    c.kernel_table = int(cfg.kernel_table)
    return c


def lib():
    global _lib
    if _lib is None:
        # SPH_ORACLE_LIBRARY: another build of the oracle (the sanitizer build)
        path = os.environ.get("SPH_ORACLE_LIBRARY") or _build.library_path()
        if not os.environ.get("SPH_ORACLE_LIBRARY") and (
                not os.path.exists(path) or
                os.path.getmtime(path) < os.path.getmtime(_build.SOURCE)):
            _build.build()
        _lib = C.CDLL(path)
        d, i64, vp = C.c_double, C.c_int64, C.c_void_p
        _lib.ora_bn.restype = d
        _lib.ora_bn.argtypes = [d]
        for f in ("ora_S", "ora_dSdv"):
            getattr(_lib, f).restype = d
            getattr(_lib, f).argtypes = [d, d]
        for f in ("ora_W", "ora_dWdh"):
            getattr(_lib, f).restype = d
            getattr(_lib, f).argtypes = [d, d, d, d]
        for f in ("ora_S_cfg", "ora_dSdv_cfg"):
            getattr(_lib, f).restype = d
            getattr(_lib, f).argtypes = [vp, d]
        _lib.ora_timestep.restype = d
        _lib.ora_timestep.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, d]
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _targets(n, targets):
    if targets is None:
        return n, None
    t = np.ascontiguousarray(targets, dtype=np.int64)
    if t.size and (t.min() < 0 or t.max() >= n):
        raise ValueError("target index out of range")
    return t.size, t


# --------------------------------------------------------------------------- kernel
def bn(n: float) -> float:
    """B_n of eq. (6) in 3-D by 96-point Gauss-Legendre."""
    return lib().ora_bn(float(n))


def S(v: float, n: float) -> float:
    return lib().ora_S(float(v), float(n))


def dSdv(v: float, n: float) -> float:
    return lib().ora_dSdv(float(v), float(n))


def S_cfg(cfg, v: float) -> float:
    """S_n(pi v/2) as cfg evaluates it (exactly, or from its lookup table)."""
    return lib().ora_S_cfg(C.byref(_cc(cfg)), float(v))


def dSdv_cfg(cfg, v: float) -> float:
    return lib().ora_dSdv_cfg(C.byref(_cc(cfg)), float(v))


def W(r2: float, h: float, n: float, b: float) -> float:
    return lib().ora_W(float(r2), float(h), float(n), float(b))


def dWdh(r2: float, h: float, n: float, b: float) -> float:
    return lib().ora_dWdh(float(r2), float(h), float(n), float(b))


# --------------------------------------------------------------------------- passes
def update_h(cfg, x, y, z, h, targets=None):
    x, y, z, h = map(_f64, (x, y, z, h))
    n = x.size
    nt, t = _targets(n, targets)
    out = h.copy()
    lib().ora_update_h(C.byref(_cc(cfg)), C.c_int64(n), _p(x), _p(y), _p(z), _p(h),
                       _p(out), C.c_int64(nt), _p(t))
    return out


def newton_terms(cfg, x, y, z, h, targets=None):
    x, y, z, h = map(_f64, (x, y, z, h))
    n = x.size
    nt, t = _targets(n, targets)
    F = np.full(n, np.nan)
    Fp = np.full(n, np.nan)
    lib().ora_newton_terms(C.byref(_cc(cfg)), C.c_int64(n), _p(x), _p(y), _p(z), _p(h),
                           C.c_int64(nt), _p(t), _p(F), _p(Fp))
    return F, Fp


def neighbors(cfg, x, y, z, h, targets=None, with_lists=True):
    """Returns (nc, ns, lists, gather) per target: lists[t] holds the ids of N_s(a)
    ascending, gather[t] flags members of N(a)."""
    x, y, z, h = map(_f64, (x, y, z, h))
    n = x.size
    nt, t = _targets(n, targets)
    nc = np.zeros(nt, np.int32)
    ns = np.zeros(nt, np.int32)
    lib().ora_neighbors(C.byref(_cc(cfg)), C.c_int64(n), _p(x), _p(y), _p(z), _p(h),
                        C.c_int64(nt), _p(t), _p(nc), _p(ns), C.c_int64(0), None, None)
    if not with_lists:
        return nc, ns, None, None
    cap = int(ns.max()) if nt else 0
    cap = max(cap, 1)
    ids = np.zeros(nt * cap, np.int64)
    gat = np.zeros(nt * cap, np.uint8)
    lib().ora_neighbors(C.byref(_cc(cfg)), C.c_int64(n), _p(x), _p(y), _p(z), _p(h),
                        C.c_int64(nt), _p(t), _p(nc), _p(ns), C.c_int64(cap), _p(ids), _p(gat))
    ids = ids.reshape(nt, cap)
    gat = gat.reshape(nt, cap)
    lists = [ids[i, : ns[i]].copy() for i in range(nt)]
    gath = [gat[i, : ns[i]].astype(bool) for i in range(nt)]
    return nc, ns, lists, gath


def density(cfg, x, y, z, h, m, u, p_ref=None, rho_ref=None, targets=None):
    x, y, z, h, m, u = map(_f64, (x, y, z, h, m, u))
    n = x.size
    if cfg.eos == 1:
        p_ref, rho_ref = _f64(p_ref), _f64(rho_ref)
    nt, t = _targets(n, targets)
    rho, om, p, c = (np.full(n, np.nan) for _ in range(4))
    lib().ora_density(C.byref(_cc(cfg)), C.c_int64(n), _p(x), _p(y), _p(z), _p(h), _p(m),
                      _p(u), _p(p_ref), _p(rho_ref), C.c_int64(nt), _p(t), _p(rho), _p(om),
                      _p(p), _p(c))
    return rho, om, p, c


def iad(cfg, x, y, z, h, m, rho, targets=None):
    """Returns (C, singular) with C of shape (6, n) ordered 11 12 13 22 23 33."""
    x, y, z, h, m, rho = map(_f64, (x, y, z, h, m, rho))
    n = x.size
    nt, t = _targets(n, targets)
    Cm = np.full((6, n), np.nan)
    sing = C.c_int32(0)
    lib().ora_iad(C.byref(_cc(cfg)), C.c_int64(n), _p(x), _p(y), _p(z), _p(h), _p(m),
                  _p(rho), C.c_int64(nt), _p(t), *[_p(Cm[k]) for k in range(6)],
                  C.byref(sing))
    return Cm, bool(sing.value)


def momentum_energy(cfg, x, y, z, vx, vy, vz, h, m, rho, omega, p, c, Cm, targets=None):
    """Returns dict with ax, ay, az, du, dt_cand, scale_a, scale_du."""
    arrs = list(map(_f64, (x, y, z, vx, vy, vz, h, m, rho, omega, p, c)))
    Cm = np.ascontiguousarray(Cm, dtype=np.float64)
    n = arrs[0].size
    nt, t = _targets(n, targets)
    out = {k: np.full(n, np.nan) for k in ("ax", "ay", "az", "du", "dt_cand", "scale_a", "scale_du")}
    lib().ora_momentum_energy(C.byref(_cc(cfg)), C.c_int64(n), *[_p(a) for a in arrs],
                              *[_p(Cm[k]) for k in range(6)], C.c_int64(nt), _p(t),
                              *[_p(out[k]) for k in ("ax", "ay", "az", "du", "dt_cand",
                                                    "scale_a", "scale_du")])
    return out


def timestep(cfg, h, c, u, ax, ay, az, du, dt_m1):
    arrs = list(map(_f64, (h, c, u, ax, ay, az, du)))
    return lib().ora_timestep(C.byref(_cc(cfg)), C.c_int64(arrs[0].size),
                              *[_p(a) for a in arrs], float(dt_m1))


STATE_FIELDS = ("x", "y", "z", "vx", "vy", "vz", "vhx", "vhy", "vhz", "h", "m", "u", "du_m1")


def integrate(cfg, st, ax, ay, az, du, dt, dt_m1):
    """Returns a new state dict (copies) advanced by dt."""
    s = {k: (_f64(v).copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    n = s["x"].size
    ax, ay, az, du = map(_f64, (ax, ay, az, du))
    lib().ora_integrate(C.byref(_cc(cfg)), C.c_int64(n),
                        *[_p(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "vhx", "vhy",
                                             "vhz", "u", "du_m1")],
                        _p(ax), _p(ay), _p(az), _p(du), C.c_double(dt), C.c_double(dt_m1))
    return s


def sums(m, x, y, z, vx, vy, vz, u):
    arrs = list(map(_f64, (m, x, y, z, vx, vy, vz, u)))
    out = np.zeros(9)
    lib().ora_sums(C.c_int64(arrs[0].size), *[_p(a) for a in arrs], _p(out))
    return {"mass": out[0], "mom": out[1:4].copy(), "ang": out[4:7].copy(),
            "e_kin": out[7], "e_int": out[8]}


def morton_keys(x, y, z, lo, hi):
    x, y, z = map(_f64, (x, y, z))
    lo, hi = _f64(lo), _f64(hi)
    keys = np.zeros(x.size, np.uint64)
    lib().ora_morton_keys(C.c_int64(x.size), _p(x), _p(y), _p(z), _p(lo), _p(hi), _p(keys))
    return keys


def bbox(x, y, z, h):
    x, y, z, h = map(_f64, (x, y, z, h))
    out = np.zeros(7)
    lib().ora_bbox(C.c_int64(x.size), _p(x), _p(y), _p(z), _p(h), _p(out))
    return out


def key_domain(cfg, x, y, z, h):
    """lo/hi used by the Morton keys: the box on periodic axes, the bbox on open ones."""
    bb = bbox(x, y, z, h)
    lo = np.array([cfg.box_lo[k] if cfg.periodic[k] else bb[k] for k in range(3)])
    hi = np.array([cfg.box_hi[k] if cfg.periodic[k] else bb[3 + k] for k in range(3)])
    return lo, hi


def sort_keys(keys, level=None):
    """Stable order of the keys (ties by index); with level L only their prefix
    of L levels (3L bits) is compared: the particle order of the cell build,
    whose finest cell level is leaf_level(n)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    perm = np.zeros(keys.size, np.int64)
    if level is None:
        lib().ora_sort_keys(C.c_int64(keys.size), _p(keys), _p(perm))
    else:
        lib().ora_sort_keys_level(C.c_int64(keys.size), _p(keys), C.c_int(int(level)),
                                  _p(perm))
    return perm


# --------------------------------------------------------------------------- gravity
def leaf_level(n: int) -> int:
    """Finest cell level L of n particles (the particle order's and the gravity
    tree's): the largest L <= 9 with 8^L <= n."""
    L = 0
    while L < 9 and 8 ** (L + 1) <= max(n, 1):
        L += 1
    return L


gravity_leaf_level = leaf_level


def gravity_direct(x, y, z, m, G, eps, targets=None):
    """(gx, gy, gz, scale): the softened Newtonian sum over all pairs."""
    x, y, z, m = map(_f64, (x, y, z, m))
    n = x.size
    nt, t = _targets(n, targets)
    out = [np.full(n, np.nan) for _ in range(4)]
    lib().ora_gravity_direct(C.c_int64(n), _p(x), _p(y), _p(z), _p(m), C.c_double(G),
                             C.c_double(eps), C.c_int64(nt), _p(t), *[_p(o) for o in out])
    return tuple(out)


def moments(idx, x, y, z, m):
    """[M, cx, cy, cz, Q11, Q12, Q13, Q22, Q23, Q33] of the particles idx."""
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    x, y, z, m = map(_f64, (x, y, z, m))
    out = np.zeros(10)
    lib().ora_moments(C.c_int64(idx.size), _p(idx), _p(x), _p(y), _p(z), _p(m), _p(out))
    return out


def multipole_accel(mo, pos, G, eps):
    mo, pos = _f64(mo), _f64(pos)
    g = np.zeros(3)
    lib().ora_multipole_accel(_p(mo), _p(pos), C.c_double(G), C.c_double(eps), _p(g))
    return g


def gravity_tree(x, y, z, m, lo, hi, L, G, eps, theta, targets=None):
    """(gx, gy, gz, scale): the multipole tree walk of section 4.1 (see the C
    header comment for the tree, the opening rule and the expansion)."""
    x, y, z, m = map(_f64, (x, y, z, m))
    lo, hi = _f64(lo), _f64(hi)
    n = x.size
    nt, t = _targets(n, targets)
    out = [np.full(n, np.nan) for _ in range(4)]
    lib().ora_gravity_tree(C.c_int64(n), _p(x), _p(y), _p(z), _p(m), _p(lo), _p(hi),
                           C.c_int(int(L)), C.c_double(G), C.c_double(eps),
                           C.c_double(theta), C.c_int64(nt), _p(t), *[_p(o) for o in out])
    return tuple(out)


# --------------------------------------------------------------------------- composed
def initial_h(cfg, st, iters=12, kappa=8.0):
    """Untimed set-up: `iters` Newton steps from the generator's guess, clamped at
    [h/kappa, kappa h] of the guess."""
    c = cfg.replace(newton_iters=iters, h_ratio_max=kappa)
    return update_h(c, st["x"], st["y"], st["z"], st["h"])


def step(cfg, st, gl):
    """One full step on a state dict; gl holds dt_m1 and t.  Returns
    (new_state, new_globals, fields) where fields holds every intermediate."""
    x, y, z = st["x"], st["y"], st["z"]
    h = update_h(cfg, x, y, z, st["h"])
    rho, om, p, c = density(cfg, x, y, z, h, st["m"], st["u"], st.get("p_ref"),
                            st.get("rho_ref"))
    Cm, sing = iad(cfg, x, y, z, h, st["m"], rho)
    me = momentum_energy(cfg, x, y, z, st["vx"], st["vy"], st["vz"], h, st["m"], rho, om, p,
                         c, Cm)
    dt = timestep(cfg, h, c, st["u"], me["ax"], me["ay"], me["az"], me["du"], gl["dt_m1"])
    s0 = dict(st)
    s0["h"] = h
    new = integrate(cfg, s0, me["ax"], me["ay"], me["az"], me["du"], dt, gl["dt_m1"])
    sm = sums(new["m"], new["x"], new["y"], new["z"], new["vx"], new["vy"], new["vz"], new["u"])
    g = {"dt": dt, "dt_m1": dt, "t": gl["t"] + dt, **sm}
    fields = {"h": h, "rho": rho, "omega": om, "p": p, "c": c, "C": Cm, "singular": sing, **me}
    return new, g, fields


def num_threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(lib().ora_num_threads())


def set_num_threads(k: int) -> None:
    """Sets the OpenMP threads of the oracle's loops (for timing on k cores)."""
    lib().ora_set_num_threads(C.c_int(int(k)))
