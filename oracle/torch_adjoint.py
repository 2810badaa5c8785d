"""Differentiable FP64 oracle of the SPH step (test infrastructure only).

A plain PyTorch CPU, float64, dense O(N^2) restatement of the same definitions
as sph_oracle.c (section 4.1, eqs. 1-5, with the readings in the design notes),
used only for reference GRADIENTS: autograd differentiates it.  The step map
is the one the adjoint differentiates, with the structure frozen:

* h of every particle and the time steps dt, dt_m1 are inputs (not differentiated);
* the neighbour sets follow from the fixed h (the indicator r^2 < (2h)^2 has a
  zero derivative almost everywhere), and so do the viscosity branches.

It shares no code with the HIP path.  Its forward values are pinned to the C
oracle's, and its gradients to central finite differences of the C oracle's
composed stages, by tests/test_oracle_adjoint.py.
"""
from __future__ import annotations

import math

import torch

T = torch.float64


def bn(n: float) -> float:
    """B_n by composite Gauss-Legendre (independent of the C oracle's routine)."""
    import numpy as np
    t, w = np.polynomial.legendre.leggauss(128)
    v = 1.0 + t
    f = np.sinc(v / 2.0) ** n * v * v
    return 1.0 / (4.0 * math.pi * float((w * f).sum()))


class Setup:
    """Fixed data of one step: box, masses, parameters."""

    def __init__(self, cfg, m, h, u_ref=None):
        self.cfg = cfg
        self.m = torch.as_tensor(m, dtype=T)
        self.h = torch.as_tensor(h, dtype=T)
        self.n = self.m.numel()
        self.bn = bn(cfg.sinc_n)
        self.L = torch.tensor([cfg.box_hi[k] - cfg.box_lo[k] for k in range(3)], dtype=T)
        self.periodic = torch.tensor([bool(p) for p in cfg.periodic])


def pair_geometry(S: Setup, x):
    """d[a, b] = x_b - x_a with the minimum image on periodic axes, r^2, masks."""
    d = x[None, :, :] - x[:, None, :]
    L = S.L
    half = 0.5 * L
    wrapped = torch.where(d > half, d - L, torch.where(d <= -half, d + L, d))
    d = torch.where(S.periodic[None, None, :], wrapped, d)
    r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    eye = torch.eye(S.n, dtype=torch.bool)
    return d, r2, eye


def kernel_S(v, n):
    """S_n(pi v / 2) = sinc(v/2)^n (torch.sinc is sin(pi t)/(pi t))."""
    return torch.sinc(v / 2.0) ** n


def density_omega(S: Setup, x):
    d, r2, eye = pair_geometry(S, x)
    h = S.h
    n = S.cfg.sinc_n
    ha2 = (2.0 * h)[:, None] * (2.0 * h)[:, None]
    inside = (r2 < ha2) & ~eye
    r = torch.sqrt(torch.where(inside, r2, torch.ones_like(r2)))
    v = r / h[:, None]
    Sv = torch.where(inside, kernel_S(v, n), torch.zeros_like(r))
    # v dS/dv through autograd of S in v would need a second graph; write it out:
    # dS/dv = n sinc^(n-1) * d sinc(v/2)/dv
    x_ = 0.5 * math.pi * v
    sinc = torch.sinc(v / 2.0)
    dsinc_dx = torch.where(x_ > 1e-3, (x_ * torch.cos(x_) - torch.sin(x_)) / (x_ * x_),
                           -x_ / 3.0 + x_ ** 3 / 30.0)
    vdS = torch.where(inside, n * sinc ** (n - 1) * dsinc_dx * x_, torch.zeros_like(r))
    m = S.m
    w0 = S.bn / h ** 3
    sS = m + (Sv * m[None, :]).sum(1)                      # self term: S = 1
    sD = 3.0 * m + ((3.0 * Sv + vdS) * m[None, :]).sum(1)  # self term: 3S + v S' = 3
    rho = w0 * sS
    omega = 1.0 - w0 * sD / (3.0 * rho)
    return rho, omega


def eos(S: Setup, rho, u, p_ref=None, rho_ref=None):
    cfg = S.cfg
    if cfg.eos == 0:
        p = (cfg.gamma - 1.0) * rho * u
        c = torch.sqrt(cfg.gamma * (cfg.gamma - 1.0) * u)
    else:
        p = torch.as_tensor(p_ref, dtype=T) + cfg.c0 ** 2 * (rho - torch.as_tensor(rho_ref, dtype=T))
        c = torch.full_like(rho, cfg.c0)
    return p, c


def W_matrix(S: Setup, r2, h_rows, eye):
    """W(r_ab, h) with h per row a (or per column when transposed by the caller)."""
    n = S.cfg.sinc_n
    hh = 2.0 * h_rows
    inside = (r2 < hh * hh) & ~eye
    r = torch.sqrt(torch.where(inside, r2, torch.ones_like(r2)))
    v = r / h_rows
    return torch.where(inside, S.bn / h_rows ** 3 * kernel_S(v, n), torch.zeros_like(r)), inside


def iad(S: Setup, x, rho):
    d, r2, eye = pair_geometry(S, x)
    Wa, _ = W_matrix(S, r2, S.h[:, None], eye)
    vol = (S.m / rho)[None, :]
    s = vol * Wa
    tau = torch.einsum("ab,abi,abj->aij", s, d, d)
    return torch.linalg.inv(tau)


def momentum_energy(S: Setup, x, v, rho, omega, p, c, Cm):
    cfg = S.cfg
    d, r2, eye = pair_geometry(S, x)
    h = S.h
    hm = torch.maximum(h[:, None], h[None, :])
    sym = (r2 < (2.0 * hm) * (2.0 * hm)) & ~eye
    Wa, _ = W_matrix(S, r2, h[:, None], eye)          # W(r_ab, h_a)
    Wb, _ = W_matrix(S, r2, h[None, :], eye)          # W(r_ab, h_b)
    Aa = torch.einsum("aij,abj->abi", Cm, d) * Wa[..., None]
    Ab = torch.einsum("bij,abj->abi", Cm, d) * Wb[..., None]
    vab = v[:, None, :] - v[None, :, :]
    xv = -(vab * d).sum(-1)
    r = torch.sqrt(torch.where(sym, r2, torch.ones_like(r2)))
    w = xv / r
    vsig = c[:, None] + c[None, :] - 3.0 * w
    Pi = torch.where(sym & (xv < 0.0), -0.5 * cfg.alpha_av * vsig * w, torch.zeros_like(w))
    m = S.m
    pa = p / (omega * rho * rho)
    g = 0.5 * m[None, :, None] * Pi[..., None] * (Aa / rho[:, None, None] + Ab / rho[None, :, None])
    f = m[None, :, None] * (pa[:, None, None] * Aa + pa[None, :, None] * Ab)
    symf = sym[..., None].to(T)
    acc = (-(f + g) * symf).sum(1)
    e1 = (m[None, :] * (vab * Aa).sum(-1) * sym.to(T)).sum(1)
    e2 = ((vab * g).sum(-1) * sym.to(T)).sum(1)
    du = pa * e1 + 0.5 * e2
    return acc, du


def step(S: Setup, st: dict, dt: float, dt_m1: float, p_ref=None, rho_ref=None):
    """One step with frozen h and dt.  st holds tensors x (n,3), v (n,3), vh (n,3),
    u (n,), du_m1 (n,).  Returns the new state dict and the intermediates."""
    x, v, vh, u, du_m1 = st["x"], st["v"], st["vh"], st["u"], st["du_m1"]
    rho, omega = density_omega(S, x)
    p, c = eos(S, rho, u, p_ref, rho_ref)
    Cm = iad(S, x, rho)
    acc, du = momentum_energy(S, x, v, rho, omega, p, c, Cm)
    kick = 0.5 * (dt_m1 + dt)
    vh1 = vh + acc * kick
    x1 = x + vh1 * dt
    # periodic wrap: a constant shift, derivative one
    lo = torch.tensor(S.cfg.box_lo, dtype=T)
    hi = torch.tensor(S.cfg.box_hi, dtype=T)
    shift = torch.where(S.periodic[None, :] & (x1 >= hi), -S.L,
                        torch.where(S.periodic[None, :] & (x1 < lo), S.L, torch.zeros_like(S.L)))
    x1 = x1 + shift.detach()
    v1 = vh1 + acc * (0.5 * dt)
    if dt_m1 > 0.0:
        q = dt / (2.0 * dt_m1)
        u1 = u + dt * ((1.0 + q) * du - q * du_m1)
    else:
        u1 = u + dt * du
    new = {"x": x1, "v": v1, "vh": vh1, "u": u1, "du_m1": du}
    return new, {"rho": rho, "omega": omega, "p": p, "c": c, "C": Cm, "a": acc, "du": du}


def rollout_density(cfg, st0: dict, v0, steps: int):
    """Final density after `steps` steps from the state st0 with v = vh = v0.

    v0 is a torch (n, 3) float64 tensor (it may require grad); st0 holds numpy
    arrays keyed like the C oracle's state.  The structure of each step is the C
    oracle's and is frozen: its Newton h and its dt (sections 4.1 and 4.2), and the
    final evaluation's h (one more h update on the final positions).  Then the
    steps are replayed with this module's differentiable step map.  Returns
    (rho, frozen) with frozen the per-step (h, dt, dt_m1) list and the final h."""
    import numpy as np
    import oracle as ora

    v = v0.detach().cpu().numpy()
    st = dict(st0)
    for c, a in enumerate("xyz"):
        st["v" + a] = v[:, c].copy()
        st["vh" + a] = v[:, c].copy()
    gl = {"dt_m1": 0.0, "t": 0.0}
    frozen = []
    for _ in range(steps):
        new, g, f = ora.step(cfg, st, gl)
        frozen.append((f["h"], g["dt"], gl["dt_m1"]))
        st, gl = new, g
    h_final = ora.update_h(cfg, st["x"], st["y"], st["z"], st["h"])
    ts = {"x": torch.tensor(np.stack([st0["x"], st0["y"], st0["z"]], 1)),
          "v": v0, "vh": v0,
          "u": torch.tensor(st0["u"]),
          "du_m1": torch.tensor(st0.get("du_m1", np.zeros(st0["u"].size)))}
    for h, dt, dt_m1 in frozen:
        ts, _ = step(Setup(cfg, st0["m"], h), ts, dt, dt_m1)
    rho, _ = density_omega(Setup(cfg, st0["m"], h_final), ts["x"])
    return rho, frozen, h_final
