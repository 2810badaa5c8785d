"""Seeded synthetic workloads for the SPH step (shared by the tests, the benchmark
and the oracle's callers).

This module holds only initial conditions: positions, velocities, masses,
internal energies, a first guess of h, the analytic pressure of the rotating
square patch and the physical parameters of each workload.  It contains none of
the SPH method's arithmetic (no kernel, no sums, no integrator); both the HIP
path and the oracle compute everything else themselves from these arrays.

Workloads (numpy ``Generator(PCG64(seed))`` everywhere):

* ``lattice``  -- simple cubic lattice in the periodic unit cube, ideal gas,
  u = 1, rho0 = 1, velocities N(0, sigma^2) per component.
* ``square_patch`` -- the rotating square patch of section 4.6: an n^3 lattice
  in [-1/2, 1/2]^3, periodic in z only, v = (omega y, -omega x, 0) (eq. 7),
  initial pressure from the double sine series of the incompressible solution
  (eq. 8, with the reading: odd m, n >= 1 only, the second factor in y,
  coordinates shifted to [0, L]), weakly compressible EOS with c0 = 10 |v|max.
* ``gaussian_blob`` -- Poisson-random particles in the periodic unit cube,
  rejection-sampled from n(x) ~ 1 + A exp(-|x-c|^2 / (2 sigma^2)) with the
  minimum-image distance to the centre, ideal gas, u = 1.
* ``random_periodic`` -- uniform random particles with random h (invariance
  tests).
"""
from __future__ import annotations

import dataclasses

import numpy as np

# guess for h in units of the local mean inter-particle spacing; the set-up then
# runs the smoothing-length Newton iteration from it
H_GUESS_SPACINGS = 1.44


@dataclasses.dataclass
class Workload:
    name: str
    arrays: dict          # numpy arrays, one entry per particle
    params: dict          # box, boundary flags, EOS and run parameters

    @property
    def n(self) -> int:
        return int(self.arrays["x"].size)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def base_params(**kw) -> dict:
    p = dict(box_lo=(0.0, 0.0, 0.0), box_hi=(1.0, 1.0, 1.0), periodic=(1, 1, 1),
             sinc_n=6.0, n_target=100.0, newton_iters=2, h_ratio_max=1.25, eos=0,
             gamma=5.0 / 3.0, c0=0.0, alpha_av=1.0, courant=0.2, dt_growth=1.1,
             acc_dt=0.2, energy_dt=0.2, ng_max=160)
    p.update(kw)
    return p


def lattice(n_side: int, seed: int = 1, sigma_v: float = 0.01, u0: float = 1.0) -> Workload:
    """Simple cubic n_side^3 lattice, x = (i + 1/2) / n_side in the periodic unit cube."""
    d = 1.0 / n_side
    g = (np.arange(n_side) + 0.5) * d
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    n = n_side ** 3
    rng = _rng(seed)
    v = rng.normal(0.0, sigma_v, size=(3, n))
    arr = dict(x=X.ravel().copy(), y=Y.ravel().copy(), z=Z.ravel().copy(),
               vx=v[0].copy(), vy=v[1].copy(), vz=v[2].copy(),
               m=np.full(n, 1.0 / n), u=np.full(n, u0),
               h=np.full(n, H_GUESS_SPACINGS * d), id=np.arange(n, dtype=np.int64))
    return Workload(f"lattice{n_side}^3", arr, base_params())


def square_patch_pressure(xs: np.ndarray, ys: np.ndarray, omega: float = 5.0, rho: float = 1.0,
                          L: float = 1.0, m_max: int = 399) -> np.ndarray:
    """Analytic initial pressure of the rotating square patch (eq. 8) on the grid
    xs x ys (patch centred on 0).  Returns an array of shape (len(xs), len(ys))."""
    k = np.arange(1, m_max + 1, 2, dtype=np.float64)
    X = (np.asarray(xs, np.float64) + 0.5 * L)[:, None]
    Y = (np.asarray(ys, np.float64) + 0.5 * L)[:, None]
    sx = np.sin(k[None, :] * np.pi * X / L)
    sy = np.sin(k[None, :] * np.pi * Y / L)
    km, kn = np.meshgrid(k, k, indexing="ij")
    coef = -32.0 * omega ** 2 / (km * kn * np.pi ** 2 * ((km * np.pi / L) ** 2 + (kn * np.pi / L) ** 2))
    return rho * (sx @ coef @ sy.T)


def square_patch(n_side: int, omega: float = 5.0, u0: float = 1.0) -> Workload:
    d = 1.0 / n_side
    g = -0.5 + (np.arange(n_side) + 0.5) * d
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    n = n_side ** 3
    P2 = square_patch_pressure(g, g, omega=omega)          # (ix, iy)
    p_ref = np.broadcast_to(P2[:, :, None], (n_side, n_side, n_side)).ravel().copy()
    x, y, z = X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy()
    arr = dict(x=x, y=y, z=z, vx=omega * y, vy=-omega * x, vz=np.zeros(n),
               m=np.full(n, 1.0 / n), u=np.full(n, u0),
               h=np.full(n, H_GUESS_SPACINGS * d), id=np.arange(n, dtype=np.int64),
               p_ref=p_ref)
    c0 = 10.0 * omega * np.sqrt(2.0) / 2.0
    prm = base_params(box_lo=(-0.5, -0.5, -0.5), box_hi=(0.5, 0.5, 0.5), periodic=(0, 0, 1),
                      eos=1, c0=c0, energy_dt=0.0)
    return Workload(f"square_patch{n_side}^3", arr, prm)


def gaussian_blob(n: int, seed: int = 3, seed_v: int = 33, amp: float = 10.0,
                  sigma: float = 0.05, sigma_v: float = 0.1, chunk: int = 1 << 22) -> Workload:
    rng = _rng(seed)
    c = 0.5
    out = []
    have = 0
    while have < n:
        p = rng.random((chunk, 3))
        d = p - c
        d = d - np.round(d)                       # minimum image in the unit cube
        dens = 1.0 + amp * np.exp(-(d * d).sum(1) / (2.0 * sigma ** 2))
        keep = rng.random(chunk) * (1.0 + amp) < dens
        out.append(p[keep])
        have += int(keep.sum())
    pos = np.concatenate(out)[:n]
    d = pos - c
    d = d - np.round(d)
    rel = 1.0 + amp * np.exp(-(d * d).sum(1) / (2.0 * sigma ** 2))
    mean_rel = 1.0 + amp * (2.0 * np.pi) ** 1.5 * sigma ** 3
    n_local = n * rel / mean_rel
    v = _rng(seed_v).normal(0.0, sigma_v, size=(3, n))
    arr = dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(),
               vx=v[0].copy(), vy=v[1].copy(), vz=v[2].copy(),
               m=np.full(n, 1.0 / n), u=np.ones(n),
               h=H_GUESS_SPACINGS * n_local ** (-1.0 / 3.0), id=np.arange(n, dtype=np.int64))
    # Poisson clumps hold up to ~260 neighbours within 2h once h has converged
    # (8M particles), so a larger list capacity than the lattices' 160
    return Workload(f"gaussian_blob{n}", arr, base_params(ng_max=320))


def random_periodic(n: int, seed: int, h_lo: float, h_hi: float, sigma_v: float = 0.3,
                    u_lo: float = 0.5, u_hi: float = 1.5) -> Workload:
    rng = _rng(seed)
    pos = rng.random((3, n))
    v = rng.normal(0.0, sigma_v, size=(3, n))
    arr = dict(x=pos[0].copy(), y=pos[1].copy(), z=pos[2].copy(), vx=v[0].copy(),
               vy=v[1].copy(), vz=v[2].copy(), m=rng.uniform(0.5, 1.5, n) / n,
               u=rng.uniform(u_lo, u_hi, n), h=rng.uniform(h_lo, h_hi, n),
               id=np.arange(n, dtype=np.int64))
    return Workload(f"random{n}", arr, base_params())


# the five workloads the benchmark and the parity tests are sized on
def evrard_sphere(n: int, seed: int = 7, u0: float = 0.05) -> Workload:
    """Self-gravitating gas sphere of radius 1 and mass 1 with density
    rho = 1/(2 pi r), at rest (the standard collapse test of SPH codes with
    gravity): enclosed mass r^2, so r = sqrt(U) for U uniform, with isotropic
    directions; equal masses 1/n, u = u0, open boundaries.  h starts at 1.44
    local mean spacings of the number density n/(2 pi r)."""
    rng = _rng(seed)
    r = np.sqrt(rng.random(n))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pos = d * r[:, None]
    nd = n / (2.0 * np.pi * np.maximum(r, 1e-3))
    arr = dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(),
               vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n), m=np.full(n, 1.0 / n),
               u=np.full(n, u0), h=H_GUESS_SPACINGS * nd ** (-1.0 / 3.0),
               id=np.arange(n, dtype=np.int64))
    return Workload(f"evrard{n}", arr, base_params(box_lo=(-1.0, -1.0, -1.0),
                                                    box_hi=(1.0, 1.0, 1.0), periodic=(0, 0, 0)))


def c1_lattice() -> Workload:
    return lattice(20, seed=1, sigma_v=0.01)


def c2_square_patch() -> Workload:
    return square_patch(100)


def c3_gaussian_blob() -> Workload:
    return gaussian_blob(8_000_000, seed=3, seed_v=33)


def c4_square_patch() -> Workload:
    return square_patch(400)


def c5_lattice() -> Workload:
    return lattice(64, seed=5, sigma_v=0.01)


def c5_target_density(n: int, seed: int = 55) -> np.ndarray:
    return 1.0 + 0.01 * _rng(seed).normal(0.0, 1.0, n)
