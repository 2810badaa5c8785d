"""ctypes binding of libsph (include/sph.h).

Argument marshalling only: torch tensors provide device memory and the stream,
every step of the SPH path runs in the library's HIP kernels.  The library must
be built (``python -m paper_2005_02656_amd.build``); if it is missing this module
raises on first use -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# SPH_LIBRARY selects another build of the library (e.g. one with other tuning flags)
LIB_PATH = os.environ.get("SPH_LIBRARY") or os.path.join(_HERE, "libsph.so")

SPH_OK = 0
STATUS_NAMES = {0: "SPH_OK", 1: "SPH_E_ARG", 2: "SPH_E_HIP", 3: "SPH_E_WORKSPACE",
                4: "SPH_E_NEIGHBOR_OVERFLOW", 5: "SPH_E_CELL_RANGE", 6: "SPH_E_NONFINITE",
                7: "SPH_E_SINGULAR_TAU"}
ERRBIT_NEIGHBOR_OVERFLOW, ERRBIT_CELL_RANGE, ERRBIT_NONFINITE, ERRBIT_SINGULAR_TAU = 1, 2, 4, 8
SHORT_REACH = 1.03   # SPH_SHORT_REACH: the fused step's short candidate reach lambda
STATIC_SCRATCH_BYTES = 64 << 20   # SPH_STATIC_SCRATCH_BYTES: sph_step_static's scratch
GRAPH_MAX_STEPS = 1024   # SPH_GRAPH_MAX_STEPS: most steps one step graph captures
KERNEL_TABLE_MAX = 65536          # SPH_KERNEL_TABLE_MAX
KERNEL_TABLE_PAPER = 20000        # the table size of section 4.5
FP64, MIXED = 0, 1

STATE_FIELDS = ("x", "y", "z", "vx", "vy", "vz", "vhx", "vhy", "vhz", "h", "m", "u", "du_m1",
                "p_ref", "rho_ref")
OUT_FIELDS = ("rho", "omega", "p", "c", "c11", "c12", "c13", "c22", "c23", "c33", "ax", "ay",
              "az", "du")
GLOBAL_FIELDS = ("dt", "dt_m1", "t", "mass", "mom0", "mom1", "mom2", "ang0", "ang1", "ang2",
                 "e_kin", "e_int")


class SphError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}")


class _Config(C.Structure):
    _fields_ = [("n", C.c_int64), ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
                ("periodic", C.c_int32 * 3), ("eos", C.c_int32), ("sinc_n", C.c_double),
                ("n_target", C.c_double), ("ng_max", C.c_int32), ("newton_iters", C.c_int32),
                ("h_ratio_max", C.c_double), ("gamma", C.c_double), ("c0", C.c_double),
                ("alpha_av", C.c_double), ("courant", C.c_double), ("dt_growth", C.c_double),
                ("acc_dt", C.c_double), ("energy_dt", C.c_double),
                ("precision", C.c_int32), ("kernel_table", C.c_int32)]


GRAD_FIELDS = ("x", "y", "z", "vx", "vy", "vz", "vhx", "vhy", "vhz", "u", "du_m1")


class _Grads(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in GRAD_FIELDS]


class _Particles(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in
                ("x", "y", "z", "vx", "vy", "vz", "vhx", "vhy", "vhz", "h", "m", "u", "du_m1",
                 "p_ref", "rho_ref", "id") + OUT_FIELDS]


@dataclasses.dataclass
class Config:
    n: int
    box_lo: tuple = (0.0, 0.0, 0.0)
    box_hi: tuple = (1.0, 1.0, 1.0)
    periodic: tuple = (1, 1, 1)
    eos: int = 0
    sinc_n: float = 6.0
    n_target: float = 100.0
    ng_max: int = 160
    newton_iters: int = 2
    h_ratio_max: float = 1.25
    gamma: float = 5.0 / 3.0
    c0: float = 0.0
    alpha_av: float = 1.0
    courant: float = 0.2
    dt_growth: float = 1.1
    acc_dt: float = 0.2
    energy_dt: float = 0.2
    precision: int = FP64
    kernel_table: int = 0   # 0: direct kernel; N: the N-entry table of section 4.5

    @classmethod
    def from_params(cls, n: int, params: dict, **kw) -> "Config":
        keys = set(cls.__dataclass_fields__)
        p = {k: v for k, v in params.items() if k in keys}
        p.update(kw)
        return cls(n=n, **p)

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)

    def c(self) -> _Config:
        s = _Config()
        s.n = int(self.n)
        s.box_lo[:] = [float(v) for v in self.box_lo]
        s.box_hi[:] = [float(v) for v in self.box_hi]
        s.periodic[:] = [int(v) for v in self.periodic]
        s.eos = int(self.eos)
        s.sinc_n = float(self.sinc_n)
        s.n_target = float(self.n_target)
        s.ng_max = int(self.ng_max)
        s.newton_iters = int(self.newton_iters)
        s.h_ratio_max = float(self.h_ratio_max)
        s.gamma = float(self.gamma)
        s.c0 = float(self.c0)
        s.alpha_av = float(self.alpha_av)
        s.courant = float(self.courant)
        s.dt_growth = float(self.dt_growth)
        s.acc_dt = float(self.acc_dt)
        s.energy_dt = float(self.energy_dt)
        s.precision = int(self.precision)
        s.kernel_table = int(self.kernel_table)
        return s


_lib = None
_SIGS = {
    "sph_workspace_bytes": (C.c_size_t, [C.c_void_p]),
    "sph_workspace_init": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sph_build_cells": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sph_update_h": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sph_find_neighbors": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sph_density": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sph_iad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sph_momentum_energy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sph_timestep": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sph_integrate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sph_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sph_neighbors_view": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "sph_order_view": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sph_candidates_view": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sph_status_sync": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sph_step_marked": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_int32]),
    "sph_adjoint_workspace_bytes": (C.c_size_t, [C.c_void_p]),
    "sph_step_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p]),
    "sph_density_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p]),
    "sph_status_string": (C.c_char_p, [C.c_int]),
    "sph_step_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sph_step_graph_create": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_int32, C.c_void_p]),
    "sph_step_graph_launch": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sph_step_graph_destroy": (None, [C.c_void_p]),
    "sph_gravity_workspace_bytes": (C.c_size_t, [C.c_void_p]),
    "sph_gravity": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
}
EXPORTED = tuple(_SIGS)


def lib():
    """Loads libsph.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2005_02656_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _check(st, what):
    if st != SPH_OK:
        raise SphError(st, what)


# --------------------------------------------------------------------------- memory
class Workspace:
    """Caller-owned workspace (a torch uint8 tensor, 256-byte aligned)."""

    def __init__(self, cfg: Config, device="cuda"):
        nbytes = lib().sph_workspace_bytes(C.byref(cfg.c()))
        if nbytes == 0:
            raise SphError(1, "sph_workspace_bytes (invalid config)")
        self.raw = torch.zeros(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.raw.data_ptr()) % 256
        self.buf = self.raw[off:off + nbytes]
        self.nbytes = nbytes

    @property
    def ptr(self):
        return C.c_void_p(self.buf.data_ptr())

    def view(self, ptr: int, count: int, dtype) -> torch.Tensor:
        """Tensor view of `count` elements of dtype at device address ptr inside ws."""
        off = ptr - self.buf.data_ptr()
        esz = torch.empty((), dtype=dtype).element_size()
        if off < 0 or off + count * esz > self.nbytes:
            raise ValueError("view outside the workspace")
        return self.buf[off:off + count * esz].view(dtype)


class Particles:
    """Device arrays of one particle set (torch tensors, FP64 SoA; id int64).
    The FP64 fields of a step's state (SNAP_FIELDS) are the rows of one block,
    so that a checkpoint is one copy."""

    def __init__(self, tensors: dict, block: torch.Tensor = None):
        self.t = tensors
        self.block = block   # (fields, n) FP64 storage of the state rows, or None

    @classmethod
    def from_arrays(cls, arrays: dict, cfg: Config, device="cuda") -> "Particles":
        n = cfg.n
        src = {}
        for k in ("x", "y", "z", "vx", "vy", "vz", "h", "m", "u"):
            src[k] = arrays[k]
        for k, s0 in (("vhx", "vx"), ("vhy", "vy"), ("vhz", "vz")):
            src[k] = arrays.get(k, arrays[s0])
        src["du_m1"] = arrays.get("du_m1", np.zeros(n))
        if cfg.eos == 1:
            src["p_ref"] = arrays["p_ref"]
            src["rho_ref"] = arrays.get("rho_ref", np.zeros(n))
        for k, v in src.items():
            if np.size(v) != n:
                raise ValueError(f"field {k} has {np.size(v)} entries, expected {n}")
        rows = [k for k in SNAP_FIELDS if k in src]
        # rows padded to 256 bytes, so that every field starts aligned
        npad = (n + 31) // 32 * 32
        block = torch.zeros((len(rows), npad), dtype=torch.float64, device=device)
        t = {}
        for i, k in enumerate(rows):
            t[k] = block[i, :n]
            t[k].copy_(torch.as_tensor(src[k], dtype=torch.float64))
        t["id"] = torch.as_tensor(arrays["id"], dtype=torch.int64).to(device).contiguous()
        for k in OUT_FIELDS:
            t[k] = torch.zeros(n, dtype=torch.float64, device=device)
        if t["id"].numel() != n:
            raise ValueError(f"field id has {t['id'].numel()} entries, expected {n}")
        return cls(t, block)

    def __getitem__(self, k):
        return self.t[k]

    def __setitem__(self, k, v):
        self.t[k].copy_(v)

    def c(self) -> _Particles:
        s = _Particles()
        for name, _ in _Particles._fields_:
            v = self.t.get(name)
            setattr(s, name, C.c_void_p(v.data_ptr()) if v is not None else None)
        return s


class Globals:
    """The 14 device doubles of sph_globals."""

    def __init__(self, device="cuda"):
        self.t = torch.zeros(14, dtype=torch.float64, device=device)

    @property
    def ptr(self):
        return C.c_void_p(self.t.data_ptr())

    def host(self) -> dict:
        v = self.t.cpu().tolist()
        return {"dt": v[0], "dt_m1": v[1], "t": v[2], "mass": v[3], "mom": v[4:7],
                "ang": v[7:10], "e_kin": v[10], "e_int": v[11]}


# --------------------------------------------------------------------------- entry points
def workspace_init(cfg: Config, ws: Workspace, stream=None):
    _check(lib().sph_workspace_init(C.byref(cfg.c()), ws.ptr, _stream(stream)), "sph_workspace_init")


def _stage(name):
    def f(cfg: Config, parts: Particles, ws: Workspace, stream=None):
        ps = parts.c()
        _check(getattr(lib(), name)(C.byref(cfg.c()), C.byref(ps), ws.ptr, _stream(stream)), name)
    f.__name__ = name[4:]
    f.__doc__ = f"Enqueues {name} (see include/sph.h)."
    return f


build_cells = _stage("sph_build_cells")
update_h = _stage("sph_update_h")
find_neighbors = _stage("sph_find_neighbors")
density = _stage("sph_density")
iad = _stage("sph_iad")
momentum_energy = _stage("sph_momentum_energy")


def timestep(cfg: Config, g: Globals, ws: Workspace, stream=None):
    _check(lib().sph_timestep(C.byref(cfg.c()), g.ptr, ws.ptr, _stream(stream)), "sph_timestep")


def integrate(cfg: Config, parts: Particles, g: Globals, ws: Workspace, stream=None):
    ps = parts.c()
    _check(lib().sph_integrate(C.byref(cfg.c()), C.byref(ps), g.ptr, ws.ptr, _stream(stream)),
           "sph_integrate")


def step(cfg: Config, parts: Particles, g: Globals, ws: Workspace, stream=None):
    ps = parts.c()
    _check(lib().sph_step(C.byref(cfg.c()), C.byref(ps), g.ptr, ws.ptr, _stream(stream)),
           "sph_step")


class StepGraph:
    """sph_step_graph_*: `steps` consecutive sph_step calls captured once as a
    HIP graph and enqueued by launch() in one go (bit-identical to the calls).
    Keeps the particles, globals and workspace alive: the graph holds their
    device pointers."""

    def __init__(self, cfg: Config, parts: Particles, g: Globals, ws: Workspace, steps: int = 1):
        ps = parts.c()
        h = C.c_void_p()
        _check(lib().sph_step_graph_create(C.byref(cfg.c()), C.byref(ps), g.ptr, ws.ptr,
                                           int(steps), C.byref(h)), "sph_step_graph_create")
        self._h = h
        self.steps = int(steps)
        self._keep = (parts, g, ws)

    def launch(self, stream=None):
        if self._h is None:
            raise RuntimeError("the step graph was closed")
        _check(lib().sph_step_graph_launch(self._h, _stream(stream)), "sph_step_graph_launch")

    def close(self):
        if self._h is not None:
            lib().sph_step_graph_destroy(self._h)
            self._h = None
            self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


STEP_PHASES = ("build_cells", "candidates", "newton_h", "lists", "density", "iad",
               "momentum_energy", "integrate")


def step_static(cfg: Config, parts: Particles, g: Globals, err: torch.Tensor = None,
                stream=None):
    """Enqueues sph_step_static: sph_step with the library's fixed device scratch
    instead of a workspace (no allocation).  err: optional int32 device tensor of
    one element that receives the step's device error bits."""
    if err is not None and (err.dtype != torch.int32 or err.numel() != 1):
        raise ValueError("err must be a one-element int32 tensor")
    ps = parts.c()
    _check(lib().sph_step_static(C.byref(cfg.c()), C.byref(ps), g.ptr,
                                 C.c_void_p(err.data_ptr()) if err is not None else None,
                                 _stream(stream)), "sph_step_static")


class StepMarks:
    """HIP events (torch.cuda.Event, timing enabled) for sph_step_marked: one
    before the step and one after each of its STEP_PHASES phases."""

    def __init__(self, stream=None):
        stream = stream or torch.cuda.current_stream()
        self.events = [torch.cuda.Event(enable_timing=True) for _ in range(len(STEP_PHASES) + 1)]
        for e in self.events:     # torch creates the underlying event on first record
            e.record(stream)
        self.handles = (C.c_void_p * len(self.events))(*[e.cuda_event for e in self.events])

    def phase_ms(self) -> dict:
        """Per-phase durations (ms) of the last marked step (synchronises)."""
        self.events[-1].synchronize()
        return {k: self.events[i].elapsed_time(self.events[i + 1])
                for i, k in enumerate(STEP_PHASES)}


def step_marked(cfg: Config, parts: Particles, g: Globals, ws: Workspace, marks: StepMarks,
                stream=None):
    ps = parts.c()
    _check(lib().sph_step_marked(C.byref(cfg.c()), C.byref(ps), g.ptr, ws.ptr, _stream(stream),
                                 marks.handles, len(marks.events)), "sph_step_marked")


def neighbors_view(cfg: Config, ws: Workspace):
    """Returns (nc, ns, list) tensor views into ws; list has shape
    (ceil(n/64), ng_max, 64): entry j of slot a is list[a // 64, j, a % 64]."""
    nc, ns, lst = C.c_void_p(), C.c_void_p(), C.c_void_p()
    cap = C.c_int32()
    _check(lib().sph_neighbors_view(C.byref(cfg.c()), ws.ptr, C.byref(nc), C.byref(ns),
                                    C.byref(lst), C.byref(cap)), "sph_neighbors_view")
    n = cfg.n
    tiles = (n + 63) // 64
    return (ws.view(nc.value, n, torch.int32), ws.view(ns.value, n, torch.int32),
            ws.view(lst.value, tiles * cap.value * 64, torch.int32).view(tiles, cap.value, 64))


def candidates_view(cfg: Config, ws: Workspace):
    """Returns (nk int32 view, capacity): true candidate counts of the fused step."""
    nk = C.c_void_p()
    cap = C.c_int32()
    _check(lib().sph_candidates_view(C.byref(cfg.c()), ws.ptr, C.byref(nk), C.byref(cap)),
           "sph_candidates_view")
    return ws.view(nk.value, cfg.n, torch.int32), cap.value


def order_view(cfg: Config, ws: Workspace):
    """Returns (keys uint64-as-int64, perm int32) views into ws."""
    k, p = C.c_void_p(), C.c_void_p()
    _check(lib().sph_order_view(C.byref(cfg.c()), ws.ptr, C.byref(k), C.byref(p)),
           "sph_order_view")
    return ws.view(k.value, cfg.n, torch.int64), ws.view(p.value, cfg.n, torch.int32)


def status_sync(ws: Workspace, stream=None):
    """Synchronises the stream; returns (status, bits) and clears the device word."""
    bits = C.c_uint32()
    st = lib().sph_status_sync(ws.ptr, _stream(stream), C.byref(bits))
    return st, bits.value


def status_string(st: int) -> str:
    return lib().sph_status_string(int(st)).decode()


# --------------------------------------------------------------------------- set-up
def initialise(cfg: Config, parts: Particles, ws: Workspace, g: Globals, iters: int = 12,
               kappa: float = 8.0, stream=None):
    """Untimed set-up of a workload: `iters` Newton steps on h from the generator's
    guess (clamped at [h/kappa, kappa h]); with the weakly compressible EOS the
    reference density rho_ref is the density at t = 0.  Leaves the particles in
    key order and the globals at t = 0 with no previous step."""
    workspace_init(cfg, ws, stream)
    build_cells(cfg, parts, ws, stream)
    update_h(cfg.replace(newton_iters=iters, h_ratio_max=kappa), parts, ws, stream)
    if cfg.eos == 1:
        find_neighbors(cfg, parts, ws, stream)
        density(cfg, parts, ws, stream)
        parts.t["rho_ref"].copy_(parts.t["rho"])
    g.t.zero_()


# --------------------------------------------------------------------------- adjoint
class AdjointWorkspace:
    """Caller-owned scratch of the reverse passes (sph_adjoint_workspace_bytes)."""

    def __init__(self, cfg: Config, device="cuda"):
        nbytes = lib().sph_adjoint_workspace_bytes(C.byref(cfg.c()))
        if nbytes == 0:
            raise SphError(1, "sph_adjoint_workspace_bytes (invalid config)")
        self.raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.raw.data_ptr()) % 256
        self.buf = self.raw[off:off + nbytes]

    @property
    def ptr(self):
        return C.c_void_p(self.buf.data_ptr())


class Grads:
    """Adjoints of the 11 fields one step maps (FP64 device tensors, length n)."""

    def __init__(self, n: int, device="cuda"):
        self.t = {k: torch.zeros(n, dtype=torch.float64, device=device) for k in GRAD_FIELDS}

    def __getitem__(self, k):
        return self.t[k]

    def zero_(self):
        for v in self.t.values():
            v.zero_()
        return self

    def c(self) -> _Grads:
        s = _Grads()
        for k in GRAD_FIELDS:
            setattr(s, k, C.c_void_p(self.t[k].data_ptr()))
        return s


def step_backward(cfg: Config, parts: Particles, g: Globals, ws: Workspace,
                  aws: AdjointWorkspace, gout: Grads, gin: Grads, stream=None):
    """Enqueues sph_step_backward: parts/g/ws must hold the step's INPUT state."""
    ps, go, gi = parts.c(), gout.c(), gin.c()
    _check(lib().sph_step_backward(C.byref(cfg.c()), C.byref(ps), g.ptr, ws.ptr, aws.ptr,
                                   C.byref(go), C.byref(gi), _stream(stream)),
           "sph_step_backward")


def density_backward(cfg: Config, parts: Particles, ws: Workspace, aws: AdjointWorkspace,
                     rho_bar: torch.Tensor, xb: torch.Tensor, yb: torch.Tensor, zb: torch.Tensor,
                     stream=None):
    """Enqueues sph_density_backward (gradients in the order before the last cell build)."""
    for t in (rho_bar, xb, yb, zb):
        if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != cfg.n:
            raise ValueError("density_backward takes contiguous FP64 tensors of length n")
    ps = parts.c()
    _check(lib().sph_density_backward(C.byref(cfg.c()), C.byref(ps), ws.ptr, aws.ptr,
                                      C.c_void_p(rho_bar.data_ptr()), C.c_void_p(xb.data_ptr()),
                                      C.c_void_p(yb.data_ptr()), C.c_void_p(zb.data_ptr()),
                                      _stream(stream)), "sph_density_backward")


# --------------------------------------------------------------------------- gravity
class _GravityParams(C.Structure):
    _fields_ = [("G", C.c_double), ("eps", C.c_double), ("theta", C.c_double)]


class GravityWorkspace:
    """Caller-owned tree storage of sph_gravity (sph_gravity_workspace_bytes)."""

    def __init__(self, cfg: Config, device="cuda"):
        nbytes = lib().sph_gravity_workspace_bytes(C.byref(cfg.c()))
        if nbytes == 0:
            raise SphError(1, "sph_gravity_workspace_bytes (invalid config)")
        self.raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.raw.data_ptr()) % 256
        self.buf = self.raw[off:off + nbytes]

    @property
    def ptr(self):
        return C.c_void_p(self.buf.data_ptr())


def gravity(cfg: Config, parts: Particles, ws: Workspace, gws: GravityWorkspace, G: float,
            eps: float, theta: float, out=None, stream=None):
    """Enqueues sph_gravity on the slot order of the last build_cells; returns
    (gx, gy, gz) device tensors per slot."""
    if out is None:
        out = tuple(torch.empty(cfg.n, dtype=torch.float64, device=parts["x"].device)
                    for _ in range(3))
    gp = _GravityParams(float(G), float(eps), float(theta))
    ps = parts.c()
    _check(lib().sph_gravity(C.byref(cfg.c()), C.byref(ps), C.byref(gp), ws.ptr, gws.ptr,
                             *[C.c_void_p(t.data_ptr()) for t in out], _stream(stream)),
           "sph_gravity")
    return out


SNAP_FIELDS = ("x", "y", "z", "vx", "vy", "vz", "vhx", "vhy", "vhz", "h", "m", "u", "du_m1",
               "p_ref", "rho_ref", "id")


def snapshot(parts: Particles, g: Globals) -> dict:
    """Device copy of the state arrays and the globals (a step checkpoint):
    one copy of the state block (its rows are also given by name), the ids and
    the globals."""
    snap = {"_globals": g.t.clone(), "id": parts.t["id"].clone()}
    if parts.block is not None:
        b = parts.block.clone()
        snap["_block"] = b
        n = parts.t["id"].numel()
        rows = [k for k in SNAP_FIELDS if k in parts.t and k != "id"]
        for i, k in enumerate(rows):
            snap[k] = b[i, :n]
    else:
        for k in SNAP_FIELDS:
            if k in parts.t and k != "id":
                snap[k] = parts.t[k].clone()
    return snap


def restore(parts: Particles, g: Globals, snap: dict):
    g.t.copy_(snap["_globals"])
    parts.t["id"].copy_(snap["id"])
    if "_block" in snap and parts.block is not None:
        parts.block.copy_(snap["_block"])
    else:
        for k in SNAP_FIELDS:
            if k in snap and k != "id":
                parts.t[k].copy_(snap[k])


def density_eval(cfg: Config, parts: Particles, ws: Workspace, stream=None):
    """Cell build, h update, lists and density of the current state (the
    rollout's final density evaluation)."""
    build_cells(cfg, parts, ws, stream)
    update_h(cfg, parts, ws, stream)
    find_neighbors(cfg, parts, ws, stream)
    density(cfg, parts, ws, stream)


class Rollout:
    """`steps` forward steps from an initial state with checkpoints every `ckpt`
    steps, then a density evaluation; reverse mode by segments (restore the
    segment's checkpoint, re-run its steps to recover each step's input state,
    then sph_step_backward in reverse order).  The structure (h, dt, lists, AV
    branches) of each step is frozen: the replays reproduce it bit for bit.

    Particles keep their ids; inputs and outputs of the differentiable map are
    keyed by id, in id order."""

    def __init__(self, cfg: Config, parts: Particles, g: Globals, ws: Workspace,
                 steps: int, ckpt: int, aws: AdjointWorkspace = None):
        if cfg.precision != FP64:
            raise ValueError("the adjoint rollout is FP64")
        if steps < 1 or ckpt < 1:
            raise ValueError("steps and ckpt must be >= 1")
        self.cfg, self.parts, self.g, self.ws = cfg, parts, g, ws
        self.steps, self.ckpt = steps, ckpt
        self.aws = aws or AdjointWorkspace(cfg)
        self.initial = snapshot(parts, g)
        self.snaps = {}
        self.final = None

    def set_velocity(self, v0: torch.Tensor):
        """Sets v and v^{n-1/2} of the initial state from v0 (n, 3), keyed by id."""
        idx = self.initial["id"]
        v = v0.to(torch.float64)[idx]
        for k, col in (("vx", 0), ("vy", 1), ("vz", 2)):
            self.initial[k].copy_(v[:, col])
            self.initial["vh" + k[1]].copy_(v[:, col])

    def forward(self) -> torch.Tensor:
        """Runs the rollout; returns the final density keyed by id."""
        cfg, parts, g, ws = self.cfg, self.parts, self.g, self.ws
        restore(parts, g, self.initial)
        self.snaps = {}
        for k in range(self.steps):
            if k % self.ckpt == 0:
                self.snaps[k] = snapshot(parts, g)
            step(cfg, parts, g, ws)
        self.final = snapshot(parts, g)
        density_eval(cfg, parts, ws)
        rho = torch.empty_like(parts["rho"])
        rho[parts["id"]] = parts["rho"]
        return rho

    def backward(self, rho_bar: torch.Tensor) -> Grads:
        """Gradient of <rho_bar, rho_final> with respect to the initial state,
        per slot of the initial order (a Grads)."""
        cfg, parts, g, ws, aws = self.cfg, self.parts, self.g, self.ws, self.aws
        n = cfg.n
        dev = parts["x"].device
        restore(parts, g, self.final)
        density_eval(cfg, parts, ws)
        rb = rho_bar.to(torch.float64)[parts["id"]].contiguous()
        gout, gin = Grads(n, dev), Grads(n, dev)
        density_backward(cfg, parts, ws, aws, rb, gout["x"], gout["y"], gout["z"])
        for s0 in reversed(range(0, self.steps, self.ckpt)):
            s1 = min(s0 + self.ckpt, self.steps)
            restore(parts, g, self.snaps[s0])
            inputs = [self.snaps[s0]]
            for k in range(s0, s1 - 1):
                step(cfg, parts, g, ws)
                inputs.append(snapshot(parts, g))
            for k in reversed(range(s0, s1)):
                restore(parts, g, inputs[k - s0])
                step_backward(cfg, parts, g, ws, aws, gout, gin)
                gout, gin = gin, gout
        return gout

    def velocity_grad(self, grads: Grads) -> torch.Tensor:
        """d/dv0 (keyed by id, (n, 3)) from the initial-state gradient: v0 sets
        both v and v^{n-1/2} of the initial state."""
        idx = self.initial["id"]
        out = torch.zeros((self.cfg.n, 3), dtype=torch.float64, device=idx.device)
        for col, a in enumerate("xyz"):
            out[idx, col] = grads["v" + a] + grads["vh" + a]
        return out


class DensityRollout(torch.autograd.Function):
    """rho_final(v0) of a Rollout as a differentiable torch function of the
    initial velocities v0 (n, 3), both keyed by particle id."""

    @staticmethod
    def forward(ctx, v0, rollout: Rollout):
        rollout.set_velocity(v0.detach())
        ctx.rollout = rollout
        return rollout.forward()

    @staticmethod
    def backward(ctx, rho_bar):
        r = ctx.rollout
        return r.velocity_grad(r.backward(rho_bar.contiguous())), None
