"""Benchmark of the SPH time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4|c3|c2|c1]
                    [--precision fp64|mixed] [--no-cpu-baseline]

A step is one sph_step (Morton sort into cells, Newton h update, neighbour
search, density, IAD, momentum/energy with AV, global dt, integration and
conservation sums) on the synthetic workload with every input resident in HBM.
The set-up (initial conditions, upload, the Newton initialisation of h and the
reference density) is untimed.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X vector FP64

WORKLOADS = {
    "c1": ("lattice 20^3 = 8,000 particles, periodic unit cube, ideal gas", "c1_lattice"),
    "c2": ("rotating square patch 100^3 = 1,000,000 particles, weakly compressible EOS",
           "c2_square_patch"),
    "c3": ("Poisson + Gaussian overdensity, 8,000,000 particles, periodic, ideal gas",
           "c3_gaussian_blob"),
    "c4": ("rotating square patch 400^3 = 64,000,000 particles, weakly compressible EOS",
           "c4_square_patch"),
}

# Algorithmic FP64 flops of each stage per unit (per neighbour pair unless noted),
# counted from the arithmetic the method needs (see the design notes): sinc^n and
# v dS/dv by even polynomials, one sqrt only in the viscosity branch.
FLOPS_PER_PAIR = {
    "update_h": 2 * 30,     # two Newton iterations, ~30 flops per pair each
    "find_neighbors": 10,   # distance test per neighbour
    "density": 45,
    "iad": 35,
    "momentum_energy": 110,
}
# algorithmic HBM bytes per particle of each stage (lists counted where read/written)
def bytes_per_particle(stage, k_g, k_s, wc):
    return {
        "build_cells": 32 + 36 + 24 + (260 if wc else 228) + 8,
        "update_h": 72,
        "find_neighbors": 36 + 4 * k_s + 8,
        "density": (96 if wc else 80) + 4 * k_g,
        "iad": 96 + 4 * k_g,
        "momentum_energy": 176 + 4 * k_s,
        "timestep_integrate": 184,
    }[stage]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stage-timing", action="store_true")
    ap.add_argument("--cpu-sample-side", type=int, default=32,
                    help="side of the square-patch lattice the oracle steps on")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (scales HBM counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stage_times(sph, cfg, parts, g, ws, steps, torch):
    """Average per-stage time (ms) over `steps` steps run stage by stage, with HIP
    events recorded on the stream the library launches on (torch's current one)."""
    names = ["build_cells", "update_h", "find_neighbors", "density", "iad",
             "momentum_energy", "timestep_integrate"]
    acc = {k: 0.0 for k in names}
    for _ in range(steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
        ev[0].record()
        sph.build_cells(cfg, parts, ws); ev[1].record()
        sph.update_h(cfg, parts, ws); ev[2].record()
        sph.find_neighbors(cfg, parts, ws); ev[3].record()
        sph.density(cfg, parts, ws); ev[4].record()
        sph.iad(cfg, parts, ws); ev[5].record()
        sph.momentum_energy(cfg, parts, ws); ev[6].record()
        sph.timestep(cfg, g, ws)
        sph.integrate(cfg, parts, g, ws); ev[7].record()
        torch.cuda.synchronize()
        for i, k in enumerate(names):
            acc[k] += ev[i].elapsed_time(ev[i + 1])
    return {k: v / steps for k, v in acc.items()}


def cpu_baseline(side):
    """The oracle (never tuned) stepping a side^3 rotating square patch once."""
    import oracle
    from paper_2005_02656_amd import inputs
    w = inputs.square_patch(side)
    keys = set(oracle.Config.__dataclass_fields__)
    ocfg = oracle.Config(**{k: v for k, v in w.params.items() if k in keys})
    st = {k: np.array(v, copy=True) for k, v in w.arrays.items()}
    st["h"] = oracle.initial_h(ocfg, st)
    st["rho_ref"] = oracle.density(ocfg, st["x"], st["y"], st["z"], st["h"], st["m"], st["u"],
                                   st["p_ref"], np.zeros(w.n))[0]
    st.update(vhx=st["vx"].copy(), vhy=st["vy"].copy(), vhz=st["vz"].copy(),
              du_m1=np.zeros(w.n))
    t0 = time.perf_counter()
    oracle.step(ocfg, st, {"dt_m1": 0.0, "t": 0.0})
    t = time.perf_counter() - t0
    return {"value": w.n / t, "unit": "particle-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"one full step of the brute-force O(N^2) FP64 oracle on a {side}^3 "
                      f"= {w.n} particle rotating square patch (same recipe as the workload, "
                      f"smaller); {t:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design, not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2005_02656_amd import inputs, sph

    desc, gen = WORKLOADS[args.workload]
    t0 = time.time()
    w = getattr(inputs, gen)()
    prec = sph.FP64 if args.precision == "fp64" else sph.MIXED
    cfg = sph.Config.from_params(w.n, w.params, precision=prec)
    log(f"[bench] {args.workload}: {desc}; IC ready in {time.time() - t0:.1f}s")
    parts = sph.Particles.from_arrays(w.arrays, cfg)
    ws = sph.Workspace(cfg)
    g = sph.Globals()
    del w
    sph.initialise(cfg, parts, ws, g)
    st, bits = sph.status_sync(ws)
    if st:
        raise RuntimeError(f"set-up raised {sph.status_string(st)} (bits {bits})")
    log(f"[bench] set-up done in {time.time() - t0:.1f}s; ws {ws.nbytes / 2**30:.1f} GiB")

    for i in range(args.warmup):
        sph.step(cfg, parts, g, ws)
    torch.cuda.synchronize()
    st, bits = sph.status_sync(ws)
    if st:
        raise RuntimeError(f"warm-up raised {sph.status_string(st)} (bits {bits})")
    log("[bench] warm-up done")

    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(args.steps):
        sph.step(cfg, parts, g, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    st, bits = sph.status_sync(ws)
    if st:
        raise RuntimeError(f"timed steps raised {sph.status_string(st)} (bits {bits})")
    log(f"[bench] {args.steps} timed steps: {ms:.3f} ms/step")

    nc, ns, _ = sph.neighbors_view(cfg, ws)
    k_g = float(nc.double().mean())
    k_s = float(ns.double().mean())
    pairs_g = float(nc.double().sum())
    pairs_s = float(ns.double().sum())
    n = cfg.n
    wc = cfg.eos == 1

    out = {
        "metric": "particle-updates/s per SPH step at 1 MI355X",
        "value": n / (ms * 1e-3),
        "unit": "particle-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == sph.FP64 else "f32-pair/f64-accumulate",
        "data": "synthetic",
        "config": {"workload": desc, "particles": n, "neighbours_gather_mean": k_g,
                   "neighbours_symmetric_mean": k_s, "ng_max": cfg.ng_max,
                   "newton_iters": cfg.newton_iters},
    }

    if not args.no_stage_timing:
        stt = stage_times(sph, cfg, parts, g, ws, args.steps, torch)
        out["stage_ms"] = {k: round(v, 4) for k, v in stt.items()}
        dom = max(stt, key=stt.get)
        t = stt[dom] * 1e-3
        unit_pairs = {"update_h": pairs_g, "find_neighbors": pairs_s, "density": pairs_g,
                      "iad": pairs_g, "momentum_energy": pairs_s}
        if dom in FLOPS_PER_PAIR:
            fl = FLOPS_PER_PAIR[dom] * unit_pairs[dom]
            ach = fl / t / 1e12
            out["roofline"] = {"bound": "alu", "kernel": dom, "achieved": ach,
                               "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": ach / FP64_VALU_PEAK_TFLOPS, "traffic": None,
                               "algorithmic": f"{FLOPS_PER_PAIR[dom]} FP64 flops per neighbour "
                                              f"pair x {unit_pairs[dom]:.3e} pairs"}
        else:
            by = bytes_per_particle(dom, k_g, k_s, wc) * n
            ach = by / t / 1e9
            out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": ach,
                               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                               "traffic": None,
                               "algorithmic": f"{bytes_per_particle(dom, k_g, k_s, wc)} B per "
                                              f"particle x {n} particles"}
        step_bytes = sum(bytes_per_particle(s, k_g, k_s, wc) for s in stt) * n
        out["step_hbm_frac"] = step_bytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)

    if args.calib_copy_mib > 0:
        # a plain copy of known size: its FETCH_SIZE/WRITE_SIZE counters calibrate
        # the byte counters of the SPH kernels in the same profiled run
        nbytes = args.calib_copy_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = nbytes
        del src, dst

    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_side)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
