"""Benchmark of the SPH time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4|c3|c2|c1]
                    [--precision fp64|mixed] [--no-cpu-baseline] [--no-graph]
                    [--no-mixed] [--no-adjoint] [--no-table] [--no-gravity]
                    [--oracle-points]

A step is one sph_step (Morton sort into cells, Newton h update, neighbour
search, density, IAD, momentum/energy with AV, global dt, integration and
conservation sums) on the synthetic workload with every input resident in HBM.
The set-up (initial conditions, upload, the Newton initialisation of h and the
reference density) is untimed.  The timed steps run through sph_step_marked
(the same launches plus HIP events between phases) so the per-phase times and
the roofline of the longest phase come from the timed steps themselves.  Then,
unless switched off: the same steps replayed from a one-step HIP graph, the
same workload in mixed precision, the kernel
lookup-table variant (FP64 and mixed), the adjoint/forward
time of the 64^3 rollout, the self-gravity tree walk on an 8 M-particle sphere,
and the FP64 oracle timed on the host on a bounded sample.  Prints ONE JSON line.
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

# Algorithmic work of each phase of sph_step: what the method itself must do,
# independent of how this implementation does it.  Flops are FP64 operations (an
# fma counts 2) of the SPH arithmetic per pair, with the kernel S_n evaluated as
# an even polynomial in v^2 (no sqrt, sin or pow per pair): Newton ~30 per
# candidate pair and iteration, density and Omega ~45 and IAD ~35 per gather
# pair, momentum, energy and viscosity ~110 per symmetric pair.  The candidate
# distance tests of the search are not counted (their number depends on the cell
# structure, not on the method).
FLOPS_PER_PAIR = {"newton_h": 30, "lists": 45, "density": 45, "iad": 35,
                  "momentum_energy": 110}


def bytes_per_particle(phase, k_g, k_s, wc, k_c=0.0, iters=2, fused=True, urec=False):
    """Algorithmic HBM bytes per particle of one phase of sph_step: every FP64
    state field and int32 list entry the phase must read or write, once.  The
    neighbours' fields are taken as served from the caches (the measured
    counter traffic against this figure is the cache amplification).  Per kernel:
    bbox 32, keys 36, sort 24 (one read and one write of key and index), permute
    228 (ideal gas) / 260 (weakly compressible), cells 8, Newton 72 (x y z h per
    iteration + h out), neighbours 36 (x y z h in, counts out), density 80 / 96,
    IAD 96, momentum/energy 176, integrate 184, and the neighbour list written
    once and read by density, IAD and momentum (4 k_s each).  The step total is
    972 + 16 k_s (ideal gas) or 1,020 + 16 k_s (weakly compressible)."""
    lst = 4.0 * k_s
    return {
        "build_cells": 32 + 36 + 24 + (260 if wc else 228) + 8,
        "candidates": 0.0,
        "newton_h": 32 * iters + 8,
        # neighbour search (write of the list) and, in the fused step, the
        # density formed while the list is filtered (its list read counted here)
        "lists": 36 + lst + ((96 if wc else 80) + lst if fused else 0.0),
        "density": 0.0 if fused else (96 if wc else 80) + lst,
        "iad": 96 + lst,
        "momentum_energy": 176 + lst,
        "integrate": 184,
    }[phase]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the timing of the step replayed from a HIP graph")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision timing of the same workload")
    ap.add_argument("--no-gravity", action="store_true",
                    help="skip the timing of the self-gravity tree walk")
    ap.add_argument("--no-table", action="store_true",
                    help="skip the timing of the kernel lookup-table variant")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward timing of the 64^3 rollout")
    ap.add_argument("--cpu-sample-side", type=int, default=48,
                    help="side of the square-patch lattice the oracle steps on")
    ap.add_argument("--oracle-points", action="store_true",
                    help="also time the oracle on the 20^3 and 32^3 lattices, all cores and one")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (scales HBM counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the kernel that does the work of each phase (its rocprofv3 name)
PHASE_KERNEL = {"build_cells": "k_radix_scatter", "candidates": "k_candidates",
                "newton_h": "k_update_h_list", "lists": "k_filter", "density": "k_density",
                "iad": "k_iad", "momentum_energy": "k_momentum_energy",
                "integrate": "k_integrate"}


def traffic_from_profile(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary of this
    workload, or None when there is none or the sources changed since."""
    from paper_2005_02656_amd import profiling
    s = profiling.read_summary(os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md"))
    if not s or s.get("source_digest") != profiling.source_digest():
        return None
    try:
        return float(s["fetch_bytes_per_launch"]) + float(s["write_bytes_per_launch"])
    except KeyError:
        return None


def roofline(phases, n, k_g, k_s, wc, iters, k_c, workload, fused, urec=False):
    """Roofline of the phase that takes the longest among those the method's
    own work is counted for (the candidate walk of the fused search has none:
    its tests depend on the cell structure).  Both ceilings are evaluated
    (algorithmic HBM bytes against 8 TB/s, algorithmic FP64 flops against the
    78.6 TFLOP/s vector peak); the binding one (larger fraction) is reported."""
    counted = [k for k in phases
               if bytes_per_particle(k, k_g, k_s, wc, k_c, iters, fused, urec) > 0]
    dom = max(counted, key=phases.get)
    t = phases[dom] * 1e-3
    by = bytes_per_particle(dom, k_g, k_s, wc, k_c, iters, fused, urec)
    hbm = by * n / t / 1e9
    kern = PHASE_KERNEL[dom]
    traffic = traffic_from_profile(kern, workload)
    res = {"kernel": kern, "phase": dom, "phase_ms": phases[dom], "traffic": traffic,
           "algorithmic_bytes": by * n,
           "traffic_over_algorithmic": traffic / (by * n) if traffic else None}
    pairs = {"newton_h": iters * k_s * n, "density": k_g * n, "lists": k_g * n,
             "iad": k_g * n, "momentum_energy": k_s * n}
    if dom in FLOPS_PER_PAIR and pairs.get(dom):
        fl = FLOPS_PER_PAIR[dom] * pairs[dom]
        alu = fl / t / 1e12
        res["alt"] = {"bound": "hbm", "achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": hbm / HBM_PEAK_GBS}
        if alu / FP64_VALU_PEAK_TFLOPS >= hbm / HBM_PEAK_GBS:
            res.update(bound="alu", achieved=alu, peak=FP64_VALU_PEAK_TFLOPS, unit="TFLOP/s",
                       frac=alu / FP64_VALU_PEAK_TFLOPS,
                       algorithmic=f"{FLOPS_PER_PAIR[dom]} FP64 flops per pair x "
                                   f"{pairs[dom]:.4e} pairs")
            return res
    res.update(bound="hbm", achieved=hbm, peak=HBM_PEAK_GBS, unit="GB/s",
               frac=hbm / HBM_PEAK_GBS,
               algorithmic=f"{by:.1f} B per particle x {n} particles")
    return res


def adjoint_timing(sph, inputs, torch, steps=20, ckpt=5):
    """Forward and reverse time of the 64^3 lattice rollout (20 steps, a
    checkpoint every 5, density loss against a seeded target field)."""
    w = inputs.c5_lattice()
    cfg = sph.Config.from_params(w.n, w.params)
    parts = sph.Particles.from_arrays(w.arrays, cfg)
    ws = sph.Workspace(cfg)
    g = sph.Globals()
    sph.initialise(cfg, parts, ws, g)
    target = torch.tensor(inputs.c5_target_density(w.n), device="cuda")
    v0 = torch.tensor(np.stack([w.arrays["vx"], w.arrays["vy"], w.arrays["vz"]], 1),
                      device="cuda", requires_grad=True)
    ro = sph.Rollout(cfg, parts, g, ws, steps=steps, ckpt=ckpt)
    for _ in range(2):   # first pass warms up
        v0.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rho = sph.DensityRollout.apply(v0, ro)
        loss = 0.5 * ((rho - target) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    st, bits = sph.status_sync(ws)
    if st:
        raise RuntimeError(f"adjoint rollout raised {sph.status_string(st)} (bits {bits})")
    fwd, bwd = (t1 - t0) * 1e3, (t2 - t1) * 1e3
    return {"workload": f"lattice 64^3 = {w.n} particles, {steps}-step rollout, checkpoint "
                        f"every {ckpt}, loss 1/2|rho - rho*|^2, gradient w.r.t. v0",
            "forward_ms": fwd, "backward_ms": bwd, "adjoint_over_forward": bwd / fwd,
            "loss": float(loss.item()), "grad_norm": float(v0.grad.norm().item())}


def gravity_timing(sph, inputs, torch, n=8_000_000, theta=0.5, eps=1e-3, reps=3):
    """sph_gravity on an Evrard sphere (rho = 1/(2 pi r), radius and mass 1) at
    opening angle theta: tree build and walk, after the cell build."""
    w = inputs.evrard_sphere(n)
    cfg = sph.Config.from_params(w.n, w.params)
    parts = sph.Particles.from_arrays(w.arrays, cfg)
    ws = sph.Workspace(cfg)
    sph.workspace_init(cfg, ws)
    gws = sph.GravityWorkspace(cfg)
    sph.build_cells(cfg, parts, ws)
    out = sph.gravity(cfg, parts, ws, gws, 1.0, eps, theta)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sph.gravity(cfg, parts, ws, gws, 1.0, eps, theta, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    st, bits = sph.status_sync(ws)
    if st:
        raise RuntimeError(f"gravity raised {sph.status_string(st)} (bits {bits})")
    res = {"workload": f"Evrard sphere, {n} particles, theta {theta}, Plummer eps {eps}",
           "ms": ms, "particles_per_s": n / (ms * 1e-3)}
    del parts, ws, gws, out
    torch.cuda.empty_cache()
    return res


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


def oracle_points():
    """The oracle's throughput on the 20^3 lattice (8,000 particles) and on a 32^3
    lattice (32,768), one full step each from the generator's state, on all host
    cores and on one (the brute-force cost does not depend on h)."""
    import oracle
    from paper_2005_02656_amd import inputs
    keys = set(oracle.Config.__dataclass_fields__)
    allc = oracle.num_threads()
    pts = []
    for side in (20, 32):
        w = inputs.lattice(side, seed=1, sigma_v=0.01)
        ocfg = oracle.Config(**{k: v for k, v in w.params.items() if k in keys})
        st = {k: np.array(v, copy=True) for k, v in w.arrays.items()}
        st.update(vhx=st["vx"].copy(), vhy=st["vy"].copy(), vhz=st["vz"].copy(),
                  du_m1=np.zeros(w.n))
        for cores in (allc, 1):
            oracle.set_num_threads(cores)
            t0 = time.perf_counter()
            oracle.step(ocfg, st, {"dt_m1": 0.0, "t": 0.0})
            t = time.perf_counter() - t0
            pts.append({"workload": f"lattice {side}^3 = {w.n} particles, one step",
                        "cores": cores, "seconds": t, "value": w.n / t})
    oracle.set_num_threads(allc)
    return pts


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library "
              "has no multi-GPU decomposition", file=sys.stderr)
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
    marks = [sph.StepMarks(stream) for _ in range(args.steps)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(args.steps):
        sph.step_marked(cfg, parts, g, ws, marks[i])
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    st, bits = sph.status_sync(ws)
    if st:
        raise RuntimeError(f"timed steps raised {sph.status_string(st)} (bits {bits})")
    phases = {k: 0.0 for k in sph.STEP_PHASES}
    per_step = []
    for mk in marks:
        pm = mk.phase_ms()
        per_step.append(sum(pm.values()))
        for k, v in pm.items():
            phases[k] += v / args.steps
    log(f"[bench] {args.steps} timed steps: {ms:.3f} ms/step; phases "
        + " ".join(f"{k}={v:.2f}" for k, v in phases.items()))

    nc, ns, _ = sph.neighbors_view(cfg, ws)
    k_g = float(nc.double().mean())
    k_s = float(ns.double().mean())
    n = cfg.n
    wc = cfg.eos == 1
    # equal masses under the weakly compressible EOS (c = c0): the momentum
    # pass reads its 112-byte neighbour records
    urec = wc and bool(torch.all(parts["m"] == parts["m"][0]))

    out = {
        "metric": "particle-updates/s per SPH step at 1 MI355X",
        "value": n / (ms * 1e-3),
        "unit": "particle-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "ms_per_step_median": float(np.median(per_step)),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == sph.FP64 else "f32-pair/f64-accumulate",
        "data": "synthetic",
        "config": {"workload": desc, "particles": n, "neighbours_gather_mean": k_g,
                   "neighbours_symmetric_mean": k_s, "ng_max": cfg.ng_max,
                   "newton_iters": cfg.newton_iters},
        "phase_ms": {k: round(v, 4) for k, v in phases.items()},
    }
    k_c = 0.0
    if cfg.h_ratio_max <= 1.25:
        nk, _ = sph.candidates_view(cfg, ws)
        k_c = float(nk.double().mean())
        out["config"]["candidates_mean"] = k_c
    out["roofline"] = roofline(phases, n, k_g, k_s, wc, cfg.newton_iters, k_c, args.workload,
                               cfg.h_ratio_max <= 1.25, urec)
    fused = cfg.h_ratio_max <= 1.25
    step_bytes = sum(bytes_per_particle(k, k_g, k_s, wc, k_c, cfg.newton_iters, fused, urec)
                     for k in phases) * n
    out["step_hbm_frac"] = step_bytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)
    step_flops = n * (FLOPS_PER_PAIR["newton_h"] * cfg.newton_iters * k_s
                      + FLOPS_PER_PAIR["lists"] * k_g + FLOPS_PER_PAIR["iad"] * k_g
                      + FLOPS_PER_PAIR["momentum_energy"] * k_s)
    out["step_fp64_valu_frac"] = step_flops / (ms * 1e-3) / (FP64_VALU_PEAK_TFLOPS * 1e12)

    if not args.no_graph:
        # the same step replayed from a one-step HIP graph (sph_step_graph):
        # what the eager steps lose to launching ~40 kernels one by one
        sg = sph.StepGraph(cfg, parts, g, ws, steps=1)
        sg.launch(stream)
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(args.steps):
            sg.launch(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        gms = e0.elapsed_time(e1) / args.steps
        sg.close()
        st, bits = sph.status_sync(ws)
        if st:
            raise RuntimeError(f"graph steps raised {sph.status_string(st)} (bits {bits})")
        out["graph"] = {"ms_per_step": gms, "value": n / (gms * 1e-3),
                        "note": "the same step replayed from a one-step HIP graph"}
        log(f"[bench] graph replay: {gms:.3f} ms/step")

    if not args.no_mixed and prec == sph.FP64:
        mcfg = cfg.replace(precision=sph.MIXED)
        sph.step(mcfg, parts, g, ws)
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(args.steps):
            sph.step_marked(mcfg, parts, g, ws, marks[i])
        e1.record(stream)
        torch.cuda.synchronize()
        mms = e0.elapsed_time(e1) / args.steps
        mph = {k: 0.0 for k in sph.STEP_PHASES}
        for mk in marks:
            for k, v in mk.phase_ms().items():
                mph[k] += v / args.steps
        st, bits = sph.status_sync(ws)
        if st:
            raise RuntimeError(f"mixed steps raised {sph.status_string(st)} (bits {bits})")
        out["mixed"] = {"ms_per_step": mms, "value": n / (mms * 1e-3),
                        "speedup_vs_fp64": ms / mms,
                        "phase_ms": {k: round(v, 4) for k, v in mph.items()},
                        "note": "same workload and state, FP32 pair terms with FP64 sums"}
        log(f"[bench] mixed precision: {mms:.3f} ms/step")
    if not args.no_table:
        # the kernel lookup table of section 4.5 (20,000 values, linear
        # interpolation in v) in place of the fitted polynomials, same state
        out["kernel_table"] = {"entries": sph.KERNEL_TABLE_PAPER}
        for name, pr in (("fp64", sph.FP64), ("mixed", sph.MIXED)):
            tcfg = cfg.replace(precision=pr, kernel_table=sph.KERNEL_TABLE_PAPER)
            sph.step(tcfg, parts, g, ws)
            torch.cuda.synchronize()
            e0.record(stream)
            for i in range(args.steps):
                sph.step_marked(tcfg, parts, g, ws, marks[i])
            e1.record(stream)
            torch.cuda.synchronize()
            tms = e0.elapsed_time(e1) / args.steps
            tph = {k: 0.0 for k in sph.STEP_PHASES}
            for mk in marks:
                for k, v in mk.phase_ms().items():
                    tph[k] += v / args.steps
            st, bits = sph.status_sync(ws)
            if st:
                raise RuntimeError(f"table steps raised {sph.status_string(st)} (bits {bits})")
            out["kernel_table"][name] = {"ms_per_step": tms,
                                         "phase_ms": {k: round(v, 4) for k, v in tph.items()}}
        log(f"[bench] kernel table: {out['kernel_table']}")
    del parts, ws
    torch.cuda.empty_cache()

    if not args.no_adjoint:
        out["adjoint"] = adjoint_timing(sph, inputs, torch)
        log(f"[bench] adjoint rollout: {out['adjoint']}")

    if not args.no_gravity:
        out["gravity"] = gravity_timing(sph, inputs, torch)
        log(f"[bench] gravity: {out['gravity']}")

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
        if args.oracle_points:
            out["cpu_baseline"]["points"] = oracle_points()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
