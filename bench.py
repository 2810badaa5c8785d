"""Benchmark of the SPH time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4|c3|c2|c1]
                    [--precision fp64|mixed] [--no-cpu-baseline] [--no-mixed]
                    [--no-adjoint]

A step is one sph_step (Morton sort into cells, Newton h update, neighbour
search, density, IAD, momentum/energy with AV, global dt, integration and
conservation sums) on the synthetic workload with every input resident in HBM.
The set-up (initial conditions, upload, the Newton initialisation of h and the
reference density) is untimed.  The timed steps run through sph_step_marked
(the same launches plus HIP events between phases) so the per-phase times and
the roofline of the longest phase come from the timed steps themselves.  Then,
unless switched off: the same workload in mixed precision, the adjoint/forward
time of the 64^3 rollout, and the FP64 oracle timed on the host on a bounded
sample.  Prints ONE JSON line.
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

# Algorithmic work of each phase of sph_step (the per-unit figures are derived in
# the design notes).  Flops are FP64 operations (an fma counts 2) of the
# arithmetic the phase needs per unit: neighbour pair for the pair passes
# (k_g gather pairs, k_s symmetric pairs per particle), candidate pair for the
# Newton iterations.  Bytes are HBM bytes with every datum read or written once.
FLOPS_PER_PAIR = {
    # r^2 (8), t (1), sinc and x sinc' polynomials (11 + 10 terms: 39), s^n, S,
    # v dS/dv (6), the two sums (2)
    "newton_h": 56,
    # as Newton, with mass-weighted sums (6); in the fused step the list filter
    # does this work for the gather pairs
    "density": 60,
    "lists": 60,
    # r^2, t, sinc polynomial and s^n (33), V W (2), six d_i d_j products summed (15)
    "iad": 50,
    # r^2, W(h_a) and W(h_b) (55), C_a d and C_b d scaled by W (36), v_ab, x.v, AV
    # (16), g, the pressure terms and a (30), e1 and e2 (13)
    "momentum_energy": 160,
}


def bytes_per_particle(phase, k_g, k_s, wc, k_c=0.0, iters=2, fused=True, urec=False):
    """Algorithmic HBM bytes per particle of one phase of sph_step.  urec: the
    momentum records take m and c from slot 0 (equal masses and sound speeds),
    112 bytes instead of 144."""
    rec = 112 if urec else 144
    return {
        # bbox (x y z h), keys, 8 radix passes over 8-byte keys and 4-byte indices,
        # permutation of the state (15 fields with the weakly compressible EOS,
        # else 13, plus the id), packed positions (32 B) and FP32 walk records
        # (16 B), cell table fill
        "build_cells": 32 + 12 + 8 * 24 + (16 if wc else 14) * 16 + 32 + 16 + 8,
        # p4 of the target and the FP32 walk records read, candidate list and
        # count written (k_c candidates per particle)
        "candidates": 32 + 16 + 4 + 4 * k_c,
        # p4 read, candidate list read once per iteration, h written
        "newton_h": 32 + 8 + 4 * k_c * iters,
        # p4 repack, candidates read, counts and the filtered list written, and
        # (fused step) the density's own fields: m u (p_ref rho_ref) in, 4 out
        "lists": 64 + 4 + 4 * k_c + 8 + 4 * k_s + ((64 if wc else 48) if fused else 0),
        # separate density pass (stage path): p4 m u (p_ref rho_ref), list, 4 out
        "density": 0 if fused else (100 if wc else 84) + 4 * k_g,
        # volume pass: m rho p4 in, m/rho and {x y z m/rho} out; the m and c
        # uniformity check; IAD pass: p4 of the target, {x y z m/rho} records,
        # count and list, the record's other sources (m rho omega p c v), C and
        # the momentum records out
        "iad": (16 + 32 + 8 + 32) + 16 + 32 + 32 + 4 + 4 * k_g + 64 + 48 + rec,
        # the target's record, its C rho omega p h, u, counts, list, 4 out
        "momentum_energy": rec + 48 + 24 + 8 + 8 + 8 + 4 * k_s + 32,
        "integrate": 13 * 8 + 4 * 8 + 11 * 8,          # state + rates in, state out
    }[phase]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision timing of the same workload")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward timing of the 64^3 rollout")
    ap.add_argument("--cpu-sample-side", type=int, default=48,
                    help="side of the square-patch lattice the oracle steps on")
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
    """Roofline of the phase that takes the longest.  Both ceilings are evaluated
    (algorithmic HBM bytes against 8 TB/s, algorithmic FP64 flops against the
    78.6 TFLOP/s vector peak); the binding one (larger fraction) is reported."""
    dom = max(phases, key=phases.get)
    t = phases[dom] * 1e-3
    by = bytes_per_particle(dom, k_g, k_s, wc, k_c, iters, fused, urec)
    hbm = by * n / t / 1e9
    kern = PHASE_KERNEL[dom]
    if dom == "momentum_energy" and urec:
        kern = "k_momentum_energy_u"   # the kernel of the 112-byte records
    res = {"kernel": kern, "phase": dom, "phase_ms": phases[dom],
           "traffic": traffic_from_profile(kern, workload)}
    pairs = {"newton_h": iters * k_c * n, "density": k_g * n, "lists": k_g * n,
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
    for mk in marks:
        for k, v in mk.phase_ms().items():
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
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
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
    step_flops = n * (FLOPS_PER_PAIR["newton_h"] * cfg.newton_iters * k_c
                      + FLOPS_PER_PAIR["lists"] * k_g + FLOPS_PER_PAIR["iad"] * k_g
                      + FLOPS_PER_PAIR["momentum_energy"] * k_s)
    out["step_fp64_valu_frac"] = step_flops / (ms * 1e-3) / (FP64_VALU_PEAK_TFLOPS * 1e12)

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
    del parts, ws
    torch.cuda.empty_cache()

    if not args.no_adjoint:
        out["adjoint"] = adjoint_timing(sph, inputs, torch)
        log(f"[bench] adjoint rollout: {out['adjoint']}")

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
