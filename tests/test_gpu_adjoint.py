"""GPU parity of the reverse mode: sph_step_backward, sph_density_backward and the
checkpointed rollout, through the C ABI, against the differentiable FP64 oracle
(oracle/torch_adjoint.py, itself pinned to central differences of the C oracle
by test_oracle_adjoint.py).

The oracle takes its frozen structure (Newton h, dt) from the C oracle, never
from the GPU.  Gradients are compared field by field relative to the field's
largest entry.  Bar: 1e-12, the FP64 field bar, for one step, the density and a
3-step rollout (both sides are FP64; the residual is summation order and the
1e-16-level differences between the GPU's and the oracle's own h and dt; the
measured errors are below 1e-13)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import torch_adjoint as TA
from paper_2005_02656_amd import inputs, sph
from gpu_support import Run, configs, rel_err

pytestmark = pytest.mark.gpu
TOL_STEP = 1e-12
TOL_ROLLOUT = 1e-12
NG = 400


def _jitter(a, rng, s):
    for k in "xyz":
        a[k] = np.mod(a[k] + rng.normal(0, s, a[k].size), 1.0)


def step_case(name):
    """(workload, arrays, dt_m1) of one single-step case, arrays in id order."""
    rng = np.random.default_rng(21)
    if name == "lattice9":       # jittered lattice, Adams-Bashforth step
        w = inputs.lattice(9, seed=2, sigma_v=0.05)
        a = dict(w.arrays)
        _jitter(a, rng, 0.01)
        dt_m1 = 0.004
    elif name == "random":       # variable h (symmetric-only list entries), first step
        w = inputs.random_periodic(1501, seed=6, h_lo=0.10, h_hi=0.13)
        a = dict(w.arrays)
        dt_m1 = 0.0
    else:                        # square patch: open x, y; weakly compressible EOS
        w = inputs.square_patch(8)
        a = dict(w.arrays)
        a["rho_ref"] = np.full(w.n, 0.97)
        dt_m1 = 0.002
    n = w.n
    a["vhx"] = a["vx"] + rng.normal(0, 0.01, n)
    a["vhy"] = a["vy"] + rng.normal(0, 0.01, n)
    a["vhz"] = a["vz"] - rng.normal(0, 0.01, n)
    a["du_m1"] = rng.normal(0, 0.1, n)
    a["u"] = a["u"] * (1.0 + 0.1 * rng.random(n))
    return w, a, dt_m1


STEP_CASES = ("lattice9", "random", "patch")


def _torch_state(a):
    return {"x": torch.tensor(np.stack([a["x"], a["y"], a["z"]], 1), requires_grad=True),
            "v": torch.tensor(np.stack([a["vx"], a["vy"], a["vz"]], 1), requires_grad=True),
            "vh": torch.tensor(np.stack([a["vhx"], a["vhy"], a["vhz"]], 1), requires_grad=True),
            "u": torch.tensor(a["u"], requires_grad=True),
            "du_m1": torch.tensor(a["du_m1"], requires_grad=True)}


def _weights(n, seed):
    rng = np.random.default_rng(seed)
    return {k: rng.normal(size=n) for k in sph.GRAD_FIELDS}


@pytest.mark.parametrize("name", STEP_CASES)
def test_step_backward_matches_oracle(name):
    w, a, dt_m1 = step_case(name)
    n = w.n
    cfg, ocfg = configs(w, ng_max=NG)
    W = _weights(n, 5)
    # oracle: frozen structure from the C oracle's step, gradient by autograd
    st = dict(a)
    new, gl, f = oracle.step(ocfg, st, {"dt_m1": dt_m1, "t": 0.0})
    S = TA.Setup(ocfg, a["m"], f["h"])
    ts = _torch_state(a)
    out, _ = TA.step(S, ts, gl["dt"], dt_m1, a.get("p_ref"), a.get("rho_ref"))
    T = {k: torch.tensor(v) for k, v in W.items()}
    L = ((T["x"] * out["x"][:, 0]).sum() + (T["y"] * out["x"][:, 1]).sum()
         + (T["z"] * out["x"][:, 2]).sum() + (T["vx"] * out["v"][:, 0]).sum()
         + (T["vy"] * out["v"][:, 1]).sum() + (T["vz"] * out["v"][:, 2]).sum()
         + (T["vhx"] * out["vh"][:, 0]).sum() + (T["vhy"] * out["vh"][:, 1]).sum()
         + (T["vhz"] * out["vh"][:, 2]).sum() + (T["u"] * out["u"]).sum()
         + (T["du_m1"] * out["du_m1"]).sum())
    L.backward()
    col = lambda g, c: None if g is None else g[:, c]
    ref = {"x": col(ts["x"].grad, 0), "y": col(ts["x"].grad, 1), "z": col(ts["x"].grad, 2),
           "vx": col(ts["v"].grad, 0), "vy": col(ts["v"].grad, 1), "vz": col(ts["v"].grad, 2),
           "vhx": col(ts["vh"].grad, 0), "vhy": col(ts["vh"].grad, 1),
           "vhz": col(ts["vh"].grad, 2), "u": ts["u"].grad, "du_m1": ts["du_m1"].grad}
    # GPU: a forward step tells the output slot order; the backward replays the
    # step from the same input state
    probe = Run(w, cfg, a)
    probe.g.t[1] = dt_m1
    sph.step(cfg, probe.parts, probe.g, probe.ws)
    assert probe.status() == (0, 0)
    out_ids = probe.ids()
    r = Run(w, cfg, a)
    r.g.t[1] = dt_m1
    gout, gin = sph.Grads(n), sph.Grads(n)
    for k in sph.GRAD_FIELDS:
        gout[k].copy_(torch.from_numpy(W[k][out_ids]))
    aws = sph.AdjointWorkspace(cfg)
    sph.step_backward(cfg, r.parts, r.g, r.ws, aws, gout, gin)
    assert r.status() == (0, 0)
    assert np.array_equal(r.ids(), out_ids)
    errs = {}
    for k in sph.GRAD_FIELDS:
        # torch leaves the gradient of an input that reaches no output (du_m1 on
        # a first step) at None: it is zero
        o = ref[k].numpy() if ref[k] is not None else np.zeros(n)
        errs[k] = rel_err(gin[k].cpu().numpy(), o)
    print(name, "dt", gl["dt"], {k: f"{v:.1e}" for k, v in errs.items()})
    for k, e in errs.items():
        assert e <= TOL_STEP, (k, e)


@pytest.mark.parametrize("name", STEP_CASES)
def test_density_backward_matches_oracle(name):
    w, a, _ = step_case(name)
    n = w.n
    cfg, ocfg = configs(w, ng_max=NG)
    wr = np.random.default_rng(8).normal(size=n)
    h = oracle.update_h(ocfg, a["x"], a["y"], a["z"], a["h"])
    x = torch.tensor(np.stack([a["x"], a["y"], a["z"]], 1), requires_grad=True)
    rho, _ = TA.density_omega(TA.Setup(ocfg, a["m"], h), x)
    (rho * torch.tensor(wr)).sum().backward()
    r = Run(w, cfg, a)
    sph.density_eval(cfg, r.parts, r.ws)
    rb = torch.from_numpy(wr[r.ids()]).cuda()
    xb, yb, zb = (torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3))
    aws = sph.AdjointWorkspace(cfg)
    sph.density_backward(cfg, r.parts, r.ws, aws, rb, xb, yb, zb)
    assert r.status() == (0, 0)
    for c, g in enumerate((xb, yb, zb)):
        e = rel_err(g.cpu().numpy(), x.grad[:, c].numpy())
        print(name, "density x_bar", c, f"{e:.1e}")
        assert e <= TOL_STEP


def test_step_backward_bitwise_reproducible():
    w, a, dt_m1 = step_case("random")
    cfg, _ = configs(w, ng_max=NG)
    W = _weights(w.n, 6)
    res = []
    for _ in range(2):
        r = Run(w, cfg, a)
        r.g.t[1] = dt_m1
        gout, gin = sph.Grads(w.n), sph.Grads(w.n)
        for k in sph.GRAD_FIELDS:
            gout[k].copy_(torch.from_numpy(W[k]))
        sph.step_backward(cfg, r.parts, r.g, r.ws, sph.AdjointWorkspace(cfg), gout, gin)
        res.append(np.stack([gin[k].cpu().numpy() for k in sph.GRAD_FIELDS]))
    assert np.array_equal(res[0].view(np.uint64), res[1].view(np.uint64))


def _frozen_step(cfg, r, dt, dt_m1):
    """The step map with its structure frozen, from the stage entry points: no
    h update (h is the input's), dt given."""
    sph.build_cells(cfg, r.parts, r.ws)
    sph.find_neighbors(cfg, r.parts, r.ws)
    sph.density(cfg, r.parts, r.ws)
    sph.iad(cfg, r.parts, r.ws)
    sph.momentum_energy(cfg, r.parts, r.ws)
    r.g.t[0] = dt
    r.g.t[1] = dt_m1
    sph.integrate(cfg, r.parts, r.g, r.ws)


def test_step_backward_finite_differences():
    """<gin, delta> against central differences of the GPU's own frozen-structure
    step (stage entry points, h and dt held), in 3 random directions over all
    inputs plus 10 single components."""
    w, a, dt_m1 = step_case("lattice9")
    n = w.n
    cfg, _ = configs(w, ng_max=NG, newton_iters=0)   # the backward's replay keeps h
    W = _weights(n, 7)
    r = Run(w, cfg, a)
    r.g.t[1] = dt_m1
    gout, gin = sph.Grads(n), sph.Grads(n)
    probe = Run(w, cfg, a)
    probe.g.t[1] = dt_m1
    sph.step(cfg, probe.parts, probe.g, probe.ws)
    dt = float(probe.g.t[0].item())
    for k in sph.GRAD_FIELDS:
        gout[k].copy_(torch.from_numpy(W[k][probe.ids()]))
    sph.step_backward(cfg, r.parts, r.g, r.ws, sph.AdjointWorkspace(cfg), gout, gin)
    assert abs(float(r.g.t[0].item()) - dt) == 0.0
    G = {k: gin[k].cpu().numpy() for k in sph.GRAD_FIELDS}

    def loss(arr):
        q = Run(w, cfg, arr)
        _frozen_step(cfg, q, dt, dt_m1)
        ids = q.ids()
        return float(sum((W[k][ids] * q.parts[k].cpu().numpy()).sum() for k in sph.GRAD_FIELDS))

    rng = np.random.default_rng(17)
    dirs = []
    for _ in range(3):
        dirs.append({k: rng.normal(size=n) for k in sph.GRAD_FIELDS})
    for c in rng.choice(n, 10, replace=False):
        k = sph.GRAD_FIELDS[int(rng.integers(len(sph.GRAD_FIELDS)))]
        d = {f: np.zeros(n) for f in sph.GRAD_FIELDS}
        d[k][c] = 1.0
        dirs.append(d)
    for d in dirs:
        eps = 1e-6
        ap, am = dict(a), dict(a)
        for k in sph.GRAD_FIELDS:
            ap[k] = a[k] + eps * d[k]
            am[k] = a[k] - eps * d[k]
        for k in "xyz":   # stay inside the periodic box (the wrap is a constant shift)
            ap[k] = np.mod(ap[k], 1.0)
            am[k] = np.mod(am[k], 1.0)
        fd = (loss(ap) - loss(am)) / (2 * eps)
        ad = sum(float((G[k] * d[k]).sum()) for k in sph.GRAD_FIELDS)
        print("fd", fd, "adjoint", ad)
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-3), (fd, ad)


def _rollout_case():
    w = inputs.lattice(7, seed=5, sigma_v=0.05)
    a = dict(w.arrays)
    _jitter(a, np.random.default_rng(31), 0.01)
    target = 1.0 + 0.01 * np.random.default_rng(32).normal(size=w.n)
    return w, a, target


def _gpu_rollout_grad(w, a, target, steps, ckpt):
    cfg, _ = configs(w, ng_max=NG)
    r = Run(w, cfg, a)
    sph.initialise(cfg, r.parts, r.ws, r.g)
    ro = sph.Rollout(cfg, r.parts, r.g, r.ws, steps=steps, ckpt=ckpt)
    v0 = torch.tensor(np.stack([a["vx"], a["vy"], a["vz"]], 1), device="cuda",
                      requires_grad=True)
    rho = sph.DensityRollout.apply(v0, ro)
    L = 0.5 * ((rho - torch.tensor(target, device="cuda")) ** 2).sum()
    L.backward()
    assert r.status() == (0, 0)
    return rho.detach().cpu().numpy(), v0.grad.cpu().numpy()


def test_rollout_matches_oracle():
    w, a, target = _rollout_case()
    steps = 3
    rho_g, g_g = _gpu_rollout_grad(w, a, target, steps, ckpt=2)
    _, ocfg = configs(w, ng_max=NG)
    st0 = dict(a)
    st0["h"] = oracle.initial_h(ocfg, st0)
    st0["du_m1"] = np.zeros(w.n)
    v0 = torch.tensor(np.stack([a["vx"], a["vy"], a["vz"]], 1), requires_grad=True)
    rho_o, _, _ = TA.rollout_density(ocfg, st0, v0, steps)
    L = 0.5 * ((rho_o - torch.tensor(target)) ** 2).sum()
    L.backward()
    e_rho = rel_err(rho_g, rho_o.detach().numpy())
    e_g = rel_err(g_g, v0.grad.numpy())
    print("rollout rho", f"{e_rho:.1e}", "grad", f"{e_g:.1e}")
    assert e_rho <= 1e-11
    assert e_g <= TOL_ROLLOUT


def test_rollout_checkpoint_interval_invariant():
    """The replays reproduce every step bit for bit, so the gradient does not
    depend on the checkpoint interval."""
    w, a, target = _rollout_case()
    grads = [_gpu_rollout_grad(w, a, target, 4, ckpt)[1] for ckpt in (1, 3, 4)]
    for g in grads[1:]:
        assert np.array_equal(g.view(np.uint64), grads[0].view(np.uint64))


def _frozen_rollout_density(cfg, w, a0, v0, hs, dts, h_fin):
    """rho (by id) at the end of the rollout with its structure frozen: step s
    runs the stage entry points with h = hs[s] and dt = dts[s] (newton_iters = 0
    in cfg), and the final density is evaluated at h_fin."""
    arr = dict(a0)
    for k, col in (("vx", 0), ("vy", 1), ("vz", 2)):
        arr[k] = v0[:, col].copy()
        arr["vh" + k[1]] = v0[:, col].copy()
    r = Run(w, cfg, arr)
    dt_m1 = 0.0
    for s in range(len(dts)):
        r.parts["h"] = torch.from_numpy(hs[s][r.ids()])
        _frozen_step(cfg, r, dts[s], dt_m1)
        dt_m1 = dts[s]
    r.parts["h"] = torch.from_numpy(h_fin[r.ids()])
    sph.build_cells(cfg, r.parts, r.ws)
    sph.find_neighbors(cfg, r.parts, r.ws)
    sph.density(cfg, r.parts, r.ws)
    assert r.status() == (0, 0)
    return r.by_id("rho")


# The C5 differences (v0 + eps d, d of RMS 0.01 or one component of 0.01).
# The AV switch (viscosity only where v_ab . x_ab < 0) is a kink of the step map:
# the adjoint follows the recorded branch, while a central difference straddles
# the switch for O(eps * pairs * steps) pairs, each an O(eps) error.  With the
# viscosity off the map is smooth, and the differences converge as eps^2 down to
# the rounding floor (eps = 1e-3 random, 1e-2 one component: 2e-8 .. 3e-7 in
# a sweep of eps from 1e-2 to 1e-7); that case carries the 1e-6 bar, with two
# step sizes Richardson-combined to remove the O(eps^2) term.  With the viscosity
# of the benchmark (alpha = 1) the same sweep leaves 1e-6 .. 9e-4 at every step
# size, scattered by the straddled switches, so that case is a plain central
# difference held to 1e-2; its adjoint is pinned at 1e-12 against the oracle's
# gradient on the small rollouts above.
C5_CASES = {0.0: (1e-3, 1e-2, 1e-6, True), 1.0: (1e-6, 1e-4, 1e-2, False)}


@pytest.mark.parametrize("alpha", sorted(C5_CASES))
def test_rollout_c5_finite_differences(alpha):
    """The 64^3 lattice rollout as benchmarked: 20 steps, a checkpoint every 5,
    loss 1/2 |rho_20 - rho*|^2, gradient with respect to v0.  Checked against
    central differences of the GPU's own frozen-structure rollout (h and dt of
    every step as recorded) in 3 random directions of RMS 0.01 and 10 single
    components of size 0.01.  The loss difference is formed as
    sum (rho+ - rho-)((rho+ + rho-)/2 - rho*), which has no cancellation of the
    loss itself."""
    eps_dir, eps_comp, bar, richardson = C5_CASES[alpha]
    w = inputs.c5_lattice()
    n = w.n
    target = inputs.c5_target_density(n)
    cfg, _ = configs(w, alpha_av=alpha)
    r = Run(w, cfg)
    sph.initialise(cfg, r.parts, r.ws, r.g)
    a0 = {k: r.by_id(k) for k in ("x", "y", "z", "h", "m", "u")}
    a0["id"] = np.arange(n)
    v0 = np.stack([w.arrays["vx"], w.arrays["vy"], w.arrays["vz"]], 1)
    # gradient through the checkpointed rollout
    ro = sph.Rollout(cfg, r.parts, r.g, r.ws, steps=20, ckpt=5)
    v0_t = torch.tensor(v0, device="cuda", requires_grad=True)
    rho = sph.DensityRollout.apply(v0_t, ro)
    L = 0.5 * ((rho - torch.tensor(target, device="cuda")) ** 2).sum()
    L.backward()
    assert r.status() == (0, 0)
    grad = v0_t.grad.cpu().numpy()
    rho_ad = rho.detach().cpu().numpy()
    # the structure of every step, recorded on a plain forward from the same state
    sph.restore(r.parts, r.g, ro.initial)
    hs, dts = [], []
    for s in range(20):
        sph.step(cfg, r.parts, r.g, r.ws)
        hs.append(r.by_id("h"))
        dts.append(float(r.g.t[0].item()))
    sph.density_eval(cfg, r.parts, r.ws)
    assert np.array_equal(r.by_id("rho"), rho_ad)     # the rollout's own forward
    h_fin = r.by_id("h")
    fz = cfg.replace(newton_iters=0)
    rho_fz = _frozen_rollout_density(fz, w, a0, v0, hs, dts, h_fin)
    assert rel_err(rho_fz, rho_ad) < 1e-13            # frozen replay = free forward

    def dL(d, eps):
        rp = _frozen_rollout_density(fz, w, a0, v0 + eps * d, hs, dts, h_fin)
        rm = _frozen_rollout_density(fz, w, a0, v0 - eps * d, hs, dts, h_fin)
        return float(np.sum((rp - rm) * (0.5 * (rp + rm) - target))) / (2 * eps)

    rng = np.random.default_rng(57)
    dirs = [(rng.normal(0.0, 0.01, (n, 3)), eps_dir) for _ in range(3)]
    # single components drawn among those whose derivative is at least the
    # median one: the differences carry an absolute rounding floor of ~1e-12
    # after 20 steps, which a relative bar cannot resolve near a zero derivative
    big = np.flatnonzero(np.abs(grad).ravel() >= np.median(np.abs(grad)))
    for c in rng.choice(big, 10, replace=False):
        d = np.zeros(3 * n)
        d[c] = 0.01
        dirs.append((d.reshape(n, 3), eps_comp))
    worst = 0.0
    for d, eps in dirs:
        ad = float(np.sum(grad * d))
        fd = (4.0 * dL(d, eps / 2) - dL(d, eps)) / 3.0 if richardson else dL(d, eps)
        err = abs(fd - ad) / abs(ad)
        worst = max(worst, err)
        print(f"c5 alpha {alpha} fd {fd:.12e} adjoint {ad:.12e} rel {err:.1e}")
        assert err <= bar, (fd, ad)
    print(f"c5 alpha {alpha} worst {worst:.1e}")
