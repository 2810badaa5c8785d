"""Pins of the differentiable oracle (oracle/torch_adjoint.py): its forward values
equal the C oracle's, and its autograd gradients equal central finite
differences of the C oracle's stages composed with the same frozen h and dt."""
import numpy as np
import pytest
import torch

from conftest import oracle_config
from paper_2005_02656_amd import inputs
from oracle import torch_adjoint as TA


def c_step_frozen(ora, cfg, st, h, dt, dt_m1):
    """The C oracle's stages with h and dt given (the frozen-structure map)."""
    x, y, z = st["x"], st["y"], st["z"]
    rho, om, p, c = ora.density(cfg, x, y, z, h, st["m"], st["u"], st.get("p_ref"),
                                st.get("rho_ref"))
    Cm, _ = ora.iad(cfg, x, y, z, h, st["m"], rho)
    me = ora.momentum_energy(cfg, x, y, z, st["vx"], st["vy"], st["vz"], h, st["m"], rho, om, p,
                             c, Cm)
    s0 = dict(st)
    s0["h"] = h
    new = ora.integrate(cfg, s0, me["ax"], me["ay"], me["az"], me["du"], dt, dt_m1)
    return new, {"rho": rho, "omega": om, "p": p, "c": c, "C": Cm, **me}


def to_torch(st):
    return {"x": torch.tensor(np.stack([st["x"], st["y"], st["z"]], 1)),
            "v": torch.tensor(np.stack([st["vx"], st["vy"], st["vz"]], 1)),
            "vh": torch.tensor(np.stack([st["vhx"], st["vhy"], st["vhz"]], 1)),
            "u": torch.tensor(st["u"]), "du_m1": torch.tensor(st["du_m1"])}


@pytest.fixture(scope="module")
def case(ora):
    w = inputs.lattice(7, seed=2, sigma_v=0.05)
    a = w.arrays
    rng = np.random.default_rng(9)
    a["x"] = np.mod(a["x"] + rng.normal(0, 0.01, a["x"].size), 1.0)   # break the symmetry
    a["y"] = np.mod(a["y"] + rng.normal(0, 0.01, a["y"].size), 1.0)
    a["z"] = np.mod(a["z"] + rng.normal(0, 0.01, a["z"].size), 1.0)
    cfg = oracle_config(w.params)
    st = dict(a)
    st["h"] = ora.initial_h(cfg, st)
    st.update(vhx=st["vx"] + 0.01, vhy=st["vy"].copy(), vhz=st["vz"] - 0.02,
              du_m1=rng.normal(0, 0.1, w.n), u=1.0 + 0.1 * rng.random(w.n))
    return cfg, st


def test_forward_matches_c_oracle(ora, case):
    cfg, st = case
    dt, dt_m1 = 0.01, 0.008
    new_c, f_c = c_step_frozen(ora, cfg, st, st["h"], dt, dt_m1)
    S = TA.Setup(cfg, st["m"], st["h"])
    new_t, f_t = TA.step(S, to_torch(st), dt, dt_m1)
    assert abs(S.bn - ora.bn(cfg.sinc_n)) < 1e-14
    for k in ("rho", "omega", "p", "c"):
        assert np.max(np.abs(f_t[k].numpy() - f_c[k])) < 1e-12 * np.max(np.abs(f_c[k])), k
    Cf = f_t["C"].numpy()
    for k, (i, j) in enumerate(((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))):
        assert np.max(np.abs(Cf[:, i, j] - f_c["C"][k])) < 1e-11 * np.max(np.abs(f_c["C"][0]))
    sa = np.max(f_c["scale_a"])
    for k, ax in enumerate(("ax", "ay", "az")):
        assert np.max(np.abs(f_t["a"][:, k].numpy() - f_c[ax])) < 1e-12 * sa
    assert np.max(np.abs(f_t["du"].numpy() - f_c["du"])) < 1e-12 * np.max(f_c["scale_du"])
    for k, key in enumerate("xyz"):
        assert np.allclose(new_t["x"][:, k].numpy(), new_c[key], rtol=0, atol=1e-14)


def test_gradient_matches_finite_differences(ora, case):
    """d/dv0 and d/dx0 of a weighted sum of the step outputs, along random
    directions: autograd of the torch oracle vs central differences of the C oracle."""
    cfg, st = case
    dt, dt_m1 = 0.01, 0.008
    rng = np.random.default_rng(4)
    n = st["x"].size
    wx, wv, wu = rng.normal(size=(n, 3)), rng.normal(size=(n, 3)), rng.normal(size=n)

    def loss_c(s):
        new, _ = c_step_frozen(ora, cfg, s, st["h"], dt, dt_m1)
        X = np.stack([new["x"], new["y"], new["z"]], 1)
        V = np.stack([new["vx"], new["vy"], new["vz"]], 1)
        return float((wx * X).sum() + (wv * V).sum() + (wu * new["u"]).sum())

    S = TA.Setup(cfg, st["m"], st["h"])
    ts = to_torch(st)
    for k in ("x", "v", "u"):
        ts[k].requires_grad_(True)
    new, _ = TA.step(S, ts, dt, dt_m1)
    L = (torch.tensor(wx) * new["x"]).sum() + (torch.tensor(wv) * new["v"]).sum() + \
        (torch.tensor(wu) * new["u"]).sum()
    L.backward()
    for field, cols in (("v", ("vx", "vy", "vz")), ("x", ("x", "y", "z")), ("u", ("u",))):
        g = ts[field].grad.numpy().reshape(n, -1)
        for trial in range(2):
            delta = rng.normal(size=g.shape)
            eps = 1e-6 if field != "x" else 1e-7
            sp, sm = dict(st), dict(st)
            for c, col in enumerate(cols):
                sp[col] = st[col] + eps * delta[:, c]
                sm[col] = st[col] - eps * delta[:, c]
            fd = (loss_c(sp) - loss_c(sm)) / (2 * eps)
            ad = float((g * delta).sum())
            assert abs(fd - ad) <= 2e-6 * max(abs(ad), 1.0), (field, fd, ad)


def test_rollout_gradient_matches_finite_differences(ora):
    """d/dv0 of L = 1/2 |rho_final - rho*|^2 after a 3-step rollout (frozen h and dt
    per step, final density with its own frozen h): autograd of the torch replay vs
    central differences of the C oracle's stages composed with the same frozen
    structure."""
    w = inputs.lattice(6, seed=3, sigma_v=0.05)
    cfg = oracle_config(w.params)
    st0 = dict(w.arrays)
    rng = np.random.default_rng(12)
    for a in "xyz":
        st0[a] = np.mod(st0[a] + rng.normal(0, 0.01, w.n), 1.0)
    st0["h"] = ora.initial_h(cfg, st0)
    st0["du_m1"] = np.zeros(w.n)
    target = 1.0 + 0.01 * rng.normal(size=w.n)
    v0 = torch.tensor(np.stack([st0["vx"], st0["vy"], st0["vz"]], 1), requires_grad=True)
    rho, frozen, h_final = TA.rollout_density(cfg, st0, v0, 3)
    L = 0.5 * ((rho - torch.tensor(target)) ** 2).sum()
    L.backward()
    g = v0.grad.numpy()
    assert np.all(np.isfinite(g)) and np.abs(g).max() > 0

    def loss_c(v):
        s = dict(st0)
        for c, a in enumerate("xyz"):
            s["v" + a] = v[:, c].copy()
            s["vh" + a] = v[:, c].copy()
        for h, dt, dt_m1 in frozen:
            s, _ = c_step_frozen(ora, cfg, s, h, dt, dt_m1)
        r, _, _, _ = ora.density(cfg, s["x"], s["y"], s["z"], h_final, s["m"], s["u"])
        return 0.5 * float(((r - target) ** 2).sum())

    v = v0.detach().numpy()
    eps = 1e-6
    for trial in range(3):
        delta = rng.normal(size=v.shape)
        fd = (loss_c(v + eps * delta) - loss_c(v - eps * delta)) / (2 * eps)
        ad = float((g * delta).sum())
        print("rollout fd", fd, ad, abs(fd - ad) / abs(ad))
        assert abs(fd - ad) <= 1e-8 * max(abs(ad), 1e-8), (fd, ad)
