"""The oracle's C code under the host AddressSanitizer and UndefinedBehavior-
Sanitizer: a sanitized build, loaded in a child process that preloads libasan,
runs every entry point on small inputs (all workload shapes, targets, the
table, gravity, keys, sorting, integration).  Any invalid access, leak-free
heap misuse or undefined behaviour aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
sys.path.insert(0, ROOT)
import numpy as np
import oracle
from paper_2005_02656_amd import inputs
keys = set(oracle.Config.__dataclass_fields__)
for w in (inputs.lattice(6, seed=1), inputs.square_patch(6),
          inputs.random_periodic(300, seed=2, h_lo=0.1, h_hi=0.16),
          inputs.gaussian_blob(400, seed=3, seed_v=33)):
    for kt in (0, 2000):
        cfg = oracle.Config(**{k: v for k, v in w.params.items() if k in keys}).replace(kernel_table=kt)
        st = {k: np.array(v, copy=True) for k, v in w.arrays.items()}
        st["h"] = oracle.initial_h(cfg, st, iters=3)
        if cfg.eos == 1:
            st["rho_ref"] = np.ones(w.n)
        st.update(vhx=st["vx"].copy(), vhy=st["vy"].copy(), vhz=st["vz"].copy(),
                  du_m1=np.zeros(w.n))
        s1, g1, f1 = oracle.step(cfg, st, {"dt_m1": 0.0, "t": 0.0})
        oracle.step(cfg, s1, g1)
        t = np.array([0, w.n - 1, w.n // 2])
        oracle.neighbors(cfg, st["x"], st["y"], st["z"], st["h"], targets=t)
        oracle.newton_terms(cfg, st["x"], st["y"], st["z"], st["h"], targets=t)
        lo, hi = oracle.key_domain(cfg, st["x"], st["y"], st["z"], st["h"])
        oracle.sort_keys(oracle.morton_keys(st["x"], st["y"], st["z"], lo, hi))
X = np.random.default_rng(1).normal(size=(700, 3))
m = np.full(700, 1.0 / 700)
for th in (0.0, 0.5):
    oracle.gravity_tree(X[:, 0], X[:, 1], X[:, 2], m, X.min(0), X.max(0),
                        oracle.gravity_leaf_level(700), 1.0, 0.01, th, targets=[0, 699])
oracle.gravity_direct(X[:, 0], X[:, 1], X[:, 2], m, 1.0, 0.01)
print("sanitized oracle ok")
""".replace("ROOT", repr(ROOT))


def test_oracle_under_address_sanitizer(tmp_path):
    from oracle import build
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("gcc has no libasan here")
    lib = build.build(out=str(tmp_path / "libsph_oracle_asan.so"), sanitize=True)
    env = dict(os.environ, SPH_ORACLE_LIBRARY=lib, LD_PRELOAD=libasan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", OMP_NUM_THREADS="2",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", SCRIPT], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
