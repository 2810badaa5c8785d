"""The HIP path's polynomial fits of the sinc kernel (csrc/sph_sinc_poly.h)
against the host C library's sin and cos, on the kernel's support.

The device evaluates sinc(x) and x sinc'(x) = cos x - sinc x, with x = (pi/2) v
and 0 <= v <= 2, as polynomials in t = x^2 (eq. 6 needs S_n = sinc^n and, for
the grad-h term, v dS_n/dv).  Bar: 1e-15 absolute for the FP64 fits and for
S_6 built from them, 2e-15 for v dS_6/dv = 6 s^5 q (its float64 reference
rounds at that level), 1e-6 for the FP32 fits of the mixed-precision path (a
few float32 ulps of values up to 1)."""
import os
import re

import numpy as np

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2005_02656_amd", "csrc", "sph_sinc_poly.h")


def _coeffs():
    src = open(HDR).read()
    out = {}
    for name, body in re.findall(r"constexpr (?:double|float) (\w+)\[\d+\] = \{([^}]*)\}", src):
        out[name] = [float(v.rstrip("f")) for v in body.replace("\n", " ").split(",")]
    return out


def _horner(c, t, dtype):
    c = np.asarray(c, dtype=dtype)
    t = t.astype(dtype)
    s = np.full_like(t, c[-1])
    for k in range(len(c) - 2, -1, -1):
        s = (s * t + c[k]).astype(dtype)
    return s


def _grid():
    x = np.linspace(0.0, np.pi, 200001)
    x[0] = 1e-300
    return x


def test_fp64_fits_against_libm():
    c = _coeffs()
    x = _grid()
    t = x * x
    sinc = np.sin(x) / x
    q = np.cos(x) - sinc                         # x sinc'(x)
    s_fit = _horner(c["kSincS64"], t, np.float64)
    q_fit = _horner(c["kSincQ64"], t, np.float64) * t
    assert np.max(np.abs(s_fit - sinc)) <= 1e-15
    assert np.max(np.abs(q_fit - q)) <= 1e-15
    # S_6 and v dS_6/dv as the kernels form them
    assert np.max(np.abs(s_fit ** 6 - sinc ** 6)) <= 1e-15
    assert np.max(np.abs(6 * s_fit ** 5 * q_fit - 6 * sinc ** 5 * q)) <= 2e-15
    assert c["kSincS64"][0] == 1.0                # S(0) = 1 exactly


def test_fp32_fits_against_libm():
    c = _coeffs()
    x = _grid()
    t = x * x
    sinc = np.sin(x) / x
    q = np.cos(x) - sinc
    s_fit = _horner(c["kSincS32"], t, np.float32).astype(np.float64)
    q_fit = (_horner(c["kSincQ32"], t, np.float32) * t.astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(s_fit - sinc)) <= 1e-6
    assert np.max(np.abs(q_fit - q)) <= 1e-6
