"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function include/sph.h declares, and rejects bad arguments before enqueuing."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "sph.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def sph():
    from paper_2005_02656_amd import sph as s
    s.lib()
    return s


def test_exports_every_declared_symbol(sph):
    names = declared()
    assert "sph_step" in names and "sph_build_cells" in names
    L = C.CDLL(sph.LIB_PATH)
    for nm in names:
        assert hasattr(L, nm), nm
    # the binding wraps exactly what the header declares
    assert sorted(sph.EXPORTED) == names


def test_constants_match_the_header(sph):
    src = open(os.path.join(ROOT, "include", "sph.h")).read()
    defs = dict(re.findall(r"#define (SPH_\w+) (.+)", src))
    assert float(defs["SPH_SHORT_REACH"]) == sph.SHORT_REACH
    assert int(defs["SPH_KERNEL_TABLE_MAX"]) == sph.KERNEL_TABLE_MAX
    m = re.fullmatch(r"\((\d+)u << (\d+)\)", defs["SPH_STATIC_SCRATCH_BYTES"].strip())
    assert int(m.group(1)) << int(m.group(2)) == sph.STATIC_SCRATCH_BYTES
    assert int(defs["SPH_STEP_PHASES"]) == len(sph.STEP_PHASES)
    assert int(defs["SPH_GRAPH_MAX_STEPS"]) == sph.GRAPH_MAX_STEPS
    shift = lambda d: 1 << int(re.fullmatch(r"\(1u << (\d+)\)", d.strip()).group(1))
    bits = {k: shift(defs["SPH_ERRBIT_" + k]) for k in
            ("NEIGHBOR_OVERFLOW", "CELL_RANGE", "NONFINITE", "SINGULAR_TAU")}
    assert bits == {"NEIGHBOR_OVERFLOW": sph.ERRBIT_NEIGHBOR_OVERFLOW,
                    "CELL_RANGE": sph.ERRBIT_CELL_RANGE, "NONFINITE": sph.ERRBIT_NONFINITE,
                    "SINGULAR_TAU": sph.ERRBIT_SINGULAR_TAU}


def test_workspace_bytes_validation(sph):
    L = sph.lib()
    good = sph.Config(n=1000)
    assert L.sph_workspace_bytes(C.byref(good.c())) > 1000 * 4 * good.ng_max
    for bad in (good.replace(n=0), good.replace(ng_max=0), good.replace(sinc_n=2.5),
                good.replace(sinc_n=12.0), good.replace(eos=7), good.replace(h_ratio_max=1.0),
                good.replace(precision=3), good.replace(eos=1, c0=0.0),
                good.replace(box_hi=(1.0, 0.0, 1.0)), good.replace(kernel_table=1),
                good.replace(kernel_table=sph.KERNEL_TABLE_MAX + 1)):
        assert L.sph_workspace_bytes(C.byref(bad.c())) == 0
    assert L.sph_workspace_bytes(None) == 0
    for ok in (2, sph.KERNEL_TABLE_PAPER, sph.KERNEL_TABLE_MAX):
        assert L.sph_workspace_bytes(C.byref(good.replace(kernel_table=ok).c())) == \
            L.sph_workspace_bytes(C.byref(good.c()))


def test_argument_errors_are_synchronous(sph):
    L = sph.lib()
    cfg = sph.Config(n=100)
    ws = C.create_string_buffer(1024)
    parts = sph._Particles()
    # NULL config / particles / misaligned workspace return before any launch
    assert L.sph_build_cells(None, C.byref(parts), ws, None) == 1
    assert L.sph_build_cells(C.byref(cfg.c()), None, C.c_void_p(256), None) == 1
    assert L.sph_build_cells(C.byref(cfg.c()), C.byref(parts), C.c_void_p(17), None) == 3
    assert L.sph_build_cells(C.byref(cfg.c()), C.byref(parts), None, None) == 3
    assert L.sph_density(C.byref(cfg.c()), C.byref(parts), C.c_void_p(256), None) == 1
    assert L.sph_timestep(C.byref(cfg.c()), None, C.c_void_p(256), None) == 1


def test_static_step_rejects_before_enqueuing(sph):
    """sph_step_static validates on the host: bad config or particles give
    SPH_E_ARG and a workspace larger than the fixed scratch SPH_E_WORKSPACE,
    before any device call."""
    L = sph.lib()
    parts = sph._Particles()
    g = C.c_void_p(256)
    assert L.sph_step_static(None, C.byref(parts), g, None, None) == 1
    assert L.sph_step_static(C.byref(sph.Config(n=0).c()), C.byref(parts), g, None, None) == 1
    big = sph.Config(n=200_000)
    assert L.sph_workspace_bytes(C.byref(big.c())) > sph.STATIC_SCRATCH_BYTES
    assert L.sph_step_static(C.byref(big.c()), C.byref(parts), g, None, None) == 3
    small = sph.Config(n=8000)
    assert L.sph_workspace_bytes(C.byref(small.c())) <= sph.STATIC_SCRATCH_BYTES
    assert L.sph_step_static(C.byref(small.c()), C.byref(parts), g, None, None) == 1


def test_step_graph_rejects_before_capturing(sph):
    """sph_step_graph_create validates on the host and leaves *graph NULL:
    SPH_E_ARG for a NULL handle, steps outside 1..SPH_GRAPH_MAX_STEPS, a bad
    config or NULL particles, SPH_E_WORKSPACE for a misaligned workspace; a
    NULL graph is refused by launch and ignored by destroy."""
    L = sph.lib()
    cfg = sph.Config(n=1000)
    parts = sph._Particles()
    g = C.c_void_p(256)
    ws = C.c_void_p(256)
    h = C.c_void_p(1234)
    assert L.sph_step_graph_create(C.byref(cfg.c()), C.byref(parts), g, ws, 1, None) == 1
    for steps in (0, -1, sph.GRAPH_MAX_STEPS + 1):
        assert L.sph_step_graph_create(C.byref(cfg.c()), C.byref(parts), g, ws, steps,
                                       C.byref(h)) == 1
        assert h.value is None
        h = C.c_void_p(1234)
    assert L.sph_step_graph_create(C.byref(cfg.replace(n=0).c()), C.byref(parts), g, ws, 1,
                                   C.byref(h)) == 1
    assert L.sph_step_graph_create(C.byref(cfg.c()), C.byref(parts), g, C.c_void_p(17), 1,
                                   C.byref(h)) == 3
    assert L.sph_step_graph_create(C.byref(cfg.c()), None, g, ws, 1, C.byref(h)) == 1
    assert L.sph_step_graph_create(C.byref(cfg.c()), C.byref(parts), g, ws, 1,
                                   C.byref(h)) == 1   # the particle arrays are NULL
    assert L.sph_step_graph_launch(None, None) == 1
    L.sph_step_graph_destroy(None)


def test_status_strings(sph):
    for st in range(8):
        assert sph.status_string(st).startswith(sph.STATUS_NAMES[st])
    assert "unknown" in sph.status_string(99)
