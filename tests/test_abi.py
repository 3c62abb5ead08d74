"""The C ABI library loads and exports every entry point declared in include/socfv.h.

No compute calls: this runs without a GPU.
"""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "socfv.h")
LIB = os.path.join(ROOT, "paper_2502_08034_amd", "libsocfv.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(socfv_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("socfv_setup_geometry", "socfv_set_velocity", "socfv_solve_soc_steady",
                 "socfv_compute_umt", "socfv_solve_soc_adjoint", "socfv_batch_solve"):
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (python -m paper_2502_08034_amd.build)"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.socfv_version.restype = ctypes.c_int
    assert lib.socfv_version() >= 1


def test_default_params_without_gpu():
    from paper_2502_08034_amd import socfv as mod
    p = mod.params(tol=1e-9, mode="pinned", precision="fp64")
    assert p.cfl == 0.4 and p.tol == 1e-9 and p.mode == mod.PINNED and p.precision == mod.FP64
    assert p.check_every == 200 and p.Da == 0.45
    # a NULL context is rejected with an error code, not a crash
    st = mod.Stats()
    code = mod.lib().socfv_solve_soc_steady(None, ctypes.byref(p), None, None, ctypes.byref(st), None)
    assert code == mod.INVALID_ARG
    assert b"context" in mod.lib().socfv_last_error()


def test_flow_params_without_gpu():
    from paper_2502_08034_amd import socfv as mod
    fp = mod.flow_params(cfl=2.0)
    assert fp.p_in == 1.0 and fp.cfl == 2.0 and fp.tol == 1e-9 and fp.cg_theta == 0.1
    assert fp.check_every == 50 and fp.cg_max == 256
    st = mod.FlowStats()
    code = mod.lib().socfv_solve_stokes(None, ctypes.byref(fp), None, None, None, None,
                                        ctypes.byref(st), None)
    assert code == mod.INVALID_ARG
    assert b"context" in mod.lib().socfv_last_error()
