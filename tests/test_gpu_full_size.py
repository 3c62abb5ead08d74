"""The benchmark's full-size workloads on the GPU, checked by the FP64 oracle (needs an MI355X).

256 x 128 x 128: against the stored oracle solves (tests/golden/fibre256.json and, for a
mid-range utilisation, fibre256_mid.json, written by tests/golden/make_golden.py from the
oracle alone).  1024 x 512 x 256 (the benchmark's slab,
in the benchmark's launch configuration): by properties the oracle evaluates on the GPU's
state at any size -- its FP64 residual over every cell, the exact flux balance, the bounds,
and U recomputed from the state.
"""
import hashlib
import json
import os
import time

import numpy as np
import pytest
import torch

from paper_2502_08034_amd import inputs as I

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


@pytest.fixture(scope="module")
def sv():
    from paper_2502_08034_amd import socfv
    return socfv


@pytest.mark.parametrize("mode", ["finite", "pinned"])
def test_fibre256_against_stored_oracle(sv, orc, mode):
    gold = json.load(open(os.path.join(HERE, "golden", "fibre256.json")))
    w = I.workload("fibre256", with_velocity=False)
    solid = w["solid"]
    assert hashlib.sha256(solid.tobytes()).hexdigest() == gold["geometry_sha256"]
    u = I.darcy_velocity(solid, 1.0, device="cuda", as_numpy=False)
    g = gold[mode]
    pb = sv.Problem.create(solid, *u)
    p = sv.params(precision="fp32", tol=1e-8, mode=1 if g["pinned"] else 0, s_in=g["s_in"],
                  s_eq=g["s_eq"], Da=g["Da"])
    s, st = sv.solve_soc_steady(pb.ctx, p)
    assert st.status == sv.OK
    Ug = g["outputs"]["U"]
    assert abs(st.U - Ug) <= 1e-6 * abs(Ug)
    print(f"{mode}: U {st.U:.12f} ref {Ug:.12f}, |dU| / (1 - U) = "
          f"{abs(st.U - Ug) / (1 - Ug):.2e}")
    if mode == "finite":
        # 1 - U ~ 3e-4: the unconverted fraction to 1e-4 relative at residual 1e-8
        assert abs(st.U - Ug) <= 1e-4 * (1 - Ug)
    # the stored references were converged to 2e-12; at 1e-8 the state is ~1e-9 away
    idx = np.asarray(gold["sample_index"])
    sg = s.view(-1)[torch.as_tensor(idx, device="cuda")].cpu().numpy()
    assert np.abs(sg - np.asarray(g["s_sample"])).max() <= 1e-5
    sn = s.cpu().numpy()
    un = tuple(a.cpu().numpy() for a in u)
    op = orc.Problem(solid, *un, s_in=g["s_in"], s_eq=g["s_eq"], Da=g["Da"], pinned=g["pinned"])
    assert orc.residual_norm(op, sn) < 1.5e-8
    pore = solid == 0
    assert sn[pore].min() >= min(g["s_in"], g["s_eq"]) - 1e-9
    assert sn[pore].max() <= max(g["s_in"], g["s_eq"]) + 1e-9


def test_fibre256_mid_range_utilisation(sv, orc):
    """A slow surface reaction (Da 0.02 per fibre face) puts U near 0.5, where an error in U is
    an error in the unconverted fraction too (at Da 0.45, 1 - U ~ 3e-4, and in the
    mass-transport limit 1 - U ~ 7e-8, so |dU| / U says little there).  FP32 mode to 1e-8
    against the stored oracle solve: |dU| <= 1e-6 min(U, 1 - U)."""
    gold = json.load(open(os.path.join(HERE, "golden", "fibre256_mid.json")))
    w = I.workload("fibre256", with_velocity=False)
    solid = w["solid"]
    assert hashlib.sha256(solid.tobytes()).hexdigest() == gold["geometry_sha256"]
    u = I.darcy_velocity(solid, 1.0, device="cuda", as_numpy=False)
    g = gold["mid"]
    pb = sv.Problem.create(solid, *u)
    s, st = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp32", tol=1e-8, Da=g["Da"]))
    assert st.status == sv.OK
    Ug = g["outputs"]["U"]
    assert 0.3 < Ug < 0.7
    err = abs(st.U - Ug)
    print(f"U {st.U:.12f} ref {Ug:.12f}: |dU| / min(U, 1 - U) = {err / min(Ug, 1 - Ug):.2e}")
    assert err <= 1e-6 * min(Ug, 1 - Ug)
    idx = np.asarray(gold["sample_index"])
    sg = s.view(-1)[torch.as_tensor(idx, device="cuda")].cpu().numpy()
    assert np.abs(sg - np.asarray(g["s_sample"])).max() <= 1e-5
    for k in ("flux_in", "flux_out", "reaction"):
        ok = {"flux_in": "F_in", "flux_out": "F_out", "reaction": "reaction"}[k]
        assert abs(getattr(st, k) - g["outputs"][ok]) <= 1e-6 * abs(g["outputs"][ok]), k


def test_slab1024_in_the_benchmark_configuration(sv, orc):
    """The benchmark's solve (FP32 mode, tolerance 1e-8, automatic tiles) at its three
    Peclet numbers, each state then evaluated by the oracle in FP64 over all 134M cells."""
    cfg = I.WORKLOADS["slab1024"]
    nx, ny, nz = cfg["shape"]
    t = time.time()
    geo = I.fibres_boolean(nx, ny, nz, cfg["radius"], cfg["porosity"], cfg["seed"])
    log(f"geometry {time.time() - t:.1f}s porosity {geo.porosity:.4f}")
    t = time.time()
    u = I.darcy_velocity(geo.solid, 1.0, device="cuda", as_numpy=False, log=log)
    log(f"darcy {time.time() - t:.1f}s")
    pb = sv.Problem.create(geo.solid, *u)
    un = tuple(a.cpu().numpy() for a in u)
    del u
    pore = geo.solid == 0
    npore = int(np.count_nonzero(pore))
    p = sv.params(precision="fp32", tol=1e-8, check_every=200)
    for pe in cfg["peclet"]:
        pb.set_flow_rate(pe)
        t = time.time()
        s, st = sv.solve_soc_steady(pb.ctx, p)
        log(f"Pe {pe}: solve {time.time() - t:.1f}s, {st.iterations} sweeps, residual "
            f"{st.residual:.3e}, U {st.U:.12f}, tiles ({st.tile_y}, {st.z_chunk})")
        assert st.status == sv.OK
        sn = s.cpu().numpy()
        del s
        t = time.time()
        op = orc.Problem(geo.solid, *(a * pe for a in un), s_in=1.0, s_eq=0.0, Da=0.45)
        res = orc.residual_norm(op, sn)
        o = orc.outputs(op, sn)
        log(f"Pe {pe}: oracle evaluation {time.time() - t:.1f}s, residual {res:.3e}, "
            f"U {o['U']:.12f}, F_in {o['F_in']:.6e}, sum R {o['sum_R']:.3e}")
        # the oracle's FP64 residual of the GPU state meets the tolerance the solve reports
        assert res < 1.5e-8
        assert abs(o["U"] - st.U) <= 1e-12
        # global balance of a steady state: inflow = outflow + reaction up to sum R, and
        # |sum R| <= npore * rms(R) = npore * res / tau
        tau = orc.time_scale(op)
        assert abs(o["sum_R"]) <= npore * res / tau * (1 + 1e-9)
        assert abs(o["F_in"] - o["F_out"] - o["reaction"]) <= 2e-8 * o["F_in"]
        assert 0.0 < o["U"] < 1.0
        assert sn[pore].min() >= -1e-9 and sn[pore].max() <= 1.0 + 1e-9
        assert np.all(sn[~pore] == 0.0)
        del sn, op
