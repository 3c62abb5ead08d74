"""Batched solve of many uneven problems in one launch per sweep (needs an MI355X).

Each problem of the batch must reach its own tolerance, agree with the same problem
solved alone, and satisfy the FP64 oracle's residual check cell by cell.
"""
import math
import time

import numpy as np
import pytest
import torch

from paper_2502_08034_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv():
    from paper_2502_08034_amd import socfv
    return socfv


def small_batch(n, seed0):
    """Uneven boxes (ragged in x, y, z) with per-problem porosity, radius and Peclet."""
    probs = []
    for k in range(n):
        rng = np.random.Generator(np.random.PCG64(seed0 + k))
        nx = int(rng.integers(40, 97))
        ny = int(rng.integers(12, 41))
        nz = int(rng.integers(10, 33))
        r = float(rng.uniform(2.0, 3.5))
        phi = float(rng.uniform(0.8, 0.92))
        pe = float(math.exp(rng.uniform(math.log(0.1), math.log(10.0))))
        g = I.fibres_nonoverlap(nx, ny, nz, r, phi, int(rng.integers(1 << 30)), max_tries=20000)
        probs.append({"solid": g.solid, "peclet": pe})
    vel = I.darcy_velocity([p["solid"] for p in probs], [p["peclet"] for p in probs],
                           device="cuda")
    for p, v in zip(probs, vel):
        p["velocity"] = v
    return probs


def run_batch(sv, probs, params):
    pbs = [sv.Problem.create(p["solid"], *p["velocity"]) for p in probs]
    states, stats = sv.batch_solve([pb.ctx for pb in pbs], params)
    return pbs, states, stats


@pytest.mark.parametrize("mode", ["finite", "pinned"])
def test_batch_matches_single_solves_and_oracle(sv, orc, mode):
    probs = small_batch(7, 500 if mode == "finite" else 600)
    kw = dict(s_in=1.0, s_eq=0.0, Da=0.45, mode=0) if mode == "finite" else \
        dict(s_in=0.0, s_eq=1.0, Da=0.0, mode=1)
    params = [sv.params(precision="fp32", tol=(1e-8 if k % 2 else 1e-9), check_every=100, **kw)
              for k in range(len(probs))]
    pbs, states, stats = run_batch(sv, probs, params)
    for k, (p, s, st) in enumerate(zip(probs, states, stats)):
        assert st.status == sv.OK, (k, st.status)
        assert st.residual < params[k].tol * 1.5
        # alone
        s1, st1 = sv.solve_soc_steady(pbs[k].ctx, params[k])
        assert np.abs(s.cpu().numpy() - s1.cpu().numpy()).max() < 50 * params[k].tol
        assert abs(st.U - st1.U) <= 1e-6 * abs(st1.U) + 1e-12
        # the oracle's FP64 residual of the batched state
        op = orc.Problem(p["solid"], *p["velocity"], s_in=kw["s_in"], s_eq=kw["s_eq"],
                         Da=kw["Da"], pinned=bool(kw["mode"]))
        assert orc.residual_norm(op, s.cpu().numpy()) < params[k].tol * 1.5
        o = orc.outputs(op, s.cpu().numpy())
        assert abs(o["U"] - st.U) <= 1e-12 * max(1.0, abs(st.U))


def test_batch_exact_on_small_cases(sv, orc):
    probs = small_batch(4, 700)
    params = [sv.params(precision="fp32", tol=1e-10, check_every=100) for _ in probs]
    _, states, stats = run_batch(sv, probs, params)
    for p, s, st in zip(probs, states, stats):
        op = orc.Problem(p["solid"], *p["velocity"], s_in=1.0, s_eq=0.0, Da=0.45)
        sx = orc.exact_steady(op)
        assert np.abs(s.cpu().numpy() - sx)[p["solid"] == 0].max() <= 1e-5
        Ux = orc.outputs(op, sx)["U"]
        assert abs(st.U - Ux) <= 1e-6 * Ux


def test_batch_polish_lengths_differ(sv, orc):
    # the batched FP64 polish runs each converged problem's first polish chunk (polish_iters,
    # else check_every) in shared launches; problems whose chunk ends earlier leave the
    # launches' table, which is rebuilt for the rest
    probs = small_batch(4, 800)
    lengths = [dict(check_every=100), dict(check_every=200, polish_iters=50),
               dict(check_every=300), dict(check_every=100, polish_iters=150)]
    params = [sv.params(precision="fp32", tol=1e-9, **kw) for kw in lengths]
    expect = [100, 50, 300, 100]   # a polish longer than check_every stops after its first
                                   # chunk once the residual is below tol, as alone
    _, states, stats = run_batch(sv, probs, params)
    for k, (p, s, st) in enumerate(zip(probs, states, stats)):
        assert st.status == sv.OK, (k, st.status)
        assert st.sweeps_fp64 == expect[k], (k, st.sweeps_fp64)
        op = orc.Problem(p["solid"], *p["velocity"], s_in=1.0, s_eq=0.0, Da=0.45)
        assert orc.residual_norm(op, s.cpu().numpy()) < 1.5e-9
        o = orc.outputs(op, s.cpu().numpy())
        assert abs(o["U"] - st.U) <= 1e-12 * max(1.0, abs(st.U))


def test_batch48_design_sweep(sv, orc):
    """48 geometries from 64^3 to 192 x 96 x 96, porosity 0.70-0.90, radius 3-6, Peclet
    0.1-10, each to its own residual 1e-8 in one batched solve."""
    t = time.time()
    probs = I.batch_workloads(48, seed0=100, device="cuda")
    print(f"batch fixtures {time.time() - t:.1f}s", flush=True)
    params = [sv.params(precision="fp32", tol=1e-8) for _ in probs]
    pbs = [sv.Problem.create(p["solid"], *p["velocity"]) for p in probs]
    torch.cuda.synchronize()
    t = time.time()
    states, stats = sv.batch_solve([pb.ctx for pb in pbs], params)
    torch.cuda.synchronize()
    makespan = time.time() - t
    print(f"batched makespan {makespan:.2f}s, tiles ({stats[0].tile_y}, {stats[0].z_chunk})",
          flush=True)
    rng = np.random.default_rng(1)
    check = set(rng.choice(48, size=6, replace=False).tolist())
    for k, (p, s, st) in enumerate(zip(probs, states, stats)):
        assert st.status == sv.OK and st.residual < 1.5e-8, (k, st.status, st.residual)
        assert abs(st.flux_in - st.flux_out - st.reaction - st.sum_R) <= 1e-9 * abs(st.flux_in)
        if k in check:
            op = orc.Problem(p["solid"], *p["velocity"], s_in=1.0, s_eq=0.0, Da=0.45)
            assert orc.residual_norm(op, s.cpu().numpy()) < 1.5e-8
    t = time.time()
    for pb, prm in zip(pbs, params):
        sv.solve_soc_steady(pb.ctx, prm, want_state=False)
    torch.cuda.synchronize()
    seq = time.time() - t
    print(f"one after another {seq:.2f}s; batched/sequential {makespan / seq:.2f}", flush=True)
