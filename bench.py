#!/usr/bin/env python3
"""Benchmark of the steady state-of-charge solve on one MI355X.

Workload: the paper-scale single-GPU slab, 1024 x 512 x 256 voxels (134,217,728 cells;
h = 1.25 um as in the paper's logpile run), overlapping fibres of radius 4 voxels with
random orientations in the y-z plane, porosity 0.78, Darcy face velocities at cell Peclet
0.2, 1 and 5 (one flow field scaled three ways).  Finite-rate surface reaction Da = 0.45
per fibre face, inlet s = 1, s_eq = 0.  Inputs are seeded and synthetic.

Step (what --steps and --warmup count): one pass of the solve's loop body at cell Peclet 1,
through the library's entry point (socfv_solve_soc_steady, FP32 mode, warm-started from the
previous step's state): the FP64 refresh of the residual r0 = b - A s, 400 FP32 correction
sweeps in two checked chunks (FP64 residual reduction and the convergence test after each),
the FP64 update s += delta with its refresh, and U and the flux balance of the new state.
The timed steps continue one trajectory toward the steady state.  value = cell updates per
second over the timed steps (all lattice cells, every sweep), in GLUPS.

The same JSON line also carries, from the same run:
  to_steady     the full solves from s = s_in to residual 1e-8 at Peclet 0.2, 1, 5: time,
                sweeps, GLUPS, U and 1 - U (the benchmark's metric "to steady s")
  roofline      the dominant kernel (the FP32 correction sweep, two per launch), its launch
                time from HIP events on the library's stream inside the timed steps
  cpu_baseline  the FP64 CPU oracle on the host's cores: per-sweep rate on the slab (value),
                a full 64 x 32 x 32 solve, and bounded samples of the 256 x 128 x 128 solve
                and adjoint (projected to the GPU's sweep counts, stated as such)
  accuracy      FP32-mode errors against the oracle: 64 x 32 x 32 exact solve; 256 x 128 x 128
                stored oracle solves (finite rate, mass-transport limit, a mid-range-U case)
  adjoint       256 x 128 x 128 with lognormal activity: adjoint / forward time, gradients
                against the stored oracle adjoint and against finite differences
  batch         48 uneven problems: batched makespan against the problems solved one by one
Legs after the step and the solves to steady state run while the wall budget (--budget
seconds from process start) allows; a skipped leg says so.  Separate runs:
--leg flow | logpile | upsampling | batch print their own line.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--budget 420]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

T_START = time.time()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GLUPS & HBM GB/s (% peak) to steady s at residual 1e-8; U_mt err; adjoint/fwd time"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per cell update of the FP32 correction sweep:
# s in 4 + s out 4 + three lower-face velocities 12 + flag byte 1 + frozen residual 4
BYTES_FP32_DC = 25
# FP64 sweep: s in 8 + s out 8 + three lower-face velocities 24 + flag byte 1
BYTES_FP64_SWEEP = 41
# FP64 refresh: s64 in 8 + correction in 4 + faces 24 + flags 1 + s64 out 8 + residual out 4
BYTES_REFRESH = 49
STEP_SWEEPS = 400
DOMINANT = "k_sweep2"


def log(msg):
    print(f"[bench {time.time() - T_START:6.1f}s] {msg}", file=sys.stderr, flush=True)


def elapsed():
    return time.time() - T_START


def parse_scale(s):
    if not s:
        return None
    nx, ny, nz = (int(v) for v in s.lower().split("x"))
    return nx, ny, nz


def kernel_sha():
    src = os.path.join(ROOT, "paper_2502_08034_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()


def counter_traffic(kernel_tag=DOMINANT):
    """HBM bytes per launch of the dominant kernel from the committed counter summary, or
    None when the kernel source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_slab1024_pmc.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if f"sha256 at measurement: {kernel_sha()}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith("| traffic per launch |"):
            return float(line.split("|")[2].split("GB")[0]) * 1e9
    return None


def build_slab(scale, device):
    from paper_2502_08034_amd import inputs as I
    cfg = I.WORKLOADS["slab1024"]
    nx, ny, nz = scale or cfg["shape"]
    t = time.time()
    geo = I.fibres_boolean(nx, ny, nz, cfg["radius"], cfg["porosity"], cfg["seed"])
    log(f"geometry {nx}x{ny}x{nz}: {geo.n_fibres} fibres, porosity {geo.porosity:.4f}, "
        f"{geo.filled} cells filled, {time.time() - t:.1f}s")
    t = time.time()
    u, info = I.darcy_velocity(geo.solid, 1.0, rtol=1e-12, device=device, return_info=True,
                               log=log, as_numpy=False)
    log(f"darcy: {info['cg_iterations']} CG iterations, rel residual "
        f"{info['rel_residual'][0]:.2e}, {time.time() - t:.1f}s")
    return geo, u


# ------------------------------------------------------------------------------------
# GPU legs
# ------------------------------------------------------------------------------------

def solve_row(st, ncell, wall=None):
    sec = st.seconds if wall is None else wall
    return {"seconds": sec, "sweeps": st.iterations, "fp32_sweeps": st.it_fp32,
            "fp64_sweeps": st.sweeps_fp64, "refreshes": st.cycles, "residual": st.residual,
            "U": st.U, "one_minus_U": 1.0 - st.U, "glups": st.iterations * ncell / sec / 1e9,
            "status": st.status,
            "balance_rel": abs(st.flux_in - st.flux_out - st.reaction - st.sum_R)
            / abs(st.flux_in)}


def to_steady(sv, torch, pb, pes, tol, ncell):
    p = sv.params(precision="fp32", tol=tol, check_every=200)
    rows = {}
    for pe in pes:
        pb.set_flow_rate(pe)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = sv.solve_soc_steady(pb.ctx, p, want_state=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        if st.status != sv.OK:
            raise RuntimeError(f"Pe {pe}: status {st.status}")
        rows[f"{pe:g}"] = solve_row(st, ncell, wall)
        log(f"to steady Pe={pe}: {st.iterations} sweeps ({st.it_fp32} fp32, {st.sweeps_fp64} "
            f"fp64, {st.cycles} refreshes), res {st.residual:.2e}, U={st.U:.12f}, {wall:.2f}s")
    sec = sum(r["seconds"] for r in rows.values())
    sw = sum(r["sweeps"] for r in rows.values())
    return {"tol": tol, "per_peclet": rows, "seconds": sec, "sweeps": sw,
            "glups": sw * ncell / sec / 1e9}


def fibre256_problem(sv, with_velocity=True):
    from paper_2502_08034_amd import inputs as I
    w = I.workload("fibre256", with_velocity=False)
    solid = w["solid"]
    u = I.darcy_velocity(solid, 1.0, rtol=1e-12, device="cuda", as_numpy=False)
    return solid, u


def accuracy_c1(sv, orc):
    """FP32 mode against the oracle's exact fixed point on 64 x 32 x 32."""
    from paper_2502_08034_amd import inputs as I
    w = I.workload("fibre64")
    solid = w["solid"]
    u = w["velocity"][0.5]
    pb = sv.Problem.create(solid, *u)
    pore = solid == 0
    p = sv.params(precision="fp32", tol=1e-10, check_every=100)
    s, st = sv.solve_soc_steady(pb.ctx, p)
    op = orc.Problem(solid, *u, s_in=1.0, s_eq=0.0, Da=0.45)
    sx = orc.exact_steady(op)
    Ux = orc.outputs(op, sx)["U"]
    umt, smt, _ = sv.compute_umt(pb.ctx, p, want_state=True)
    opm = orc.Problem(solid, *u, s_in=0.0, s_eq=1.0, pinned=True)
    smx = orc.exact_steady(opm)
    umx = orc.outputs(opm, smx)["U"]
    return {"max_abs_ds": float(np.abs(s.cpu().numpy() - sx)[pore].max()),
            "U": st.U, "U_rel_err": abs(st.U - Ux) / abs(Ux),
            "one_minus_U_rel_err": abs(st.U - Ux) / min(abs(Ux), abs(1 - Ux)),
            "U_mt": umt, "U_mt_rel_err": abs(umt - umx) / abs(umx),
            "U_mt_max_abs_ds": float(np.abs(smt.cpu().numpy() - smx)[pore].max()),
            "reference": "oracle sparse direct solve", "tol": 1e-10}


def accuracy_c2(sv, torch, solid, u, ncell):
    """FP32 mode against the stored FP64 oracle solves of 256 x 128 x 128.  U saturates near
    1 at Da 0.45 (1 - U ~ 3e-4) and in the mass-transport limit (1 - U ~ 7e-8), so the error
    is also stated relative to min(U, 1 - U); the mid-range case (smaller Da) has U ~ 0.5."""
    out = {}
    for fname in ("fibre256.json", "fibre256_mid.json"):
        gpath = os.path.join(ROOT, "tests", "golden", fname)
        if not os.path.exists(gpath):
            continue
        gold = json.load(open(gpath))
        if hashlib.sha256(solid.tobytes()).hexdigest() != gold["geometry_sha256"]:
            out[fname] = {"skipped": "geometry differs from the stored references"}
            continue
        pb = sv.Problem.create(solid, *u)
        idx = torch.as_tensor(np.asarray(gold["sample_index"]), device="cuda")
        for mode in [k for k in ("finite", "pinned", "mid") if k in gold]:
            g = gold[mode]
            p = sv.params(precision="fp32", tol=1e-8, mode=1 if g["pinned"] else 0,
                          s_in=g["s_in"], s_eq=g["s_eq"], Da=g["Da"])
            torch.cuda.synchronize()
            t = time.perf_counter()
            s, st = sv.solve_soc_steady(pb.ctx, p)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t
            Ug = g["outputs"]["U"]
            ds = np.abs(s.view(-1)[idx].cpu().numpy() - np.asarray(g["s_sample"])).max()
            out[mode] = {"Da": g["Da"], "U": st.U, "U_ref": Ug,
                         "U_rel_err": abs(st.U - Ug) / abs(Ug),
                         "one_minus_U_rel_err": abs(st.U - Ug) / max(abs(1 - Ug), 1e-300),
                         "err_rel_min_U_1mU": abs(st.U - Ug) / min(abs(Ug), abs(1 - Ug)),
                         "max_abs_ds_sampled": float(ds), "n_sampled": int(idx.numel()),
                         "sweeps": st.iterations, "residual": st.residual, "seconds": wall,
                         "glups": st.iterations * ncell / wall / 1e9}
            log(f"C2 {mode}: U {st.U:.10f} (ref {Ug:.10f}), {st.iterations} sweeps, {wall:.2f}s")
        out["reference"] = "stored FP64 oracle solves to residual %.0e" % gold["tol"]
        pb.ctx.destroy()
    return out


def adjoint_c5(sv, torch, solid, u, budget_end):
    """256 x 128 x 128 with lognormal activity (sigma 0.3, seed 5): FP32-mode forward solve to
    residual 1e-8 and adjoint to relative residual 1e-9, adjoint time against the forward's; gradients against the stored oracle adjoint and
    against central differences of FP64 forward solves at the stored 20 voxels (relative
    step 1e-2, warm-started from the base state) while the budget lasts."""
    from paper_2502_08034_amd import inputs as I
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "adjoint256.json")))
    if hashlib.sha256(solid.tobytes()).hexdigest() != gold["geometry_sha256"]:
        return {"skipped": "geometry differs from the stored references"}
    kappa = torch.as_tensor(I.lognormal_activity(solid, 0.3, seed=5), device="cuda")
    pb = sv.Problem.create(solid, *u, kappa=kappa)
    p = sv.params(precision="fp32", tol=1e-8)
    sv.solve_soc_steady(pb.ctx, p, want_state=False)              # untimed priming
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, stf = sv.solve_soc_steady(pb.ctx, p, want_state=False)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t
    t = time.perf_counter()
    g, dlnq, _, sta = sv.solve_soc_adjoint(pb.ctx, sv.params(precision="fp32", tol=1e-9))
    torch.cuda.synchronize()
    ta = time.perf_counter() - t
    gn = g.cpu().numpy().ravel()
    gmax = gold["grad_abs_max"]
    errs = {}
    for key_c, key_v in (("fd_cells", "dU_dkappa_fd_cells"), ("sample_cells", "dU_dkappa_sample")):
        cells = np.asarray(gold[key_c])
        ref = np.asarray(gold[key_v])
        errs[key_c] = float((np.abs(gn[cells] - ref) / np.maximum(np.abs(ref), 1e-3 * gmax)).max())
    out = {"forward_seconds": tf, "adjoint_seconds": ta, "adjoint_fwd_ratio": ta / tf,
           "forward_sweeps": stf.iterations, "adjoint_sweeps": sta.iterations,
           "status": sta.status, "dU_dlnq": dlnq,
           "dU_dlnq_rel_err_vs_oracle": abs(dlnq - gold["dU_dlnq"]) / abs(gold["dU_dlnq"]),
           "grad_rel_err_vs_oracle_fd_cells": errs["fd_cells"],
           "grad_rel_err_vs_oracle_2000_cells": errs["sample_cells"],
           "reference": "stored FP64 oracle adjoint to relative residual 1e-12"}
    log(f"C5 adjoint {ta:.2f}s vs forward {tf:.2f}s (ratio {ta / tf:.2f}), grad err vs oracle "
        f"{errs['sample_cells']:.2e}")
    # central differences at the stored voxels (FP64 forward solves, 20000 sweeps from the
    # converged base state), as many as the budget allows
    p64 = sv.params(precision="fp64", tol=1e-12, max_iter=200000)
    base, _ = sv.solve_soc_steady(pb.ctx, p64)
    pfd = sv.params(precision="fp64", tol=0.0, max_iter=20000)
    scale = p64.s_eq - p64.s_in
    kflat = kappa.view(-1)
    fd_rows = []
    t_one = None
    for c in gold["fd_cells"]:
        if t_one is not None and time.time() + 1.5 * t_one > budget_end:
            break
        t = time.time()
        k0 = float(kflat[int(c)])
        h = 1e-2 * k0
        so = []
        for sgn in (1.0, -1.0):
            k2 = kappa.clone()
            k2.view(-1)[int(c)] = k0 + sgn * h
            pb.set_activity(k2)
            _, st = sv.solve_soc_steady(pb.ctx, pfd, s_init=base, want_state=False)
            so.append(st.s_out)
        fd = (so[0] - so[1]) / (2 * h) / scale
        gv = float(gn[int(c)])
        bound = 1e-4 * abs(fd) if abs(fd) >= 1e-3 * gmax else 1e-4 * gmax
        fd_rows.append(abs(fd - gv) / bound)
        t_one = time.time() - t
    pb.set_activity(kappa)
    out["fd_voxels"] = len(fd_rows)
    out["fd_worst_err_over_bound"] = max(fd_rows) if fd_rows else None
    out["fd_protocol"] = ("central differences in kappa at the stored voxels, relative step "
                          "1e-2, FP64 solves; bound 1e-4 |fd| (1e-4 max|grad| where |fd| < 1e-3 "
                          "max|grad|)")
    pb.ctx.destroy()
    return out


def batch_c4(sv, torch, budget_end):
    """48 uneven problems (seeds 100-147): one batched solve against the same problems one
    after another, each to residual 1e-8 in FP32 mode."""
    from paper_2502_08034_amd import inputs as I
    t = time.time()
    probs = I.batch_workloads(48, seed0=100, device="cuda")
    log(f"C4: 48 geometries + Darcy in {time.time() - t:.1f}s")
    pbs = [sv.Problem.create(p["solid"], *p["velocity"]) for p in probs]
    ctxs = [pb.ctx for pb in pbs]
    params = [sv.params(precision="fp32", tol=1e-8) for _ in probs]
    cells = np.array([p["solid"].size for p in probs])
    sv.batch_solve(ctxs[:2], params[:2], want_states=False)       # untimed priming
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, stats = sv.batch_solve(ctxs, params, want_states=False)
    torch.cuda.synchronize()
    mk = time.perf_counter() - t
    sweeps = np.array([st.iterations for st in stats])
    ok = all(st.status == sv.OK for st in stats)
    upd = float((sweeps * cells).sum())
    out = {"problems": len(probs), "cells_total": int(cells.sum()), "makespan_s": mk,
           "glups_aggregate": upd / mk / 1e9, "all_converged": ok,
           "sweeps_min": int(sweeps.min()), "sweeps_median": float(np.median(sweeps)),
           "sweeps_max": int(sweeps.max())}
    log(f"C4 batched: {mk:.2f}s, {upd / mk / 1e9:.1f} GLUPS, sweeps {sweeps.min()}-{sweeps.max()}")
    if time.time() + 2.0 * mk < budget_end:
        torch.cuda.synchronize()
        t = time.perf_counter()
        for pb, p in zip(pbs, params):
            sv.solve_soc_steady(pb.ctx, p, want_state=False)
        torch.cuda.synchronize()
        seq = time.perf_counter() - t
        out.update({"sequential_s": seq, "speedup_vs_sequential": seq / mk,
                    "glups_sequential": upd / seq / 1e9})
        log(f"C4 one by one: {seq:.2f}s ({seq / mk:.2f}x)")
    else:
        out["sequential_s"] = "skipped: wall budget"
    for pb in pbs:
        pb.ctx.destroy()
    return out


# ------------------------------------------------------------------------------------
# CPU oracle (the reported baseline)
# ------------------------------------------------------------------------------------

def cpu_baseline(orc, geo, u_np, seconds):
    """The FP64 oracle on the host's cores.  value: per-sweep rate on the slab (a bounded
    sample, not run to steady state); plus the full 64 x 32 x 32 solve to residual 1e-10."""
    from paper_2502_08034_amd import inputs as I
    ux, uy, uz = u_np
    op = orc.Problem(geo.solid, ux, uy, uz, s_in=1.0, s_eq=0.0, Da=0.45)
    n = geo.solid.size
    dt = 0.4 / orc.max_diag(op)
    s = orc.iterate(op, op.initial_state(), dt, 1)    # untimed: first touch of the arrays
    t = time.time()
    s = orc.iterate(op, s, dt, 1)
    t1 = time.time() - t                               # one warm sweep sizes the sample
    m = max(1, int(seconds / max(t1, 1e-3)))
    t = time.time()
    s = orc.iterate(op, s, dt, m)
    el = time.time() - t
    del s, op
    out = {"value": m * n / el / 1e9, "unit": "GLUPS", "cores": orc.num_threads(),
           "kind": "oracle",
           "sample": f"{m} FP64 explicit sweeps (after 2 untimed) of the "
                     f"{geo.solid.shape[2]}x{geo.solid.shape[1]}x{geo.solid.shape[0]} slab at "
                     f"Peclet 1 from s = s_in ({el:.1f} s); per-sweep rate, not run to steady "
                     f"state", "nproc": os.cpu_count()}
    w = I.workload("fibre64")
    o1 = orc.Problem(w["solid"], *w["velocity"][0.5], s_in=1.0, s_eq=0.0, Da=0.45)
    t = time.time()
    _, info = orc.solve(o1, cfl=0.4, tol=1e-10, check_every=100)
    e1 = time.time() - t
    out["c1_full_solve"] = {"seconds": e1, "sweeps": info["iterations"],
                            "glups": info["iterations"] * w["solid"].size / e1 / 1e9,
                            "residual": info["residual"], "tol": 1e-10,
                            "workload": "fibre64 (64x32x32, Peclet 0.5, Da 0.45)"}
    return out


def cpu_samples_256(orc, solid2, u2, counts):
    """Bounded samples of the oracle's explicit solve and adjoint iteration on 256 x 128 x 128
    (a full FP64 solve takes minutes on the host), projected to the sweep counts the GPU
    needed; stated as projections."""
    from paper_2502_08034_amd import inputs as I
    n2 = solid2.size
    o2 = orc.Problem(solid2, *u2, s_in=1.0, s_eq=0.0, Da=0.45)
    dt2 = 0.4 / orc.max_diag(o2)
    s2 = orc.iterate(o2, o2.initial_state(), dt2, 1)
    k2 = 60
    t = time.time()
    orc.iterate(o2, s2, dt2, k2)
    per = (time.time() - t) / k2
    c2 = {"sample_sweeps": k2, "seconds_per_sweep": per, "glups": n2 / per / 1e9}
    if counts.get("c2_sweeps"):
        c2["projected_seconds_to_1e-8"] = per * counts["c2_sweeps"]
        c2["projection"] = (f"{counts['c2_sweeps']} sweeps (the GPU's count at 1e-8 for the "
                            "same explicit iteration) x the sampled time per sweep")
    out = {"c2_solve": c2}
    kappa = I.lognormal_activity(solid2, 0.3, seed=5).astype(np.float64)
    o5 = orc.Problem(solid2, *u2, s_in=1.0, s_eq=0.0, Da=0.45, kappa=kappa)
    k5 = 40
    t = time.time()
    orc.adjoint(o5, tol=0.0, max_iter=k5, check_every=k5)
    per5 = (time.time() - t) / k5
    c5 = {"sample_sweeps": k5, "seconds_per_sweep": per5}
    if counts.get("c5_adjoint_sweeps"):
        c5["projected_adjoint_seconds"] = per5 * counts["c5_adjoint_sweeps"]
        c5["projected_forward_seconds"] = per * counts["c5_forward_sweeps"]
        c5["projection"] = "the GPU's sweep counts x the sampled time per sweep"
    out["c5_adjoint"] = c5
    return out


# ------------------------------------------------------------------------------------
# Separate legs (own JSON line)
# ------------------------------------------------------------------------------------

def logpile_sweep(sv, torch, pes, volts=(-2.0, 0.0, 2.0), s_in=1.7e-7):
    """Voltage x flow-rate sweep on the logpile lattice (h = 1.25 um, 1024 x 512 x 128):
    one batched FP32 solve of every (V, Pe) problem to residual 1e-8; s_eq = sigma(V),
    Da = 0.45 cosh(V / 2), the paper's inlet SOC."""
    from paper_2502_08034_amd import inputs as I
    t = time.time()
    g = I.logpile(1.25)
    u, info = I.darcy_velocity(g.solid, 1.0, device="cuda", return_info=True, log=log,
                               as_numpy=False)
    log(f"logpile {g.solid.shape[::-1]}, porosity {g.porosity:.4f}, Darcy {info['cg_iterations']} "
        f"iterations, {time.time() - t:.1f}s")
    pbs = {V: sv.Problem.create(g.solid, *u) for V in volts}
    n = g.solid.size
    table, total, sweeps = {}, 0.0, 0
    for pe in pes:
        params = [sv.params(precision="fp32", tol=1e-8, s_in=s_in, **I.voltage_params(V))
                  for V in volts]
        for V in volts:
            pbs[V].set_flow_rate(pe)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, stats = sv.batch_solve([pbs[V].ctx for V in volts], params, want_states=False)
        torch.cuda.synchronize()
        mk = time.perf_counter() - t
        total += mk
        k = sum(st.iterations for st in stats)
        sweeps += k
        for V, st in zip(volts, stats):
            table[f"V={V:+g},Pe={pe:g}"] = {"U": st.U, "sweeps": st.iterations,
                                            "status": st.status}
        log(f"Pe {pe}: batch of {len(volts)} in {mk:.1f}s, {k} sweeps, "
            f"{k * n / mk / 1e9:.1f} GLUPS")
    return {"metric": "logpile voltage x flow sweep (batched per flow rate)",
            "problems": len(volts) * len(pes), "cells": n, "seconds": total,
            "sweeps": sweeps, "glups": sweeps * n / total / 1e9,
            "porosity": g.porosity, "s_in": s_in, "results": table}


def stokes_flow(sv, torch, name="fibre256", cfl=0.5, tol=1e-9, max_steps=10**7, scale=None):
    """Upstream flow step on a fibre workload: steady Stokes flow from rest by projection
    steps (eps_flow = 1e-9), then the SOC solve on that flow at cell Peclet 1."""
    from paper_2502_08034_amd import inputs as I
    log(f"flow workload {name}: building the geometry")
    w = I.workload(name, with_velocity=False, scale=scale)
    solid = w["solid"]
    nz, ny, nx = solid.shape
    n = solid.size
    phi = float((solid == 0).mean())
    ctx = sv.setup_geometry(torch.as_tensor(solid, device="cuda"))
    sv.solve_stokes(ctx, cfl=cfl, max_steps=10, check_every=10)       # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    if n < 50_000_000:
        ux, uy, uz, _, st = sv.solve_stokes(ctx, cfl=cfl, tol=tol, max_steps=max_steps)
    else:
        # large boxes: resumed calls of 2000 steps, each reporting its progress
        ux, uy, uz, pr, st = sv.solve_stokes(ctx, cfl=cfl, tol=tol,
                                             max_steps=min(2000, max_steps), want_pressure=True)
        steps, cg = st.steps, st.cg_iterations
        while st.status == sv.NOT_CONVERGED and steps < max_steps:
            log(f"flow {nx}x{ny}x{nz}: {steps} steps, change {st.change:.2e}, "
                f"{time.perf_counter() - t:.1f}s")
            ux, uy, uz, pr, st = sv.solve_stokes(ctx, cfl=cfl, tol=tol, start=(ux, uy, uz, pr),
                                                 max_steps=min(2000, max_steps - steps))
            steps += st.steps
            cg += st.cg_iterations
        st.steps, st.cg_iterations = steps, cg
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    log(f"Stokes flow {nx}x{ny}x{nz}: {st.steps} steps, {st.cg_iterations} CG iterations, "
        f"{el:.2f}s, change {st.change:.2e}")
    out = {"metric": "steady Stokes flow by projection steps", "workload": name,
           "shape": [nx, ny, nz], "cells": n, "porosity": phi, "cfl": cfl, "tol": tol,
           "status": st.status, "steps": st.steps, "cg_iterations": st.cg_iterations,
           "seconds": el, "ms_per_step": 1e3 * el / st.steps,
           "cell_steps_per_s": n * st.steps / el, "change": st.change,
           "divergence_rel": st.divergence / st.u_max, "Q": st.Q, "Q_out": st.Q_out}
    if st.status == sv.OK:
        q = 1.0 / ((st.Q / (ny * nz)) / phi)
        sv.set_velocity(ctx, ux, uy, uz, q=q)
        _, sst = sv.solve_soc_steady(ctx, sv.params(precision="fp32", tol=1e-8),
                                     want_state=False)
        out["soc_pe1"] = {"U": sst.U, "sweeps": sst.iterations, "status": sst.status}
    return out


def upsampling_leg(sv, torch, pb, tol):
    """Iterative upsampling at Peclet 1: the coarse (2x) steady state as the fine solve's
    start, against the plain solve from s = s_in."""
    p = sv.params(precision="fp32", tol=tol, check_every=200)
    pb.set_flow_rate(1.0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, stp = sv.solve_soc_steady(pb.ctx, p, want_state=False)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t
    t = time.perf_counter()
    _, stu, stc = sv.solve_soc_upsampled(pb.ctx, p, want_state=False)
    torch.cuda.synchronize()
    tu = time.perf_counter() - t
    return {"metric": "iterative upsampling of the SOC solve (slab, Peclet 1)",
            "plain_seconds": tp, "upsampled_seconds": tu, "speedup": tp / tu,
            "plain_sweeps": stp.iterations, "fine_sweeps": stu.iterations,
            "coarse_sweeps": stc.iterations, "U_plain": stp.U, "U_upsampled": stu.U}


# ------------------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--budget", type=float, default=420.0,
                    help="wall seconds from process start within which the legs after the "
                         "solves to steady state may run")
    ap.add_argument("--scale", default=None, help="override the slab box, e.g. 256x128x64")
    ap.add_argument("--peclet", default="0.2,1,5")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--cpu-seconds", type=float, default=24.0)
    ap.add_argument("--skip", default="", help="comma list of legs to leave out: steady, cpu, "
                    "accuracy, adjoint, batch")
    ap.add_argument("--leg", default=None,
                    choices=["flow", "logpile", "upsampling", "batch", "adjoint"],
                    help="run one separate leg and print its own JSON line")
    ap.add_argument("--flow-cfl", type=float, default=3.5)
    ap.add_argument("--flow-workload", default="fibre256")
    ap.add_argument("--flow-max-steps", type=int, default=10**7)
    ap.add_argument("--calibrate", action="store_true",
                    help="start with the counter-calibration copies (for rocprofv3 --pmc runs)")
    ap.add_argument("--tiles", default=None, help="tile_y,z_chunk,z_chunk2,two for the sweeps")
    ap.add_argument("--profile-sweeps", type=int, default=0,
                    help="profiling run: this many FP32 correction sweeps at Peclet 1 on the "
                         "slab, and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    skip = set(filter(None, args.skip.split(",")))
    budget_end = T_START + args.budget

    import torch
    from paper_2502_08034_amd import socfv as sv

    assert torch.cuda.is_available(), "bench needs a GPU"
    log(f"torch {torch.__version__} on {torch.cuda.get_device_name(0)}")
    if args.profile_sweeps or args.calibrate:
        # counter calibration, first kernels of the process: 4 converting copies of 2^28
        # FP32 values to FP64 (1 GiB read, 2 GiB written each)
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        c = torch.empty(1 << 28, dtype=torch.float64, device="cuda")
        for _ in range(4):
            c.copy_(a)
        torch.cuda.synchronize()
        del a, c
    pes = [float(v) for v in args.peclet.split(",")]
    if args.leg == "logpile":
        print(json.dumps(logpile_sweep(sv, torch, pes)), flush=True)
        return
    if args.leg == "batch":
        out = batch_c4(sv, torch, budget_end)
        out["metric"] = "batched solve of 48 uneven problems (seeds 100-147) to residual 1e-8"
        print(json.dumps(out), flush=True)
        return
    if args.leg == "adjoint":
        solid2, u2 = fibre256_problem(sv)
        out = adjoint_c5(sv, torch, solid2, u2, budget_end)
        out["metric"] = "adjoint / forward time on 256x128x128 with a lognormal activity field"
        print(json.dumps(out), flush=True)
        return
    if args.leg == "flow":
        print(json.dumps(stokes_flow(sv, torch, name=args.flow_workload, cfl=args.flow_cfl,
                                     max_steps=args.flow_max_steps,
                                     scale=parse_scale(args.scale))), flush=True)
        return

    geo, u1 = build_slab(parse_scale(args.scale), "cuda")
    nz, ny, nx = geo.solid.shape
    ncell = nx * ny * nz
    t = time.time()
    pb = sv.Problem.create(geo.solid, *u1)
    info = pb.ctx.info()
    log(f"setup_geometry + set_velocity: {time.time() - t:.1f}s, {info['pore']} pore cells, "
        f"{info['reactive']} reactive")
    tiles = None
    if args.tiles:
        vals = [int(v) for v in args.tiles.split(",")] + [0, 0, 0, -1]
        sv.set_tiles(pb.ctx, *vals[:4])
        tiles = tuple(vals[:4])
    if args.profile_sweeps:
        pb.set_flow_rate(1.0)
        pp = sv.params(precision="fp32", tol=0.0, max_iter=args.profile_sweeps, check_every=200)
        _, st = sv.solve_soc_steady(pb.ctx, pp, want_state=False)
        avg = st.ms_fp32 / max(st.it_fp32, 1)
        # the FP64 plane-march kernels: 100 FP64 sweeps (partials on the last), and 20 short
        # FP32 solves, each of which starts with a refresh and ends with the outputs
        _, s64 = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp64", tol=0.0, max_iter=100,
                                                        check_every=100), want_state=False)
        ms_ref, n_ref = 0.0, 0
        for _ in range(20):
            _, sr = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp32", tol=0.0, max_iter=4,
                                                           check_every=4), want_state=False)
            ms_ref += sr.ms_refresh
            n_ref += sr.cycles
        sw64 = s64.ms_fp64 / max(s64.iterations, 1)
        ref = ms_ref / max(n_ref, 1)
        print(json.dumps({"profile_sweeps": st.it_fp32, "avg_sweep_ms": avg,
                          "avg_launch_us": 2e3 * avg,
                          "achieved_GBs": BYTES_FP32_DC * ncell / (avg / 1e3) / 1e9,
                          "fp64_sweeps": s64.iterations, "fp64_sweep_ms": sw64,
                          "fp64_sweep_GBs": BYTES_FP64_SWEEP * ncell / (sw64 / 1e3) / 1e9,
                          "refreshes": n_ref, "refresh_ms": ref,
                          "refresh_GBs": BYTES_REFRESH * ncell / (ref / 1e3) / 1e9,
                          "cells": ncell, "tiles": tiles}), flush=True)
        return
    if args.leg == "upsampling":
        print(json.dumps(upsampling_leg(sv, torch, pb, args.tol)), flush=True)
        return

    # ---- the timed steps -------------------------------------------------------------
    pb.set_flow_rate(1.0)
    p_step = sv.params(precision="fp32", tol=0.0, max_iter=STEP_SWEEPS, check_every=200)
    state = None

    def step():
        nonlocal state
        s, st = sv.solve_soc_steady(pb.ctx, p_step, s_init=state)
        if st.status < 0 or st.iterations != STEP_SWEEPS:
            raise RuntimeError(f"step: status {st.status}, {st.iterations} sweeps")
        state = s
        return st

    step()                                   # untimed priming: buffers, kernels, first state
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sweeps = sum(st.iterations for st in stats)
    glups = sweeps * ncell / el / 1e9
    ms32 = sum(st.ms_fp32 for st in stats)
    n32 = sum(st.it_fp32 for st in stats)
    avg32 = ms32 / n32
    avg_launch_s = 2.0 * avg32 / 1e3
    achieved = 2 * BYTES_FP32_DC * ncell / avg_launch_s / 1e9
    traffic = counter_traffic() if (nx, ny, nz) == (1024, 512, 256) else None
    log(f"{args.steps} steps in {el:.2f}s: {glups:.1f} GLUPS, {DOMINANT} {2e3 * avg32:.1f} us "
        f"per launch, {achieved:.0f} GB/s algorithmic; residual after the steps "
        f"{stats[-1].residual:.3e}")
    del state
    result = {
        "metric": METRIC, "value": glups, "unit": "GLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"slab1024: {nx}x{ny}x{nz} fibre slab (boolean fibres r=4 in the "
                               f"y-z plane, porosity {geo.porosity:.3f}), Darcy velocity, Da "
                               f"0.45/face; step = one {STEP_SWEEPS}-sweep pass of the FP32 "
                               f"correction solve at cell Peclet 1 (FP64 refreshes, "
                               f"reductions, convergence test, U and balance)",
                   "cells": ncell, "pore_cells": info["pore"], "sweeps_per_step": STEP_SWEEPS,
                   "precision": "fp32 sweeps + fp64 refresh/reductions",
                   "tiles": list(tiles) if tiles else None},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"{DOMINANT}<correction> (FP32 correction sweeps, two per launch)",
                     "achieved_is": "algorithmic bytes (25 B per cell update, two updates per "
                                    "launch) / average launch time",
                     "bytes_per_launch": 2 * BYTES_FP32_DC * ncell,
                     "avg_launch_us": avg_launch_s * 1e6, "launches_timed": n32 // 2,
                     "measured_GBs": traffic / avg_launch_s / 1e9 if traffic else None,
                     "measured_frac": traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS
                     if traffic else None,
                     "kernel_source_sha256": kernel_sha()},
        "glups_pore_only": glups * info["pore"] / ncell,
    }
    log(f"main part done at {elapsed():.0f}s")

    # ---- to steady state at the three flow rates -------------------------------------
    if "steady" not in skip:
        result["to_steady"] = to_steady(sv, torch, pb, pes, args.tol, ncell)
        ts = result["to_steady"]
        log(f"to steady: {ts['seconds']:.1f}s, {ts['glups']:.1f} GLUPS")
    u_np = tuple(a.cpu().numpy() for a in u1) if "cpu" not in skip else None
    del u1
    pb.ctx.destroy()
    torch.cuda.empty_cache()
    import oracle as orc
    if u_np is not None:
        t = time.time()
        result["cpu_baseline"] = cpu_baseline(orc, geo, u_np, args.cpu_seconds)
        del u_np
        log(f"cpu baseline {time.time() - t:.1f}s: {result['cpu_baseline']['value']:.2f} GLUPS "
            f"on {result['cpu_baseline']['cores']} threads")

    def budget_ok(need, leg):
        ok = time.time() + need < budget_end
        if not ok:
            result.setdefault("skipped", []).append(leg)
            log(f"{leg}: skipped (wall budget: {elapsed():.0f}s used, needs ~{need:.0f}s)")
        return ok

    counts = {}
    solid2 = u2 = None
    if {"accuracy", "adjoint"} - skip and budget_ok(25, "256x128x128 workload"):
        t = time.time()
        solid2, u2 = fibre256_problem(sv)
        log(f"256x128x128 geometry + Darcy {time.time() - t:.1f}s")
    if "accuracy" not in skip and solid2 is not None and budget_ok(15, "accuracy 256x128x128"):
        result["accuracy"] = {"fibre256": accuracy_c2(sv, torch, solid2, u2, solid2.size)}
        counts["c2_sweeps"] = result["accuracy"]["fibre256"].get("finite", {}).get("sweeps")
    if "adjoint" not in skip and solid2 is not None and budget_ok(20, "adjoint"):
        result["adjoint"] = adjoint_c5(sv, torch, solid2, u2, min(budget_end - 150,
                                                                   time.time() + 60))
        counts["c5_adjoint_sweeps"] = result["adjoint"].get("adjoint_sweeps")
        counts["c5_forward_sweeps"] = result["adjoint"].get("forward_sweeps")
    if "batch" not in skip and budget_ok(90, "batch"):
        result["batch"] = batch_c4(sv, torch, budget_end - 60)
    if "accuracy" not in skip and budget_ok(20, "accuracy 64x32x32"):
        result.setdefault("accuracy", {})["fibre64"] = accuracy_c1(sv, orc)
    if "cpu_baseline" in result and solid2 is not None and budget_ok(30, "cpu 256x128x128"):
        u2n = tuple(a.cpu().numpy() for a in u2)
        result["cpu_baseline"].update(cpu_samples_256(orc, solid2, u2n, counts))
    result["wall_seconds"] = elapsed()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
