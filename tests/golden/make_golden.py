"""Write the stored oracle references for the 256x128x128 workloads.

Calls only the FP64 CPU oracle (``oracle/``) and the seeded input generator.  The
references are too slow to recompute inside a GPU test (tens of thousands of explicit
FP64 sweeps over 4.2M cells on the host), so they are stored here as small JSON files:
scalar outputs plus the state at seeded sample cells.

    python tests/golden/make_golden.py fibre256      # finite rate + mass-transport limit
    python tests/golden/make_golden.py fibre256_mid  # finite rate with U in mid-range
    python tests/golden/make_golden.py adjoint256    # lognormal activity + adjoint

Each file also stores a digest of the generated geometry so a test can tell when the
generator no longer reproduces the inputs the references were computed from.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O                                        # noqa: E402
from paper_2502_08034_amd import inputs as I               # noqa: E402

TOL = 2e-12            # explicit-iteration residual for the references
CHECK = 200
N_SAMPLE = 4096


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def sample_cells(solid, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    pore = np.flatnonzero(solid.ravel() == 0)
    return np.sort(rng.choice(pore, size=min(n, pore.size), replace=False))


def solve_ref(pb, label):
    t = time.time()
    s, info = O.solve(pb, cfl=0.4, tol=TOL, max_iter=2_000_000, check_every=CHECK)
    info["seconds"] = time.time() - t
    info["threads"] = O.num_threads()
    log(f"{label}: {info}")
    return s, info


def fibre256():
    w = I.workload("fibre256", log=log)
    solid = w["solid"]
    ux, uy, uz = w["velocity"][1.0]
    idx = sample_cells(solid, N_SAMPLE, 2024)
    res = {"workload": "fibre256", "shape": list(w["shape"]), "geometry_sha256": digest(solid),
           "porosity": w["geometry"].porosity, "n_fibres": w["geometry"].n_fibres,
           "darcy": w["darcy"], "tol": TOL, "check_every": CHECK, "sample_index": idx.tolist()}
    for mode, (s_in, s_eq, pinned) in {"finite": (1.0, 0.0, False),
                                       "pinned": (0.0, 1.0, True)}.items():
        pb = O.Problem(solid, ux, uy, uz, s_in=s_in, s_eq=s_eq, Da=0.45, pinned=pinned)
        s, info = solve_ref(pb, mode)
        out = O.outputs(pb, s)
        pore = solid == 0
        res[mode] = {"s_in": s_in, "s_eq": s_eq, "Da": 0.45, "pinned": pinned,
                     "solve": info, "outputs": out,
                     "s_sample": s.ravel()[idx].tolist(),
                     "s_min": float(s[pore].min()), "s_max": float(s[pore].max()),
                     "s_sum": float(s[pore].sum())}
        with open(os.path.join(HERE, "fibre256.json"), "w") as f:
            json.dump(res, f)
    log("wrote fibre256.json")


def fibre256_mid():
    """The same geometry and flow with a slow surface reaction (Da 0.02 per fibre face, about
    1/20 of the benchmark's), which puts U near 0.5: at Da 0.45 U saturates (1 - U ~ 3e-4)
    and an error in U says little about the unconverted fraction."""
    w = I.workload("fibre256", log=log)
    solid = w["solid"]
    ux, uy, uz = w["velocity"][1.0]
    idx = sample_cells(solid, N_SAMPLE, 2025)
    res = {"workload": "fibre256, Da 0.02", "shape": list(w["shape"]),
           "geometry_sha256": digest(solid), "tol": TOL, "check_every": CHECK,
           "sample_index": idx.tolist()}
    pb = O.Problem(solid, ux, uy, uz, s_in=1.0, s_eq=0.0, Da=0.02)
    s, info = solve_ref(pb, "mid")
    pore = solid == 0
    res["mid"] = {"s_in": 1.0, "s_eq": 0.0, "Da": 0.02, "pinned": False, "solve": info,
                  "outputs": O.outputs(pb, s), "s_sample": s.ravel()[idx].tolist(),
                  "s_min": float(s[pore].min()), "s_max": float(s[pore].max()),
                  "s_sum": float(s[pore].sum())}
    with open(os.path.join(HERE, "fibre256_mid.json"), "w") as f:
        json.dump(res, f)
    log("wrote fibre256_mid.json")


def adjoint256():
    w = I.workload("fibre256", log=log)
    solid = w["solid"]
    ux, uy, uz = w["velocity"][1.0]
    kappa = I.lognormal_activity(solid, 0.3, seed=5).astype(np.float64)
    pb = O.Problem(solid, ux, uy, uz, s_in=1.0, s_eq=0.0, Da=0.45, kappa=kappa)
    s, info = solve_ref(pb, "forward")
    t = time.time()
    psi, ainfo = O.adjoint(pb, cfl=0.4, tol=1e-12, max_iter=2_000_000, check_every=CHECK)
    ainfo["seconds"] = time.time() - t
    log(f"adjoint: {ainfo}")
    gk, dlnq = O.gradients(pb, s, psi)
    reactive = np.flatnonzero((pb.nf.ravel() > 0))
    rng = np.random.Generator(np.random.PCG64(6))
    fd_cells = np.sort(rng.choice(reactive, size=20, replace=False))
    more = np.sort(rng.choice(reactive, size=2000, replace=False))
    out = O.outputs(pb, s)
    res = {"workload": "fibre256+lognormal(0.3, seed 5)", "geometry_sha256": digest(solid),
           "kappa_sha256": digest(kappa.astype(np.float32)),
           "forward": info, "adjoint": ainfo, "U": out["U"], "outputs": out,
           "dU_dlnq": dlnq, "fd_cells": fd_cells.tolist(),
           "dU_dkappa_fd_cells": gk.ravel()[fd_cells].tolist(),
           "sample_cells": more.tolist(), "dU_dkappa_sample": gk.ravel()[more].tolist(),
           "grad_abs_max": float(np.abs(gk).max())}
    with open(os.path.join(HERE, "adjoint256.json"), "w") as f:
        json.dump(res, f)
    log("wrote adjoint256.json")


if __name__ == "__main__":
    which = sys.argv[1:] or ["fibre256", "fibre256_mid", "adjoint256"]
    for name in which:
        {"fibre256": fibre256, "fibre256_mid": fibre256_mid, "adjoint256": adjoint256}[name]()
