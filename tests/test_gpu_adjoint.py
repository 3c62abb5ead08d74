"""Discrete adjoint on the GPU (needs an MI355X).

The adjoint solve A^T psi = dU/ds runs the reversed-advection stencil; gradients are
checked against the FP64 oracle's adjoint (sparse solve of the same rows), against central
finite differences of the GPU's own forward solves, and through torch.autograd.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

from paper_2502_08034_amd import inputs as I

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def sv():
    from paper_2502_08034_amd import socfv
    return socfv


def case(nx, ny, nz, seed, pe=1.0):
    g = I.fibres_nonoverlap(nx, ny, nz, 3.0, 0.85, seed)
    return g.solid, I.darcy_velocity(g.solid, pe)


@pytest.mark.parametrize("shape,prec", [((64, 32, 32), "fp64"), ((70, 37, 29), "fp64"),
                                        ((64, 32, 32), "fp32"), ((70, 37, 29), "fp32")])
def test_adjoint_matches_oracle(sv, orc, shape, prec):
    solid, u = case(*shape, seed=41)
    kappa = I.lognormal_activity(solid, 0.3, seed=5)
    pb = sv.Problem.create(solid, *u, kappa=kappa)
    p = sv.params(precision=prec, tol=1e-11, check_every=100)
    s, st = sv.solve_soc_steady(pb.ctx, p)
    g, dlnq, psi, sta = sv.solve_soc_adjoint(pb.ctx, p, want_psi=True)
    assert sta.status == sv.OK
    op = orc.Problem(solid, *u, s_in=1.0, s_eq=0.0, Da=0.45, kappa=kappa.astype(np.float64))
    sx = orc.exact_steady(op)
    px = orc.exact_adjoint(op)
    gx, dlnqx = orc.gradients(op, sx, px)
    tol = 1e-8 if prec == "fp64" else 1e-5
    assert np.abs(psi.cpu().numpy() - px).max() <= tol * np.abs(px).max()
    assert np.abs(g.cpu().numpy() - gx).max() <= tol * np.abs(gx).max()
    assert abs(dlnq - dlnqx) <= tol * abs(dlnqx)


@pytest.mark.parametrize("shape,pinned", [((128, 40, 33), False), ((128, 40, 33), True),
                                          ((95, 37, 29), False)])
def test_adjoint_two_sweep_launches_match_oracle(sv, orc, shape, pinned):
    """FP32-mode adjoint with one and with two transpose sweeps per launch (several tiles,
    ragged in y and z; odd nx takes one cell per lane), each against the oracle's exact
    adjoint; held and fibre cells keep psi = 0."""
    solid, u = case(*shape, seed=45)
    kappa = None if pinned else I.lognormal_activity(solid, 0.3, seed=8)
    pb = sv.Problem.create(solid, *u, kappa=kappa)
    kw = dict(mode=1, s_in=0.0, s_eq=1.0, Da=0.0) if pinned else {}
    p = sv.params(precision="fp32", tol=1e-10, check_every=100, **kw)
    sv.solve_soc_steady(pb.ctx, p)
    if pinned:
        op = orc.Problem(solid, *u, s_in=0.0, s_eq=1.0, pinned=True)
    else:
        op = orc.Problem(solid, *u, s_in=1.0, s_eq=0.0, Da=0.45, kappa=kappa.astype(np.float64))
    sx = orc.exact_steady(op)
    px = orc.exact_adjoint(op)
    gx, dlnqx = orc.gradients(op, sx, px)
    held = (op.nf > 0) & (solid == 0) if pinned else np.zeros(solid.shape, bool)
    for two in (0, 1):
        sv.set_tiles(pb.ctx, 0, 0, 0, two)
        g, dlnq, psi, st = sv.solve_soc_adjoint(pb.ctx, p, want_psi=True)
        assert st.status == sv.OK
        pn = psi.cpu().numpy()
        # the oracle also defines psi on held cells (after the solve); the library keeps 0
        assert np.abs(pn - px)[~held].max() <= 1e-5 * np.abs(px).max(), two
        assert abs(dlnq - dlnqx) <= 1e-5 * abs(dlnqx), two
        if not pinned:
            assert np.abs(g.cpu().numpy() - gx).max() <= 1e-5 * np.abs(gx).max(), two
        assert np.all(pn[solid == 1] == 0.0) and np.all(pn[held] == 0.0)


def test_adjoint_pinned_mode(sv, orc):
    solid, u = case(64, 32, 32, seed=42)
    pb = sv.Problem.create(solid, *u)
    p = sv.params(precision="fp64", tol=1e-11, mode=1, s_in=0.0, s_eq=1.0, Da=0.0)
    sv.solve_soc_steady(pb.ctx, p)
    g, dlnq, psi, _ = sv.solve_soc_adjoint(pb.ctx, p, want_psi=True)
    op = orc.Problem(solid, *u, s_in=0.0, s_eq=1.0, pinned=True)
    sx = orc.exact_steady(op)
    px = orc.exact_adjoint(op)
    _, dlnqx = orc.gradients(op, sx, px)
    free = (solid == 0) & (op.nf == 0)
    assert np.abs(psi.cpu().numpy() - px)[free].max() <= 1e-8 * np.abs(px).max()
    assert np.all(psi.cpu().numpy()[op.nf > 0] == 0.0)
    assert abs(dlnq - dlnqx) <= 1e-8 * abs(dlnqx)
    assert np.all(g.cpu().numpy() == 0.0)


def fd_check(sv, pb, kappa_t, p, cells, grad, rel_step, sweeps=None):
    """Central differences of the outlet mean s in kappa at single voxels; FP64 solves
    warm-started from the converged base state (with ``sweeps``: a fixed number of sweeps
    from it, enough to converge the perturbation below rounding)."""
    base, st0 = sv.solve_soc_steady(pb.ctx, p)
    if sweeps:
        p = sv.params(precision="fp64", tol=0.0, max_iter=sweeps, s_in=p.s_in, s_eq=p.s_eq,
                      Da=p.Da, mode=p.mode)
    scale = p.s_eq - p.s_in
    gmax = float(np.abs(grad).max())
    errs = []
    for c in cells:
        z, y, x = np.unravel_index(int(c), kappa_t.shape)
        k0 = float(kappa_t[z, y, x])
        h = rel_step * k0
        so = []
        for sgn in (1.0, -1.0):
            k2 = kappa_t.clone()
            k2[z, y, x] = k0 + sgn * h
            pb.set_activity(k2)
            _, st = sv.solve_soc_steady(pb.ctx, p, s_init=base, want_state=False)
            so.append(st.s_out)
        fd = (so[0] - so[1]) / (2 * h) / scale
        g = float(grad.reshape(-1)[int(c)])
        bound = 1e-4 * abs(fd) if abs(fd) >= 1e-3 * gmax else 1e-4 * gmax
        errs.append((abs(fd - g), bound, fd, g))
        print(f"  voxel {int(c)}: fd {fd:.6e} adjoint {g:.6e} err/bound {abs(fd - g) / bound:.3f}",
              flush=True)
    pb.set_activity(kappa_t)
    return errs


def test_gradient_against_finite_differences_small(sv):
    solid, u = case(64, 32, 32, seed=43)
    kappa = torch.as_tensor(I.lognormal_activity(solid, 0.3, seed=5), device="cuda")
    pb = sv.Problem.create(solid, *u, kappa=kappa)
    p64 = sv.params(precision="fp64", tol=1e-13, check_every=100)
    sv.solve_soc_steady(pb.ctx, p64)
    g, dlnq, _, _ = sv.solve_soc_adjoint(pb.ctx, p64)
    gn = g.cpu().numpy()
    rng = np.random.default_rng(6)
    reactive = np.flatnonzero((gn != 0).ravel())
    cells = rng.choice(reactive, size=12, replace=False)
    for err, bound, fd, gv in fd_check(sv, pb, kappa, p64, cells, gn, 1e-3):
        assert err <= bound, (fd, gv)
    # flow rate: u = q u0, d U / d ln q by central differences in q
    sv.solve_soc_steady(pb.ctx, p64)
    sv_ = []
    base, _ = sv.solve_soc_steady(pb.ctx, p64)
    for q in (1.0 + 1e-4, 1.0 - 1e-4):
        pb.set_flow_rate(q)
        _, st = sv.solve_soc_steady(pb.ctx, p64, s_init=base, want_state=False)
        sv_.append(st.s_out)
    pb.set_flow_rate(1.0)
    fdq = (sv_[0] - sv_[1]) / 2e-4 / (p64.s_eq - p64.s_in)
    assert abs(fdq - dlnq) <= 1e-4 * abs(fdq)


def test_adjoint256_against_oracle_and_fd(sv):
    """The 256 x 128 x 128 workload with lognormal activity (sigma 0.3): FP32-mode adjoint
    against the stored FP64 oracle adjoint, and against central differences at 20 voxels."""
    gold = json.load(open(os.path.join(HERE, "golden", "adjoint256.json")))
    w = I.workload("fibre256", with_velocity=False)
    solid = w["solid"]
    import hashlib
    assert hashlib.sha256(solid.tobytes()).hexdigest() == gold["geometry_sha256"]
    u = I.darcy_velocity(solid, 1.0, device="cuda", as_numpy=False)
    kappa = torch.as_tensor(I.lognormal_activity(solid, 0.3, seed=5), device="cuda")
    pb = sv.Problem.create(solid, *u, kappa=kappa)
    p = sv.params(precision="fp32", tol=1e-8)
    _, stf = sv.solve_soc_steady(pb.ctx, p)
    assert abs(stf.U - gold["U"]) <= 1e-6 * gold["U"]
    torch.cuda.synchronize()
    g, dlnq, _, sta = sv.solve_soc_adjoint(pb.ctx, sv.params(precision="fp32", tol=1e-9))
    print(f"forward {stf.seconds:.2f}s {stf.iterations} sweeps; adjoint {sta.seconds:.2f}s "
          f"{sta.iterations} sweeps; ratio {sta.seconds / stf.seconds:.2f}", flush=True)
    gn = g.cpu().numpy().ravel()
    gmax = gold["grad_abs_max"]
    for key_c, key_v in (("fd_cells", "dU_dkappa_fd_cells"), ("sample_cells", "dU_dkappa_sample")):
        cells = np.asarray(gold[key_c])
        ref = np.asarray(gold[key_v])
        err = np.abs(gn[cells] - ref)
        bound = np.where(np.abs(ref) >= 1e-3 * gmax, 1e-4 * np.abs(ref), 1e-4 * gmax)
        assert np.all(err <= bound), (key_c, float((err / bound).max()))
    assert abs(dlnq - gold["dU_dlnq"]) <= 1e-4 * abs(gold["dU_dlnq"])
    # Finite differences of FP64 forward solves at the 20 voxels.  U depends on one
    # voxel's activity as a rank-one rational function (A changes by a diagonal entry), so
    # the central difference's truncation error is about (Da n_f (A^-1)_PP h)^2 ~ 1e-7
    # at a relative step h = 1e-2; a step of 1e-3 would leave the difference of the outlet
    # means (~1e-13) too close to their FP64 rounding noise (~1e-16).
    p64 = sv.params(precision="fp64", tol=1e-12, max_iter=200000)
    errs = fd_check(sv, pb, kappa, p64, np.asarray(gold["fd_cells"]), g.cpu().numpy(), 1e-2,
                    sweeps=20000)
    worst = max(e / b for e, b, _, _ in errs)
    print(f"finite differences: worst error / bound {worst:.3f}", flush=True)
    assert worst <= 1.0


def test_autograd_function(sv):
    from paper_2502_08034_amd.autograd import SocSteady
    solid, u = case(64, 32, 32, seed=44)
    kappa = torch.as_tensor(I.lognormal_activity(solid, 0.3, seed=5), device="cuda")
    pb = sv.Problem.create(solid, *u)
    p = sv.params(precision="fp64", tol=1e-13, check_every=100)
    k = kappa.clone().requires_grad_(True)
    q = torch.tensor(1.3, dtype=torch.float64, requires_grad=True)
    U = SocSteady.apply(k, q, pb, p)
    U.backward()
    # direct adjoint at the same point
    pb.set_flow_rate(1.3)
    pb.set_activity(kappa)
    sv.solve_soc_steady(pb.ctx, p)
    g, dlnq, _, _ = sv.solve_soc_adjoint(pb.ctx, p)
    assert torch.allclose(k.grad.double(), g, rtol=1e-6, atol=1e-12 * float(g.abs().max()))
    assert abs(float(q.grad) - dlnq / 1.3) <= 1e-9 * abs(dlnq)
    # finite differences in q through the autograd forward
    with torch.no_grad():
        Up = SocSteady.apply(kappa, torch.tensor(1.3 + 1e-4, dtype=torch.float64), pb, p)
        Um = SocSteady.apply(kappa, torch.tensor(1.3 - 1e-4, dtype=torch.float64), pb, p)
    fd = float(Up - Um) / 2e-4
    assert abs(fd - float(q.grad)) <= 1e-4 * abs(fd)
