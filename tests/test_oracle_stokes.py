"""Pins of the oracle's flow step: steady Stokes flow on the voxel grid and the projection
step of the flow simulation (CPU only).

Pinned against: the fully developed rectangular-duct solution of the same discretisation (a
separable 2D problem solved through the eigenvectors of the 1D wall operator), the same duct
walled by fibre voxels, the continuum square-duct flow rate (series solution), an independent
ghost-value evaluation of the viscous operator, mirror and y-z symmetry, the discrete power
balance, mass conservation, and the projection iteration's convergence to the direct solve.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import stokes as S
from paper_2502_08034_amd import inputs as I


def duct_profile(ny, nz):
    """w with (T_z (+) T_y) w = 1, T = tridiag(-1, 2, -1) with 3 at both ends (no-slip wall on
    the boundary face), by the eigen-decomposition of each 1D operator."""
    def eig(n):
        d = np.full(n, 2.0)
        d[0] = d[-1] = 3.0
        return sla.eigh_tridiagonal(d, -np.ones(n - 1))
    ly, vy = eig(ny)
    lz, vz = eig(nz)
    rhs = vz.T @ np.ones((nz, ny)) @ vy
    return vz @ (rhs / (lz[:, None] + ly[None, :])) @ vy.T


@pytest.mark.parametrize("nx,ny,nz,p_in", [(6, 5, 4, 1.0), (9, 3, 7, 2.5)])
def test_duct_is_the_separable_solution(nx, ny, nz, p_in):
    solid = np.zeros((nz, ny, nx), np.uint8)
    ux, uy, uz, p = S.stokes_steady(solid, p_in)
    w = duct_profile(ny, nz) * (p_in / nx)
    assert np.abs(ux - w[:, :, None]).max() <= 1e-12 * w.max()
    assert np.abs(uy).max() <= 1e-13 * w.max() and np.abs(uz).max() <= 1e-13 * w.max()
    # linear pressure, p_in at the inlet face and 0 at the outlet face
    lin = p_in * (1.0 - (np.arange(nx) + 0.5) / nx)
    assert np.abs(p - lin[None, None, :]).max() <= 1e-12 * p_in


def test_fibre_walls_act_as_domain_walls():
    nx, ny, nz = 6, 7, 4
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    ux, uy, uz, p = S.stokes_steady(solid)
    dx, dy, dz, dp = S.stokes_steady(np.zeros((nz, ny - 2, nx), np.uint8))
    assert np.abs(ux[:, 1:ny - 1, :] - dx).max() <= 1e-13
    assert np.abs(p[:, 1:ny - 1, :] - dp).max() <= 1e-13
    assert np.all(ux[:, 0, :] == 0) and np.all(ux[:, ny - 1, :] == 0)
    assert np.abs(uy).max() <= 1e-14 and np.abs(uz).max() <= 1e-14


def square_duct_rate():
    """Continuum flow rate of a unit square duct under unit pressure gradient (mu = 1): the
    series solution Q = (1/12) (1 - (192 / pi^5) sum_{n odd} tanh(n pi / 2) / n^5)."""
    s = sum(math.tanh(n * math.pi / 2) / n ** 5 for n in range(1, 200, 2))
    return (1.0 - 192.0 / math.pi ** 5 * s) / 12.0


def test_square_duct_converges_to_the_continuum_rate():
    exact = square_duct_rate()
    assert abs(exact - 0.0351443) < 1e-6
    errs = []
    for a in (6, 12, 24):
        nx = 2
        ux, _, _, _ = S.stokes_steady(np.zeros((a, a, nx), np.uint8), p_in=1.0)
        q = S.flow_rate(ux) / ((1.0 / nx) * a ** 4)      # Q / (G a^4)
        errs.append(abs(q - exact) / exact)
    assert errs[2] < 0.02
    # second order: the error falls about fourfold per halving of the voxel
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


@pytest.fixture(scope="module")
def fibre_geom():
    g = I.fibres_nonoverlap(16, 10, 10, 1.6, 0.8, 7)
    return g.solid


def ghost_laplacian(opens, u_fields):
    """The viscous operator by explicit ghost values: pad each face array by one, fill the
    padding and every closed face with the value the boundary rule prescribes for the face
    being updated, apply the plain 7-point Laplacian."""
    out = []
    for a, (o, u) in enumerate(zip(opens, u_fields)):
        res = np.zeros(u.shape)
        nzf, nyf, nxf = u.shape
        for (k, j, i) in zip(*np.nonzero(o)):
            acc = 0.0
            for axis, (dk, dj, di) in ((0, (0, 0, 1)), (0, (0, 0, -1)), (1, (0, 1, 0)),
                                       (1, (0, -1, 0)), (2, (1, 0, 0)), (2, (-1, 0, 0))):
                kk, jj, ii = k + dk, j + dj, i + di
                inside = 0 <= kk < nzf and 0 <= jj < nyf and 0 <= ii < nxf
                if inside and o[kk, jj, ii]:
                    g = u[kk, jj, ii]
                elif not inside and axis == 0:
                    g = u[k, j, i]                 # zero gradient through the open planes
                elif axis == a:
                    g = 0.0                        # no penetration one cell away
                else:
                    g = -u[k, j, i]                # no-slip wall halfway: reflected value
                acc += g - u[k, j, i]
            res[k, j, i] = acc
        out.append(res)
    return out


def test_viscous_operator_matches_ghost_values(fibre_geom):
    ops = S.StokesOperators(fibre_geom)
    rng = np.random.default_rng(3)
    fields = [np.where(o, rng.standard_normal(o.shape), 0.0) for o in ops.opens]
    Lu = ops.unpack(ops.L @ ops.pack(*fields))
    ref = ghost_laplacian(ops.opens, fields)
    for got, want in zip(Lu, ref):
        assert np.abs(got - want).max() <= 1e-13
    # -L is symmetric positive definite
    L = ops.L.toarray()
    assert np.abs(L - L.T).max() == 0.0
    assert np.linalg.eigvalsh(-L).min() > 0


def test_fibre_flow_invariants(fibre_geom):
    ops = S.StokesOperators(fibre_geom, 1.0)
    ux, uy, uz, p = S.stokes_steady(fibre_geom, ops=ops)
    mom, div, closed = S.stokes_residual(fibre_geom, ux, uy, uz, p, ops=ops)
    umax = max(np.abs(ux).max(), np.abs(uy).max(), np.abs(uz).max())
    assert mom <= 1e-12 and div <= 1e-13 * umax and closed == 0.0
    # mass: inflow = outflow; the mean pressure falls from inlet to outlet plane (Stokes
    # pressure has no pointwise maximum principle next to walls)
    assert abs(ux[:, :, 0].sum() - ux[:, :, -1].sum()) <= 1e-13 * ux[:, :, 0].sum()
    pore = fibre_geom == 0
    means = [p[:, :, i][pore[:, :, i]].mean() for i in range(p.shape[2])]
    assert 1.0 > means[0] and means[-1] > 0.0 and np.all(np.diff(means) < 0)
    # power balance: -u.L u = sum_in u (2 p_in - p_0) + sum_out u p_last
    u, pv = ops.pack(ux, uy, uz, p)
    diss = -u @ (ops.L @ u)
    work = (ux[:, :, 0] * (2.0 - p[:, :, 0]))[pore[:, :, 0]].sum() + \
        (ux[:, :, -1] * p[:, :, -1])[pore[:, :, -1]].sum()
    assert diss > 0 and abs(diss - work) <= 1e-12 * diss
    # Stokes: the field is linear in the applied pressure
    vx, _, _, vp = S.stokes_steady(fibre_geom, p_in=3.0)
    assert np.abs(vx - 3.0 * ux).max() <= 1e-12 * np.abs(vx).max()


def test_mirror_and_transpose_symmetry(fibre_geom):
    ux, uy, uz, p = S.stokes_steady(fibre_geom)
    mx, my, mz, mp = S.stokes_steady(fibre_geom[:, ::-1, :].copy())
    tol = 1e-12 * np.abs(ux).max()
    assert np.abs(mx - ux[:, ::-1, :]).max() <= tol
    assert np.abs(my + uy[:, ::-1, :]).max() <= tol
    assert np.abs(mz - uz[:, ::-1, :]).max() <= tol
    assert np.abs(mp - p[:, ::-1, :]).max() <= 1e-12
    # y <-> z exchange (square cross-section)
    tx, ty, tz, tp = S.stokes_steady(fibre_geom.transpose(1, 0, 2).copy())
    assert np.abs(tx - ux.transpose(1, 0, 2)).max() <= tol
    assert np.abs(ty - uz.transpose(1, 0, 2)).max() <= tol
    assert np.abs(tz - uy.transpose(1, 0, 2)).max() <= tol


def test_projection_steps_reach_the_steady_flow(fibre_geom):
    ops = S.StokesOperators(fibre_geom)
    sx, sy, sz, sp_ = S.stokes_steady(fibre_geom, ops=ops)
    dt = S.flow_time_step(2.0)
    assert abs(dt - 2.0 / 24.0) < 1e-15
    # each step leaves a discretely divergence-free field
    u = np.zeros(ops.nu)
    p = np.zeros(ops.np_)
    for _ in range(3):
        u, p = S.chorin_step(ops, u, p, dt)
        assert np.abs(ops.D @ u).max() <= 1e-13
    ux, uy, uz, pp, steps = S.flow_sim(fibre_geom, cfl=2.0, eps=1e-12, ops=ops)
    umax = np.abs(sx).max()
    for got, want in ((ux, sx), (uy, sy), (uz, sz)):
        assert np.abs(got - want).max() <= 1e-9 * umax
    assert np.abs(pp - sp_).max() <= 1e-9
    assert 50 < steps < 20000


def test_implicit_diffusion_steps_reach_the_steady_flow(fibre_geom):
    """The algorithm's implicit-diffusion branch: each step solves (I - dt L) v = u - dt (G p +
    gbc) exactly and projects to a divergence-free field, and it reaches the same steady flow.
    With the lagged pressure each step is a pressure-correction (Uzawa-like) iteration, so the
    step count has an optimum in dt (here near C_CFL 16, about four times fewer steps than
    explicit diffusion at C_CFL 2) instead of falling without bound."""
    ops = S.StokesOperators(fibre_geom)
    sx, sy, sz, sp_ = S.stokes_steady(fibre_geom, ops=ops)
    dt = S.flow_time_step(200.0)
    u = np.zeros(ops.nu)
    p = np.zeros(ops.np_)
    for _ in range(3):
        un, pn = S.chorin_step(ops, u, p, dt, implicit=True)
        gp = ops.G @ p + ops.gbc
        v = un + dt * (ops.G @ pn + ops.gbc) - dt * gp      # the Helmholtz solution
        lhs = v - dt * (ops.L @ v)
        assert np.abs(lhs - (u - dt * gp)).max() <= 1e-11 * max(1.0, np.abs(u - dt * gp).max())
        assert np.abs(ops.D @ un).max() <= 1e-12
        u, p = un, pn
    ux, uy, uz, pp, steps = S.flow_sim(fibre_geom, cfl=16.0, eps=1e-12, ops=ops, implicit=True)
    umax = np.abs(sx).max()
    for got, want in ((ux, sx), (uy, sy), (uz, sz)):
        assert np.abs(got - want).max() <= 1e-9 * umax
    assert np.abs(pp - sp_).max() <= 1e-9
    _, _, _, _, steps_explicit = S.flow_sim(fibre_geom, cfl=2.0, eps=1e-12, ops=ops)
    print(f"implicit {steps} steps, explicit {steps_explicit}")
    assert steps < steps_explicit / 3


def paper_flow_dt(cfl, CA, CV, CF):
    """Eq. (time-step-flow) as printed: dt = 1/2 C_CFL (C_A + C_V + sqrt((C_A + C_V)^2 +
    4 C_F^2))^-1."""
    return 0.5 * cfl / (CA + CV + math.sqrt((CA + CV) ** 2 + 4.0 * CF * CF))


@pytest.mark.parametrize("cfl,nu,h", [(0.5, 1.0, 1.0), (3.5, 1.0, 1.0), (1.0, 2.0, 0.5),
                                      (0.25, 0.3, 1.25)])
def test_flow_time_step_is_the_paper_formula_without_advection_and_force(cfl, nu, h):
    # C_V from Eq. (time-step-flow-viscous) on a cubic grid: (2 nu)(3 / h^2); no momentum
    # advection (C_A = 0) and the pressure acting through the projection only (C_F = 0):
    # dt = C_CFL / (4 C_V) = C_CFL h^2 / (24 nu)
    CV = 2.0 * nu * (1.0 / h ** 2 + 1.0 / h ** 2 + 1.0 / h ** 2)
    ref = paper_flow_dt(cfl, 0.0, CV, 0.0)
    assert abs(ref - cfl * h * h / (24.0 * nu)) <= 1e-15 * ref
    assert abs(S.flow_time_step(cfl, nu=nu, h=h) - ref) <= 1e-15 * ref


@pytest.mark.parametrize("kind", ["open", "fibres"])
def test_flow_time_step_reaches_the_explicit_stability_limit_at_cfl_4(kind):
    # explicit momentum diffusion u* = u + dt L u is stable iff dt lambda_max(-L) <= 2; the
    # viscous operator's spectrum reaches up to 4 per axis (12 in 3D), so C_CFL = 4 sits at
    # the limit (dt lambda_max just below 2) and the paper's C_CFL = 1/2 far inside it
    import scipy.sparse.linalg as spl
    if kind == "open":
        solid = np.zeros((12, 12, 16), np.uint8)
    else:
        solid = I.fibres_nonoverlap(24, 14, 12, 2.5, 0.8, 3).solid
    L = S.StokesOperators(solid).L
    assert abs(L - L.T).max() == 0.0
    lmax = spl.eigsh(-L.tocsc(), k=1, which="LA", return_eigenvectors=False)[0]
    assert 1.95 < S.flow_time_step(4.0) * lmax <= 2.0
    assert S.flow_time_step(0.5) * lmax <= 0.25
