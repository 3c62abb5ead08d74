"""Pins of the oracle's coarsening and prolongation for iterative upsampling (CPU only).

Coarse problem: fibre iff all eight children are fibre; coarse face velocity = half the sum
of its four fine faces (same physical flux in coarse grid units); reaction per coarse face
2 Da.  Pinned against brute-force loops, exact flux identities, and the agreement of U
across three grid levels of a walled slit (which a wrong velocity or reaction scaling
breaks).
"""
import numpy as np
import pytest

from paper_2502_08034_amd import inputs as I


@pytest.fixture(scope="module")
def fibre_case(orc):
    g = I.fibres_nonoverlap(20, 12, 8, 2.0, 0.8, 3)
    u = I.darcy_velocity(g.solid, 1.0)
    return orc.Problem(g.solid, *u)


def test_coarse_mask_and_faces_by_brute_force(orc, fibre_case):
    pb = fibre_case
    c = orc.coarsen(pb)
    nz, ny, nx = pb.solid.shape
    for kc in range(nz // 2):
        for jc in range(ny // 2):
            for ic in range(nx // 2):
                kids = [pb.solid[2 * kc + a, 2 * jc + b, 2 * ic + d]
                        for a in (0, 1) for b in (0, 1) for d in (0, 1)]
                assert c.solid[kc, jc, ic] == (1 if all(kids) else 0)
    for kc in range(nz // 2):
        for jc in range(ny // 2):
            for ic in range(nx // 2 + 1):
                tot = sum(pb.ux[2 * kc + a, 2 * jc + b, 2 * ic] for a in (0, 1) for b in (0, 1))
                assert abs(c.ux[kc, jc, ic] - tot / 2) <= 1e-15 * (1 + abs(tot))
    for kc in range(nz // 2):
        for jc in range(ny // 2 + 1):
            for ic in range(nx // 2):
                tot = sum(pb.uy[2 * kc + a, 2 * jc, 2 * ic + d] for a in (0, 1) for d in (0, 1))
                assert abs(c.uy[kc, jc, ic] - tot / 2) <= 1e-15 * (1 + abs(tot))
    for kc in range(nz // 2 + 1):
        for jc in range(ny // 2):
            for ic in range(nx // 2):
                tot = sum(pb.uz[2 * kc, 2 * jc + b, 2 * ic + d] for b in (0, 1) for d in (0, 1))
                assert abs(c.uz[kc, jc, ic] - tot / 2) <= 1e-15 * (1 + abs(tot))
    assert c.Da == 2 * pb.Da


def test_coarse_flux_identities(orc, fibre_case):
    pb = fibre_case
    c = orc.coarsen(pb)
    umax = max(np.abs(pb.ux).max(), np.abs(pb.uy).max(), np.abs(pb.uz).max())
    # a coarse cell's divergence is half the sum of its eight children's (any field), so a
    # divergence-free fine field gives a divergence-free coarse one
    def div(q):
        return (q.ux[:, :, 1:] - q.ux[:, :, :-1]) + (q.uy[:, 1:, :] - q.uy[:, :-1, :]) + \
               (q.uz[1:] - q.uz[:-1])
    nz, ny, nx = pb.solid.shape
    kids = div(pb).reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2).sum(axis=(1, 3, 5))
    assert np.abs(div(c) - kids / 2).max() <= 1e-14 * umax
    assert np.abs(div(c)).max() <= 4 * np.abs(div(pb)).max() + 1e-14 * umax
    # no flux through any face of a coarse fibre cell
    f = c.solid == 1
    assert np.all(c.ux[:, :, :-1][f] == 0) and np.all(c.ux[:, :, 1:][f] == 0)
    assert np.all(c.uy[:, :-1, :][f] == 0) and np.all(c.uy[:, 1:, :][f] == 0)
    assert np.all(c.uz[:-1][f] == 0) and np.all(c.uz[1:][f] == 0)
    # same physical inlet flux: Q h D is kept, h doubles
    assert abs(c.ux[:, :, 0].sum() - pb.ux[:, :, 0].sum() / 2) <= 1e-13 * pb.ux[:, :, 0].sum()
    # a valid problem: every coarse pore cell reaches the inlet
    assert orc.disconnected(c.solid) == 0


def slit(orc, nx, ny, nz, wall, u, Da):
    """Plug flow u along x between fibre walls `wall` voxels thick at y = 0 and y = ny-1."""
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, :wall, :] = 1
    solid[:, ny - wall:, :] = 1
    ux = np.zeros((nz, ny, nx + 1))
    ux[:, wall:ny - wall, :] = u
    uy = np.zeros((nz, ny + 1, nx))
    uz = np.zeros((nz + 1, ny, nx))
    return orc.Problem(solid, ux, uy, uz, s_in=1.0, s_eq=0.0, Da=Da)


def test_coarsening_is_the_same_physics(orc):
    """Three levels of a walled slit (fine 128 x 16 x 4, 4-voxel fibre walls, plug flow 1.0,
    Da 0.05, U ~ 0.78): the coarse discretisations give the fine U within 1%, while a coarse
    problem with the velocity not halved, or with Da not doubled, is off by more than 0.2."""
    fine = slit(orc, 128, 16, 4, 4, 1.0, 0.05)
    lv = [fine, orc.coarsen(fine)]
    lv.append(orc.coarsen(lv[1]))
    U = [orc.outputs(p, orc.exact_steady(p))["U"] for p in lv]
    assert 0.5 < U[0] < 0.95
    assert abs(U[1] - U[0]) < 0.01 * U[0] and abs(U[2] - U[0]) < 0.02 * U[0], U
    c = lv[1]
    for bad in (orc.Problem(c.solid, 2 * c.ux, c.uy, c.uz, s_in=1.0, s_eq=0.0, Da=c.Da),
                orc.Problem(c.solid, c.ux, c.uy, c.uz, s_in=1.0, s_eq=0.0, Da=fine.Da)):
        Ub = orc.outputs(bad, orc.exact_steady(bad))["U"]
        assert abs(Ub - U[0]) > 0.2, (Ub, U)


def test_prolongation_takes_the_parent_value(orc, fibre_case):
    pb = fibre_case
    rng = np.random.default_rng(4)
    nz, ny, nx = pb.solid.shape
    sc = rng.random((nz // 2, ny // 2, nx // 2))
    s = orc.prolongate(pb, sc)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                want = 0.0 if pb.solid[k, j, i] else sc[k // 2, j // 2, i // 2]
                assert s[k, j, i] == want


def test_upsampled_start_keeps_the_fixed_point(orc, fibre_case):
    """Starting from the prolongated coarse steady state changes the sweep count, not the
    steady state."""
    pb = fibre_case
    c = orc.coarsen(pb)
    s0 = orc.prolongate(pb, orc.exact_steady(c))
    sx = orc.exact_steady(pb)
    st, info = orc.solve(pb, tol=1e-11, s0=s0)
    cold, info_cold = orc.solve(pb, tol=1e-11)
    assert np.abs(st - sx)[pb.solid == 0].max() < 1e-9
    assert info["iterations"] < info_cold["iterations"]
