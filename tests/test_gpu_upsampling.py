"""Iterative upsampling on the GPU against the oracle (needs an MI355X).

The coarse problem the library builds (mask and face velocities) equals the oracle's
coarsening bit for bit; the upsampled solve reaches the oracle's fixed point of the fine
problem, from a start that needs fewer fine sweeps than the cold start; the coarse solve
reaches the oracle's fixed point of the coarse problem.
"""
import numpy as np
import pytest
import torch

from paper_2502_08034_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv():
    from paper_2502_08034_amd import socfv
    return socfv


def case(nx, ny, nz, seed, pe=1.0):
    g = I.fibres_nonoverlap(nx, ny, nz, 3.0, 0.85, seed)
    return g.solid, I.darcy_velocity(g.solid, pe)


@pytest.mark.parametrize("shape,q", [((64, 32, 32), 1.0), ((70, 38, 30), 1.7)])
def test_coarse_problem_is_the_oracle_coarsening(sv, orc, shape, q):
    solid, u = case(*shape, seed=51)
    pb = sv.Problem.create(solid, *u, q=q)
    cs, cux, cuy, cuz = sv.coarsen(pb.ctx)
    op = orc.Problem(solid, *(a * q for a in u))
    oc = orc.coarsen(op)
    assert np.array_equal(cs.cpu().numpy(), oc.solid)
    for got, want in ((cux, oc.ux), (cuy, oc.uy), (cuz, oc.uz)):
        assert np.array_equal(got.cpu().numpy(), want)


@pytest.mark.parametrize("prec,mode", [("fp64", "finite"), ("fp32", "finite"), ("fp32", "pinned")])
def test_upsampled_solve_reaches_the_fixed_point(sv, orc, prec, mode):
    solid, u = case(64, 32, 32, seed=52)
    pb = sv.Problem.create(solid, *u)
    kw = dict(mode=1, s_in=0.0, s_eq=1.0, Da=0.0) if mode == "pinned" else {}
    p = sv.params(precision=prec, tol=1e-10, check_every=100, **kw)
    s, st, cst = sv.solve_soc_upsampled(pb.ctx, p)
    assert st.status == sv.OK and cst.status == sv.OK
    okw = dict(s_in=0.0, s_eq=1.0, pinned=True) if mode == "pinned" else {}
    op = orc.Problem(solid, *u, **okw)
    sx = orc.exact_steady(op)
    pore = solid == 0
    tol = 1e-8 if prec == "fp64" else 1e-5
    assert np.abs(s.cpu().numpy() - sx)[pore].max() <= tol
    Ux = orc.outputs(op, sx)["U"]
    assert abs(st.U - Ux) <= 1e-6 * abs(Ux) + 1e-12
    # the coarse solve is the oracle's coarse problem at its fixed point
    oc = orc.coarsen(op)
    Uc = orc.outputs(oc, orc.exact_steady(oc))["U"]
    assert abs(cst.U - Uc) <= 1e-6 * abs(Uc) + 1e-12
    # the warm start saves fine sweeps
    _, cold = sv.solve_soc_steady(pb.ctx, p, want_state=False)
    print(f"{prec} {mode}: fine sweeps {st.iterations} (cold {cold.iterations}), coarse "
          f"{cst.iterations}", flush=True)
    assert st.iterations < cold.iterations


def test_odd_dimensions_are_rejected(sv):
    solid, u = case(63, 32, 32, seed=53)
    pb = sv.Problem.create(solid, *u)
    with pytest.raises(sv.SocfvError) as e:
        sv.coarsen(pb.ctx)
    assert e.value.code == sv.INVALID_ARG
    with pytest.raises(sv.SocfvError):
        sv.solve_soc_upsampled(pb.ctx, sv.params(precision="fp64"))
