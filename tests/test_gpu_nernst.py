"""Explicit Nernst model on the GPU against the oracle (needs an MI355X).

Equal iteration counts against the oracle's Nernst iteration (state and overpotential, FP64,
rounding order only), and the steady state against the oracle's sparse solve of the affine
finite-rate problem, which has the same fixed point.
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


# with the lognormal activity, low-activity electrode cells bring the stability bound of the
# relaxation (omega < ~2 / (1 + M), M ~ 1 / (a k0)) down to ~0.055; omega 0.02 keeps it clear
@pytest.mark.parametrize("shape,activity,omega", [((64, 32, 32), False, 0.05),
                                                  ((70, 37, 29), True, 0.02)])
def test_nernst_matches_oracle_at_equal_count(sv, orc, shape, activity, omega):
    solid, u = case(*shape, seed=61)
    kappa = I.lognormal_activity(solid, 0.3, seed=9) if activity else None
    pb = sv.Problem.create(solid, *u, kappa=kappa)
    p = sv.params(precision="fp64", tol=0.0, max_iter=600, check_every=100, s_in=0.2,
                  s_eq=0.7, Da=0.45)
    s, eta, st = sv.solve_nernst(pb.ctx, p, omega=omega, want_eta=True)
    assert st.iterations == 600
    op = orc.Problem(solid, *u, s_in=0.2, s_eq=0.7, Da=0.45,
                     kappa=None if kappa is None else kappa.astype(np.float64))
    so, etao, info = orc.nernst(op, omega=omega, tol=0.0, max_iter=600, check_every=100)
    assert info["iterations"] == 600
    ds = np.abs(s.cpu().numpy() - so).max()
    print(f"max |s - s_oracle| {ds:.2e}", flush=True)
    assert ds <= 1e-11
    assert np.abs(eta.cpu().numpy() - etao).max() <= 1e-9 * max(1.0, np.abs(etao).max())


@pytest.mark.parametrize("Da,omega", [(0.45, 0.05), (5.0, 0.5)])
def test_nernst_steady_state_is_the_finite_rate_one(sv, orc, Da, omega):
    solid, u = case(64, 32, 32, seed=62)
    pb = sv.Problem.create(solid, *u)
    p = sv.params(precision="fp64", tol=1e-11, check_every=100, s_in=0.2, s_eq=0.7, Da=Da)
    s, _, st = sv.solve_nernst(pb.ctx, p, omega=omega)
    assert st.status == sv.OK
    op = orc.Problem(solid, *u, s_in=0.2, s_eq=0.7, Da=Da)
    sx = orc.exact_steady(op)
    assert np.abs(s.cpu().numpy() - sx)[solid == 0].max() <= 1e-8
    Ux = orc.outputs(op, sx)["U"]
    assert abs(st.U - Ux) <= 1e-8 * abs(Ux)
    # the same fixed point from the finite-rate solve
    s2, st2 = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp64", tol=1e-11, s_in=0.2,
                                                    s_eq=0.7, Da=Da))
    print(f"Da {Da}: Nernst {st.iterations} iterations, finite-rate solve {st2.iterations}",
          flush=True)
    assert np.abs(s.cpu().numpy() - s2.cpu().numpy())[solid == 0].max() <= 2e-8


def test_nernst_error_paths(sv):
    solid, u = case(64, 32, 32, seed=63)
    pb = sv.Problem.create(solid, *u)
    for kw in (dict(mode=1, s_in=0.0, s_eq=1.0, Da=0.0), dict(s_in=1.0, s_eq=0.0),
               dict(s_in=0.2, s_eq=0.7, Da=0.0)):
        with pytest.raises(sv.SocfvError) as e:
            sv.solve_nernst(pb.ctx, sv.params(precision="fp64", **kw))
        assert e.value.code == sv.INVALID_ARG
    with pytest.raises(sv.SocfvError) as e:
        sv.solve_nernst(pb.ctx, sv.params(precision="fp64", s_in=0.2, s_eq=0.7), omega=0.0)
    assert e.value.code == sv.INVALID_ARG
    # a relaxation too strong for slow kinetics ends as DIVERGED, not as a wrong answer
    with pytest.raises(sv.SocfvError) as e:
        sv.solve_nernst(pb.ctx, sv.params(precision="fp64", tol=1e-11, max_iter=4000,
                                          check_every=100, s_in=0.2, s_eq=0.7, Da=0.45),
                        omega=1.0)
    assert e.value.code == sv.DIVERGED
