"""Voltage x flow-rate sweep on the logpile lattice through the batched solve (needs an
MI355X).  At 5 um voxels (256 x 128 x 32): each batched problem reaches its own residual,
agrees with its single solve, and passes the oracle's FP64 residual check; U rises with the
voltage's Damkohler number and falls with the flow rate."""
import numpy as np
import pytest
import torch

from paper_2502_08034_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv():
    from paper_2502_08034_amd import socfv
    return socfv


def test_logpile_sweep_batched(sv, orc):
    g = I.logpile(5.0)
    u = I.darcy_velocity(g.solid, 1.0)
    grid = [(V, pe) for V in (-1.0, 1.5) for pe in (0.5, 2.0)]
    s_in = 1e-3
    params, pbs = [], []
    for V, pe in grid:
        vp = I.voltage_params(V)
        params.append(sv.params(precision="fp32", tol=1e-8, s_in=s_in, **vp))
        pbs.append(sv.Problem.create(g.solid, *u, q=pe))
    states, stats = sv.batch_solve([pb.ctx for pb in pbs], params)
    U = {}
    for (V, pe), pb, p, s, st in zip(grid, pbs, params, states, stats):
        assert st.status == sv.OK and st.residual < 1.5e-8
        _, st1 = sv.solve_soc_steady(pb.ctx, p, want_state=False)
        assert abs(st.U - st1.U) <= 1e-6 * abs(st1.U)
        op = orc.Problem(g.solid, *(a * pe for a in u), s_in=s_in, s_eq=p.s_eq, Da=p.Da)
        assert orc.residual_norm(op, s.cpu().numpy()) < 1.5e-8
        U[(V, pe)] = st.U
        print(f"V {V:+.1f} Pe {pe}: U {st.U:.6f} ({st.iterations} sweeps)", flush=True)
    for pe in (0.5, 2.0):
        assert U[(1.5, pe)] > U[(-1.0, pe)]
    for V in (-1.0, 1.5):
        assert U[(V, 0.5)] > U[(V, 2.0)]
