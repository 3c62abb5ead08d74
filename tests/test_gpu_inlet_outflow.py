"""Flow leaving through part of the inlet, on the GPU against the oracle (needs an MI355X).

A slab under a fibre row with plug flow plus a divergence-free loop that leaves through the
inlet at y = 0: the velocity is accepted, and the forward solves (FP64 single sweeps, FP32
two-sweep launches over several tiles), the upwinded inlet flux of the balance and the
adjoint gradients agree with the oracle.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv():
    from paper_2502_08034_amd import socfv
    return socfv


def looped_slab(nx, ny, nz):
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, ny - 1, :] = 1
    ux = np.zeros((nz, ny, nx + 1))
    ux[:, :ny - 1, :] = 0.5
    uy = np.zeros((nz, ny + 1, nx))
    uz = np.zeros((nz + 1, ny, nx))
    ux[:, 0, 0] -= 1.0
    ux[:, 1, 0] += 1.0
    uy[:, 1, 0] = -1.0
    return solid, (ux, uy, uz)


@pytest.mark.parametrize("shape", [(10, 6, 3), (130, 40, 9)])
def test_inlet_outflow_matches_oracle(sv, orc, shape):
    solid, u = looped_slab(*shape)
    assert (u[0][:, 0, 0] < 0).all()
    pb = sv.Problem.create(solid, *u)
    op = orc.Problem(solid, *u, s_in=1.0, s_eq=0.0, Da=0.45)
    sx = orc.exact_steady(op)
    ox = orc.outputs(op, sx)
    s, st = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp64", tol=1e-12,
                                                  check_every=100))
    assert st.status == sv.OK
    assert np.abs(s.cpu().numpy() - sx)[solid == 0].max() <= 1e-9
    for got, key in ((st.flux_in, "F_in"), (st.flux_in_adv, "F_in_adv"), (st.U, "U")):
        assert abs(got - ox[key]) <= 1e-9 * max(1.0, abs(ox[key])), (key, got, ox[key])
    s32, st32 = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp32", tol=1e-8))
    assert st32.status == sv.OK
    assert np.abs(s32.cpu().numpy() - sx)[solid == 0].max() <= 1e-5
    assert abs(st32.U - ox["U"]) <= 1e-6 * abs(ox["U"])
    # adjoint gradients through the same faces
    g, dlnq, psi, sta = sv.solve_soc_adjoint(pb.ctx, sv.params(precision="fp64", tol=1e-12,
                                                               check_every=100), want_psi=True)
    assert sta.status == sv.OK
    px = orc.exact_adjoint(op)
    gx, dlnqx = orc.gradients(op, sx, px)
    assert np.abs(psi.cpu().numpy() - px).max() <= 1e-8 * np.abs(px).max()
    assert np.abs(g.cpu().numpy() - gx).max() <= 1e-8 * np.abs(gx).max()
    assert abs(dlnq - dlnqx) <= 1e-8 * abs(dlnqx)
    print(f"{shape}: U {st.U:.8f} (oracle {ox['U']:.8f}), F_in {st.flux_in:.6f}", flush=True)
