"""Pins of the oracle with outflow through part of the inlet plane (CPU only).

A pressure-driven Stokes flow can leave through the inlet next to an obstacle close to it.
Through such a face the upwind value is the cell's own (the same upwind rule as every other
face), while the diffusive Dirichlet term is unchanged.  Pinned by the exact flux balance
F_in - F_out - reaction = sum R at the exact steady state (a non-upwind inlet flux breaks it),
the bounds, the lam = 0 invariant, and the explicit iteration reaching the exact steady state.
"""
import numpy as np

from paper_2502_08034_amd import inputs as I  # noqa: F401  (shared seeded generators)


def looped_slab(orc, Da=0.45, s_in=1.0, s_eq=0.0):
    """Plug flow 0.5 along x in a slab under a fibre row (y = ny-1), plus a divergence-free
    loop at the inlet: inflow 1.5 at y = 1, outflow 0.5 at y = 0, linked by the y face
    between them."""
    nz, ny, nx = 3, 6, 10
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, ny - 1, :] = 1
    ux = np.zeros((nz, ny, nx + 1))
    ux[:, :ny - 1, :] = 0.5
    uy = np.zeros((nz, ny + 1, nx))
    uz = np.zeros((nz + 1, ny, nx))
    ux[:, 0, 0] -= 1.0
    ux[:, 1, 0] += 1.0
    uy[:, 1, 0] = -1.0
    return orc.Problem(solid, ux, uy, uz, s_in=s_in, s_eq=s_eq, Da=Da)


def divergence(pb):
    return (pb.ux[:, :, 1:] - pb.ux[:, :, :-1]) + (pb.uy[:, 1:, :] - pb.uy[:, :-1, :]) + \
        (pb.uz[1:] - pb.uz[:-1])


def test_fixture_has_inlet_outflow_and_no_divergence(orc):
    pb = looped_slab(orc)
    assert (pb.ux[:, 0, 0] < 0).all()
    assert np.abs(divergence(pb)[pb.solid == 0]).max() == 0.0


def test_balance_is_exact_with_inlet_outflow(orc):
    pb = looped_slab(orc)
    sx = orc.exact_steady(pb)
    out = orc.outputs(pb, sx)
    scale = abs(out["F_in"]) + abs(out["F_out"]) + abs(out["reaction"])
    assert abs(out["sum_R"]) <= 1e-12 * scale
    assert abs(out["F_in"] - out["F_out"] - out["reaction"] - out["sum_R"]) <= 1e-12 * scale
    # the advective inlet flux counts the outflowing faces with the cell value
    adv = (np.maximum(pb.ux[:, :, 0], 0) * pb.s_in + np.minimum(pb.ux[:, :, 0], 0) * sx[:, :, 0])
    assert abs(out["F_in_adv"] - adv[pb.solid[:, :, 0] == 0].sum()) <= 1e-13
    pore = pb.solid == 0
    assert sx[pore].min() >= -1e-14 and sx[pore].max() <= 1.0 + 1e-14


def test_no_reaction_keeps_the_inlet_value(orc):
    pb = looped_slab(orc, Da=0.0, s_in=0.3)
    sx = orc.exact_steady(pb)
    assert np.abs(sx - 0.3)[pb.solid == 0].max() <= 1e-13


def test_iteration_reaches_the_exact_state(orc):
    pb = looped_slab(orc)
    s, info = orc.solve(pb, tol=1e-12)
    assert info["status"] == 0
    assert np.abs(s - orc.exact_steady(pb))[pb.solid == 0].max() <= 1e-10
