"""The synthetic inputs every workload uses (CPU).

Darcy stand-in velocity: staggered layout, no flux through closed faces, discrete
divergence-free pore cells, inflow equal to outflow, linearity in the Peclet scale.  Fibre
boxes: porosity near its target, every pore cell reachable from the inlet.
"""
import numpy as np
import pytest

from paper_2502_08034_amd import inputs as I


@pytest.fixture(scope="module")
def box():
    g = I.fibres_nonoverlap(40, 20, 16, 3.0, 0.85, 7)
    return g.solid, I.darcy_velocity(g.solid, 1.0)


def test_layout_and_closed_faces(box):
    solid, (ux, uy, uz) = box
    nz, ny, nx = solid.shape
    assert ux.shape == (nz, ny, nx + 1) and uy.shape == (nz, ny + 1, nx)
    assert uz.shape == (nz + 1, ny, nx)
    pore = solid == 0
    # a face between two cells is open only if both are pore
    assert np.all(ux[:, :, 1:nx][~(pore[:, :, :-1] & pore[:, :, 1:])] == 0)
    assert np.all(uy[:, 1:ny, :][~(pore[:, :-1, :] & pore[:, 1:, :])] == 0)
    assert np.all(uz[1:nz, :, :][~(pore[:-1] & pore[1:])] == 0)
    # y and z walls are closed; the inlet and outlet faces of fibre cells carry nothing
    assert np.all(uy[:, 0, :] == 0) and np.all(uy[:, ny, :] == 0)
    assert np.all(uz[0] == 0) and np.all(uz[nz] == 0)
    assert np.all(ux[:, :, 0][~pore[:, :, 0]] == 0) and np.all(ux[:, :, nx][~pore[:, :, -1]] == 0)


def test_divergence_free_with_balanced_flux(box):
    solid, (ux, uy, uz) = box
    div = (ux[:, :, 1:] - ux[:, :, :-1]) + (uy[:, 1:, :] - uy[:, :-1, :]) + \
        (uz[1:] - uz[:-1])
    umax = max(np.abs(ux).max(), np.abs(uy).max(), np.abs(uz).max())
    assert np.abs(div[solid == 0]).max() <= 1e-9 * umax
    q_in, q_out = ux[:, :, 0].sum(), ux[:, :, -1].sum()
    assert q_in > 0 and abs(q_in - q_out) <= 1e-9 * q_in
    assert np.all(ux[:, :, 0] >= 0)                     # no backflow through the inlet


def test_linear_in_the_peclet_scale(box):
    solid, u1 = box
    u3 = I.darcy_velocity(solid, 3.0)
    for a, b in zip(u1, u3):
        assert np.allclose(b, 3.0 * a, rtol=1e-9, atol=1e-12 * np.abs(b).max())


def reachable_from_inlet(pore):
    # flood fill through shared faces by repeated dilation (independent of the generator's
    # labelling): the pore cells a fluid parcel entering at x = 0 can reach
    r = np.zeros_like(pore)
    r[:, :, 0] = pore[:, :, 0]
    while True:
        g = r.copy()
        g[:, :, 1:] |= r[:, :, :-1]
        g[:, :, :-1] |= r[:, :, 1:]
        g[:, 1:, :] |= r[:, :-1, :]
        g[:, :-1, :] |= r[:, 1:, :]
        g[1:] |= r[:-1]
        g[:-1] |= r[1:]
        g &= pore
        if np.array_equal(g, r):
            return r
        r = g


@pytest.mark.parametrize("kind", ["nonoverlap", "boolean"])
def test_fibre_boxes_reach_their_porosity_and_the_inlet(kind):
    if kind == "nonoverlap":
        geo = I.fibres_nonoverlap(64, 32, 32, 3.0, 0.85, 11)
    else:
        geo = I.fibres_boolean(64, 32, 32, 3.0, 0.80, 12)
    pore = geo.solid == 0
    assert geo.porosity == pytest.approx(pore.mean(), abs=1e-12)
    assert abs(geo.porosity - (0.85 if kind == "nonoverlap" else 0.80)) < 0.03
    assert np.array_equal(reachable_from_inlet(pore), pore)
    assert pore[:, :, -1].any()                          # the flow can leave
