"""The logpile input geometry (CPU only): rod count, porosity against the rods' exact volume
fraction, the lattice's mirror symmetries, and the voltage parameters."""
import math

import numpy as np
import pytest

from paper_2502_08034_amd import inputs as I


@pytest.mark.parametrize("h", [5.0, 1.25])
def test_logpile_porosity_and_symmetry(h):
    g = I.logpile(h)
    assert g.solid.shape == (round(160 / h), round(640 / h), round(1280 / h))
    assert g.n_fibres == 43 and g.filled == 0
    # adjacent layers are tangent and rods of one layer are apart: no overlap, so the solid
    # fraction is the rods' volume over the box's
    exact = 1.0 - math.pi * 10.0 ** 2 * (16 * 1280 + 27 * 640) / (1280 * 640 * 160)
    assert abs(g.porosity - exact) < (0.002 if h <= 1.25 else 0.015)
    s = g.solid
    assert np.array_equal(s, s[::-1, :, :]) and np.array_equal(s, s[:, ::-1, :])
    assert np.array_equal(s, s[:, :, ::-1])


def test_logpile_layers():
    g = I.logpile(2.5)
    s = g.solid
    # the mid-plane of layer 1 (z = 20 um) cuts its four x rods; of layer 2 (z = 40 um) its
    # nine y rods
    z1, z2 = int(20 / 2.5), int(40 / 2.5)
    runs = lambda v: int(np.count_nonzero(np.diff(np.concatenate([[0], v.astype(int), [0]])) == 1))
    assert runs(s[z1, :, 100]) == 4 and np.all(s[z1, :, :].any(axis=1) == s[z1, :, 0].astype(bool))
    assert runs(s[z2, 50, :]) == 9


def test_voltage_params():
    p0 = I.voltage_params(0.0)
    assert p0 == {"s_eq": 0.5, "Da": 0.45}
    p = I.voltage_params(2.0)
    assert abs(p["s_eq"] - 1 / (1 + math.exp(-2))) < 1e-15
    assert abs(p["Da"] - 0.45 * math.cosh(1.0)) < 1e-15
