"""Pins of the oracle's explicit Nernst model (CPU only).

The explicit Nernst model holds electrode cells at sigma(V - eta) and relaxes eta toward the
overpotential that balances the transport step.  Its fixed point is the steady state of the
simplified Butler-Volmer rate 2 a k0 sqrt(s (1 - s)) sinh(eta / 2), which for s = sigma(V - eta)
equals the affine rate a k0 K (s_eq - s) at alpha = 1/2 (K = 2 cosh(V / 2), s_eq = sigma(V)):
the paper states both models converge to the same steady state.  Pinned against the sparse
solve of the affine finite-rate problem, the rate identity, and the fast-kinetics limit.
"""
import numpy as np
import pytest

from paper_2502_08034_amd import inputs as I


@pytest.fixture(scope="module")
def fibre64():
    w = I.workload("fibre64")
    return w["solid"], w["velocity"][0.5]


@pytest.mark.parametrize("s_in,s_eq,Da,omega", [(0.2, 0.7, 0.45, 0.05), (0.05, 0.9, 0.45, 0.05),
                                                (0.2, 0.7, 5.0, 0.5)])
def test_nernst_fixed_point_is_the_affine_steady_state(orc, fibre64, s_in, s_eq, Da, omega):
    solid, u = fibre64
    op = orc.Problem(solid, *u, s_in=s_in, s_eq=s_eq, Da=Da)
    s, eta, info = orc.nernst(op, omega=omega, tol=1e-11, check_every=100)
    assert info["status"] == 0
    sx = orc.exact_steady(op)
    assert np.abs(s - sx)[solid == 0].max() < 1e-9
    # the electrode holds sigma(V - eta), and the rate identity holds there
    el = (solid == 0) & (op.nf > 0)
    V = np.log(s_eq / (1 - s_eq))
    assert np.abs(s[el] - 1 / (1 + np.exp(eta[el] - V))).max() < 1e-14
    K = 1 / np.sqrt(s_eq * (1 - s_eq))
    assert abs(K - 2 * np.cosh(V / 2)) < 1e-12 * K
    lam = op.lam[el]
    sbv = 2 * (lam / K) * np.sqrt(s[el] * (1 - s[el])) * np.sinh(eta[el] / 2)
    assert np.abs(sbv - lam * (s_eq - s[el])).max() < 1e-12 * np.abs(lam).max()


def test_nernst_fast_kinetics_limit(orc, fibre64):
    """k0 -> infinity: the electrode approaches s_eq, and U approaches the pinned (mass
    transport limit) solution's, with the gap shrinking like 1/Da."""
    solid, u = fibre64
    pin = orc.Problem(solid, *u, s_in=0.2, s_eq=0.7, pinned=True)
    Upin = orc.outputs(pin, orc.exact_steady(pin))["U"]
    gaps = []
    for Da in (50.0, 500.0):
        op = orc.Problem(solid, *u, s_in=0.2, s_eq=0.7, Da=Da)
        s, eta, info = orc.nernst(op, omega=0.5, tol=1e-11, check_every=100)
        assert info["status"] == 0
        el = (solid == 0) & (op.nf > 0)
        assert np.abs(s[el] - 0.7).max() < 20.0 / Da
        gaps.append(abs(orc.outputs(op, s)["U"] - Upin))
    assert gaps[1] < 0.2 * gaps[0]
