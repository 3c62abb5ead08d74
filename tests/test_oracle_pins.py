"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

Each test ties the oracle to something other than its own code: reaction-rate identities
the paper states, hand-derived tiny systems, the exact discrete solution and the
continuum solution of 1D plug flow with a homogeneous sink, exact conservation
(telescoping fluxes), mirror symmetry, the bound principle, the limits of the
mass-transport utilisation, adjoint duality and finite differences.
"""
import math

import numpy as np
import pytest

from paper_2502_08034_amd import inputs as I


# ------------------------------------------------------------------------------------
# Reaction algebra: Eqs. (rate-soc-eta), (rate-from-soc), (rate-from-soc-gen),
# (seq-from-Var)
# ------------------------------------------------------------------------------------

def test_rate_half_alpha_matches_sinh_form(orc):
    # alpha = 1/2: 2 sqrt(s(1-s)) sinh(eta/2) == exp(V/2) - 2 cosh(V/2) s
    for V in (-3.0, -0.7, 0.0, 0.4, 2.5):
        for s in (0.01, 0.2, 0.5, 0.77, 0.99):
            lhs = orc.rate_sinh(s, V)
            rhs = math.exp(V / 2) - 2 * math.cosh(V / 2) * s
            assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(rhs))
            assert abs(orc.rate_affine(s, V, 0.5) - rhs) <= 1e-13 * max(1.0, abs(rhs))


def test_rate_general_alpha_is_affine(orc):
    for alpha in (0.3, 0.5, 0.62):
        for V in (-1.5, 0.0, 1.1):
            K, seq = orc.rate_slope_and_seq(V, alpha)
            for s in (0.05, 0.3, 0.6, 0.95):
                bv = orc.rate_bv_general(s, V, alpha)
                aff = orc.rate_affine(s, V, alpha)
                assert abs(bv - aff) <= 1e-12 * max(1.0, abs(aff))
                assert abs(aff - K * (seq - s)) <= 1e-12 * max(1.0, abs(aff))
            # zero rate at the equilibrium state of charge sigma(V)
            assert abs(orc.rate_affine(seq, V, alpha)) <= 1e-14
    # the slope at alpha = 1/2 is 2 cosh(V/2)
    K, _ = orc.rate_slope_and_seq(0.8, 0.5)
    assert abs(K - 2 * math.cosh(0.4)) < 1e-14


def test_damkohler_paper_parameters(orc):
    # k0 = 7.2e-5 m/s, D = 4e-10 m^2/s, h = 1.25 um, V = 0, alpha = 1/2: K = 2
    Da = orc.damkohler_per_face(7.2e-5, 0.0, 0.5, 1.25e-6, 4e-10)
    assert abs(Da - 0.45) < 1e-12


# ------------------------------------------------------------------------------------
# Hand-derived tiny systems
# ------------------------------------------------------------------------------------

def _problem(orc, solid, ux, uy, uz, **kw):
    return orc.Problem(solid, ux, uy, uz, **kw)


def test_single_cell_with_one_fibre_face(orc):
    # nx=1, ny=2: the pore cell (y=0) has a fibre voxel above it (one reactive face).
    solid = np.array([[[0], [1]]], dtype=np.uint8)            # (nz=1, ny=2, nx=1)
    u, Da, s_in, s_eq = 0.7, 0.45, 1.0, 0.2
    ux = np.zeros((1, 2, 2)); ux[0, 0, :] = u
    uy = np.zeros((1, 3, 1)); uz = np.zeros((2, 2, 1))
    pb = _problem(orc, solid, ux, uy, uz, s_in=s_in, s_eq=s_eq, Da=Da)
    # inlet: u s_in + 2 (s_in - s); outlet: -u s; reaction: Da (s_eq - s)
    expect = ((u + 2) * s_in + Da * s_eq) / (u + 2 + Da)
    s = orc.exact_steady(pb)
    assert abs(s[0, 0, 0] - expect) < 1e-15
    se, info = orc.solve(pb, tol=1e-14)
    assert info["status"] == 0 and abs(se[0, 0, 0] - expect) < 1e-13


def test_two_cell_chain(orc):
    solid = np.array([[[0, 0], [1, 1]]], dtype=np.uint8)      # (1, 2, 2): row y=1 fibre
    u, Da, s_in, s_eq = 1.3, 0.8, 0.9, 0.1
    ux = np.zeros((1, 2, 3)); ux[0, 0, :] = u
    uy = np.zeros((1, 3, 2)); uz = np.zeros((2, 2, 2))
    pb = _problem(orc, solid, ux, uy, uz, s_in=s_in, s_eq=s_eq, Da=Da)
    lam = Da
    # R_A = (u+2) s_in - (u+3+lam) s_A + s_B + lam s_eq
    # R_B = (u+1) s_A - (u+1+lam) s_B + lam s_eq
    M = np.array([[u + 3 + lam, -1.0], [-(u + 1), u + 1 + lam]])
    b = np.array([(u + 2) * s_in + lam * s_eq, lam * s_eq])
    sA, sB = np.linalg.solve(M, b)
    s = orc.exact_steady(pb)
    assert abs(s[0, 0, 0] - sA) < 1e-14 and abs(s[0, 0, 1] - sB) < 1e-14
    se, info = orc.solve(pb, tol=1e-14)
    assert abs(se[0, 0, 0] - sA) < 1e-13 and abs(se[0, 0, 1] - sB) < 1e-13


@pytest.mark.parametrize("axis", ["y", "z"])
def test_four_cell_turning_flow(orc, axis):
    """Flow enters at (x=0, t=0), turns along the transverse axis t, leaves at (x=1, t=1).

    Cells a=(0,0) b=(1,0) c=(0,1) d=(1,1) in (x, t); uniform sink lam everywhere."""
    u, lam, s_in, s_eq = 0.9, 0.3, 1.0, 0.25
    if axis == "y":
        solid = np.zeros((1, 2, 2), dtype=np.uint8)
        ux = np.zeros((1, 2, 3)); uy = np.zeros((1, 3, 2)); uz = np.zeros((2, 2, 2))
        ux[0, 0, 0] = u            # inlet face of a
        ux[0, 1, 1] = u            # c -> d
        ux[0, 1, 2] = u            # outlet face of d
        uy[0, 1, 0] = u            # a -> c
        idx = {"a": (0, 0, 0), "b": (0, 0, 1), "c": (0, 1, 0), "d": (0, 1, 1)}
    else:
        solid = np.zeros((2, 1, 2), dtype=np.uint8)
        ux = np.zeros((2, 1, 3)); uy = np.zeros((2, 2, 2)); uz = np.zeros((3, 1, 2))
        ux[0, 0, 0] = u
        ux[1, 0, 1] = u
        ux[1, 0, 2] = u
        uz[1, 0, 0] = u
        idx = {"a": (0, 0, 0), "b": (0, 0, 1), "c": (1, 0, 0), "d": (1, 0, 1)}
    pb = _problem(orc, solid, ux, uy, uz, s_in=s_in, s_eq=s_eq, lam_field=np.full(solid.shape, lam))
    # rows derived by hand from the face table (order a, b, c, d); A s = b
    A = np.array([
        [u + 4 + lam, -1.0, -1.0, 0.0],
        [-1.0, 2 + lam, 0.0, -1.0],
        [-(u + 1), 0.0, u + 4 + lam, -1.0],
        [0.0, -1.0, -(u + 1), u + 2 + lam],
    ])
    rhs = np.array([(u + 2) * s_in + lam * s_eq, lam * s_eq, 2 * s_in + lam * s_eq, lam * s_eq])
    ref = np.linalg.solve(A, rhs)
    s = orc.exact_steady(pb)
    se, info = orc.solve(pb, tol=1e-14)
    for k, key in enumerate("abcd"):
        assert abs(s[idx[key]] - ref[k]) < 1e-14
        assert abs(se[idx[key]] - ref[k]) < 1e-13


# ------------------------------------------------------------------------------------
# 1D plug flow with a homogeneous sink: exact discrete and continuum solutions
# ------------------------------------------------------------------------------------

def plug_flow_discrete(n, u, lam, s_in, s_eq):
    """Exact solution of the 1D recurrence written from the face table.

    c = (s - s_eq)/(s_in - s_eq).  Interior cells: (u+1) c_{i-1} - (u+2+lam) c_i + c_{i+1}
    = 0, so c_i = A r1^i + B r2^{i-(n-1)} with r1 r2 = u+1, r1 + r2 = u+2+lam.  Inlet row:
    (u+2) - (u+3+lam) c_0 + c_1 = 0.  Outlet row: (u+1) c_{n-2} - (u+1+lam) c_{n-1} = 0.
    """
    disc = math.sqrt((2 + u + lam) ** 2 - 4 * (1 + u))
    r1 = ((2 + u + lam) - disc) / 2
    r2 = ((2 + u + lam) + disc) / 2
    i = np.arange(n, dtype=np.float64)
    e1 = r1 ** i                          # decaying from the inlet
    e2 = r2 ** (i - (n - 1))              # decaying from the outlet (scaled to avoid overflow)
    # two boundary rows in the unknowns (A, B)
    row0 = [-(u + 3 + lam) * e1[0] + e1[1], -(u + 3 + lam) * e2[0] + e2[1]]
    rowN = [(u + 1) * e1[n - 2] - (u + 1 + lam) * e1[n - 1],
            (u + 1) * e2[n - 2] - (u + 1 + lam) * e2[n - 1]]
    AB = np.linalg.solve(np.array([row0, rowN]), np.array([-(u + 2), 0.0]))
    c = AB[0] * e1 + AB[1] * e2
    return s_eq + (s_in - s_eq) * c


@pytest.mark.parametrize("n,u,lam,ny,nz", [(48, 0.8, 0.05, 1, 1), (64, 2.5, 0.3, 3, 2),
                                           (40, 0.05, 0.2, 2, 3), (72, 5.0, 0.01, 1, 2)])
def test_plug_flow_discrete_closed_form(orc, n, u, lam, ny, nz):
    solid, (ux, uy, uz) = I.plug_flow_case(n, ny, nz, u)
    pb = orc.Problem(solid, ux, uy, uz, s_in=1.0, s_eq=0.0, lam_field=np.full(solid.shape, lam))
    ref = plug_flow_discrete(n, u, lam, 1.0, 0.0)
    s = orc.exact_steady(pb)
    assert np.abs(s - ref[None, None, :]).max() < 1e-13
    se, info = orc.solve(pb, tol=5e-12)
    assert info["status"] == 0
    assert np.abs(se - ref[None, None, :]).max() < 1e-10
    # general (s_in, s_eq): affine image of the normalised profile
    pb2 = orc.Problem(solid, ux, uy, uz, s_in=0.3, s_eq=0.9, lam_field=np.full(solid.shape, lam))
    assert np.abs(orc.exact_steady(pb2) - plug_flow_discrete(n, u, lam, 0.3, 0.9)).max() < 1e-13


def test_plug_flow_continuum_first_order(orc):
    """D c'' - U c' - k c = 0, c(0) = 1, c'(L) = 0: the FV solution converges at first order."""
    L, U, k, D = 8.0, 1.0, 0.5, 1.0
    m1 = (U - math.sqrt(U * U + 4 * k * D)) / (2 * D)
    m2 = (U + math.sqrt(U * U + 4 * k * D)) / (2 * D)
    a_b = np.linalg.solve(np.array([[1.0, 1.0], [m1 * math.exp(m1 * L), m2 * math.exp(m2 * L)]]),
                          np.array([1.0, 0.0]))
    errs = []
    for n in (32, 64, 128, 256):
        h = L / n
        solid, (ux, uy, uz) = I.plug_flow_case(n, 1, 1, U * h / D)
        pb = orc.Problem(solid, ux, uy, uz, s_in=1.0, s_eq=0.0,
                         lam_field=np.full(solid.shape, k * h * h / D))
        s = orc.exact_steady(pb)[0, 0]
        x = (np.arange(n) + 0.5) * h
        cont = a_b[0] * np.exp(m1 * x) + a_b[1] * np.exp(m2 * x)
        errs.append(np.abs(s - cont).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    # upwind advection: the observed order rises toward 1 under refinement
    assert all(0.8 < p < 1.1 for p in orders) and 0.9 < orders[-1], (errs, orders)
    assert errs[-1] < 2e-3


# ------------------------------------------------------------------------------------
# Fibre geometries: conservation, bounds, symmetry, constant state, limits
# ------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small_fibre():
    g = I.fibres_nonoverlap(40, 20, 16, 3.0, 0.85, 7)
    u = I.darcy_velocity(g.solid, 1.0)
    return g.solid, u


@pytest.mark.parametrize("pinned", [False, True])
def test_conservation_is_exact(orc, small_fibre, pinned):
    solid, u = small_fibre
    pb = orc.Problem(solid, *u, s_in=0.0 if pinned else 1.0, s_eq=1.0 if pinned else 0.0,
                     Da=0.45, pinned=pinned)
    rng = np.random.default_rng(3)
    for s in (rng.uniform(0, 1, solid.shape), orc.exact_steady(pb)):
        if pinned:
            s = np.where(pb.nf > 0, pb.s_eq, s)
        o = orc.outputs(pb, s)
        R, _ = orc.residual(pb, s)
        lhs = o["F_in"] - o["F_out"] - o["reaction"]
        assert abs(lhs - R.sum()) <= 1e-10 * max(1.0, abs(o["F_in"]))
        assert abs(o["sum_R"] - R.sum()) <= 1e-10 * max(1.0, abs(o["F_in"]))
    # at the fixed point the net transport balances the electrode
    assert abs(lhs) <= 1e-10 * abs(o["F_in"])


def test_bounds_hold_for_every_iterate(orc, small_fibre):
    solid, u = small_fibre
    pb = orc.Problem(solid, *u, s_in=1.0, s_eq=0.0, Da=0.45)
    dt = 0.4 / orc.max_diag(pb)
    s = pb.initial_state()
    pore = solid == 0
    for _ in range(30):
        s = orc.iterate(pb, s, dt, 25)
        assert s[pore].min() >= -1e-15 and s[pore].max() <= 1.0 + 1e-15
    # a time step beyond the positivity bound must be able to break it (cfl 1.9)
    s2 = orc.iterate(pb, pb.initial_state(), 1.9 / orc.max_diag(pb), 60)
    assert s2[pore].min() < -1e-6 or s2[pore].max() > 1 + 1e-6


def test_no_reaction_keeps_inlet_state(orc, small_fibre):
    solid, u = small_fibre
    pb = orc.Problem(solid, *u, s_in=0.37, s_eq=0.0, Da=0.0)
    R, _ = orc.residual(pb, pb.initial_state())
    assert np.abs(R).max() < 1e-10
    s = orc.exact_steady(pb)
    assert np.abs(s[solid == 0] - 0.37).max() < 1e-9


def test_mirror_symmetry(orc, small_fibre):
    solid, (ux, uy, uz) = small_fibre
    pb = orc.Problem(solid, ux, uy, uz, s_in=1.0, s_eq=0.0, Da=0.45)
    s = orc.exact_steady(pb)
    # mirror in y: flip cells, flip y faces and negate their velocity
    pm = orc.Problem(solid[:, ::-1, :], ux[:, ::-1, :], -uy[:, ::-1, :], uz[:, ::-1, :],
                     s_in=1.0, s_eq=0.0, Da=0.45)
    assert np.abs(orc.exact_steady(pm)[:, ::-1, :] - s).max() < 1e-13
    # mirror in z
    pz = orc.Problem(solid[::-1], ux[::-1], uy[::-1], -uz[::-1], s_in=1.0, s_eq=0.0, Da=0.45)
    assert np.abs(orc.exact_steady(pz)[::-1] - s).max() < 1e-13
    # swap y and z
    pt = orc.Problem(solid.transpose(1, 0, 2), ux.transpose(1, 0, 2), uz.transpose(1, 0, 2),
                     uy.transpose(1, 0, 2), s_in=1.0, s_eq=0.0, Da=0.45)
    assert np.abs(orc.exact_steady(pt).transpose(1, 0, 2) - s).max() < 1e-13


def test_utilisation_limits(orc, small_fibre):
    solid, u = small_fibre
    # no fibres: nothing is pinned, U_mt = 0
    s0, u0 = I.plug_flow_case(24, 6, 6, 0.7)
    p0 = orc.Problem(s0, *u0, s_in=0.0, s_eq=1.0, pinned=True)
    assert orc.outputs(p0, orc.exact_steady(p0))["U"] == 0.0
    pm = orc.Problem(solid, *u, s_in=0.0, s_eq=1.0, pinned=True)
    umt = orc.outputs(pm, orc.exact_steady(pm))["U"]
    assert 0.0 < umt < 1.0
    prev = 0.0
    for Da in (0.045, 0.45, 4.5, 45.0, 450.0, 45000.0):
        pb = orc.Problem(solid, *u, s_in=0.0, s_eq=1.0, Da=Da)
        U = orc.outputs(pb, orc.exact_steady(pb))["U"]
        assert prev < U <= umt + 1e-12
        prev = U
    assert umt - prev < 1e-3
    # same geometry and s_in / s_eq swapped: U is the same figure
    pb1 = orc.Problem(solid, *u, s_in=1.0, s_eq=0.0, Da=0.45)
    pb2 = orc.Problem(solid, *u, s_in=0.0, s_eq=1.0, Da=0.45)
    assert abs(orc.outputs(pb1, orc.exact_steady(pb1))["U"]
               - orc.outputs(pb2, orc.exact_steady(pb2))["U"]) < 1e-12
    # faster flow, lower utilisation
    Us = []
    for q in (0.5, 1.0, 2.0):
        pq = orc.Problem(solid, *(a * q for a in u), s_in=0.0, s_eq=1.0, pinned=True)
        Us.append(orc.outputs(pq, orc.exact_steady(pq))["U"])
    assert Us[0] > Us[1] > Us[2]


def test_explicit_iteration_reaches_the_fixed_point(orc):
    w = I.workload("fibre64")
    solid = w["solid"]
    u = w["velocity"][0.5]
    for pinned in (False, True):
        pb = orc.Problem(solid, *u, s_in=0.0 if pinned else 1.0, s_eq=1.0 if pinned else 0.0,
                         Da=0.45, pinned=pinned)
        s, info = orc.solve(pb, tol=1e-12, check_every=50)
        assert info["status"] == 0
        sx = orc.exact_steady(pb)
        assert np.abs(s - sx)[solid == 0].max() < 1e-11
        assert orc.residual_norm(pb, sx) < 1e-11


# ------------------------------------------------------------------------------------
# Geometry classification
# ------------------------------------------------------------------------------------

def test_fibre_face_counts_and_pockets(orc):
    solid = np.zeros((3, 3, 4), dtype=np.uint8)
    solid[1, 1, 1] = 1
    nf = orc.fibre_faces(solid)
    assert nf[1, 1, 1] == -1
    # six face neighbours of the fibre voxel react (one face each); corners do not
    for (z, y, x) in [(1, 1, 0), (1, 1, 2), (1, 0, 1), (1, 2, 1), (0, 1, 1), (2, 1, 1)]:
        assert nf[z, y, x] == 1
    assert nf[0, 0, 0] == 0 and nf[0, 0, 1] == 0       # edge / corner contact only
    assert orc.disconnected(solid) == 0
    # an enclosed pocket: a pore cell surrounded by fibre on all six sides
    s2 = np.ones((3, 3, 5), dtype=np.uint8)
    s2[:, :, 0] = 0                 # inlet plane open
    s2[1, 1, 3] = 0                 # isolated pocket
    assert orc.disconnected(s2) == 1
    g = I.fibres_nonoverlap(48, 24, 24, 3.0, 0.80, 11)
    assert orc.disconnected(g.solid) == 0


# ------------------------------------------------------------------------------------
# Adjoint: duality and finite differences
# ------------------------------------------------------------------------------------

def test_adjoint_duality_and_gradients(orc, small_fibre):
    solid, u = small_fibre
    kappa = I.lognormal_activity(solid, 0.3, seed=5).astype(np.float64)
    pb = orc.Problem(solid, *u, s_in=1.0, s_eq=0.0, Da=0.45, kappa=kappa)
    s = orc.exact_steady(pb)
    psi = orc.exact_adjoint(pb)
    A, b = orc.assemble(pb)
    g = orc.adjoint_rhs(pb)
    assert abs((g * s).sum() - (psi.ravel() * b).sum()) < 1e-13
    # the explicit adjoint iteration converges to the same psi
    pe, info = orc.adjoint(pb, tol=1e-13)
    assert np.abs(pe - psi).max() <= 1e-10 * np.abs(psi).max()
    gk, dlnq = orc.gradients(pb, s, psi)
    U0 = orc.outputs(pb, s)["U"]
    rng = np.random.default_rng(9)
    cells = rng.choice(np.flatnonzero(pb.nf.ravel() > 0), size=8, replace=False)
    for c in cells:
        z, y, x = np.unravel_index(c, solid.shape)
        h = 1e-3 * kappa[z, y, x]
        Us = []
        for sgn in (1, -1):
            k2 = kappa.copy(); k2[z, y, x] += sgn * h
            p2 = orc.Problem(solid, *u, s_in=1.0, s_eq=0.0, Da=0.45, kappa=k2)
            Us.append(orc.outputs(p2, orc.exact_steady(p2))["U"])
        fd = (Us[0] - Us[1]) / (2 * h)
        assert abs(fd - gk[z, y, x]) <= 1e-5 * abs(fd) + 1e-12
    # d U / d ln q against a central difference in the velocity scale
    Uq = []
    for eps in (1e-4, -1e-4):
        pq = orc.Problem(solid, *(a * (1 + eps) for a in u), s_in=1.0, s_eq=0.0, Da=0.45,
                         kappa=kappa)
        Uq.append(orc.outputs(pq, orc.exact_steady(pq))["U"])
    fdq = (Uq[0] - Uq[1]) / (2e-4)
    assert abs(fdq - dlnq) <= 1e-6 * abs(fdq)
    assert U0 > 0


def test_adjoint_pinned_mode_flow_gradient(orc, small_fibre):
    solid, u = small_fibre
    pb = orc.Problem(solid, *u, s_in=0.0, s_eq=1.0, pinned=True)
    s = orc.exact_steady(pb)
    psi = orc.exact_adjoint(pb)
    pe, _ = orc.adjoint(pb, tol=1e-13)
    assert np.abs(pe - psi).max() <= 1e-10 * np.abs(psi).max()
    A, b = orc.assemble(pb)
    assert abs((orc.adjoint_rhs(pb) * s).sum() - (psi.ravel() * b).sum()) < 1e-13
    _, dlnq = orc.gradients(pb, s, psi)
    Uq = []
    for eps in (1e-4, -1e-4):
        pq = orc.Problem(solid, *(a * (1 + eps) for a in u), s_in=0.0, s_eq=1.0, pinned=True)
        Uq.append(orc.outputs(pq, orc.exact_steady(pq))["U"])
    fdq = (Uq[0] - Uq[1]) / (2e-4)
    assert dlnq < 0 and abs(fdq - dlnq) <= 1e-6 * abs(fdq)


# ------------------------------------------------------------------------------------
# Scale of the stop rule (Eq. (convergence-bv-change)): tau = V / Q with the nominal box
# volume V and the inlet flow Q; RMS over the pore cells
# ------------------------------------------------------------------------------------

@pytest.mark.parametrize("n,ny,nz,u", [(40, 3, 2, 0.7), (17, 1, 1, 2.5), (64, 5, 4, 0.05)])
def test_time_scale_is_flow_through_time_of_plug_flow(orc, n, ny, nz, u):
    # uniform velocity u through an open box: Q = u ny nz, V = n ny nz, so tau = n / u
    solid, vel = I.plug_flow_case(n, ny, nz, u)
    pb = orc.Problem(solid, *vel)
    assert abs(orc.time_scale(pb) - n / u) <= 1e-13 * n / u


@pytest.mark.parametrize("n,ny,nz,u,lam", [(40, 3, 2, 0.7, 0.3), (25, 2, 2, 3.0, 0.05)])
def test_residual_norm_hand_value_in_plug_flow(orc, n, ny, nz, u, lam):
    # s = s_in = 1 everywhere, s_eq = 0: advection and diffusion cancel in every cell (the
    # inlet face brings u s_in and nothing diffuses; the outlet removes u s_P), leaving
    # R_P = -lam in every cell, so rms(R) = lam and res = tau lam = n lam / u
    solid, vel = I.plug_flow_case(n, ny, nz, u)
    pb = orc.Problem(solid, *vel, s_in=1.0, s_eq=0.0, lam_field=np.full(solid.shape, lam))
    s = np.ones(solid.shape)
    R, _ = orc.residual(pb, s)
    assert np.abs(R + lam).max() <= 1e-14
    assert abs(orc.residual_norm(pb, s) - n * lam / u) <= 1e-12 * n * lam / u


def test_residual_norm_uses_box_volume_and_pore_count(orc):
    # a one-cell channel between two fibre layers: V = 3 n (box), Q = u, N = n pore cells,
    # two fibre faces per cell (lam = 2 Da).  At s = 1: R = -2 Da, res = (3 n / u) 2 Da.
    # Pore volume in tau (n / u) or the box cell count in the RMS would each fail this.
    n, u, Da = 30, 1.3, 0.45
    solid = np.ones((3, 1, n), dtype=np.uint8)
    solid[1] = 0
    ux = np.zeros((3, 1, n + 1)); ux[1] = u
    uy = np.zeros((3, 2, n)); uz = np.zeros((4, 1, n))
    pb = orc.Problem(solid, ux, uy, uz, s_in=1.0, s_eq=0.0, Da=Da)
    s = np.where(solid == 0, 1.0, 0.0)
    assert abs(orc.time_scale(pb) - 3 * n / u) <= 1e-13 * 3 * n / u
    assert abs(orc.residual_norm(pb, s) - (3 * n / u) * 2 * Da) <= 1e-12 * (3 * n / u) * 2 * Da


@pytest.mark.parametrize("pinned", [False, True])
def test_residual_norm_is_scaled_state_change(orc, small_fibre, pinned):
    # (tau / dt) ||s' - s||_rms over one explicit update equals tau rms(R), any dt
    solid, u = small_fibre
    pb = orc.Problem(solid, *u, s_in=0.0 if pinned else 1.0, s_eq=1.0 if pinned else 0.0,
                     Da=0.45, pinned=pinned)
    rng = np.random.default_rng(11)
    s = np.where(solid == 0, rng.uniform(0, 1, solid.shape), 0.0)
    if pinned:
        s = np.where(pb.nf > 0, 1.0, s)
    pore = solid == 0
    for dt in (0.4 / orc.max_diag(pb), 1e-3):
        s1 = orc.iterate(pb, s, dt, 1)
        rms = math.sqrt(np.mean(((s1 - s)[pore] / dt) ** 2))
        Q = u[0][:, :, 0][solid[:, :, 0] == 0].sum()
        ref = solid.size / Q * rms
        assert abs(orc.residual_norm(pb, s) - ref) <= 1e-9 * ref


# ------------------------------------------------------------------------------------
# Correction (defect) form of the explicit iteration: the FP32 bulk sweeps iterate
# delta <- delta + dt (r0 - A delta) on a frozen residual r0 = b - A s
# ------------------------------------------------------------------------------------

@pytest.mark.parametrize("pinned", [False, True])
def test_correction_iteration_continues_the_explicit_iteration(orc, small_fibre, pinned):
    # linearity: s + delta_k == the k-th explicit iterate from s, for any start s
    solid, u = small_fibre
    pb = orc.Problem(solid, *u, s_in=0.0 if pinned else 1.0, s_eq=1.0 if pinned else 0.0,
                     Da=0.45, pinned=pinned)
    rng = np.random.default_rng(5)
    s = np.where(solid == 0, rng.uniform(0, 1, solid.shape), 0.0)
    if pinned:
        s = np.where(pb.nf > 0, 1.0, s)
    dt = 0.4 / orc.max_diag(pb)
    r0, _ = orc.residual(pb, s)
    d = orc.correction_iterate(pb, r0, dt, 37)
    assert np.abs(s + d - orc.iterate(pb, s, dt, 37)).max() <= 1e-13
    # split into two calls
    d2 = orc.correction_iterate(pb, r0, dt, 20, delta=orc.correction_iterate(pb, r0, dt, 17))
    assert np.abs(d2 - d).max() <= 1e-15
    held = (solid == 1) | ((pb.nf > 0) & pinned)
    assert np.all(d[held] == 0.0)


def test_correction_iteration_fixed_point_is_the_defect(orc, small_fibre):
    # delta* = A^{-1} r0 = s* - s
    solid, u = small_fibre
    pb = orc.Problem(solid, *u, s_in=1.0, s_eq=0.0, Da=0.45)
    s = pb.initial_state()
    dt = 0.4 / orc.max_diag(pb)
    r0, _ = orc.residual(pb, s)
    d = orc.correction_iterate(pb, r0, dt, 6000)
    sx = orc.exact_steady(pb)
    assert np.abs((s + d - sx)[solid == 0]).max() < 1e-8
