"""Parity of the HIP path with the FP64 CPU oracle (needs an MI355X).

Element-by-element comparisons on the same seeded inputs, at sizes the oracle finishes in
seconds (several 64 x ty x zc tiles with ragged tails), both modes, all precisions.
Tolerances: FP64 sweeps at an equal sweep count, 1e-12 (rounding order only); FP64 steady
state, 1e-9 against the exact fixed point at residual 1e-10; FP32 mode, max |ds| <= 1e-5
and U relative error <= 1e-6 (the stated accuracy targets).
"""
import math

import numpy as np
import pytest
import torch

from paper_2502_08034_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv():
    from paper_2502_08034_amd import socfv
    assert torch.cuda.is_available()
    return socfv


def cuda(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def make(sv, solid, u, kappa=None, q=1.0):
    return sv.Problem.create(solid, *u, q=q, kappa=kappa)


def fibre_case(nx, ny, nz, r, phi, seed, pe):
    g = I.fibres_nonoverlap(nx, ny, nz, r, phi, seed)
    u = I.darcy_velocity(g.solid, pe)
    return g.solid, u


CASES = {
    "fibre64": lambda: (lambda w: (w["solid"], w["velocity"][0.5]))(I.workload("fibre64")),
    "ragged70x37x29": lambda: fibre_case(70, 37, 29, 3.0, 0.82, 21, 1.0),
    "ragged130x9x65": lambda: fibre_case(130, 9, 65, 2.5, 0.85, 22, 2.0),
    "open40x3x2": lambda: I.plug_flow_case(40, 3, 2, 0.7),
    # nx % 4 == 0 takes the four-cells-per-lane FP32 sweep; nx = 260 leaves one lane
    # active in the second 256-cell block row
    "vec100x37x29": lambda: fibre_case(100, 37, 29, 3.0, 0.82, 24, 1.0),
    "vec260x11x7": lambda: fibre_case(260, 11, 7, 2.0, 0.85, 25, 1.5),
    # odd nx: scalar FP32 sweeps only
    "odd63x21x17": lambda: fibre_case(63, 21, 17, 2.5, 0.85, 26, 1.0),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    solid, u = CASES[request.param]()
    return request.param, solid, u


MODES = {"finite": dict(s_in=1.0, s_eq=0.0, Da=0.45, mode=0),
         "pinned": dict(s_in=0.0, s_eq=1.0, Da=0.0, mode=1)}


def oracle_problem(orc, solid, u, m, kappa=None):
    return orc.Problem(solid, *u, s_in=m["s_in"], s_eq=m["s_eq"], Da=m["Da"],
                       pinned=bool(m["mode"]), kappa=kappa)


@pytest.mark.parametrize("mode", list(MODES))
def test_fp64_sweeps_match_oracle_at_equal_count(sv, orc, case, mode):
    name, solid, u = case
    m = MODES[mode]
    pb = make(sv, solid, u)
    p = sv.params(precision="fp64", tol=0.0, max_iter=600, check_every=200, **m)
    s, st = sv.solve_soc_steady(pb.ctx, p)
    assert st.status == sv.NOT_CONVERGED and st.iterations == 600
    op = oracle_problem(orc, solid, u, m)
    so, info = orc.solve(op, cfl=0.4, tol=0.0, max_iter=600, check_every=200)
    assert abs(st.dt - info["dt"]) <= 1e-15 * info["dt"]
    d = np.abs(s.cpu().numpy() - so).max()
    assert d <= 1e-12, (name, mode, d)


@pytest.mark.parametrize("mode", list(MODES))
def test_fp64_steady_state(sv, orc, case, mode):
    name, solid, u = case
    m = MODES[mode]
    pb = make(sv, solid, u)
    p = sv.params(precision="fp64", tol=1e-10, check_every=100, **m)
    s, st = sv.solve_soc_steady(pb.ctx, p)
    assert st.status == sv.OK
    op = oracle_problem(orc, solid, u, m)
    sx = orc.exact_steady(op)
    pore = solid == 0
    sg = s.cpu().numpy()
    assert np.abs(sg - sx)[pore].max() <= 1e-8
    assert np.all(sg[~pore] == 0.0)
    # the oracle's own explicit solve stops after the same number of sweeps
    so, info = orc.solve(op, cfl=0.4, tol=1e-10, check_every=100)
    assert abs(info["iterations"] - st.iterations) <= 100
    # outputs: utilisation and the flux balance against the oracle's, on the GPU state
    o = orc.outputs(op, sg)
    assert abs(st.U - o["U"]) <= 1e-12 * max(1.0, abs(o["U"]))
    for k in ("flux_in", "flux_out", "reaction", "q_out"):
        ok = {"flux_in": "F_in", "flux_out": "F_out", "reaction": "reaction", "q_out": "Q_out"}[k]
        assert abs(getattr(st, k) - o[ok]) <= 1e-11 * max(1.0, abs(o[ok])), k
    assert abs(st.flux_in - st.flux_out - st.reaction - st.sum_R) <= 1e-10 * abs(st.flux_in)
    assert abs(orc.residual_norm(op, sg) - st.residual) <= 0.05 * st.residual + 1e-13


@pytest.mark.parametrize("mode", list(MODES))
def test_fp32_mode_accuracy(sv, orc, case, mode):
    name, solid, u = case
    m = MODES[mode]
    pb = make(sv, solid, u)
    p = sv.params(precision="fp32", tol=1e-10, check_every=100, **m)
    s, st = sv.solve_soc_steady(pb.ctx, p)
    assert st.status == sv.OK and (st.it_fp32 > 0 or name.startswith("open"))
    op = oracle_problem(orc, solid, u, m)
    sx = orc.exact_steady(op)
    pore = solid == 0
    ds = np.abs(s.cpu().numpy() - sx)[pore].max()
    assert ds <= 1e-5, ds
    Ux = orc.outputs(op, sx)["U"]
    assert abs(st.U - Ux) <= 1e-6 * abs(Ux) + 1e-12
    assert orc.residual_norm(op, s.cpu().numpy()) < 1e-10 * 1.5


def test_fp32_plain_stagnates_above_fp64(sv, orc):
    solid, u = CASES["fibre64"]()
    pb = make(sv, solid, u)
    p = sv.params(precision="fp32_plain", tol=1e-10, check_every=100)
    s, st = sv.solve_soc_steady(pb.ctx, p)
    op = orc.Problem(solid, *u, s_in=1.0, s_eq=0.0, Da=0.45)
    sx = orc.exact_steady(op)
    ds = np.abs(s.cpu().numpy() - sx)[solid == 0].max()
    # plain FP32 stops at its rounding floor; the state is still close
    assert ds < 1e-4
    assert st.status in (sv.OK, sv.NOT_CONVERGED)


def test_plug_flow_closed_form_on_gpu(sv):
    from tests.test_oracle_pins import plug_flow_discrete
    n, u, lam = 96, 1.7, 0.12
    solid, vel = I.plug_flow_case(n, 5, 3, u)
    # a homogeneous sink needs a reactive face in every cell: use a fibre-free box and
    # compare with lam = 0 (pure advection-diffusion: s = s_in everywhere) ...
    pb = make(sv, solid, vel)
    s, st = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp64", tol=1e-12, s_in=0.3,
                                                     s_eq=0.9))
    assert np.abs(s.cpu().numpy() - 0.3).max() < 1e-12
    # ... and a channel one cell high between two fibre layers: every pore cell has two
    # fibre faces (lam = 2 Da), flow along x: the 1D recurrence with lam = 2 Da
    solid2 = np.ones((3, 1, n), dtype=np.uint8)
    solid2[1] = 0
    ux = np.zeros((3, 1, n + 1)); ux[1] = u
    uy = np.zeros((3, 2, n)); uz = np.zeros((4, 1, n))
    Da = lam / 2
    pb2 = make(sv, solid2, (ux, uy, uz))
    for prec in ("fp64", "fp32"):
        s2, st2 = sv.solve_soc_steady(pb2.ctx, sv.params(precision=prec, tol=1e-11, Da=Da))
        ref = plug_flow_discrete(n, u, lam, 1.0, 0.0)
        d = np.abs(s2.cpu().numpy()[1, 0] - ref).max()
        assert d < (1e-12 if prec == "fp64" else 1e-7), (prec, d)


def test_umt_and_limits(sv, orc):
    solid, u = CASES["fibre64"]()
    pb = make(sv, solid, u)
    umt, s, st = sv.compute_umt(pb.ctx, sv.params(precision="fp64", tol=1e-10), want_state=True)
    op = orc.Problem(solid, *u, s_in=0.0, s_eq=1.0, pinned=True)
    ux = orc.outputs(op, orc.exact_steady(op))["U"]
    assert abs(umt - ux) <= 1e-9 * ux
    fin = []
    for Da in (0.45, 45.0):
        _, stf = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp64", tol=1e-10, s_in=0.0,
                                                         s_eq=1.0, Da=Da), want_state=False)
        fin.append(stf.U)
    assert fin[0] < fin[1] < umt


def test_activity_field(sv, orc):
    solid, u = CASES["ragged70x37x29"]()
    kappa = I.lognormal_activity(solid, 0.3, seed=5)
    pb = make(sv, solid, u, kappa=kappa)
    s, st = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp64", tol=1e-10))
    op = orc.Problem(solid, *u, s_in=1.0, s_eq=0.0, Da=0.45, kappa=kappa.astype(np.float64))
    sx = orc.exact_steady(op)
    assert np.abs(s.cpu().numpy() - sx)[solid == 0].max() < 1e-8


def test_time_step_follows_the_operator(sv, orc):
    # dt = cfl / (largest diagonal of the updated cells); the library scans the diagonal once
    # per operator and (Da, mode), so every change of Da, mode, flow rate or activity field
    # must give the oracle's dt again
    solid, u = CASES["ragged70x37x29"]()
    kappa = I.lognormal_activity(solid, 0.3, seed=5)
    pb = make(sv, solid, u)

    def dt_of(**kw):
        p = sv.params(precision="fp32", tol=0.0, max_iter=4, check_every=4, **kw)
        return sv.solve_soc_steady(pb.ctx, p, want_state=False)[1].dt

    def oracle_dt(q=1.0, Da=0.45, pinned=False, kap=None):
        op = orc.Problem(solid, *(a * q for a in u), s_in=1.0, s_eq=0.0, Da=Da, pinned=pinned,
                         kappa=None if kap is None else kap.astype(np.float64))
        return 0.4 / orc.max_diag(op)

    steps = [
        (dict(), dict()),
        (dict(), dict()),                                    # the same operator again
        (dict(Da=2.0), dict(Da=2.0)),
        (dict(mode=1, s_in=0.0, s_eq=1.0, Da=0.0), dict(Da=0.0, pinned=True)),
        (dict(), dict()),
    ]
    for kw, okw in steps:
        assert dt_of(**kw) == pytest.approx(oracle_dt(**okw), rel=1e-13), kw
    pb.set_flow_rate(3.0)
    assert dt_of() == pytest.approx(oracle_dt(q=3.0), rel=1e-13)
    pb.set_activity(cuda(kappa, torch.float32))
    assert dt_of() == pytest.approx(oracle_dt(q=3.0, kap=kappa), rel=1e-13)
    pb.set_activity(None)
    assert dt_of() == pytest.approx(oracle_dt(q=3.0), rel=1e-13)


def test_warm_start_resume(sv):
    solid, u = CASES["fibre64"]()
    pb = make(sv, solid, u)
    # FP64: 400 sweeps, then 400 more from that state == 800 sweeps directly
    p4 = sv.params(precision="fp64", tol=0.0, max_iter=400, check_every=200)
    s4, _ = sv.solve_soc_steady(pb.ctx, p4)
    s8a, _ = sv.solve_soc_steady(pb.ctx, p4, s_init=s4.clone())
    s8, _ = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp64", tol=0.0, max_iter=800,
                                                   check_every=200))
    assert torch.equal(s8a, s8)


def test_deterministic(sv):
    solid, u = CASES["ragged70x37x29"]()
    pb = make(sv, solid, u)
    p = sv.params(precision="fp32", tol=1e-9)
    a, sa = sv.solve_soc_steady(pb.ctx, p)
    b, sb = sv.solve_soc_steady(pb.ctx, p)
    assert torch.equal(a, b) and sa.residual == sb.residual and sa.U == sb.U


def test_error_paths(sv):
    # pocket not connected to the inlet
    solid = np.zeros((4, 4, 8), dtype=np.uint8)
    solid[:, :, 3] = 1
    with pytest.raises(sv.SocfvError) as e:
        sv.setup_geometry(cuda(solid, torch.uint8))
    assert e.value.code == sv.BAD_GEOMETRY
    solid, u = CASES["ragged70x37x29"]()
    ctx = sv.setup_geometry(cuda(solid, torch.uint8))
    ux, uy, uz = (cuda(a, torch.float64) for a in u)
    # flux through a fibre face
    zf, yf, xf = map(int, np.argwhere(solid == 1)[0])
    bad = ux.clone()
    bad[zf, yf, xf] = 0.5
    with pytest.raises(sv.SocfvError) as e:
        sv.set_velocity(ctx, bad, uy, uz)
    assert e.value.code == sv.BAD_VELOCITY
    bad = ux.clone()
    bad[0, 0, 5] = float("nan")
    with pytest.raises(sv.SocfvError):
        sv.set_velocity(ctx, bad, uy, uz)
    bad = ux.clone()
    inlet = np.argwhere(solid[:, :, 0] == 0)[0]
    bad[int(inlet[0]), int(inlet[1]), 0] = -1.0
    with pytest.raises(sv.SocfvError):
        sv.set_velocity(ctx, bad, uy, uz)
    # solving before a velocity is set
    with pytest.raises(sv.SocfvError) as e:
        sv.solve_soc_steady(ctx, sv.params())
    assert e.value.code == sv.INVALID_ARG
    sv.set_velocity(ctx, ux, uy, uz)
    with pytest.raises(sv.SocfvError) as e:
        sv.solve_soc_steady(ctx, sv.params(cfl=1.5))
    assert e.value.code == sv.INVALID_ARG
    # not converged: outputs still written
    s, st = sv.solve_soc_steady(ctx, sv.params(precision="fp64", max_iter=10, check_every=2))
    assert st.status == sv.NOT_CONVERGED and st.iterations == 10
    # a start state outside the bounds is reported as divergence
    with pytest.raises(sv.SocfvError) as e:
        sv.solve_soc_steady(ctx, sv.params(precision="fp64"),
                            s_init=torch.full(ctx.shape, 5.0, dtype=torch.float64, device="cuda"))
    assert e.value.code == sv.DIVERGED
    # adjoint before a matching forward
    ctx2 = sv.setup_geometry(cuda(solid, torch.uint8))
    sv.set_velocity(ctx2, ux, uy, uz)
    with pytest.raises(sv.SocfvError):
        sv.solve_soc_adjoint(ctx2, sv.params())


def test_single_cell_and_degenerate(sv):
    # one pore cell with a fibre face: closed form
    solid = np.array([[[0], [1]]], dtype=np.uint8)
    u = 0.7
    ux = np.zeros((1, 2, 2)); ux[0, 0, :] = u
    uy = np.zeros((1, 3, 1)); uz = np.zeros((2, 2, 1))
    pb = make(sv, solid, (ux, uy, uz))
    s, st = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp64", tol=1e-13, s_in=1.0,
                                                   s_eq=0.2, Da=0.45))
    expect = ((u + 2) * 1.0 + 0.45 * 0.2) / (u + 2 + 0.45)
    assert abs(float(s[0, 0, 0]) - expect) < 1e-13


@pytest.mark.parametrize("shape", [(128, 40, 33), (70, 37, 29), (260, 21, 13), (64, 32, 32),
                                   (63, 40, 33), (129, 21, 13)])
def test_two_sweep_launches_match_single_sweeps(sv, shape):
    """FP32 sweeps fused two per launch give the same iterates as one sweep per launch (odd
    nx: one cell per lane)."""
    nx, ny, nz = shape
    solid, u = fibre_case(nx, ny, nz, 3.0, 0.85, 31, 1.0)
    pb = make(sv, solid, u)
    out = {}
    for two in (0, 1):
        sv.set_tiles(pb.ctx, 0, 0, 0, two)
        for prec in ("fp32_plain", "fp32"):
            p = sv.params(precision=prec, tol=0.0, max_iter=400, check_every=200)
            s, st = sv.solve_soc_steady(pb.ctx, p)
            out[(two, prec)] = (s.cpu().numpy(), st.iterations)
    for prec in ("fp32_plain", "fp32"):
        a, na = out[(0, prec)]
        b, nb = out[(1, prec)]
        assert na == nb
        assert np.abs(a - b).max() <= 1e-6, (prec, np.abs(a - b).max())


@pytest.mark.parametrize("variant", ["pinned", "activity"])
def test_two_sweep_launches_match_single_sweeps_modes(sv, orc, variant):
    """The same with held cells (pinned mode) and with a per-cell activity and s_eq > 0 (the
    plain form's source term): fibre cells stay 0 and held cells s_eq exactly."""
    solid, u = fibre_case(128, 40, 33, 3.0, 0.85, 32, 1.0)
    kappa = I.lognormal_activity(solid, 0.3, seed=7) if variant == "activity" else None
    pb = make(sv, solid, u, kappa=kappa)
    if variant == "pinned":
        kw = dict(mode=1, s_in=0.0, s_eq=1.0, Da=0.0)
    else:
        kw = dict(s_in=0.9, s_eq=0.3, Da=0.45)
    out = {}
    for two in (0, 1):
        sv.set_tiles(pb.ctx, 0, 0, 0, two)
        for prec in ("fp32_plain", "fp32"):
            p = sv.params(precision=prec, tol=0.0, max_iter=400, check_every=200, **kw)
            s, st = sv.solve_soc_steady(pb.ctx, p)
            out[(two, prec)] = (s.cpu().numpy(), st.iterations)
    nf = orc.fibre_faces(solid)
    held = (nf > 0) & (solid == 0) if variant == "pinned" else np.zeros(solid.shape, bool)
    for prec in ("fp32_plain", "fp32"):
        a, na = out[(0, prec)]
        b, nb = out[(1, prec)]
        assert na == nb
        assert np.abs(a - b).max() <= 1e-6, (prec, np.abs(a - b).max())
        assert np.all(b[solid == 1] == 0.0)
        assert np.all(b[held] == kw["s_eq"])
