"""Equal-count parity of the FP32 sweeps with the FP64 oracle (needs an MI355X).

Each FP32 launch form runs the same number of explicit updates as the oracle, at the same
dt and from the same start, and is compared cell by cell:

* plain form (the state itself in FP32): against ``oracle.iterate``;
* correction form (the bulk of every FP32-mode solve: an FP32 correction on a frozen FP64
  residual r0 = b - A s0 of the start): the solve returns s0 + delta after one cycle, compared
  with s0 + ``oracle.correction_iterate(r0)``.

Launch forms, by box and the two-sweep switch: two sweeps per launch on rows of 64 lanes or
of 32 lanes (two per wave), with two cells per lane (even nx) or one (odd nx); one sweep per
launch with four cells per lane (nx a multiple of 4) or one cell per lane.  Boxes span several
tiles in x, y and z with ragged tails; 401 updates end every two-sweep run with one single
sweep.

Tolerance 1e-5 absolute (|s| <= 1): an FP32 update rounds about ten operations (6e-8 each),
and the iteration is non-expansive (every update coefficient is >= 0 at cfl <= 1), so 400
updates accumulate ~1e-6 in practice.  A 0.1% error in one coefficient moves the iterates by
more than the tolerance (``test_tolerance_sees_a_coefficient_error`` plants one in the
oracle, on the CPU).
"""
import numpy as np
import pytest
import torch

from paper_2502_08034_amd import inputs as I

TOL = 1e-5
SWEEPS = 401

SHAPES = {
    # nx % 4 == 0: two-sweep kernel with two cells per lane / four cells per lane
    "260x45x70": (260, 45, 70, 3.0, 0.82, 41, 1.0),
    # odd nx: two-sweep kernel with one cell per lane / scalar sweep
    "131x33x41": (131, 33, 41, 2.5, 0.85, 42, 1.5),
    # even nx, not a multiple of 4: two cells per lane / scalar sweep
    "130x19x37": (130, 19, 37, 2.5, 0.85, 43, 0.7),
}
MODES = {"finite": dict(s_in=1.0, s_eq=0.0, Da=0.45, mode=0),
         "pinned": dict(s_in=0.0, s_eq=1.0, Da=0.0, mode=1)}


def build_case(name):
    nx, ny, nz, r, phi, seed, pe = SHAPES[name]
    g = I.fibres_nonoverlap(nx, ny, nz, r, phi, seed)
    return g.solid, I.darcy_velocity(g.solid, pe)


@pytest.fixture(scope="module", params=list(SHAPES))
def case(request):
    solid, u = build_case(request.param)
    return request.param, solid, u


def oracle_refs(orc, solid, u, m, kappa=None):
    op = orc.Problem(solid, *u, s_in=m["s_in"], s_eq=m["s_eq"], Da=m["Da"],
                     pinned=bool(m["mode"]), kappa=kappa)
    dt = 0.4 / orc.max_diag(op)
    s0 = op.initial_state()
    plain = orc.iterate(op, s0, dt, SWEEPS)
    r0, _ = orc.residual(op, s0)
    corr = s0 + orc.correction_iterate(op, r0, dt, SWEEPS)
    return dt, plain, corr


def run_forms(sv, pb, m, forms):
    out = {}
    for two in forms:
        sv.set_tiles(pb.ctx, 0, 0, 0, two)
        for prec in ("fp32_plain", "fp32"):
            p = sv.params(precision=prec, tol=0.0, max_iter=SWEEPS, check_every=200, **m)
            s, st = sv.solve_soc_steady(pb.ctx, p)
            out[(two, prec)] = (s.cpu().numpy(), st)
    return out


def test_tolerance_sees_a_coefficient_error(orc):
    # CPU only: a 0.1% error planted in the oracle's reaction coefficient or in the x-face
    # velocities moves 401 updates by well over TOL, so the comparison above would catch it
    solid, u = build_case("130x19x37")
    for mode, m in MODES.items():
        op = orc.Problem(solid, *u, s_in=m["s_in"], s_eq=m["s_eq"], Da=m["Da"],
                         pinned=bool(m["mode"]))
        dt = 0.4 / orc.max_diag(op)
        ref = orc.iterate(op, op.initial_state(), dt, SWEEPS)
        bad = [orc.Problem(solid, u[0] * 1.001, u[1], u[2], s_in=m["s_in"], s_eq=m["s_eq"],
                           Da=m["Da"], pinned=bool(m["mode"]))]
        if mode == "finite":
            bad.append(orc.Problem(solid, *u, s_in=m["s_in"], s_eq=m["s_eq"], Da=m["Da"] * 1.001))
        for ob in bad:
            d = np.abs(orc.iterate(ob, ob.initial_state(), dt, SWEEPS) - ref).max()
            assert d > 5 * TOL, (mode, d)


@pytest.fixture(scope="module")
def sv():
    from paper_2502_08034_amd import socfv
    assert torch.cuda.is_available()
    return socfv


@pytest.mark.gpu
@pytest.mark.parametrize("mode", list(MODES))
def test_fp32_sweeps_match_oracle_at_equal_count(sv, orc, case, mode):
    name, solid, u = case
    m = MODES[mode]
    dt, plain, corr = oracle_refs(orc, solid, u, m)
    pb = sv.Problem.create(solid, *u)
    runs = run_forms(sv, pb, m, (2, 3, 0))
    pore = solid == 0
    for (two, prec), (s, st) in runs.items():
        assert st.status == sv.NOT_CONVERGED and st.iterations == SWEEPS, (two, prec)
        assert st.it_fp32 == SWEEPS and st.sweeps_fp64 == 0
        assert abs(st.dt - dt) <= 1e-15 * dt
        ref = plain if prec == "fp32_plain" else corr
        d = np.abs(s - ref)[pore].max()
        print(f"{name} {mode} two={two} {prec}: max |ds| {d:.2e}")
        assert d <= TOL, (name, mode, two, prec, d)
        assert np.all(s[~pore] == 0.0)
        if mode == "pinned":
            held = pore & (orc.fibre_faces(solid) > 0)
            assert np.all(s[held] == 1.0)


@pytest.mark.gpu
def test_fp32_sweeps_with_activity_field(sv, orc):
    # the activity variant of each launch form (activity loaded with the plane), s_eq > 0
    solid, u = build_case("131x33x41")
    kappa = I.lognormal_activity(solid, 0.3, seed=9)
    m = dict(s_in=0.9, s_eq=0.3, Da=0.45, mode=0)
    dt, plain, corr = oracle_refs(orc, solid, u, m, kappa=kappa.astype(np.float64))
    pb = sv.Problem.create(solid, *u, kappa=kappa)
    pore = solid == 0
    for (two, prec), (s, st) in run_forms(sv, pb, m, (2, 3, 0)).items():
        ref = plain if prec == "fp32_plain" else corr
        d = np.abs(s - ref)[pore].max()
        print(f"activity two={two} {prec}: max |ds| {d:.2e}")
        assert d <= TOL, (two, prec, d)


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["fibre64", "260x45x70", "131x33x41"])
@pytest.mark.parametrize("mode", list(MODES))
def test_fp32_mode_takes_the_fp64_sweep_count(sv, name, mode):
    # the correction cycles continue one explicit trajectory (linearity), and each cycle and
    # the FP64 iteration stop on the same residual test at the same chunk boundaries, so the
    # FP32 sweeps equal the FP64 count up to one chunk where FP32 rounding moves a crossing
    if name == "fibre64":
        w = I.workload("fibre64")
        solid, u = w["solid"], w["velocity"][0.5]
    else:
        solid, u = build_case(name)
    m = MODES[mode]
    pb = sv.Problem.create(solid, *u)
    K = 100
    _, s64 = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp64", tol=1e-10, check_every=K,
                                                    **m), want_state=False)
    _, s32 = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp32", tol=1e-10, check_every=K,
                                                    **m), want_state=False)
    print(f"{name} {mode}: FP64 {s64.iterations} sweeps; FP32 {s32.it_fp32} + polish "
          f"{s32.sweeps_fp64} in {s32.cycles} cycles")
    assert s64.status == sv.OK and s32.status == sv.OK
    assert abs(s32.it_fp32 - s64.iterations) <= K
    assert s32.sweeps_fp64 == K and s32.iterations == s32.it_fp32 + K


@pytest.mark.gpu
def test_max_iter_caps_every_sweep(sv):
    # the FP64 polish runs only after convergence and within what max_iter leaves
    w = I.workload("fibre64")
    pb = sv.Problem.create(w["solid"], *w["velocity"][0.5])
    _, st = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp32", tol=1e-10, check_every=100),
                                want_state=False)
    cap = st.it_fp32 + 40                       # converged, with 40 sweeps left for the polish
    _, sc = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp32", tol=1e-10, check_every=100,
                                                  max_iter=cap), want_state=False)
    assert sc.iterations <= cap and sc.sweeps_fp64 == 40
    _, sn = sv.solve_soc_steady(pb.ctx, sv.params(precision="fp32", tol=1e-10, check_every=100,
                                                  max_iter=st.it_fp32 - 100), want_state=False)
    assert sn.status == sv.NOT_CONVERGED and sn.iterations == st.it_fp32 - 100
    assert sn.sweeps_fp64 == 0
