"""FP64 CPU oracle for the steady state-of-charge solve (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package.  It shares no code with the GPU library: the arithmetic lives in
``soc_oracle.c`` (plain C loops, FP64) and, for the exact steady state, in a sparse
solve of the same rows with SciPy.

Functions (each cites what it follows; the discretisation is described at the top of
``soc_oracle.c``):

* ``fibre_faces`` / ``disconnected``      geometry classification (specific area of
  surface cells, Sec. "Direct Reaction Models": a = A / V per cell)
* ``reaction_coeff``                      lam = Da * kappa * n_f, from the affine rate
  of Eq. (rate-from-soc-gen): S / C_T = a k0 (e^{alpha V}) (1 - (1 + e^{-V}) s)
* ``residual`` / ``solve`` / ``iterate``  the explicit pseudo-time iteration of the
  Algorithm "SOC at Mass Transport Limit" with the stop rule of
  Eq. (convergence-bv-change)
* ``outputs``                             U (Eq. (utilization-def); U_mt of
  Eq. (umt-def) in pinned mode) and the flux balance of Eqs. (electron-flow) -
  (convergence-bv-flow)
* ``exact_steady`` / ``exact_adjoint``    the fixed point A s = b (and A^T psi = g)
  by a sparse direct or Krylov solve of the same rows
* ``adjoint`` / ``gradients``             explicit iteration for A^T psi = g and the
  design gradients dU/dkappa, dU/dln q
* ``oracle.stokes``                       the upstream flow step: steady Stokes flow on
  the voxel grid and the projection step of the Algorithm "Flow Simulation"
* ``rate_*``                              the reaction-rate algebra of
  Eqs. (rate-soc-eta), (rate-from-soc), (rate-from-soc-gen), (seq-from-Var)
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "soc_oracle.c")
_LIB = os.path.join(_HERE, "libsoc_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc -O3, OpenMP) next to its source."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i, l, d = C.c_int, C.c_long, C.c_double
        L.orc_fibre_faces.argtypes = [i, i, i, P, P]; L.orc_fibre_faces.restype = l
        L.orc_disconnected.argtypes = [i, i, i, P]; L.orc_disconnected.restype = l
        L.orc_reaction_coeff.argtypes = [i, i, i, P, P, d, P]; L.orc_reaction_coeff.restype = None
        L.orc_residual.argtypes = [i, i, i, P, P, P, P, P, P, d, d, i, P, P]
        L.orc_residual.restype = d
        L.orc_max_diag.argtypes = [i, i, i, P, P, P, P, P, P, i]; L.orc_max_diag.restype = d
        L.orc_inflow.argtypes = [i, i, i, P, P]; L.orc_inflow.restype = d
        L.orc_solve.argtypes = [i, i, i, P, P, P, P, P, P, d, d, i, d, d, l, i, P, P]
        L.orc_solve.restype = i
        L.orc_iterate.argtypes = [i, i, i, P, P, P, P, P, P, d, d, i, d, l, P, P]
        L.orc_iterate.restype = None
        L.orc_outputs.argtypes = [i, i, i, P, P, P, P, P, P, d, d, i, P, P]
        L.orc_outputs.restype = None
        L.orc_adjoint_rhs.argtypes = [i, i, i, P, P, d, d, P]; L.orc_adjoint_rhs.restype = None
        L.orc_adjoint.argtypes = [i, i, i, P, P, P, P, P, P, d, d, i, d, d, l, i, P, P]
        L.orc_adjoint.restype = i
        L.orc_gradients.argtypes = [i, i, i, P, P, P, P, P, d, d, d, i, P, P, P]
        L.orc_gradients.restype = d
        L.orc_export_rows.argtypes = [i, i, i, P, P, P, P, P, P, d, d, i, P, P, P, P, P]
        L.orc_export_rows.restype = None
        L.orc_apply_AT.argtypes = [i, i, i, P, P, P, P, P, P, i, P, P, i]
        L.orc_apply_AT.restype = None
        L.orc_nernst.argtypes = [i, i, i, P, P, P, P, P, P, d, d, d, d, d, l, i, P, P, P]
        L.orc_nernst.restype = i
        L.orc_num_threads.argtypes = []; L.orc_num_threads.restype = i
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ------------------------------------------------------------------------------------
# Reaction-rate algebra (Sec. "Electrochemical Reaction with Uniform Potential in
# Electrolyte"); V is the dimensionless applied reducing voltage.
# ------------------------------------------------------------------------------------

def sigmoid(x):
    return 1.0 / (1.0 + math.exp(-x))


def rate_sinh(s, V):
    """Eq. (rate-soc-eta) with the overpotential of Eq. (etat-from-s):
    R = 2 sqrt(s(1-s)) sinh(eta/2), eta = V - log(s/(1-s))."""
    eta = V - math.log(s / (1.0 - s))
    return 2.0 * math.sqrt(s * (1.0 - s)) * math.sinh(eta / 2.0)


def rate_bv_general(s, V, alpha):
    """Eq. (source-term-bv-gen) divided by a k0 C_T, with eta from Eq. (etat-from-s)."""
    eta = V - math.log(s / (1.0 - s))
    return s ** alpha * (1.0 - s) ** (1.0 - alpha) * (math.exp(alpha * eta)
                                                      - math.exp((alpha - 1.0) * eta))


def rate_affine(s, V, alpha):
    """Eq. (rate-from-soc-gen): R = e^{alpha V} (1 - (1 + e^{-V}) s)."""
    return math.exp(alpha * V) * (1.0 - (1.0 + math.exp(-V)) * s)


def rate_slope_and_seq(V, alpha):
    """R = K (s_eq - s): K = e^{alpha V} + e^{(alpha-1) V}, s_eq = sigma(V)
    (Eq. (seq-from-Var) with phi_L = 0)."""
    K = math.exp(alpha * V) + math.exp((alpha - 1.0) * V)
    return K, sigmoid(V)


def damkohler_per_face(k0, V, alpha, h, D):
    """Per fibre face reaction number Da = k0 K h / D (specific area a = n_f / h)."""
    K, _ = rate_slope_and_seq(V, alpha)
    return k0 * K * h / D


# ------------------------------------------------------------------------------------
# Problem wrapper
# ------------------------------------------------------------------------------------

@dataclass
class Problem:
    solid: np.ndarray          # uint8 (nz, ny, nx)
    ux: np.ndarray             # float64 (nz, ny, nx+1)
    uy: np.ndarray             # float64 (nz, ny+1, nx)
    uz: np.ndarray             # float64 (nz+1, ny, nx)
    s_in: float = 1.0
    s_eq: float = 0.0
    Da: float = 0.45
    pinned: bool = False
    kappa: np.ndarray | None = None   # per-cell activity (None: 1)
    lam_field: np.ndarray | None = None   # explicit per-cell sink (overrides Da*kappa*n_f)

    def __post_init__(self):
        self.solid = _c(self.solid, np.uint8)
        self.ux = _c(self.ux, np.float64)
        self.uy = _c(self.uy, np.float64)
        self.uz = _c(self.uz, np.float64)
        nz, ny, nx = self.solid.shape
        assert self.ux.shape == (nz, ny, nx + 1)
        assert self.uy.shape == (nz, ny + 1, nx)
        assert self.uz.shape == (nz + 1, ny, nx)
        if self.kappa is not None:
            self.kappa = _c(self.kappa, np.float64)
            assert self.kappa.shape == self.solid.shape
        self.nf = fibre_faces(self.solid)
        if self.lam_field is not None:
            self.lam = np.where(self.solid == 0, _c(self.lam_field, np.float64), 0.0)
            self.lam = np.ascontiguousarray(self.lam)
        else:
            self.lam = reaction_coeff(self.nf, self.kappa, 0.0 if self.pinned else self.Da)

    @property
    def dims(self):
        nz, ny, nx = self.solid.shape
        return nx, ny, nz

    def _args(self):
        nx, ny, nz = self.dims
        return (nx, ny, nz, _p(self.solid), _p(self.ux), _p(self.uy), _p(self.uz),
                _p(self.lam), _p(self.nf))

    def initial_state(self):
        s = np.where(self.solid == 0, self.s_in, 0.0)
        if self.pinned:
            s = np.where(self.nf > 0, self.s_eq, s)
        return s.astype(np.float64)


def fibre_faces(solid):
    solid = _c(solid, np.uint8)
    nz, ny, nx = solid.shape
    nf = np.empty(solid.shape, dtype=np.int8)
    lib().orc_fibre_faces(nx, ny, nz, _p(solid), _p(nf))
    return nf


def disconnected(solid) -> int:
    solid = _c(solid, np.uint8)
    nz, ny, nx = solid.shape
    return int(lib().orc_disconnected(nx, ny, nz, _p(solid)))


def reaction_coeff(nf, kappa, Da):
    nz, ny, nx = nf.shape
    lam = np.empty(nf.shape, dtype=np.float64)
    lib().orc_reaction_coeff(nx, ny, nz, _p(nf), _p(_c(kappa, np.float64)), float(Da), _p(lam))
    return lam


def residual(pb: Problem, s):
    s = _c(s, np.float64)
    R = np.empty_like(s)
    ss = lib().orc_residual(*pb._args(), pb.s_in, pb.s_eq, int(pb.pinned), _p(s), _p(R))
    return R, ss


def max_diag(pb: Problem) -> float:
    return float(lib().orc_max_diag(*pb._args(), int(pb.pinned)))


def inflow(pb: Problem) -> float:
    nx, ny, nz = pb.dims
    return float(lib().orc_inflow(nx, ny, nz, _p(pb.solid), _p(pb.ux)))


def time_scale(pb: Problem) -> float:
    nx, ny, nz = pb.dims
    return nx * ny * nz / inflow(pb)


def solve(pb: Problem, cfl=0.4, tol=1e-10, max_iter=10**7, check_every=1, s0=None):
    """Explicit pseudo-time iteration to res < tol.  Returns (s, info)."""
    s = pb.initial_state() if s0 is None else np.array(s0, dtype=np.float64)
    out = np.zeros(4)
    st = lib().orc_solve(*pb._args(), pb.s_in, pb.s_eq, int(pb.pinned), float(cfl), float(tol),
                         int(max_iter), int(check_every), _p(s), _p(out))
    return s, {"status": int(st), "iterations": int(out[0]), "residual": float(out[1]),
               "dt": float(out[2]), "tau": float(out[3])}


def iterate(pb: Problem, s, dt, iters):
    """``iters`` explicit updates with a given dt (no checks); returns the new state."""
    s = np.array(s, dtype=np.float64)
    R = np.empty_like(s)
    lib().orc_iterate(*pb._args(), pb.s_in, pb.s_eq, int(pb.pinned), float(dt), int(iters),
                      _p(s), _p(R))
    return s


def outputs(pb: Problem, s) -> dict:
    s = _c(s, np.float64)
    out = np.zeros(8)
    lib().orc_outputs(*pb._args(), pb.s_in, pb.s_eq, int(pb.pinned), _p(s), _p(out))
    keys = ["U", "s_out", "F_in", "F_in_adv", "F_out", "reaction", "sum_R", "Q_out"]
    return dict(zip(keys, map(float, out)))


def residual_norm(pb: Problem, s) -> float:
    """tau * rms over pore cells of R (Eq. (convergence-bv-change), RMS norm)."""
    R, ss = residual(pb, s)
    npore = int(np.count_nonzero(pb.solid == 0))
    return time_scale(pb) * math.sqrt(ss / npore)


def correction_iterate(pb: Problem, r0, dt, iters, delta=None):
    """The inner iteration of iterative refinement on A s = b (the mixed-precision form of
    the explicit iteration): for a frozen residual r0 = b - A s of some state s,
    ``iters`` updates delta <- delta + dt (r0 - A delta) from delta = 0 (or ``delta``).
    A delta is the residual operator with zero boundary values (s_in = s_eq = 0), so
    fibre and held cells keep delta = 0.  By linearity s + delta_k is the k-th iterate of
    the explicit iteration started from s.  Returns delta."""
    z = Problem.__new__(Problem)
    z.__dict__.update(pb.__dict__)
    z.s_in, z.s_eq = 0.0, 0.0
    upd = (pb.solid == 0) & ~((pb.nf > 0) & bool(pb.pinned))
    r0 = np.where(upd, np.asarray(r0, dtype=np.float64), 0.0)
    d = np.zeros(pb.solid.shape) if delta is None else np.array(delta, dtype=np.float64)
    for _ in range(int(iters)):
        Az, _ = residual(z, d)           # = -A delta on updated cells, 0 elsewhere
        d = d + dt * (r0 + Az)
    return d


def adjoint_rhs(pb: Problem):
    nx, ny, nz = pb.dims
    g = np.empty(pb.solid.shape, dtype=np.float64)
    lib().orc_adjoint_rhs(nx, ny, nz, _p(pb.solid), _p(pb.ux), pb.s_in, pb.s_eq, _p(g))
    return g


def adjoint(pb: Problem, cfl=0.4, tol=1e-12, max_iter=10**7, check_every=1):
    """Explicit iteration psi <- psi + dt (g - A^T psi).  Returns (psi, info)."""
    psi = np.zeros(pb.solid.shape, dtype=np.float64)
    out = np.zeros(2)
    st = lib().orc_adjoint(*pb._args(), pb.s_in, pb.s_eq, int(pb.pinned), float(cfl), float(tol),
                           int(max_iter), int(check_every), _p(psi), _p(out))
    return psi, {"status": int(st), "iterations": int(out[0]), "rel_residual": float(out[1])}


def apply_AT(pb: Problem, psi, scatter=False):
    """A^T psi over all cells, by gathering (default) or by scattering each row."""
    psi = _c(psi, np.float64)
    t = np.empty_like(psi)
    lib().orc_apply_AT(*pb._args(), int(pb.pinned), _p(psi), _p(t), int(bool(scatter)))
    return t


def gradients(pb: Problem, s, psi):
    """(dU/dkappa field, dU/dln q)."""
    nx, ny, nz = pb.dims
    g = np.zeros(pb.solid.shape, dtype=np.float64)
    dq = lib().orc_gradients(nx, ny, nz, _p(pb.solid), _p(pb.ux), _p(pb.uy), _p(pb.uz),
                             _p(pb.nf), float(pb.Da), pb.s_in, pb.s_eq, int(pb.pinned),
                             _p(_c(s, np.float64)), _p(_c(psi, np.float64)), _p(g))
    return g, float(dq)


# ------------------------------------------------------------------------------------
# The fixed point by a sparse solve of the same rows
# ------------------------------------------------------------------------------------

def rows(pb: Problem):
    nx, ny, nz = pb.dims
    n = nx * ny * nz
    diag = np.empty(n); rhs = np.empty(n); held = np.empty(n, dtype=np.uint8)
    nb = np.empty(6 * n, dtype=np.int64); coef = np.empty(6 * n)
    lib().orc_export_rows(*pb._args(), pb.s_in, pb.s_eq, int(pb.pinned), _p(diag), _p(rhs),
                          _p(held), _p(nb), _p(coef))
    return diag, rhs, held, nb, coef


def assemble(pb: Problem):
    """Sparse A (CSR) and b of A s = b over all cells (fibre cells: identity rows)."""
    import scipy.sparse as sp
    diag, rhs, held, nb, coef = rows(pb)
    n = diag.size
    r6 = np.repeat(np.arange(n), 6)
    m = nb >= 0
    ri = np.concatenate([np.arange(n), r6[m]])
    ci = np.concatenate([np.arange(n), nb[m]])
    va = np.concatenate([diag, coef[m]])
    A = sp.csr_matrix((va, (ri, ci)), shape=(n, n))
    return A, rhs


def _krylov(A, b, tol, x0=None, maxiter=20000):
    import scipy.sparse.linalg as sla
    n = A.shape[0]
    dinv = 1.0 / A.diagonal()
    M = sla.LinearOperator((n, n), matvec=lambda v: dinv * v)
    x, info = sla.gmres(A, b, x0=x0, rtol=tol, atol=0.0, restart=200, maxiter=maxiter, M=M)
    if info != 0:
        raise RuntimeError(f"Krylov solve did not converge (info={info})")
    return x


def exact_steady(pb: Problem, method="auto", tol=1e-14):
    """s* = A^{-1} b on the grid (the unique fixed point of the explicit iteration)."""
    import scipy.sparse.linalg as sla
    A, b = assemble(pb)
    n = b.size
    if method == "auto":
        method = "direct" if n <= 300000 else "krylov"
    if method == "direct":
        x = sla.spsolve(A.tocsc(), b)
    else:
        x = _krylov(A, b, tol)
    return x.reshape(pb.solid.shape)


def exact_adjoint(pb: Problem, method="auto", tol=1e-14):
    """psi = A^{-T} g (g = dU/ds), full field including held cells."""
    import scipy.sparse.linalg as sla
    A, _ = assemble(pb)
    g = adjoint_rhs(pb).ravel()
    n = g.size
    AT = A.T.tocsr()
    # fibre rows are identity with g = 0, so psi = 0 there
    if method == "auto":
        method = "direct" if n <= 300000 else "krylov"
    if method == "direct":
        x = sla.spsolve(AT.tocsc(), g)
    else:
        x = _krylov(AT, g, tol)
    return x.reshape(pb.solid.shape)


# ------------------------------------------------------------------------------------
# Iterative upsampling (Sec. "Incompressible Fluid Flow", its part on iterative upsampling:
# converge on the unrefined grid, then start the refined problem from the interpolated
# steady state).  Applied to the SOC solve with a grid coarsened by two in every direction.
# ------------------------------------------------------------------------------------

def _pair_sum_half(a, b, c, d):
    """((a + b) + (c + d)) / 2: the four fine faces under a coarse face, in a fixed order."""
    return ((a + b) + (c + d)) * 0.5


def coarsen(pb: Problem) -> Problem:
    """The problem on the grid coarsened by two in every direction (even nx, ny, nz).

    A coarse cell is fibre iff all eight children are fibre (so every face of a coarse fibre
    cell lies on fine fibre faces and carries no flux, and every coarse pore cell holds a
    fine pore cell connected to the inlet).  A coarse face velocity, in coarse grid units
    (h doubled, D unchanged), is half the sum of its four fine face velocities: the same
    physical flux.  Reaction per coarse fibre face 2 Da (Da = k h / D with h doubled).  The
    activity field is not carried (the coarse solve is only a starting state)."""
    nz, ny, nx = pb.solid.shape
    assert nx % 2 == 0 and ny % 2 == 0 and nz % 2 == 0, "coarsening needs even dimensions"
    sol = pb.solid.astype(bool).reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2)
    csolid = sol.all(axis=(1, 3, 5)).astype(np.uint8)
    fx = pb.ux[:, :, 0::2]                       # x faces at even fine x: (nz, ny, nx/2 + 1)
    ux = _pair_sum_half(fx[0::2, 0::2], fx[0::2, 1::2], fx[1::2, 0::2], fx[1::2, 1::2])
    fy = pb.uy[:, 0::2, :]                       # (nz, ny/2 + 1, nx)
    uy = _pair_sum_half(fy[0::2, :, 0::2], fy[0::2, :, 1::2], fy[1::2, :, 0::2], fy[1::2, :, 1::2])
    fz = pb.uz[0::2]                             # (nz/2 + 1, ny, nx)
    uz = _pair_sum_half(fz[:, 0::2, 0::2], fz[:, 0::2, 1::2], fz[:, 1::2, 0::2], fz[:, 1::2, 1::2])
    return Problem(csolid, ux, uy, uz, s_in=pb.s_in, s_eq=pb.s_eq, Da=2.0 * pb.Da,
                   pinned=pb.pinned)


def prolongate(pb: Problem, s_coarse):
    """Fine starting state from a coarse one: each fine pore cell takes its parent's value
    (piecewise-constant interpolation), fibre cells 0."""
    s = np.repeat(np.repeat(np.repeat(_c(s_coarse, np.float64), 2, axis=0), 2, axis=1), 2, axis=2)
    return np.where(pb.solid == 0, s, 0.0)


# ------------------------------------------------------------------------------------
# Explicit Nernst model (Sec. "Steady State Reaction Model (Nernst)", Algorithm "Explicit
# Nernst Model"; electrode value sigma(V - eta) of Eq. (nernst-model-s-update))
# ------------------------------------------------------------------------------------

def nernst(pb: Problem, omega=0.5, cfl=0.4, tol=1e-10, max_iter=10**7, check_every=1,
           s0=None, eta0=None):
    """Electrode cells (reactive pore cells) held at sigma(V - eta), eta relaxed toward the
    overpotential that balances the transport step (steps in the order of ``orc_nernst``).  Finite-rate problems with 0 < s_eq < 1 and Da > 0.  Returns
    (s, eta, info)."""
    assert not pb.pinned and 0.0 < pb.s_eq < 1.0 and pb.Da > 0.0
    s = pb.initial_state() if s0 is None else np.array(s0, dtype=np.float64)
    eta = np.zeros(pb.solid.shape) if eta0 is None else np.array(eta0, dtype=np.float64)
    s = _c(s, np.float64)
    eta = _c(eta, np.float64)
    out = np.zeros(4)
    st = lib().orc_nernst(*pb._args(), pb.s_in, pb.s_eq, float(omega), float(cfl), float(tol),
                          int(max_iter), int(check_every), _p(s), _p(eta), _p(out))
    return s, eta, {"status": int(st), "iterations": int(out[0]), "residual": float(out[1]),
                    "dt": float(out[2]), "tau": float(out[3])}
