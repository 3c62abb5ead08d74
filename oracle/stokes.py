"""FP64 CPU oracle for the upstream flow step (test infrastructure only).

Steady Stokes flow through the voxel pore space, the velocity field that the state-of-charge
solve takes as input.  The paper solves the incompressible Navier-Stokes equations
(Eqs. (navier-stokes), (incompressibility)) to steady state with Chorin's projection method
(Eqs. (cp1)-(cp4), Algorithm "Flow Simulation") and works in the Stokes regime, where the
steady velocity is linear in the applied pressure (Eq. (stokes-flow)).  This module writes the
discrete problem out on the voxel grid:

* unknowns: normal velocity on every open face (a face whose cells are both pore, or an
  inlet / outlet face of a pore cell) and pressure in every pore cell; faces that touch a fibre
  voxel or lie on a y / z domain wall are no-slip and carry zero velocity
* boundary conditions (Fig. "Boundary conditions"): applied pressure p_in at the inlet face
  x = 0, zero pressure at the outlet face x = nx, both half a cell from the first / last cell
  centre; no-slip on fibre voxel faces and on the y / z walls; zero normal gradient of every
  velocity component across the inlet and outlet planes
* viscous operator L (nondimensional: h = rho = mu = 1), per open face and per neighbour face of
  the same orientation one cell away along each axis:
    - neighbour open                               -> u_nb - u
    - along the face normal, neighbour closed      -> -u    (zero velocity one cell away)
    - across the face, neighbour closed or beyond
      a y / z wall                                 -> -2 u  (wall on the voxel face, reflection)
    - beyond the inlet / outlet plane              ->  0    (zero gradient)
* pressure gradient G on open faces: p_right - p_left inside, 2 (p_0 - p_in) on an inlet face,
  2 (0 - p_last) on an outlet face; divergence D of a pore cell: sum over its six faces of
  outward normal velocity
* steady Stokes: L u = G p on open faces, D u = 0 on pore cells (``stokes_steady``, by a sparse
  direct solve of this saddle-point system: the plain definition of the fixed point)
* one step of the flow simulation (``chorin_step``): with explicit momentum diffusion the
  predictor u* = u + dt L u (Eq. (cp1) without advection); with implicit diffusion (the
  algorithm's other branch) (I - dt L) v = u - dt (G p + gbc) with the lagged pressure, then
  u* = v + dt (G p + gbc); pressure from D G p' = D u* / dt - D gbc (Eq. (cp4)), projection
  u' = u* - dt (G p' + gbc) (Eq. (cp2)); time step from Eq. (time-step-flow) with the advective
  and force terms absent (``flow_time_step``); stop rule of Eq. (flow-cnvg)

The momentum advection term is omitted: the flow feeding the state-of-charge solve is taken in
the Stokes regime, where the paper scales one simulation to all applied pressures.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl


def open_faces(solid):
    """Open-face masks (ox, oy, oz) of shapes (nz, ny, nx+1), (nz, ny+1, nx), (nz+1, ny, nx)."""
    solid = np.asarray(solid)
    nz, ny, nx = solid.shape
    pore = solid == 0
    ox = np.zeros((nz, ny, nx + 1), bool)
    oy = np.zeros((nz, ny + 1, nx), bool)
    oz = np.zeros((nz + 1, ny, nx), bool)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx + 1):
                if i == 0:
                    ox[k, j, i] = pore[k, j, 0]
                elif i == nx:
                    ox[k, j, i] = pore[k, j, nx - 1]
                else:
                    ox[k, j, i] = pore[k, j, i - 1] and pore[k, j, i]
    for k in range(nz):
        for j in range(1, ny):
            for i in range(nx):
                oy[k, j, i] = pore[k, j - 1, i] and pore[k, j, i]
    for k in range(1, nz):
        for j in range(ny):
            for i in range(nx):
                oz[k, j, i] = pore[k - 1, j, i] and pore[k, j, i]
    return ox, oy, oz


class StokesOperators:
    """L, G (+ boundary vector), D of the discrete Stokes problem, over open faces and pore
    cells.  Face numbering: all x faces, then y faces, then z faces, each in (z, y, x) order;
    only open faces get an unknown."""

    def __init__(self, solid, p_in=1.0):
        solid = np.asarray(solid)
        self.shape = solid.shape
        nz, ny, nx = solid.shape
        self.p_in = float(p_in)
        self.opens = open_faces(solid)
        self.pore = solid == 0
        # unknown numbers of open faces and pore cells
        self.face_id = []
        n = 0
        for o in self.opens:
            ids = np.full(o.shape, -1, np.int64)
            for idx in zip(*np.nonzero(o)):
                ids[idx] = n
                n += 1
            self.face_id.append(ids)
        self.nu = n
        self.cell_id = np.full(solid.shape, -1, np.int64)
        m = 0
        for idx in zip(*np.nonzero(self.pore)):
            self.cell_id[idx] = m
            m += 1
        self.np_ = m
        self._assemble()
        self._lu = None

    def _assemble(self):
        nz, ny, nx = self.shape
        Lr, Lc, Lv = [], [], []
        Gr, Gc, Gv = [], [], []
        self.gbc = np.zeros(self.nu)
        for a in range(3):                       # face orientation: 0 = x, 1 = y, 2 = z
            o, ids = self.opens[a], self.face_id[a]
            dims = o.shape                       # (z, y, x) extents of this face array
            for (k, j, i) in zip(*np.nonzero(o)):
                f = ids[k, j, i]
                diag = 0.0
                for b in range(3):               # neighbour direction: 0 = x, 1 = y, 2 = z
                    for step in (-1, 1):
                        kk, jj, ii = k, j, i
                        if b == 0:
                            ii += step
                        elif b == 1:
                            jj += step
                        else:
                            kk += step
                        inside = 0 <= kk < dims[0] and 0 <= jj < dims[1] and 0 <= ii < dims[2]
                        if inside and o[kk, jj, ii]:
                            Lr.append(f)
                            Lc.append(ids[kk, jj, ii])
                            Lv.append(1.0)
                            diag -= 1.0
                        elif not inside and b == 0:
                            pass                 # beyond the inlet / outlet plane
                        elif b == a:
                            diag -= 1.0          # closed face along the normal
                        else:
                            diag -= 2.0          # wall across the face
                Lr.append(f)
                Lc.append(f)
                Lv.append(diag)
                # pressure gradient on the face
                if a == 0:
                    if i == 0:
                        Gr.append(f); Gc.append(self.cell_id[k, j, 0]); Gv.append(2.0)
                        self.gbc[f] = -2.0 * self.p_in
                    elif i == nx:
                        Gr.append(f); Gc.append(self.cell_id[k, j, nx - 1]); Gv.append(-2.0)
                    else:
                        Gr += [f, f]; Gc += [self.cell_id[k, j, i], self.cell_id[k, j, i - 1]]
                        Gv += [1.0, -1.0]
                elif a == 1:
                    Gr += [f, f]; Gc += [self.cell_id[k, j, i], self.cell_id[k, j - 1, i]]
                    Gv += [1.0, -1.0]
                else:
                    Gr += [f, f]; Gc += [self.cell_id[k, j, i], self.cell_id[k - 1, j, i]]
                    Gv += [1.0, -1.0]
        self.L = sp.csr_matrix((Lv, (Lr, Lc)), shape=(self.nu, self.nu))
        self.G = sp.csr_matrix((Gv, (Gr, Gc)), shape=(self.nu, self.np_))
        Dr, Dc, Dv = [], [], []
        fx, fy, fz = self.face_id
        for (k, j, i) in zip(*np.nonzero(self.pore)):
            c = self.cell_id[k, j, i]
            for fid, sign in ((fx[k, j, i + 1], 1.0), (fx[k, j, i], -1.0),
                              (fy[k, j + 1, i], 1.0), (fy[k, j, i], -1.0),
                              (fz[k + 1, j, i], 1.0), (fz[k, j, i], -1.0)):
                if fid >= 0:
                    Dr.append(c); Dc.append(fid); Dv.append(sign)
        self.D = sp.csr_matrix((Dv, (Dr, Dc)), shape=(self.np_, self.nu))

    # field <-> unknown vector
    def unpack(self, u, p=None):
        out = []
        for a in range(3):
            arr = np.zeros(self.opens[a].shape)
            m = self.face_id[a] >= 0
            arr[m] = u[self.face_id[a][m]]
            out.append(arr)
        if p is not None:
            pf = np.zeros(self.shape)
            pf[self.pore] = p[self.cell_id[self.pore]]
            out.append(pf)
        return tuple(out)

    def pack(self, ux, uy, uz, p=None):
        u = np.zeros(self.nu)
        for a, arr in enumerate((ux, uy, uz)):
            m = self.face_id[a] >= 0
            u[self.face_id[a][m]] = np.asarray(arr)[m]
        if p is None:
            return u
        pv = np.zeros(self.np_)
        pv[self.cell_id[self.pore]] = np.asarray(p)[self.pore]
        return u, pv

    def pressure_matrix(self):
        """-D G: the SPD pore-cell Laplacian the projection solves with (unit conductance on
        interior open faces, 2 on inlet / outlet faces)."""
        return -(self.D @ self.G)

    def pressure_solve(self, rhs):
        if self._lu is None:
            self._lu = spl.splu(self.pressure_matrix().tocsc())
        return self._lu.solve(rhs)

    def helmholtz_solve(self, dt, rhs):
        """(I - dt L) v = rhs, the implicit momentum-diffusion system (SPD)."""
        if getattr(self, "_hdt", None) != dt:
            self._hlu = spl.splu((sp.identity(self.nu) - dt * self.L).tocsc())
            self._hdt = dt
        return self._hlu.solve(rhs)


def flow_time_step(cfl=0.5, nu=1.0, h=1.0):
    """Eq. (time-step-flow) with C_V of Eq. (time-step-flow-viscous) and the advective and
    external-force terms absent (no momentum advection; the pressure enters through the
    projection only): dt = cfl / 2 * (2 C_V)^-1."""
    CV = 2.0 * nu * 3.0 / (h * h)
    CA = 0.0
    CF = 0.0
    return 0.5 * cfl / (CA + CV + math.sqrt((CA + CV) ** 2 + 4.0 * CF * CF))


def stokes_steady(solid, p_in=1.0, ops=None):
    """Steady discrete Stokes flow by a sparse direct solve of [L -G; D 0] [u; p] = [gbc; 0].
    Returns (ux, uy, uz, p) as float64 arrays (p = 0 in fibre cells)."""
    ops = ops or StokesOperators(solid, p_in)
    K = sp.bmat([[ops.L, -ops.G], [ops.D, None]]).tocsc()
    rhs = np.concatenate([ops.gbc, np.zeros(ops.np_)])
    x = spl.spsolve(K, rhs)
    return ops.unpack(x[:ops.nu], x[ops.nu:])


def chorin_step(ops, u, p, dt, implicit=False):
    """One step of the flow simulation on unknown vectors (u over open faces, p over pore
    cells): predictor (explicit or implicit momentum diffusion), exact pressure Poisson
    solve, projection.  Returns (u_next, p_next)."""
    if implicit:
        gp = ops.G @ p + ops.gbc
        u_star = ops.helmholtz_solve(dt, u - dt * gp) + dt * gp
    else:
        u_star = u + dt * (ops.L @ u)
    # D (u* - dt (G p + gbc)) = 0  <=>  (-D G) p = D gbc - D u* / dt
    p_next = ops.pressure_solve(ops.D @ ops.gbc - (ops.D @ u_star) / dt)
    u_next = u_star - dt * (ops.G @ p_next + ops.gbc)
    return u_next, p_next


def flow_sim(solid, p_in=1.0, cfl=0.5, eps=1e-9, max_steps=10**6, ops=None, implicit=False):
    """The flow simulation from rest to the stop rule ||u' - u|| < eps ||u'||.  Returns
    (ux, uy, uz, p, steps)."""
    ops = ops or StokesOperators(solid, p_in)
    dt = flow_time_step(cfl)
    u = np.zeros(ops.nu)
    p = np.zeros(ops.np_)
    for n in range(1, max_steps + 1):
        un, p = chorin_step(ops, u, p, dt, implicit)
        du = np.linalg.norm(un - u)
        u = un
        if du < eps * np.linalg.norm(u):
            break
    return (*ops.unpack(u, p), n)


def stokes_residual(solid, ux, uy, uz, p, p_in=1.0, ops=None):
    """Max-abs momentum residual (L u - G p over open faces) and continuity residual (D u over
    pore cells) of a given field; also the max-abs velocity on closed faces (must be 0)."""
    ops = ops or StokesOperators(solid, p_in)
    u, pv = ops.pack(ux, uy, uz, p)
    mom = ops.L @ u - (ops.G @ pv + ops.gbc)
    div = ops.D @ u
    closed = max(np.abs(np.asarray(arr)[~o]).max(initial=0.0)
                 for arr, o in zip((ux, uy, uz), ops.opens))
    return float(np.abs(mom).max()), float(np.abs(div).max()), float(closed)


def flow_rate(ux):
    """Volumetric flow rate Q through the inlet plane (h = 1)."""
    return float(np.asarray(ux)[:, :, 0].sum())
