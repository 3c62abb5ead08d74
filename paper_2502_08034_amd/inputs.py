"""Seeded synthetic inputs: fibrous voxel electrodes and their face velocities.

This module only *generates inputs*.  It holds none of the state-of-charge
arithmetic: no advection, diffusion, reaction, residual or utilisation.  The
solver under test and the FP64 CPU checker both consume what it returns.

Geometry (stands in for the paper's logpile / fibrous electrodes, Sec. "Incompressible
Flow Simulation for a Logpile Lattice"; cylinders from an implicit function as in the
embedded-boundary description of Sec. "Computational Methods"):

* ``fibres_nonoverlap``: cylinders of radius ``r`` whose axes run along y or z
  (uniform choice) through the whole box, axis centre continuous-uniform, added one
  at a time and rejected when they would share a voxel with an earlier fibre, until
  the porosity drops to the target.
* ``fibres_boolean``: overlapping cylinders whose axes lie in the y-z plane with a
  uniform random angle, through a uniform random point, until the porosity drops to
  the target (non-overlap is infeasible at that density).

A voxel is solid iff its centre lies strictly inside a cylinder.  Fibre axes keep
``r + 2`` voxels from the inlet and ``r + 3`` from the outlet plane, so those planes
stay fibre-free.  Pore cells not face-connected to the inlet plane are filled.

Velocity (stands in for the paper's Navier-Stokes field): a Darcy pressure Laplace
problem on the pore graph (Sec. "Incompressible Fluid Flow", Darcy's law), face
conductance 1 between pore cells, 2 to the inlet (p = 1) and outlet (p = 0) faces,
solved by Jacobi-preconditioned conjugate gradients to a relative residual of
``rtol``; face velocities ``u_f = G_f (p_P - p_nb)`` are then divergence-free up to
that residual and scaled so that the mean interstitial velocity times h / D equals
the requested cell Peclet number.

Layouts (x fastest): ``solid`` is ``uint8 (nz, ny, nx)``; staggered velocities are
``ux (nz, ny, nx+1)``, ``uy (nz, ny+1, nx)``, ``uz (nz+1, ny, nx)`` in units of D/h,
positive along +axis.  Zero on every face that touches a fibre voxel or a y/z wall.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Geometry", "fibres_nonoverlap", "fibres_boolean", "fill_disconnected",
    "darcy_velocity", "lognormal_activity", "plug_flow_case", "workload",
    "batch_workloads", "WORKLOADS", "logpile", "voltage_params",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Geometry:
    solid: np.ndarray                      # uint8 (nz, ny, nx), 1 = fibre voxel
    radius: float
    n_fibres: int
    porosity: float                        # after filling disconnected pockets
    filled: int = 0                        # pore cells filled as disconnected
    info: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.solid.shape


def _x_range(nx: int, r: float):
    lo, hi = r + 2.0, nx - r - 3.0
    if hi <= lo:
        raise ValueError(f"box too short (nx={nx}) for fibres of radius {r}")
    return lo, hi


def _cyl_window(nx, ny, nz, axis, x0, c0, r):
    """Voxels of a cylinder along y (c0 = z centre) or z (c0 = y centre), returned as a
    window of the box (index slices) and the boolean mask inside it."""
    n_c = nz if axis == "y" else ny
    xa, xb = max(0, int(math.floor(x0 - r - 0.5))), min(nx, int(math.ceil(x0 + r + 0.5)) + 1)
    ca, cb = max(0, int(math.floor(c0 - r - 0.5))), min(n_c, int(math.ceil(c0 + r + 0.5)) + 1)
    xs = np.arange(xa, xb) + 0.5
    cs = np.arange(ca, cb) + 0.5
    m2 = (xs[None, :] - x0) ** 2 + (cs[:, None] - c0) ** 2 < r * r     # (c, x)
    if axis == "y":
        return (slice(ca, cb), slice(None), slice(xa, xb)), m2[:, None, :]
    return (slice(None), slice(ca, cb), slice(xa, xb)), m2[None, :, :]


def fibres_nonoverlap(nx, ny, nz, radius, porosity, seed, max_tries=200000,
                      fill=True) -> Geometry:
    rng = _rng(seed)
    solid = np.zeros((nz, ny, nx), dtype=bool)
    n_cells = nx * ny * nz
    n_solid = 0
    lo, hi = _x_range(nx, radius)
    n_fib = tries = 0
    while (n_cells - n_solid) / n_cells > porosity:
        tries += 1
        if tries > max_tries:
            raise RuntimeError(f"porosity {porosity} unreachable without overlap "
                               f"({n_fib} fibres, phi={(n_cells - n_solid) / n_cells:.4f})")
        axis = "y" if rng.random() < 0.5 else "z"
        x0 = rng.uniform(lo, hi)
        c0 = rng.uniform(0.0, nz if axis == "y" else ny)
        win, m = _cyl_window(nx, ny, nz, axis, x0, c0, radius)
        sub = solid[win]
        m = np.broadcast_to(m, sub.shape)
        if np.any(sub & m):
            continue
        sub |= m
        n_solid += int(np.count_nonzero(m))
        n_fib += 1
    geo = Geometry(solid.astype(np.uint8), radius, n_fib, 0.0,
                   info={"kind": "nonoverlap", "seed": seed, "target_porosity": porosity})
    return fill_disconnected(geo) if fill else _finish(geo)


def fibres_boolean(nx, ny, nz, radius, porosity, seed, fill=True, device=None) -> Geometry:
    """Overlapping fibres with axes in the y-z plane at uniform random angles."""
    rng = _rng(seed)
    lo, hi = _x_range(nx, radius)
    solid_x = np.zeros((nx, nz, ny), dtype=bool)       # x-major while voxelising
    zz = (np.arange(nz) + 0.5)[:, None]
    yy = (np.arange(ny) + 0.5)[None, :]
    n_cells = nx * ny * nz
    n_solid = 0
    n_fib = 0
    r2 = radius * radius
    while (n_cells - n_solid) / n_cells > porosity:
        th = rng.uniform(0.0, math.pi)
        x0 = rng.uniform(lo, hi)
        y0 = rng.uniform(0.0, ny)
        z0 = rng.uniform(0.0, nz)
        # squared distance, in the y-z plane, from the voxel centre to the axis line
        dp = (yy - y0) * math.sin(th) - (zz - z0) * math.cos(th)
        dp2 = dp * dp                                            # (nz, ny)
        xa = max(0, int(math.floor(x0 - radius - 0.5)))
        xb = min(nx - 1, int(math.ceil(x0 + radius + 0.5)))
        added = 0
        for x in range(xa, xb + 1):
            dx = x + 0.5 - x0
            rem = r2 - dx * dx
            if rem <= 0.0:
                continue
            m = dp2 < rem
            sl = solid_x[x]
            added += int(np.count_nonzero(m & ~sl))
            sl |= m
        n_solid += added
        n_fib += 1
    solid = np.ascontiguousarray(solid_x.transpose(1, 2, 0))
    del solid_x
    geo = Geometry(solid.astype(np.uint8), radius, n_fib, 0.0,
                   info={"kind": "boolean", "seed": seed, "target_porosity": porosity})
    return fill_disconnected(geo) if fill else _finish(geo)


def _finish(geo: Geometry) -> Geometry:
    geo.porosity = float(1.0 - geo.solid.mean())
    return geo


def fill_disconnected(geo: Geometry) -> Geometry:
    """Fill pore cells that are not face-connected to a pore cell of the inlet plane."""
    from scipy import ndimage
    pore = geo.solid == 0
    lab, _ = ndimage.label(pore, structure=ndimage.generate_binary_structure(3, 1))
    keep = np.unique(lab[:, :, 0])
    keep = keep[keep > 0]
    ok = np.isin(lab, keep)
    filled = int(np.count_nonzero(pore & ~ok))
    if filled:
        geo.solid = np.where(ok, 0, 1).astype(np.uint8)
    geo.filled = filled
    return _finish(geo)


# ---------------------------------------------------------------------------------
# Darcy face velocities (batched Jacobi-PCG in torch; CPU or GPU)
# ---------------------------------------------------------------------------------

def darcy_velocity(solid, peclet, rtol=1e-12, device=None, max_iter=400000,
                   return_info=False, log=None, as_numpy=True):
    """Face velocities of the Darcy pressure-Laplace flow, scaled to cell Peclet ``peclet``.

    ``solid`` is one (nz, ny, nx) mask or a list of masks (boxes may differ; they are
    padded with solid voxels to a common box and solved as one batch, each problem with
    its own CG scalars and its own outlet plane).  Returns float64 arrays ``(ux, uy, uz)``
    (numpy, or contiguous torch tensors on ``device`` with ``as_numpy=False``), or a list of
    them for a list input.
    """
    import torch
    batched = isinstance(solid, (list, tuple))
    masks = list(solid) if batched else [solid]
    pes = list(peclet) if (batched and np.ndim(peclet)) else [peclet] * len(masks)
    dev = torch.device(device) if device is not None else torch.device("cpu")
    f64 = torch.float64
    B = len(masks)
    nz = max(m.shape[0] for m in masks)
    ny = max(m.shape[1] for m in masks)
    nx = max(m.shape[2] for m in masks)
    pore_np = np.zeros((B, nz, ny, nx), dtype=bool)
    gin_np = np.zeros((B, nz, ny), dtype=np.float64)
    gout_np = np.zeros((B, nz, ny, nx), dtype=np.float64)   # outlet conductance per cell
    for b, m in enumerate(masks):
        mz, my, mx = m.shape
        if not (m[:, :, 0] == 0).any() or not (m[:, :, mx - 1] == 0).any():
            raise ValueError(f"geometry {b}: no pore cell in the inlet or outlet plane (no flow)")
        pore_np[b, :mz, :my, :mx] = (m == 0)
        gin_np[b, :mz, :my] = 2.0 * (m[:, :, 0] == 0)
        gout_np[b, :mz, :my, mx - 1] = 2.0 * (m[:, :, mx - 1] == 0)
    pore = torch.from_numpy(pore_np).to(dev).to(f64)
    gin = torch.from_numpy(gin_np).to(dev)
    gout = torch.from_numpy(gout_np).to(dev)
    del pore_np, gout_np
    gx = pore[..., 1:] * pore[..., :-1]
    gy = pore[:, :, 1:, :] * pore[:, :, :-1, :]
    gz = pore[:, 1:] * pore[:, :-1]
    diag = gout.clone()
    diag[..., 1:] += gx
    diag[..., :-1] += gx
    diag[:, :, 1:, :] += gy
    diag[:, :, :-1, :] += gy
    diag[:, 1:] += gz
    diag[:, :-1] += gz
    diag[..., 0] += gin
    diag = torch.where(pore == 0, torch.ones_like(diag), diag)
    rhs = torch.zeros_like(pore)
    rhs[..., 0] = gin                                   # inlet pressure 1

    def lap(p):
        out = diag * p
        out[..., 1:].addcmul_(gx, p[..., :-1], value=-1.0)
        out[..., :-1].addcmul_(gx, p[..., 1:], value=-1.0)
        out[:, :, 1:, :].addcmul_(gy, p[:, :, :-1, :], value=-1.0)
        out[:, :, :-1, :].addcmul_(gy, p[:, :, 1:, :], value=-1.0)
        out[:, 1:].addcmul_(gz, p[:, :-1], value=-1.0)
        out[:, :-1].addcmul_(gz, p[:, 1:], value=-1.0)
        return out

    def bdot(a, c):
        return (a * c).reshape(B, -1).sum(dim=1).view(B, 1, 1, 1)

    inv_d = 1.0 / diag
    lens = torch.tensor([m.shape[2] for m in masks], dtype=f64, device=dev).view(B, 1, 1, 1)
    xs = torch.arange(nx, dtype=f64, device=dev).view(1, 1, 1, nx) + 0.5
    p = (torch.clamp(1.0 - xs / lens, min=0.0) * pore).contiguous()   # linear start
    r = rhs - lap(p)
    z = r * inv_d
    d = z.clone()
    rz = bdot(r, z)
    bnorm = torch.sqrt(bdot(rhs, rhs))
    it = 0
    check = 25
    active = torch.ones(B, 1, 1, 1, dtype=f64, device=dev)
    one = torch.ones_like(rz)
    while it < max_iter:
        Ad = lap(d)
        dAd = bdot(d, Ad)
        alpha = torch.where(dAd > 0, rz / torch.where(dAd > 0, dAd, one), 0.0 * one) * active
        p.addcmul_(alpha.expand_as(d), d)
        r.addcmul_(alpha.expand_as(Ad), Ad, value=-1.0)
        torch.mul(r, inv_d, out=z)
        rz_new = bdot(r, z)
        beta = torch.where(rz > 0, rz_new / torch.where(rz > 0, rz, one), 0.0 * one)
        d.mul_(beta).add_(z)
        rz = rz_new
        it += 1
        if it % check == 0:
            rel = (torch.sqrt(bdot(r, r)) / bnorm).view(B)
            done = rel < rtol
            active = (~done).to(f64).view(B, 1, 1, 1)
            if log is not None and it % (check * 80) == 0:
                log(f"darcy cg it={it} max rel residual={float(rel.max()):.3e}")
            if bool(done.all()):
                break
    rtrue = rhs - lap(p)
    rel_true = (torch.sqrt(bdot(rtrue, rtrue)) / bnorm).view(B).cpu().numpy()
    p = p * pore
    ux = torch.zeros(B, nz, ny, nx + 1, dtype=f64, device=dev)
    uy = torch.zeros(B, nz, ny + 1, nx, dtype=f64, device=dev)
    uz = torch.zeros(B, nz + 1, ny, nx, dtype=f64, device=dev)
    ux[..., 1:nx] = gx * (p[..., :-1] - p[..., 1:])
    ux[..., 1:] += gout * p                             # outlet faces (pressure 0 outside)
    ux[..., 0] = gin * (1.0 - p[..., 0])
    uy[:, :, 1:ny, :] = gy * (p[:, :, :-1, :] - p[:, :, 1:, :])
    uz[:, 1:nz] = gz * (p[:, :-1] - p[:, 1:])
    # scale to cell Peclet: mean interstitial velocity (q_sup / porosity) * h / D = Pe
    out = []
    for b, m in enumerate(masks):
        mz, my, mx = m.shape
        Q = float(ux[b, :mz, :my, 0].sum())
        phi = float((m == 0).mean())
        scale = pes[b] / ((Q / (my * mz)) / phi)
        trip = (ux[b, :mz, :my, :mx + 1].mul(scale).contiguous(),
                uy[b, :mz, :my + 1, :mx].mul(scale).contiguous(),
                uz[b, :mz + 1, :my, :mx].mul(scale).contiguous())
        out.append(tuple(t.cpu().numpy() for t in trip) if as_numpy else trip)
    info = {"cg_iterations": it, "rel_residual": [float(v) for v in rel_true]}
    res = out if batched else out[0]
    return (res, info) if return_info else res


def lognormal_activity(solid, sigma, seed):
    """Per-voxel reaction activity exp(sigma Z), Z ~ N(0,1), float32 (nz, ny, nx).

    Drawn for every voxel (so the field does not depend on which cells react);
    only pore cells that touch a fibre face use it.
    """
    rng = _rng(seed)
    z = rng.standard_normal(solid.shape)
    return np.exp(sigma * z).astype(np.float32)


def plug_flow_case(nx, ny, nz, u):
    """No fibres, uniform +x velocity ``u`` on every x face (y/z faces closed)."""
    solid = np.zeros((nz, ny, nx), dtype=np.uint8)
    ux = np.full((nz, ny, nx + 1), float(u))
    uy = np.zeros((nz, ny + 1, nx))
    uz = np.zeros((nz + 1, ny, nx))
    return solid, (ux, uy, uz)


# ---------------------------------------------------------------------------------
# Named workloads (sizes of the paper-derived benchmark configurations)
# ---------------------------------------------------------------------------------

def logpile(h_um=1.25) -> Geometry:
    """The logpile lattice of Sec. "Incompressible Flow Simulation for a Logpile Lattice":
    a 1280 x 640 x 160 um box with 43 rods of diameter 20 um in seven layers at z = 20, 40,
    ..., 140 um; odd layers run along x (four rods, 128 um apart in y), even layers along y
    (nine rods, 128 um apart in x).  Voxel size h_um (1.25 um: 1024 x 512 x 128); a voxel is
    fibre when its centre is strictly inside a rod.  Flow enters at x = 0."""
    nx, ny, nz = int(round(1280 / h_um)), int(round(640 / h_um)), int(round(160 / h_um))
    xc = (np.arange(nx) + 0.5) * h_um
    yc = (np.arange(ny) + 0.5) * h_um
    zc = (np.arange(nz) + 0.5) * h_um
    r = 10.0
    solid = np.zeros((nz, ny, nx), dtype=bool)
    n = 0
    for layer in range(7):
        z0 = 20.0 * (layer + 1)
        dz2 = (zc - z0) ** 2
        if layer % 2 == 0:                       # along x, spaced in y
            for yr in np.arange(1, 5) * 128.0:
                m = (dz2[:, None] + (yc[None, :] - yr) ** 2) < r * r
                solid |= m[:, :, None]
                n += 1
        else:                                    # along y, spaced in x
            for xr in np.arange(1, 10) * 128.0:
                m = (dz2[:, None] + (xc[None, :] - xr) ** 2) < r * r
                solid |= m[:, None, :]
                n += 1
    geo = Geometry(solid.astype(np.uint8), r / h_um, n, 0.0,
                   info={"kind": "logpile", "h_um": h_um})
    return fill_disconnected(geo)


def voltage_params(V, Da0=0.45):
    """Reaction parameters at dimensionless voltage V for the affine rate at alpha = 1/2:
    s_eq = sigma(V) (Eq. (seq-from-Var)) and Da = Da0 K(V) / K(0) with K = 2 cosh(V / 2), Da0
    the per-face Damkohler number at V = 0 (0.45: the paper's k0, D and h = 1.25 um)."""
    return {"s_eq": float(1.0 / (1.0 + np.exp(-V))), "Da": float(Da0 * np.cosh(V / 2.0))}


WORKLOADS = {
    # 64x32x32, r = 3, porosity 0.85, cell Peclet 0.5
    "fibre64": dict(shape=(64, 32, 32), radius=3.0, porosity=0.85, peclet=0.5, seed=1,
                    kind="nonoverlap"),
    # 256x128x128, r = 4, porosity 0.80, cell Peclet 1.0
    "fibre256": dict(shape=(256, 128, 128), radius=4.0, porosity=0.80, peclet=1.0, seed=2,
                     kind="nonoverlap"),
    # paper-scale slab 1024x512x256 at h = 1.25 um, r = 4, porosity 0.78, Pe 0.2 / 1 / 5
    "slab1024": dict(shape=(1024, 512, 256), radius=4.0, porosity=0.78,
                     peclet=(0.2, 1.0, 5.0), seed=3, kind="boolean"),
    # the paper's logpile lattice at h = 1.25 um (1024 x 512 x 128), Pe 0.2 / 1 / 5
    "logpile": dict(shape=(1024, 512, 128), radius=8.0, peclet=(0.2, 1.0, 5.0), seed=0,
                    kind="logpile"),
}


def workload(name, device=None, rtol=1e-12, log=None, with_velocity=True, scale=None):
    """Build a named workload; returns dict with solid, velocities (per Peclet), geometry.

    ``scale`` (optional) overrides the box size, keeping every other parameter.
    """
    cfg = dict(WORKLOADS[name])
    nx, ny, nz = scale if scale is not None else cfg["shape"]
    if cfg["kind"] == "logpile":
        geo = logpile(1.25 * cfg["shape"][0] / nx)
    elif cfg["kind"] == "nonoverlap":
        geo = fibres_nonoverlap(nx, ny, nz, cfg["radius"], cfg["porosity"], cfg["seed"])
    else:
        geo = fibres_boolean(nx, ny, nz, cfg["radius"], cfg["porosity"], cfg["seed"])
    out = {"name": name, "shape": (nx, ny, nz), "geometry": geo, "solid": geo.solid,
           "config": cfg}
    if with_velocity:
        pes = cfg["peclet"] if isinstance(cfg["peclet"], tuple) else (cfg["peclet"],)
        # the flow is linear in the driving pressure: solve once, scale per Peclet
        (u1, info) = darcy_velocity(geo.solid, 1.0, rtol=rtol, device=device,
                                    return_info=True, log=log)
        out["darcy"] = info
        out["velocity"] = {pe: tuple(a * pe for a in u1) for pe in pes}
    return out


def batch_workloads(n=48, seed0=100, device=None, rtol=1e-12, log=None, max_fibre_tries=200000):
    """Uneven batch of fibre boxes: Nx in [64,192], Ny = Nz in [64,96] (Nx >= Ny),
    porosity U(0.70, 0.90), radius U[3, 6], cell Peclet log-uniform in [0.1, 10]."""
    probs = []
    for k in range(n):
        rng = _rng(seed0 + k)
        ny = int(rng.integers(64, 97))
        nx = int(rng.integers(max(64, ny), 193))
        nz = ny
        phi = float(rng.uniform(0.70, 0.90))
        r = float(rng.uniform(3.0, 6.0))
        pe = float(math.exp(rng.uniform(math.log(0.1), math.log(10.0))))
        gseed = int(rng.integers(0, 2**31 - 1))
        try:
            geo = fibres_nonoverlap(nx, ny, nz, r, phi, gseed, max_tries=20000)
        except RuntimeError:
            geo = fibres_boolean(nx, ny, nz, r, phi, gseed)      # porosity unreachable
            geo.info["relaxed_to_overlap"] = True
        probs.append({"shape": (nx, ny, nz), "geometry": geo, "solid": geo.solid,
                      "peclet": pe, "seed": seed0 + k})
    vel = darcy_velocity([p["solid"] for p in probs], [p["peclet"] for p in probs],
                         rtol=rtol, device=device, log=log)
    for p, v in zip(probs, vel):
        p["velocity"] = v
    return probs
