"""Python binding of libsocfv (the C ABI in include/socfv.h): argument marshalling only.

Every step of the solve runs in the HIP library; torch provides device memory and the
stream.  Importing this module loads the library and raises if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsocfv.so")

OK, NOT_CONVERGED, INVALID_ARG, BAD_GEOMETRY, BAD_VELOCITY, DIVERGED, HIP_ERROR, OOM = \
    0, 1, -1, -2, -3, -4, -5, -6
FINITE_RATE, PINNED = 0, 1
FP64, FP32, FP32_PLAIN = 0, 1, 2

_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "INVALID_ARG", -2: "BAD_GEOMETRY",
          -3: "BAD_VELOCITY", -4: "DIVERGED", -5: "HIP_ERROR", -6: "OOM"}


class Params(C.Structure):
    _fields_ = [("s_in", C.c_double), ("s_eq", C.c_double), ("Da", C.c_double),
                ("mode", C.c_int), ("precision", C.c_int), ("cfl", C.c_double),
                ("tol", C.c_double), ("max_iter", C.c_long), ("check_every", C.c_int),
                ("polish_iters", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_long), ("it_fp32", C.c_long), ("it_fp64", C.c_long),
                ("cycles", C.c_int), ("status", C.c_int), ("residual", C.c_double),
                ("dt", C.c_double), ("tau", C.c_double), ("U", C.c_double),
                ("s_out", C.c_double), ("flux_in", C.c_double), ("flux_in_adv", C.c_double),
                ("flux_out", C.c_double), ("reaction", C.c_double), ("sum_R", C.c_double),
                ("q_out", C.c_double), ("seconds", C.c_double), ("ms_fp32", C.c_double),
                ("ms_fp64", C.c_double), ("ms_refresh", C.c_double),
                ("sweeps_fp64", C.c_long), ("tile_y", C.c_int), ("z_chunk", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FlowParams(C.Structure):
    _fields_ = [("p_in", C.c_double), ("cfl", C.c_double), ("tol", C.c_double),
                ("cg_theta", C.c_double), ("max_steps", C.c_long), ("check_every", C.c_int),
                ("cg_max", C.c_int), ("resume", C.c_int)]


class FlowStats(C.Structure):
    _fields_ = [("steps", C.c_long), ("cg_iterations", C.c_long), ("change", C.c_double),
                ("divergence", C.c_double), ("Q", C.c_double), ("Q_out", C.c_double),
                ("u_max", C.c_double), ("dt", C.c_double), ("seconds", C.c_double),
                ("status", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SocfvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2502_08034_amd.build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    P, i, l, d = C.c_void_p, C.c_int, C.c_long, C.c_double
    PP = C.POINTER(C.c_void_p)
    sig = {
        "socfv_default_params": (None, [C.POINTER(Params)]),
        "socfv_setup_geometry": (i, [PP, i, i, i, P, P]),
        "socfv_set_velocity": (i, [P, P, P, P, d, P]),
        "socfv_set_activity": (i, [P, P, P]),
        "socfv_solve_soc_steady": (i, [P, C.POINTER(Params), P, P, C.POINTER(Stats), P]),
        "socfv_compute_umt": (i, [P, C.POINTER(Params), C.POINTER(d), P, C.POINTER(Stats), P]),
        "socfv_evaluate": (i, [P, C.POINTER(Params), P, C.POINTER(Stats), P]),
        "socfv_evaluate_noalloc": (i, [P, C.POINTER(Params), P, C.POINTER(Stats), P]),
        "socfv_solve_soc_adjoint": (i, [P, C.POINTER(Params), P, C.POINTER(d), P,
                                        C.POINTER(Stats), P]),
        "socfv_batch_solve": (i, [i, PP, C.POINTER(Params), PP, C.POINTER(Stats), P]),
        "socfv_coarsen": (i, [P, P, P, P, P, P]),
        "socfv_solve_nernst": (i, [P, C.POINTER(Params), d, P, P, C.POINTER(Stats), P]),
        "socfv_solve_soc_upsampled": (i, [P, C.POINTER(Params), P, C.POINTER(Stats),
                                          C.POINTER(Stats), P]),
        "socfv_default_flow_params": (None, [C.POINTER(FlowParams)]),
        "socfv_solve_stokes": (i, [P, C.POINTER(FlowParams), P, P, P, P,
                                   C.POINTER(FlowStats), P]),
        "socfv_set_tiles": (i, [P, i, i, i, i]),
        "socfv_autotune": (i, [P, i, C.POINTER(C.c_int), P]),
        "socfv_info": (i, [P, C.POINTER(C.c_int), C.POINTER(C.c_long)]),
        "socfv_destroy": (None, [P]),
        "socfv_last_error": (C.c_char_p, []),
        "socfv_version": (i, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


_lib = _load()


def lib():
    return _lib


def _check(code):
    if code < 0:
        raise SocfvError(code, _lib.socfv_last_error().decode())
    return code


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype, shape=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def params(**kw) -> Params:
    """socfv_default_params, then overrides (mode / precision may be given as names)."""
    p = Params()
    _lib.socfv_default_params(C.byref(p))
    for k, v in kw.items():
        if k == "mode" and isinstance(v, str):
            v = {"finite": FINITE_RATE, "finite_rate": FINITE_RATE, "pinned": PINNED}[v.lower()]
        if k == "precision" and isinstance(v, str):
            v = {"fp64": FP64, "fp32": FP32, "fp32_plain": FP32_PLAIN}[v.lower()]
        if not hasattr(p, k):
            raise AttributeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


class Context:
    """Owns one socfv_ctx (geometry, velocity, activity, last state)."""

    def __init__(self, handle, shape):
        self._h = handle
        self.shape = shape          # (nz, ny, nx)

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("context destroyed")
        return self._h

    def destroy(self):
        if self._h:
            _lib.socfv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def info(self):
        dims = (C.c_int * 3)()
        cnt = (C.c_long * 3)()
        _check(_lib.socfv_info(self.handle, dims, cnt))
        return {"nx": dims[0], "ny": dims[1], "nz": dims[2], "pore": cnt[0], "reactive": cnt[1]}


def setup_geometry(solid: torch.Tensor) -> Context:
    """solid: CUDA uint8 (nz, ny, nx), nonzero = fibre voxel."""
    if solid.dim() != 3:
        raise ValueError("solid must be (nz, ny, nx)")
    nz, ny, nx = solid.shape
    h = C.c_void_p()
    _check(_lib.socfv_setup_geometry(C.byref(h), nx, ny, nz, _ptr(solid, torch.uint8, name="solid"),
                                     _stream()))
    return Context(h, (nz, ny, nx))


def set_velocity(ctx: Context, ux, uy, uz, q: float = 1.0):
    nz, ny, nx = ctx.shape
    _check(_lib.socfv_set_velocity(ctx.handle, _ptr(ux, torch.float64, (nz, ny, nx + 1), "ux"),
                                   _ptr(uy, torch.float64, (nz, ny + 1, nx), "uy"),
                                   _ptr(uz, torch.float64, (nz + 1, ny, nx), "uz"), float(q),
                                   _stream()))


def set_activity(ctx: Context, kappa=None):
    _check(_lib.socfv_set_activity(ctx.handle, _ptr(kappa, torch.float32, ctx.shape, "kappa"),
                                   _stream()))


def solve_soc_steady(ctx: Context, p: Params, s_init=None, want_state=True):
    """Returns (s, stats); s is a CUDA float64 (nz, ny, nx) tensor or None."""
    s = torch.empty(ctx.shape, dtype=torch.float64, device="cuda") if want_state else None
    st = Stats()
    code = _lib.socfv_solve_soc_steady(ctx.handle, C.byref(p),
                                       _ptr(s_init, torch.float64, ctx.shape, "s_init"),
                                       _ptr(s, torch.float64), C.byref(st), _stream())
    _check(code)
    return s, st


def compute_umt(ctx: Context, p: Params | None = None, want_state=False):
    """U_mt (mass-transport limit: s_in = 0, electrode cells held at 1)."""
    s = torch.empty(ctx.shape, dtype=torch.float64, device="cuda") if want_state else None
    st = Stats()
    u = C.c_double()
    _check(_lib.socfv_compute_umt(ctx.handle, C.byref(p) if p is not None else None, C.byref(u),
                                  _ptr(s, torch.float64), C.byref(st), _stream()))
    return u.value, s, st


def evaluate(ctx: Context, p: Params, s=None) -> Stats:
    st = Stats()
    _check(_lib.socfv_evaluate(ctx.handle, C.byref(p), _ptr(s, torch.float64, ctx.shape, "s"),
                               C.byref(st), _stream()))
    return st


def evaluate_noalloc(ctx: Context, p: Params, s=None) -> Stats:
    """socfv_evaluate through the allocation-free entry point (static device scratch)."""
    st = Stats()
    _check(_lib.socfv_evaluate_noalloc(ctx.handle, C.byref(p),
                                       _ptr(s, torch.float64, ctx.shape, "s"), C.byref(st),
                                       _stream()))
    return st


def solve_soc_adjoint(ctx: Context, p: Params, want_grad=True, want_psi=False):
    """Returns (dU_dkappa or None, dU_dlnq, psi or None, stats)."""
    g = torch.empty(ctx.shape, dtype=torch.float64, device="cuda") if want_grad else None
    psi = torch.empty(ctx.shape, dtype=torch.float64, device="cuda") if want_psi else None
    st = Stats()
    dq = C.c_double()
    _check(_lib.socfv_solve_soc_adjoint(ctx.handle, C.byref(p), _ptr(g, torch.float64),
                                        C.byref(dq), _ptr(psi, torch.float64), C.byref(st),
                                        _stream()))
    return g, dq.value, psi, st


def batch_solve(ctxs, ps, want_states=True):
    n = len(ctxs)
    hs = (C.c_void_p * n)(*[c.handle for c in ctxs])
    pa = (Params * n)(*ps)
    sts = (Stats * n)()
    states = [torch.empty(c.shape, dtype=torch.float64, device="cuda") if want_states else None
              for c in ctxs]
    outs = (C.c_void_p * n)(*[(s.data_ptr() if s is not None else None) for s in states])
    code = _lib.socfv_batch_solve(n, hs, pa, outs, sts, _stream())
    _check(code)
    return states, list(sts)


def solve_nernst(ctx: Context, p: Params, omega=0.05, want_state=True, want_eta=False):
    """Explicit Nernst model (FP64).  Returns (s or None, eta or None, stats)."""
    s = torch.empty(ctx.shape, dtype=torch.float64, device="cuda") if want_state else None
    eta = torch.empty(ctx.shape, dtype=torch.float64, device="cuda") if want_eta else None
    st = Stats()
    code = _lib.socfv_solve_nernst(ctx.handle, C.byref(p), float(omega), _ptr(s, torch.float64),
                                   _ptr(eta, torch.float64), C.byref(st), _stream())
    _check(code)
    return s, eta, st


def flow_params(**kw) -> FlowParams:
    """Flow-step parameters: library defaults overridden by keyword."""
    fp = FlowParams()
    _lib.socfv_default_flow_params(C.byref(fp))
    for k, v in kw.items():
        if not hasattr(fp, k):
            raise AttributeError(f"unknown flow parameter {k}")
        setattr(fp, k, v)
    return fp


def solve_stokes(ctx: Context, fp: FlowParams | None = None, want_pressure=False, start=None,
                 **kw):
    """Steady Stokes flow through the context's pore space (projection steps).  Returns
    (ux, uy, uz, p or None, stats); float64 CUDA tensors in the staggered layout.  ``start``
    = (ux, uy, uz, p) of an earlier call resumes from that state (updated in place and
    returned)."""
    fp = fp if fp is not None else flow_params(**kw)
    nz, ny, nx = ctx.shape
    dev = "cuda"
    if start is not None:
        ux, uy, uz, pr = start
        fp = FlowParams.from_buffer_copy(fp)        # leave the caller's parameters as given
        fp.resume = 1
        _ptr(ux, torch.float64, (nz, ny, nx + 1), "ux")
        _ptr(uy, torch.float64, (nz, ny + 1, nx), "uy")
        _ptr(uz, torch.float64, (nz + 1, ny, nx), "uz")
    else:
        ux = torch.empty((nz, ny, nx + 1), dtype=torch.float64, device=dev)
        uy = torch.empty((nz, ny + 1, nx), dtype=torch.float64, device=dev)
        uz = torch.empty((nz + 1, ny, nx), dtype=torch.float64, device=dev)
        pr = torch.empty((nz, ny, nx), dtype=torch.float64, device=dev) if want_pressure else None
    st = FlowStats()
    code = _lib.socfv_solve_stokes(ctx.handle, C.byref(fp), _ptr(ux, torch.float64),
                                   _ptr(uy, torch.float64), _ptr(uz, torch.float64),
                                   _ptr(pr, torch.float64), C.byref(st), _stream())
    _check(code)
    return ux, uy, uz, pr, st


def coarsen(ctx: Context):
    """The problem coarsened by two in every direction: (solid_c uint8, ux_c, uy_c, uz_c
    float64), CUDA tensors in the staggered layout of the coarse grid."""
    nz, ny, nx = ctx.shape
    nzc, nyc, nxc = nz // 2, ny // 2, nx // 2
    dev = "cuda"
    solid = torch.empty((nzc, nyc, nxc), dtype=torch.uint8, device=dev)
    ux = torch.empty((nzc, nyc, nxc + 1), dtype=torch.float64, device=dev)
    uy = torch.empty((nzc, nyc + 1, nxc), dtype=torch.float64, device=dev)
    uz = torch.empty((nzc + 1, nyc, nxc), dtype=torch.float64, device=dev)
    _check(_lib.socfv_coarsen(ctx.handle, _ptr(solid, torch.uint8), _ptr(ux, torch.float64),
                              _ptr(uy, torch.float64), _ptr(uz, torch.float64), _stream()))
    return solid, ux, uy, uz


def solve_soc_upsampled(ctx: Context, p: Params, want_state=True):
    """Iterative upsampling: coarse steady state, prolongated, as the fine solve's start.
    Returns (s, stats of the fine solve, stats of the coarse solve)."""
    s = torch.empty(ctx.shape, dtype=torch.float64, device="cuda") if want_state else None
    st, cst = Stats(), Stats()
    _check(_lib.socfv_solve_soc_upsampled(ctx.handle, C.byref(p), _ptr(s, torch.float64),
                                          C.byref(st), C.byref(cst), _stream()))
    return s, st, cst


def set_tiles(ctx: Context, tile_y=0, z_chunk=0, z_chunk2=0, two_sweeps=-1):
    _check(_lib.socfv_set_tiles(ctx.handle, int(tile_y), int(z_chunk), int(z_chunk2),
                                int(two_sweeps)))


def autotune(ctx: Context, sweeps=20):
    best = (C.c_int * 3)()
    _check(_lib.socfv_autotune(ctx.handle, int(sweeps), best, _stream()))
    return tuple(best)


@dataclass
class Problem:
    """Geometry + base velocity field u0 on the GPU, with the flow rate q and activity."""
    ctx: Context
    u0: tuple
    q: float = 1.0
    kappa: torch.Tensor | None = None

    @classmethod
    def create(cls, solid, ux, uy, uz, q=1.0, kappa=None):
        dev = torch.device("cuda")
        as_t = (lambda a, dt: a.to(dev, dt).contiguous() if isinstance(a, torch.Tensor)
                else torch.as_tensor(a, dtype=dt, device=dev).contiguous())
        ctx = setup_geometry(as_t(solid, torch.uint8))
        u0 = (as_t(ux, torch.float64), as_t(uy, torch.float64), as_t(uz, torch.float64))
        pb = cls(ctx, u0, float(q), None)
        set_velocity(ctx, *u0, q=pb.q)
        if kappa is not None:
            pb.set_activity(as_t(kappa, torch.float32))
        return pb

    def set_flow_rate(self, q: float):
        q = float(q)
        if q != self.q:
            set_velocity(self.ctx, *self.u0, q=q)
            self.q = q

    def set_activity(self, kappa):
        self.kappa = kappa
        set_activity(self.ctx, kappa)
