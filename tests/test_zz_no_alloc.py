"""The allocation-free entry point socfv_evaluate_noalloc against socfv_evaluate (needs an
MI355X).

Both run the same kernels on the same state, one with its reduction scratch in a static
device array, the other in the context's buffers, so the results agree bit for bit.  Two
problems in a row, the second smaller, so the second call reads nothing the first left in the
shared array; plus a state passed explicitly, and the size limit.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_2502_08034_amd import inputs as I

pytestmark = pytest.mark.gpu

FIELDS = ("U", "s_out", "flux_in", "flux_in_adv", "flux_out", "reaction", "sum_R", "q_out",
          "residual", "tau")


@pytest.fixture(scope="module")
def sv():
    from paper_2502_08034_amd import socfv
    assert torch.cuda.is_available()
    return socfv


def noalloc_abi(sv, ctx, p, s=None):
    """The entry point called through the C ABI directly."""
    st = sv.Stats()
    code = sv.lib().socfv_evaluate_noalloc(
        ctx.handle, ctypes.byref(p), None if s is None else ctypes.c_void_p(s.data_ptr()),
        ctypes.byref(st), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return code, st


def test_noalloc_matches_evaluate_twice_second_smaller(sv):
    cases = [(130, 45, 70, 3.0, 0.82, 51, 1.0, "finite"), (40, 18, 12, 2.5, 0.85, 52, 0.7, "pinned")]
    for nx, ny, nz, r, phi, seed, pe, mode in cases:
        g = I.fibres_nonoverlap(nx, ny, nz, r, phi, seed)
        u = I.darcy_velocity(g.solid, pe)
        pb = sv.Problem.create(g.solid, *u)
        kw = dict(s_in=1.0, s_eq=0.0, Da=0.45, mode=0) if mode == "finite" else \
            dict(s_in=0.0, s_eq=1.0, Da=0.0, mode=1)
        p = sv.params(precision="fp64", tol=1e-9, **kw)
        s, _ = sv.solve_soc_steady(pb.ctx, p)
        ref = sv.evaluate(pb.ctx, p)
        code, got = noalloc_abi(sv, pb.ctx, p)
        assert code == sv.OK, sv.lib().socfv_last_error()
        for k in FIELDS:
            assert getattr(got, k) == getattr(ref, k), (nx, k, getattr(got, k), getattr(ref, k))
        # an explicit state (not the context's): the steady state moved by an affine map (a
        # pure scaling would only scale R in the pinned case, where b = 0 with s_in = 0)
        s2 = (s * 0.97 + 0.01).contiguous()
        ref2 = sv.evaluate(pb.ctx, p, s2)
        got2 = sv.evaluate_noalloc(pb.ctx, p, s2)
        for k in FIELDS:
            assert getattr(got2, k) == getattr(ref2, k), (nx, k)
        assert got2.residual > 10 * got.residual


def test_noalloc_rejects_a_grid_beyond_its_scratch(sv):
    # 2 x 262144 x 16 cells of fibre-free channel (8.4M cells): 1 x 65,536 x 1 reduction
    # blocks, one more than the static array holds; the check precedes any launch
    nx, ny, nz = 2, 4 * 65536, 16
    solid = torch.zeros((nz, ny, nx), dtype=torch.uint8, device="cuda")
    ctx = sv.setup_geometry(solid)
    ux = torch.ones((nz, ny, nx + 1), dtype=torch.float64, device="cuda")
    uy = torch.zeros((nz, ny + 1, nx), dtype=torch.float64, device="cuda")
    uz = torch.zeros((nz + 1, ny, nx), dtype=torch.float64, device="cuda")
    sv.set_velocity(ctx, ux, uy, uz)
    s = torch.ones((nz, ny, nx), dtype=torch.float64, device="cuda")
    p = sv.params()
    code, _ = noalloc_abi(sv, ctx, p, s)
    assert code == sv.INVALID_ARG
    assert b"static scratch" in sv.lib().socfv_last_error()
    # the allocating entry point handles the same grid
    st = sv.evaluate(ctx, p, s)
    assert st.U == 0.0
    ctx.destroy()
