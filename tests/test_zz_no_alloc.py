"""ok_bicgstab_static (the solve on the library's fixed per-GPU workspace, no device
allocation) against ok_bicgstab with a caller's workspace on the same inputs: two calls
in a row, the second on a smaller lattice, each bit-identical to the workspace form
(same kernels, same fixed-order reductions) and within the oracle's residual bound.

The first call is the batched FP32 sigma-layout solve (4 Gaussian sources, FP64 reliable
updates with the sigma FP64 W) at 8^3 x 12; the second the plain FP64 solve of one
source at 4^4.  The workspace form runs with its workspace filled with NaN, the static
form after the previous call left its data in the fixed array, so neither result depends
on what the workspace held before.
"""
import numpy as np
import pytest

from oracle.route_b import OKOperatorB
from paper_1311_5029_amd import inputs as I

from gpu_util import Lattice, lib

pytestmark = pytest.mark.gpu

SIGMA, INNER = 0x200, 0x20


def _case(dims, nrhs, seed):
    U = I.random_su3_links(dims, 0.3, seed)
    c = I.standin_coeffs(m0=0.5, u0=I.tadpole_u0(U))
    xi = I.gaussian_sources(dims, nrhs, seed + 1)
    return U, c, xi


def _both(L, xi, low, w64_layout):
    ok = L.ok
    torch = L.torch
    nrhs = xi.shape[0]
    d_xi = ok.to_device_complex(xi)
    W64 = L.precompute(ok.OK_F64 | w64_layout)
    Wlo = None if low is None else L.precompute(low & ~INNER)
    lo_prec = -1 if low is None else low
    p = ok.SolverParams(tol=1e-10, W64_layout=w64_layout)
    need = ok.ok_bicgstab_workspace_bytes(L.dims, nrhs, lo_prec)
    assert need <= ok.ok_bicgstab_static_max_bytes()

    psi_s = torch.zeros_like(d_xi)
    rc_s, st_s = ok.ok_bicgstab_static(L.dims, L.c, p, W64, Wlo, lo_prec, d_xi, psi_s, nrhs)
    torch.cuda.synchronize()

    work = torch.full((need // 8 + 1,), float("nan"), dtype=torch.float64, device="cuda")
    psi_w = torch.zeros_like(d_xi)
    rc_w, st_w = ok.ok_bicgstab(L.dims, L.c, p, W64, Wlo, lo_prec, d_xi, psi_w, nrhs, work)
    torch.cuda.synchronize()
    return (rc_s, st_s, ok.to_host_complex(psi_s, xi.shape)), (rc_w, st_w, ok.to_host_complex(psi_w, xi.shape))


def _check(U, c, xi, static, withwork):
    ok = lib()
    (rc_s, st_s, x_s), (rc_w, st_w, x_w) = static, withwork
    assert rc_s == ok.OK_SUCCESS and rc_w == ok.OK_SUCCESS
    assert np.array_equal(x_s, x_w)
    for a, b in zip(st_s, st_w):
        for key in ("status", "iterations", "matvec_hi", "matvec_lo", "reliable_updates", "restarts"):
            assert a[key] == b[key], key
        assert a["true_rel_resid"] == b["true_rel_resid"]
    op = OKOperatorB(U, c)
    for k in range(xi.shape[0]):
        r = np.linalg.norm(xi[k] - op.apply(x_s[k])) / np.linalg.norm(xi[k])
        assert r <= 1.05e-10, (k, r)


def test_static_workspace_solve_twice_then_smaller():
    ok = lib()
    dims1 = (8, 8, 8, 12)
    U1, c1, xi1 = _case(dims1, 4, 811)
    L1 = Lattice(dims1, U1, c1)
    first = _both(L1, xi1, ok.OK_F32 | SIGMA | INNER, SIGMA)
    _check(U1, c1, xi1, *first)
    del L1

    dims2 = (4, 4, 4, 4)
    U2, c2, xi2 = _case(dims2, 1, 813)
    L2 = Lattice(dims2, U2, c2)
    second = _both(L2, xi2, None, 0)
    _check(U2, c2, xi2, *second)


def test_static_workspace_rejects_oversized_solve():
    ok = lib()
    dims = (32, 32, 32, 8)
    assert ok.ok_bicgstab_workspace_bytes(dims, 1) > ok.ok_bicgstab_static_max_bytes()
    stats = (ok.ok_solver_stats * 1)()
    import ctypes
    p = ok.SolverParams().c()
    rc = ok._lib.ok_bicgstab_static(ctypes.byref(ok.geom(dims)), ctypes.byref(ok.coeffs(I.standin_coeffs())),
                                    ctypes.byref(p), 0x10000000, None, -1, None, 0x20000000, 0x30000000, 1, stats,
                                    None)
    assert rc == ok.OK_ESIZE and "static workspace" in ok.ok_last_error()
