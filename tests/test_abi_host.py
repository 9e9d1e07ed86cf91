"""Host-side checks of the C-ABI library: it loads, exports every declared symbol,
and rejects bad arguments before any HIP call (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1311_5029_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "okinv.h")
LIB = os.path.join(ROOT, "paper_1311_5029_amd", "libokinv.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libokinv.so not built")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(ok_\w+)\s*\(", txt, flags=re.M)))


def test_every_declared_symbol_is_exported():
    from paper_1311_5029_amd import okinv
    lib = okinv._lib
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_1311_5029_amd import okinv
    assert sorted(okinv.EXPORTED) == declared_functions()


def test_abi_version():
    from paper_1311_5029_amd import okinv
    assert okinv.ok_abi_version() == 3


def test_saved_layout_size_and_flags():
    from paper_1311_5029_amd import okinv
    dims = (5, 6, 7, 3)
    for prec in (okinv.OK_F64, okinv.OK_F32, okinv.OK_BF16):
        full = okinv.ok_W_bytes(dims, prec)
        assert okinv.ok_W_bytes(dims, prec | okinv.OK_LAYOUT_SAVED) * 27 == full * 14
    with pytest.raises(okinv.OkError) as e:
        okinv.ok_W_bytes(dims, okinv.OK_F32 | okinv.OK_LAYOUT_SAVED | okinv.OK_LAYOUT_SITE)
    assert e.value.status == okinv.OK_EINVAL


def test_sigma_layout_size_and_flags():
    from paper_1311_5029_amd import okinv
    dims = (5, 6, 7, 3)
    for prec in (okinv.OK_F64, okinv.OK_F32):
        full = okinv.ok_W_bytes(dims, prec)
        assert okinv.ok_W_bytes(dims, prec | okinv.OK_LAYOUT_SIGMA) * 27 * 144 == full * 46 * 9
    for bad in (okinv.OK_BF16 | okinv.OK_LAYOUT_SIGMA, okinv.OK_F32 | okinv.OK_LAYOUT_SIGMA | okinv.OK_LAYOUT_SITE,
                okinv.OK_F64 | okinv.OK_LAYOUT_SIGMA | okinv.OK_LAYOUT_SAVED):
        with pytest.raises(okinv.OkError) as e:
            okinv.ok_W_bytes(dims, bad)
        assert e.value.status == okinv.OK_EINVAL


def test_size_queries():
    from paper_1311_5029_amd import okinv
    dims = (20, 20, 20, 64)
    V = 20 ** 3 * 64
    assert okinv.ok_W_bytes(dims, okinv.OK_F32) == 27 * 144 * 8 * V
    assert okinv.ok_W_bytes(dims, okinv.OK_F64) == 27 * 144 * 16 * V
    assert okinv.ok_W_bytes(dims, okinv.OK_BF16) == 27 * 144 * 4 * V
    # site stride padded to a multiple of 64
    assert okinv.ok_W_bytes((5, 5, 5, 5), okinv.OK_F32) == 27 * 144 * 8 * 640
    assert okinv.ok_precompute_scratch_bytes((4, 4, 4, 4)) == 6 * 9 * 16 * 256
    assert okinv.ok_bicgstab_workspace_bytes((4, 4, 4, 4), 1) >= 6 * 256 * 192
    assert okinv.ok_bicgstab_workspace_bytes((4, 4, 4, 4), 1, okinv.OK_F32) >= 7 * 256 * 96


@pytest.mark.parametrize("dims", [(2, 4, 4, 4), (4, 4, 4, 0), (4, 4, -1, 4), (5000, 4, 4, 4)])
def test_bad_geometry_rejected(dims):
    from paper_1311_5029_amd import okinv
    with pytest.raises(okinv.OkError) as e:
        okinv.ok_W_bytes(dims, okinv.OK_F32)
    assert e.value.status == okinv.OK_EINVAL
    assert "L[" in okinv.ok_last_error()


def test_bad_precision_rejected():
    from paper_1311_5029_amd import okinv
    with pytest.raises(okinv.OkError) as e:
        okinv.ok_W_bytes((4, 4, 4, 4), 7)
    assert e.value.status == okinv.OK_EINVAL


def test_apply_validation_before_device():
    from paper_1311_5029_amd import okinv
    c = I.standin_coeffs()
    g = okinv.geom((4, 4, 4, 4))
    cc = okinv.coeffs(c)
    lib = okinv._lib
    # null pointers
    rc = lib.ok_apply_M(ctypes.byref(g), ctypes.byref(cc), None, okinv.OK_F32, None, None, okinv.OK_F32, 1, None)
    assert rc == okinv.OK_EINVAL
    # misaligned pointers
    rc = lib.ok_apply_M(ctypes.byref(g), ctypes.byref(cc), 0x1001, okinv.OK_F32, 0x2000, 0x900000, okinv.OK_F32, 1, None)
    assert rc == okinv.OK_EALIGN
    # unsupported precision pair (FP64 W with FP32 spinors)
    rc = lib.ok_apply_M(ctypes.byref(g), ctypes.byref(cc), 0x1000, okinv.OK_F64, 0x2000, 0x900000, okinv.OK_F32, 1, None)
    assert rc == okinv.OK_EINVAL
    # aliasing in and out
    rc = lib.ok_apply_M(ctypes.byref(g), ctypes.byref(cc), 0x1000, okinv.OK_F32, 0x2000, 0x2100, okinv.OK_F32, 1, None)
    assert rc == okinv.OK_EINVAL and "overlap" in okinv.ok_last_error()
    # nrhs out of range
    rc = lib.ok_apply_M(ctypes.byref(g), ctypes.byref(cc), 0x1000, okinv.OK_F32, 0x2000, 0x900000, okinv.OK_F32, 0, None)
    assert rc == okinv.OK_EINVAL
    # non-finite coefficient
    cc.c_3 = float("nan")
    rc = lib.ok_apply_M(ctypes.byref(g), ctypes.byref(cc), 0x1000, okinv.OK_F32, 0x2000, 0x900000, okinv.OK_F32, 1, None)
    assert rc == okinv.OK_EINVAL


def test_precompute_validation_before_device():
    from paper_1311_5029_amd import okinv
    c = okinv.coeffs(I.standin_coeffs())
    g = okinv.geom((4, 4, 4, 4))
    lib = okinv._lib
    need = okinv.ok_W_bytes((4, 4, 4, 4), okinv.OK_F32)
    scr = okinv.ok_precompute_scratch_bytes((4, 4, 4, 4))
    # W too small
    rc = lib.ok_precompute_W(ctypes.byref(g), ctypes.byref(c), 0x10000000, okinv.OK_F32, 0x20000000, need - 16,
                             0x40000000, scr, None)
    assert rc == okinv.OK_ESIZE
    # scratch too small
    rc = lib.ok_precompute_W(ctypes.byref(g), ctypes.byref(c), 0x10000000, okinv.OK_F32, 0x20000000, need,
                             0x40000000, scr - 1, None)
    assert rc == okinv.OK_ESIZE
    # u0 <= 0
    c.u0 = 0.0
    rc = lib.ok_precompute_W(ctypes.byref(g), ctypes.byref(c), 0x10000000, okinv.OK_F32, 0x20000000, need,
                             0x40000000, scr, None)
    assert rc == okinv.OK_EINVAL


def test_solver_validation_before_device():
    from paper_1311_5029_amd import okinv
    dims = (4, 4, 4, 4)
    c = okinv.coeffs(I.standin_coeffs())
    g = okinv.geom(dims)
    lib = okinv._lib
    stats = (okinv.ok_solver_stats * 1)()
    need = okinv.ok_bicgstab_workspace_bytes(dims, 1)
    good = okinv.SolverParams().c()
    args = lambda p, work, wlo=None, wlo_prec=-1, net=None: (
        ctypes.byref(g), ctypes.byref(c), ctypes.byref(p), 0x10000000, wlo, wlo_prec, net, 0x20000000, 0x30000000, 1,
        0x40000000, work, stats, None)
    assert lib.ok_bicgstab(*args(good, need - 256)) == okinv.OK_ESIZE
    bad = okinv.SolverParams(tol=-1.0).c()
    assert lib.ok_bicgstab(*args(bad, need)) == okinv.OK_EINVAL
    bad = okinv.SolverParams(delta=1.5).c()
    assert lib.ok_bicgstab(*args(bad, need)) == okinv.OK_EINVAL
    # low-precision W given with an FP64 precision tag
    need2 = okinv.ok_bicgstab_workspace_bytes(dims, 1, okinv.OK_F32)
    assert lib.ok_bicgstab(*args(good, need2, 0x50000000, okinv.OK_F64)) == okinv.OK_EINVAL
    # a network needs the low-precision solve, a valid depth and room for its fields
    net = okinv.ok_net(4, 0, 0x60000000, 0x70000000)
    with pytest.raises(okinv.OkError):
        okinv.ok_bicgstab_workspace_bytes(dims, 1, -1, net)
    assert lib.ok_bicgstab(*args(good, need, None, -1, ctypes.byref(net))) == okinv.OK_EINVAL
    need3 = okinv.ok_bicgstab_workspace_bytes(dims, 1, okinv.OK_F32, net)
    assert need3 >= need2 + 4 * 256 * 96
    assert lib.ok_bicgstab(*args(good, need3 - 256, 0x50000000, okinv.OK_F32, ctypes.byref(net))) == okinv.OK_ESIZE
    bad_net = okinv.ok_net(0, 0, 0x60000000, 0x70000000)
    assert lib.ok_bicgstab(*args(good, need3, 0x50000000, okinv.OK_F32, ctypes.byref(bad_net))) == okinv.OK_EINVAL
    bad = okinv.SolverParams(stall_window=-1).c()
    assert lib.ok_bicgstab(*args(bad, need2, 0x50000000, okinv.OK_F32)) == okinv.OK_EINVAL
    # W64 layout: 0, saved or sigma only; low-precision sigma W only in FP32, one layout flag
    bad = okinv.SolverParams(W64_layout=okinv.OK_LAYOUT_SITE).c()
    assert lib.ok_bicgstab(*args(bad, need)) == okinv.OK_EINVAL
    for wlo in (okinv.OK_BF16 | okinv.OK_LAYOUT_SIGMA, okinv.OK_F32 | okinv.OK_LAYOUT_SIGMA | okinv.OK_LAYOUT_SITE):
        assert lib.ok_bicgstab(*args(good, need2, 0x50000000, wlo)) == okinv.OK_EINVAL
        with pytest.raises(okinv.OkError):
            okinv.ok_bicgstab_workspace_bytes(dims, 1, wlo)
    assert okinv.ok_bicgstab_workspace_bytes(dims, 1, okinv.OK_F32 | okinv.OK_LAYOUT_SIGMA) == need2
    # the batched solve: site-major W, or FP32 sigma W with right-hand-side-inner fields
    inner = okinv.OK_SPINOR_RHS_INNER
    assert (okinv.ok_bicgstab_workspace_bytes(dims, 4, okinv.OK_F32 | okinv.OK_LAYOUT_SIGMA | inner) ==
            okinv.ok_bicgstab_workspace_bytes(dims, 4, okinv.OK_F32 | okinv.OK_LAYOUT_SITE))
    for wlo in (okinv.OK_F32 | inner, okinv.OK_BF16 | okinv.OK_LAYOUT_SIGMA | inner,
                okinv.OK_F32 | okinv.OK_LAYOUT_SITE | inner):
        with pytest.raises(okinv.OkError):
            okinv.ok_bicgstab_workspace_bytes(dims, 4, wlo)


def test_cgnr_validation_before_device():
    from paper_1311_5029_amd import okinv
    dims = (4, 4, 4, 4)
    c = okinv.coeffs(I.standin_coeffs())
    g = okinv.geom(dims)
    lib = okinv._lib
    stats = (okinv.ok_solver_stats * 1)()
    need = okinv.ok_cgnr_workspace_bytes(dims, 1)
    assert need == okinv.ok_bicgstab_workspace_bytes(dims, 1)
    args = lambda p, work, nrhs=1: (ctypes.byref(g), ctypes.byref(c), ctypes.byref(p), 0x10000000, 0x20000000,
                                    0x30000000, nrhs, 0x40000000, work, stats, None)
    good = okinv.SolverParams().c()
    assert lib.ok_cgnr(*args(good, need - 256)) == okinv.OK_ESIZE
    assert lib.ok_cgnr(*args(okinv.SolverParams(tol=0.0).c(), need)) == okinv.OK_EINVAL
    assert lib.ok_cgnr(*args(okinv.SolverParams(W64_layout=okinv.OK_LAYOUT_SITE).c(), need)) == okinv.OK_EINVAL
    assert lib.ok_cgnr(*args(good, need, 0)) == okinv.OK_EINVAL
    with pytest.raises(okinv.OkError):
        okinv.ok_cgnr_workspace_bytes(dims, 0)


def test_net_sizes_and_validation_before_device():
    from paper_1311_5029_amd import okinv
    dims = (4, 5, 6, 7)
    V = 4 * 5 * 6 * 7
    Vs = (V + 63) // 64 * 64
    assert okinv.ok_net_param_count(4) == 4 * 27 * 16 * 2
    assert okinv.ok_net_transports_bytes(dims) == 13 * 9 * 8 * Vs
    fb = V * 12 * 8
    # apply: ping-pong fields for deep networks, none for one layer
    assert okinv.ok_net_workspace_bytes(dims, 1, 3, 0) == 256
    assert okinv.ok_net_workspace_bytes(dims, 4, 3, 0) >= 2 * 3 * fb
    # training keeps every layer's output
    assert okinv.ok_net_workspace_bytes(dims, 4, 3, 1) >= 4 * 3 * fb
    for bad in [(0, 1, 0), (17, 1, 0), (4, 0, 0), (4, 1, 3)]:
        with pytest.raises(okinv.OkError) as e:
            okinv.ok_net_workspace_bytes(dims, *bad)
        assert e.value.status == okinv.OK_EINVAL
    with pytest.raises(okinv.OkError):
        okinv.ok_net_param_count(0)
    g = okinv.geom(dims)
    lib = okinv._lib
    # transports buffer too small
    need = okinv.ok_net_transports_bytes(dims)
    assert lib.ok_net_transports(ctypes.byref(g), 0x10000000, 0x20000000, need - 8, None) == okinv.OK_ESIZE
    # layer: overlapping fields, unknown flag, misaligned pointer
    assert lib.ok_net_layer(ctypes.byref(g), 0x10000000, 0x20000000, 0x30000000, 0x30000000 + 64, 1, 0,
                            None) == okinv.OK_EINVAL
    assert lib.ok_net_layer(ctypes.byref(g), 0x10000000, 0x20000000, 0x30000000, 0x40000000, 1, 0x80,
                            None) == okinv.OK_EINVAL
    assert lib.ok_net_layer(ctypes.byref(g), 0x10000008, 0x20000000, 0x30000000, 0x40000000, 1, 0,
                            None) == okinv.OK_EALIGN
    # training step: workspace too small, missing loss pointer
    wt = okinv.ok_net_workspace_bytes(dims, 2, 2, 1)
    cfg = okinv.adam_cfg()
    base = [ctypes.byref(g), 2, 0x10000000, 0x11000000, 0x12000000, 0x13000000, 0x20000000, 0x30000000, 2, 0,
            ctypes.byref(cfg), 1, 0x14000000, 0x15000000, 0x40000000]
    assert lib.ok_net_train_step(*base, wt - 256, None) == okinv.OK_ESIZE
    nol = list(base)
    nol[12] = None
    assert lib.ok_net_train_step(*nol, wt, None) == okinv.OK_EINVAL
    # Adam settings
    badcfg = okinv.adam_cfg(beta1=1.0)
    assert lib.ok_adam_step(0x10000000, 0x11000000, 0x12000000, 0x13000000, 10, ctypes.byref(badcfg), 1,
                            None) == okinv.OK_EINVAL
    assert lib.ok_adam_step(0x10000000, 0x11000000, 0x12000000, 0x13000000, 10, ctypes.byref(cfg), 0,
                            None) == okinv.OK_EINVAL


def test_host_complex_roundtrip():
    torch = pytest.importorskip("torch")
    from paper_1311_5029_amd import okinv
    a = I.gaussian_sources((3, 3, 3, 3), 1, 1)[0]
    t = okinv.to_device_complex(a, device="cpu")
    assert t.dtype == torch.float64 and t.numel() == a.size * 2
    assert np.array_equal(okinv.to_host_complex(t, a.shape), a)


def test_static_solve_validation_before_device():
    from paper_1311_5029_amd import okinv
    assert okinv.ok_bicgstab_static_max_bytes() == 64 << 20
    c = okinv.coeffs(I.standin_coeffs())
    stats = (okinv.ok_solver_stats * 1)()
    good = okinv.SolverParams().c()
    bad = okinv.SolverParams(tol=-1.0).c()

    def call(dims, p):
        return okinv._lib.ok_bicgstab_static(ctypes.byref(okinv.geom(dims)), ctypes.byref(c), ctypes.byref(p),
                                             0x10000000, None, -1, None, 0x20000000, 0x30000000, 1, stats, None)
    big = (32, 32, 32, 8)
    assert okinv.ok_bicgstab_workspace_bytes(big, 1) > 64 << 20
    assert call(big, good) == okinv.OK_ESIZE and "static workspace" in okinv.ok_last_error()
    assert call((4, 4, 4, 4), bad) == okinv.OK_EINVAL
    assert call((2, 4, 4, 4), good) == okinv.OK_EINVAL


def test_binding_loads_one_hip_runtime():
    """Importing the binding before torch must not load a second HIP / HSA runtime next to
    torch's (two runtimes in one process leave the second without a device)."""
    import subprocess
    import sys
    code = ("import paper_1311_5029_amd.okinv, torch\n"
            "maps = open('/proc/self/maps').read().split('\\n')\n"
            "libs = sorted(set(l.split()[-1] for l in maps if 'libamdhip64' in l or 'libhsa-runtime64' in l))\n"
            "print(len([l for l in libs if 'amdhip64' in l]), len([l for l in libs if 'hsa-runtime' in l]))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.split()[-2:] == ["1", "1"], out.stdout
