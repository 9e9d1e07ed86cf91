"""Full-size parity of the HIP path against the FP64 oracle at the lattices whose
performance is reported: 20^3 x 64 (12 point sources), 24^3 x 64 and 32^3 x 64.

* M psi at 20^3 x 64 at EVERY site, for every W form (one right-hand side) and for
  the batched kernels (three of twelve right-hand sides), against route B evaluated
  slab by slab in worker processes (the same operator as the global route B).
* M psi at 24^3 x 64 and 32^3 x 64 (W byte offsets far past 2^32) at sampled sites,
  the first and last sites and the last time slice included.
* Solutions: the chosen solve at 20^3 x 64 (12 point sources, FP32 sigma-layout W,
  FP64 reliable updates) recomputed with the oracle's M, its error against the
  plain FP64 solution, the same solver on a pure-gauge field against the exact FFT
  solution, and network-preconditioned batched solves at 24^3 x 64 and 32^3 x 64
  recomputed with the oracle's M.

Tolerances as in test_gpu_operator (M psi: 1e-12 FP64, 1e-6 FP32, 1e-2 BF16 W,
norm-relative, and 1x / 3x that for the largest deviation relative to the largest
entry) and test_gpu_solver (residual <= 1.05e-10 with the oracle's M).
"""
import numpy as np
import pytest

from oracle.free import pure_gauge_point_solution
from oracle.local import apply_at_sites, apply_slabs
from paper_1311_5029_amd import inputs as I

from gpu_util import Lattice, lib, maxrel, rel

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

TOL = {0: 1e-12, 1: 1e-6, 2: 1e-2}
RES_TOL = 1.05e-10
SITE, SAVED, SIGMA, INNER = 0x10, 0x100, 0x200, 0x20
NPROC = 8


def _release(L, *precs):
    for p in precs:
        L.W.pop(p, None)
    L.torch.cuda.empty_cache()


def _solve(L, xi, low, w64, net=None, group_params=None):
    ok = L.ok
    torch = L.torch
    nrhs = xi.shape[0] if xi.ndim == 7 else 1
    d_xi = ok.to_device_complex(xi)
    psi = torch.zeros_like(d_xi)
    lo_prec = -1 if low is None else low
    work = ok.empty_bytes(ok.ok_bicgstab_workspace_bytes(L.dims, nrhs, lo_prec, net))
    W64 = L.precompute(ok.OK_F64 | w64)
    Wlo = None if low is None else L.precompute(low & ~INNER)
    p = group_params or ok.SolverParams(tol=1e-10)
    p.W64_layout = w64
    rc, st = ok.ok_bicgstab(L.dims, L.c, p, W64, Wlo, lo_prec, d_xi, psi, nrhs, work, net=net)
    torch.cuda.synchronize()
    x = ok.to_host_complex(psi, xi.shape)
    del work, psi, d_xi
    return rc, st, x


def _oracle_resid(U, c, xi, x):
    r = xi - apply_slabs(U, x, c, nproc=NPROC)
    ax = tuple(range(-6, 0))
    return np.sqrt(np.sum(np.abs(r) ** 2, axis=ax) / np.sum(np.abs(xi) ** 2, axis=ax))


def _small_net(name):
    """A 4-layer network trained on 16 pairs of the named ensemble's generator at 8^4 (the
    weights are colour blind, so they carry over to the full lattice with its own transports)."""
    from gpu_util import train_net
    ok = lib()
    dims = (8, 8, 8, 8)
    cfg = I.make_config(name, dims=dims, with_sources=False)
    L = Lattice(dims, cfg["U"], cfg["coeffs"])
    xi = I.gaussian_sources(dims, 16, I.SEED_TRAIN)
    rc, st, psi = _solve(L, xi, 2 | SITE, 0)
    assert rc == ok.OK_SUCCESS
    net, loss = train_net(L, xi, psi, steps=300)
    return net.params


def _full_net(L, params):
    ok = L.ok
    T = ok.empty_bytes(ok.ok_net_transports_bytes(L.dims))
    ok.ok_net_transports(L.dims, L.links, T)
    return ok.Net(4, params, T)


# --- 20^3 x 64, every site -------------------------------------------------------------------
@pytest.fixture(scope="module")
def c3():
    lib()
    cfg = I.make_config("batched_20x20x20x64", with_sources=False)
    L = Lattice(cfg["dims"], cfg["U"], cfg["coeffs"])
    L.psi1 = I.gaussian_sources(L.dims, 1, 131)[0]
    L.ref1 = apply_slabs(L.U, L.psi1, L.c, nproc=NPROC)
    L.psi12 = I.gaussian_sources(L.dims, 12, 133).astype(np.complex64)
    L.cols = [0, 5, 11]
    L.ref3 = apply_slabs(L.U, L.psi12[L.cols].astype(np.complex128), L.c, nproc=NPROC)
    return L


@pytest.mark.parametrize("prec", [0, 1, 2, SAVED, SAVED | 1, SAVED | 2, SIGMA, SIGMA | 1],
                         ids=["f64", "f32", "bf16", "f64-saved", "f32-saved", "bf16-saved", "f64-sigma",
                              "f32-sigma"])
def test_c3_every_site_one_rhs(c3, prec):
    got = c3.apply(prec, c3.psi1)
    _release(c3, prec)
    tol = TOL[prec & 3]
    assert rel(got, c3.ref1) <= tol
    assert maxrel(got, c3.ref1) <= tol * (1.0 if (prec & 3) == 0 else 3.0)


@pytest.mark.parametrize("prec,inner", [(1 | SITE, True), (2 | SITE, True), (1 | SITE, False), (1 | SIGMA, True)],
                         ids=["f32-site-inner", "bf16-site-inner", "f32-site", "f32-sigma-inner"])
def test_c3_every_site_batched(c3, prec, inner):
    """Twelve right-hand sides through one batched application; three of them checked at every site."""
    got = c3.apply(prec, c3.psi12, rhs_inner=inner)
    _release(c3, prec)
    tol = TOL[prec & 3]
    for n, k in enumerate(c3.cols):
        assert rel(got[k], c3.ref3[n]) <= tol
        assert maxrel(got[k], c3.ref3[n]) <= 3.0 * tol


# --- 20^3 x 64, the chosen solve and the FFT closed form ----------------------------------------
CHOSEN = 1 | SIGMA | INNER   # twelve together, FP32 sigma-layout W; FP64 sigma W for the reliable updates


def test_c3_chosen_solve_oracle_residual(c3):
    """The 12 point sources by the chosen form; three solutions recomputed with the oracle's M, and
    the first against the plain FP64 solve (27 dense FP64 blocks, one source)."""
    ok = lib()
    xi = I.point_sources(c3.dims)
    # the benchmark's chosen configuration: FP64 reliable updates when the FP32 residual has dropped
    # by delta = 0.003
    rc, st, x = _solve(c3, xi, CHOSEN, SIGMA, group_params=ok.SolverParams(tol=1e-10, delta=0.003))
    assert rc == ok.OK_SUCCESS
    res = _oracle_resid(c3.U, c3.c, xi[c3.cols], x[c3.cols])
    print("20^3x64 chosen: iterations %s, oracle residuals %s" % ([s["iterations"] for s in st], res))
    assert np.all(res <= RES_TOL)
    rc0, st0, x0 = _solve(c3, xi[0], None, 0)
    _release(c3, ok.OK_F64, ok.OK_F64 | SIGMA, 1 | SIGMA)
    assert rc0 == ok.OK_SUCCESS
    err = np.linalg.norm(x[0] - x0) / np.linalg.norm(x0)
    print("20^3x64 chosen vs plain FP64 solution, source 0: %.2e" % err)
    assert err < 1e-8


def test_c3_pure_gauge_chosen_solver_fft():
    """P12 at full size: a pure-gauge 20^3 x 64 field, the 12 point sources through the chosen
    batched solver, against the exact FFT solution (kappa(M) x 1e-10 bound)."""
    ok = lib()
    dims = (20, 20, 20, 64)
    U, g = I.pure_gauge_links(dims, 151)
    c = I.standin_coeffs(m0=0.5, u0=1.0)
    L = Lattice(dims, U, c)
    xi = I.point_sources(dims)
    rc, st, x = _solve(L, xi, CHOSEN, SIGMA, group_params=ok.SolverParams(tol=1e-10, delta=0.003))
    assert rc == ok.OK_SUCCESS
    exact = pure_gauge_point_solution(dims, c, g, xi[:, 0, 0, 0, 0])
    errs = [np.linalg.norm(x[k] - exact[k]) / np.linalg.norm(exact[k]) for k in range(12)]
    print("20^3x64 pure gauge, chosen solver vs FFT: max error %.2e" % max(errs))
    assert max(errs) < 1e-8


# --- 24^3 x 64 and 32^3 x 64: sampled sites, preconditioned solves --------------------------------
def _sites(dims, n, seed):
    rng = np.random.default_rng(seed)
    last = tuple(d - 1 for d in dims)
    near_end = (dims[0] - 2, dims[1] - 1, dims[2] - 3, dims[3] - 1)
    return [(0, 0, 0, 0), last, near_end] + [tuple(int(v) for v in rng.integers(0, dims)) for _ in range(n)]


def _sampled(L, prec, sites, nrhs=1, inner=False, seed=161):
    psi = I.gaussian_sources(L.dims, nrhs, seed)
    if nrhs == 1:
        psi = psi[0]
    if (prec & 3) != 0:
        psi = psi.astype(np.complex64)
    got = L.apply(prec, psi, rhs_inner=inner)
    _release(L, prec)
    tol = TOL[prec & 3]
    cols = [0] if nrhs == 1 else [0, nrhs - 1]
    for k in cols:
        pk = psi if nrhs == 1 else psi[k]
        gk = got if nrhs == 1 else got[k]
        ref = apply_at_sites(L.U, pk.astype(np.complex128), L.c, sites)
        gs = np.stack([gk[t, z, y, x] for (x, y, z, t) in sites])
        assert rel(gs, ref) <= tol, (prec, k)


@pytest.fixture(scope="module")
def c4():
    lib()
    cfg = I.make_config("learned_24x24x24x64", with_sources=False)
    return Lattice(cfg["dims"], cfg["U"], cfg["coeffs"])


@pytest.fixture(scope="module")
def c5():
    lib()
    cfg = I.make_config("learned_batched_32x32x32x64", with_sources=False)
    return Lattice(cfg["dims"], cfg["U"], cfg["coeffs"])


FORMS = [(0, 1, False), (1, 1, False), (1 | SITE, 12, True), (0 | SIGMA, 1, False), (1 | SIGMA, 12, True)]
FORM_IDS = ["f64", "f32", "f32-site-12", "f64-sigma", "f32-sigma-12"]


@pytest.mark.parametrize("prec,nrhs,inner", FORMS, ids=FORM_IDS)
def test_c4_sampled_sites(c4, prec, nrhs, inner):
    _sampled(c4, prec, _sites(c4.dims, 5, 171), nrhs, inner)


@pytest.mark.parametrize("prec,nrhs,inner", FORMS, ids=FORM_IDS)
def test_c5_sampled_sites(c5, prec, nrhs, inner):
    _sampled(c5, prec, _sites(c5.dims, 5, 181), nrhs, inner)


def test_c4_preconditioned_batched_solve_oracle_residual(c4):
    """Four Gaussian sources at 24^3 x 64 by the batched FP32 sigma solver right-preconditioned by
    the network; two solutions recomputed with the oracle's M."""
    ok = lib()
    net = _full_net(c4, _small_net("learned_24x24x24x64"))
    xi = I.gaussian_sources(c4.dims, 4, I.SEED_EVAL)
    rc, st, x = _solve(c4, xi, CHOSEN, SIGMA, net=net,
                       group_params=lib().SolverParams(tol=1e-10, delta=0.003))
    assert rc == ok.OK_SUCCESS
    assert all(s["fallbacks"] == 0 and s["net_applies"] > 0 for s in st)
    res = _oracle_resid(c4.U, c4.c, xi[:2], x[:2])
    print("24^3x64 preconditioned: iterations %s, oracle residuals %s" % ([s["iterations"] for s in st], res))
    assert np.all(res <= RES_TOL)


def test_c5_preconditioned_batched_point_sources_oracle_residual(c5):
    """The 12 point sources at 32^3 x 64: network + FP32 sigma W + FP64 reliable updates, batched;
    two solutions recomputed with the oracle's M."""
    ok = lib()
    net = _full_net(c5, _small_net("learned_batched_32x32x32x64"))
    xi = I.point_sources(c5.dims)
    rc, st, x = _solve(c5, xi, CHOSEN, SIGMA, net=net,
                       group_params=lib().SolverParams(tol=1e-10, delta=0.003))
    assert rc == ok.OK_SUCCESS
    assert all(s["fallbacks"] == 0 and s["net_applies"] > 0 for s in st)
    res = _oracle_resid(c5.U, c5.c, xi[[0, 7]], x[[0, 7]])
    print("32^3x64 preconditioned: iterations %s, oracle residuals %s" % ([s["iterations"] for s in st], res))
    assert np.all(res <= RES_TOL)
