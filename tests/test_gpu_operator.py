"""GPU parity of ok_precompute_W and ok_apply_M against the FP64 oracle.

Tolerances:
  * W, FP64 storage: max |dW| <= 1e-13 max |W| (FP64 arithmetic, different order);
  * W, FP32 storage: every entry the correctly rounded FP32 of the FP64 value,
    |dW| <= 2^-24 |W| (+1e-15 max|W| for the FP64 evaluation-order noise);
  * W, BF16 storage: |dW| <= 2^-8 |W| (round-to-nearest via FP32);
  * M psi: 1e-12 relative in FP64, 1e-6 in FP32 (FP32 W and psi, FP32
    accumulation of 324 products per component), and 1e-2 with BF16 W (relative
    rounding 2^-9 per W entry, random signs over 324 terms).
"""
import os

import numpy as np
import pytest

from oracle.local import apply_at_sites
from oracle.route_a import WForm
from oracle.route_b import OKOperatorB
from paper_1311_5029_amd import inputs as I

from gpu_util import Lattice, lib, maxrel, rel

pytestmark = pytest.mark.gpu

DIMS = [(4, 4, 4, 4), (5, 6, 7, 3), (6, 5, 4, 7), (8, 6, 10, 4)]
TOL_APPLY = {0: 1e-12, 1: 1e-6, 2: 1e-2}


def make(dims, eps=0.45, seed=11, u0=None):
    U = I.random_su3_links(dims, eps, seed)
    c = I.standin_coeffs(m0=0.5, u0=u0 if u0 is not None else I.tadpole_u0(U))
    return U, c


@pytest.fixture(scope="module", params=DIMS, ids=lambda d: "x".join(map(str, d)))
def lat(request):
    dims = request.param
    U, c = make(dims)
    L = Lattice(dims, U, c)
    L.oracle_W = WForm(U, c).W
    L.oracle_B = OKOperatorB(U, c)
    return L


def test_precompute_f64_blockwise(lat):
    ok = lib()
    got = lat.dense_W(ok.OK_F64)
    ref = lat.oracle_W
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_precompute_f32_correctly_rounded(lat):
    ok = lib()
    got = lat.dense_W(ok.OK_F32)
    ref = lat.oracle_W
    m = np.max(np.abs(ref))
    for part in (np.real, np.imag):
        d = np.abs(part(got) - part(ref))
        assert np.all(d <= 2.0 ** -24 * np.abs(part(ref)) + 1e-15 * m)


def test_precompute_bf16_rounding(lat):
    ok = lib()
    got = lat.dense_W(ok.OK_BF16)
    ref = lat.oracle_W
    m = np.max(np.abs(ref))
    for part in (np.real, np.imag):
        d = np.abs(part(got) - part(ref))
        assert np.all(d <= 2.0 ** -8 * np.abs(part(ref)) + 1e-15 * m)


def test_backward_blocks_exact_gamma5_partners(lat):
    """Backward blocks are bit-exact gamma5 conjugates of the stored forward blocks."""
    ok = lib()
    from oracle.basis import gamma5_conj
    from oracle.lattice import shift_vec
    from oracle.route_a import FWD_OF_BWD, offsets
    offs = offsets()
    for prec in (ok.OK_F64, ok.OK_F32, ok.OK_BF16):
        W = lat.dense_W(prec)
        for kb, kf in FWD_OF_BWD.items():
            src = shift_vec(W[..., kf, :, :], [-v for v in offs[kf]])
            assert np.array_equal(W[..., kb, :, :], gamma5_conj(src))


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "bf16"])
@pytest.mark.parametrize("tps", [1, 2, 4])
def test_apply_matches_oracle(lat, prec, tps, monkeypatch):
    monkeypatch.setenv("OKINV_TPS", str(tps))
    psi = I.gaussian_sources(lat.dims, 1, 21)[0]
    ref = lat.oracle_B.apply(psi)
    got = lat.apply(prec, psi)
    tol = TOL_APPLY[prec]
    assert rel(got, ref) <= tol
    assert maxrel(got, ref) <= tol * (1.0 if prec == 0 else 3.0)


@pytest.mark.parametrize("prec", [1, 2], ids=["f32", "bf16"])
@pytest.mark.parametrize("nrhs", [2, 12, 16, 20])
def test_apply_batched_mfma_matches_oracle(lat, prec, nrhs):
    """The multi-right-hand-side MFMA kernel (nrhs > 16 runs in groups of 16)."""
    psi = I.gaussian_sources(lat.dims, nrhs, 40 + nrhs)
    ref = lat.oracle_B.apply(psi)
    got = lat.apply(prec, psi)
    tol = TOL_APPLY[prec]
    for k in range(nrhs):
        assert rel(got[k], ref[k]) <= tol
        assert maxrel(got[k], ref[k]) <= 3.0 * tol


@pytest.mark.parametrize("prec", [1, 2], ids=["f32", "bf16"])
def test_apply_batched_equals_single(lat, prec, monkeypatch):
    psi = I.gaussian_sources(lat.dims, 12, 43)
    batched = lat.apply(prec, psi)
    monkeypatch.setenv("OKINV_MRHS", "0")
    single = lat.apply(prec, psi)
    # same W and spinors, different FP32 summation order (each within ~5e-7 of exact);
    # the BF16 kernel also splits the FP32 spinor into bf16 hi + lo (2^-18 per element)
    assert rel(batched, single) <= (1e-6 if prec == 1 else 3e-5)


SITE = 0x10   # OK_LAYOUT_SITE


@pytest.mark.parametrize("prec", [1, 2], ids=["f32", "bf16"])
def test_site_layout_holds_same_numbers(lat, prec):
    assert np.array_equal(lat.dense_W(prec | SITE), lat.dense_W(prec))


@pytest.mark.parametrize("prec", [1, 2], ids=["f32", "bf16"])
@pytest.mark.parametrize("nrhs", [1, 2, 12, 16, 20])
def test_apply_site_layout_matches_oracle(lat, prec, nrhs):
    psi = I.gaussian_sources(lat.dims, nrhs, 50 + nrhs)
    ref = lat.oracle_B.apply(psi)
    got = lat.apply(prec | SITE, psi if nrhs > 1 else psi[0])
    if nrhs == 1:
        got = got[None]
    tol = TOL_APPLY[prec]
    for k in range(nrhs):
        assert rel(got[k], ref[k]) <= tol
        assert maxrel(got[k], ref[k]) <= 3.0 * tol


@pytest.mark.parametrize("prec", [1, 2], ids=["f32", "bf16"])
@pytest.mark.parametrize("nrhs", [1, 5, 12, 16])
def test_apply_site_rhs_inner_matches_oracle(lat, prec, nrhs):
    """Site-major W with spinors [V][4][3][nrhs] (right-hand side fastest)."""
    psi = I.gaussian_sources(lat.dims, nrhs, 60 + nrhs)
    ref = lat.oracle_B.apply(psi)
    got = lat.apply(prec | SITE, psi, rhs_inner=True)
    tol = TOL_APPLY[prec]
    for k in range(nrhs):
        assert rel(got[k], ref[k]) <= tol
        assert maxrel(got[k], ref[k]) <= 3.0 * tol


def test_apply_multiple_rhs(lat):
    ok = lib()
    psi = I.gaussian_sources(lat.dims, 3, 22)
    got = lat.apply(ok.OK_F64, psi)
    for k in range(3):
        assert np.array_equal(got[k], lat.apply(ok.OK_F64, psi[k]))


def test_apply_mass_change_needs_no_precompute(lat):
    ok = lib()
    psi = I.gaussian_sources(lat.dims, 1, 23)[0]
    c2 = I.OKCoeffs(**{**lat.c.__dict__, "mhat": lat.c.mhat + 0.7})
    a = lat.apply(ok.OK_F64, psi)
    b = lat.apply(ok.OK_F64, psi, c=c2)
    assert rel(b - a, 0.7 * psi) < 1e-13


def test_apply_deterministic(lat):
    ok = lib()
    psi = I.gaussian_sources(lat.dims, 1, 24)[0]
    for prec in (ok.OK_F64, ok.OK_F32):
        assert np.array_equal(lat.apply(prec, psi), lat.apply(prec, psi))


SAVED = 0x100   # OK_LAYOUT_SAVED


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "bf16"])
def test_saved_layout_holds_same_numbers(lat, prec):
    """The 14-block layout expands to exactly the 27 blocks of the full layout (the backward
    ones are gamma5 conjugates of stored values, formed without rounding)."""
    assert np.array_equal(lat.dense_W(prec | SAVED), lat.dense_W(prec))


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "bf16"])
def test_apply_saved_layout_matches_oracle(lat, prec):
    psi = I.gaussian_sources(lat.dims, 2, 26)
    ref = lat.oracle_B.apply(psi)
    got = lat.apply(prec | SAVED, psi)
    tol = TOL_APPLY[prec]
    assert rel(got, ref) <= tol
    assert maxrel(got, ref) <= tol * (1.0 if prec == 0 else 3.0)
    # the same operator as the 27-block layout up to summation order
    assert rel(got, lat.apply(prec, psi)) <= (1e-14 if prec == 0 else 1e-6 if prec == 1 else 1e-5)


SIGMA = 0x200   # OK_LAYOUT_SIGMA


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_sigma_layout_expands_to_oracle_blocks(lat, prec):
    """The 46 Pauli-component colour matrices per site expand to the oracle's 27 dense blocks:
    FP64 to 1e-13 of max|W|; FP32 within a few roundings (an entry is a sum of at most four
    stored FP32 values, each within 2^-24 of its own magnitude)."""
    got = lat.dense_W(prec | SIGMA)
    ref = lat.oracle_W
    m = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= (1e-13 if prec == 0 else 2.0 ** -21) * m


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_apply_sigma_layout_matches_oracle(lat, prec):
    psi = I.gaussian_sources(lat.dims, 2, 28)
    ref = lat.oracle_B.apply(psi)
    got = lat.apply(prec | SIGMA, psi)
    tol = TOL_APPLY[prec]
    assert rel(got, ref) <= tol
    assert maxrel(got, ref) <= tol * (1.0 if prec == 0 else 3.0)
    assert rel(got, lat.apply(prec, psi)) <= (1e-14 if prec == 0 else 1e-6)


def test_apply_sigma_f64_columns(lat):
    """FP64 sigma W on five [V][12] fields (one pass of four with W read once, then one): each
    against the oracle (FP64 bar) and against the one-at-a-time kernel."""
    ok = lib()
    psi = I.gaussian_sources(lat.dims, 5, 45)
    got = lat.apply(ok.OK_F64 | SIGMA, psi)
    ref = lat.oracle_B.apply(psi)
    for k in range(5):
        assert rel(got[k], ref[k]) <= TOL_APPLY[0]
        assert rel(got[k], lat.apply(ok.OK_F64 | SIGMA, psi[k])) <= 1e-15


@pytest.mark.parametrize("nrhs", [1, 2, 5, 6, 12, 16])
def test_apply_sigma_rhs_inner_matches_single(lat, nrhs):
    """FP32 sigma W on nrhs right-hand-side-inner fields (the batched solver's operator): every
    right-hand side against the oracle (FP32 bar) and against the one-at-a-time sigma kernel,
    which runs the same arithmetic per right-hand side."""
    ok = lib()
    psi = I.gaussian_sources(lat.dims, nrhs, 40 + nrhs).astype(np.complex64)
    got = lat.apply(ok.OK_F32 | SIGMA, psi, rhs_inner=True)
    one = lat.apply(ok.OK_F32 | SIGMA, psi)
    assert rel(got, one) <= 1e-7
    ref = lat.oracle_B.apply(psi.astype(np.complex128))
    for k in range(nrhs):
        assert rel(got[k], ref[k]) <= TOL_APPLY[1]


@pytest.mark.parametrize("dims", [(3, 4, 3, 5), (4, 4, 3, 4), (3, 3, 3, 3)], ids=["3x4x3x5", "4x4x3x4", "3^4"])
def test_apply_sigma_small_lattices(dims):
    """L = 3 and 4: coinciding offsets and backward blocks read at the site itself or at a
    coinciding neighbour still add up to M (FP64 and FP32)."""
    ok = lib()
    U, c = make(dims, seed=9)
    L = Lattice(dims, U, c)
    psi = I.gaussian_sources(dims, 1, 29)[0]
    ref = OKOperatorB(U, c).apply(psi)
    assert rel(L.apply(ok.OK_F64 | SIGMA, psi), ref) < 1e-12
    assert rel(L.apply(ok.OK_F32 | SIGMA, psi.astype(np.complex64)), ref) < 1e-6


def test_free_field_plane_wave_sigma():
    """Unit links: the sigma-layout operator on a plane wave is the closed-form momentum-space
    symbol (FP64)."""
    ok = lib()
    from oracle.free import symbol_matrix
    dims = (5, 6, 4, 7)
    c = I.standin_coeffs(u0=0.91)
    L = Lattice(dims, I.unit_links(dims), c)
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    n = (1, 2, 3, 2)
    k = [2 * np.pi * n[m] / dims[m] for m in range(4)]
    ph = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z + k[3] * t))
    chi = np.arange(12).reshape(4, 3) * (1 - 0.5j) + 0.25
    got = L.apply(ok.OK_F64 | SIGMA, ph[..., None, None] * chi)
    want = ph[..., None, None] * (symbol_matrix(k, c) @ chi)
    assert rel(got, want) < 1e-13


@pytest.mark.parametrize("dims", [(3, 4, 3, 5), (4, 4, 3, 4)], ids=["3x4x3x5", "4x4x3x4"])
def test_apply_saved_small_lattices(dims):
    """L = 3 and 4: the forward block read for a backward offset may be the site's own or a
    coinciding neighbour's; the contributions still add up to M."""
    ok = lib()
    U, c = make(dims, seed=6)
    L = Lattice(dims, U, c)
    psi = I.gaussian_sources(dims, 1, 27)[0]
    assert rel(L.apply(ok.OK_F64 | SAVED, psi), OKOperatorB(U, c).apply(psi)) < 1e-12


def test_apply_l3_coinciding_offsets():
    """L = 3: x + 2i coincides with x - i, the contributions add."""
    ok = lib()
    dims = (3, 4, 3, 5)
    U, c = make(dims, seed=5)
    L = Lattice(dims, U, c)
    psi = I.gaussian_sources(dims, 1, 25)[0]
    assert rel(L.apply(ok.OK_F64, psi), OKOperatorB(U, c).apply(psi)) < 1e-12


def test_free_field_plane_wave_f64():
    ok = lib()
    from oracle.free import symbol_matrix
    dims = (6, 4, 5, 8)
    c = I.standin_coeffs(u0=0.93)
    L = Lattice(dims, I.unit_links(dims), c)
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    n = (2, 1, 3, 5)
    k = [2 * np.pi * n[m] / dims[m] for m in range(4)]
    ph = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z + k[3] * t))
    chi = np.arange(12).reshape(4, 3) + 1j
    got = L.apply(ok.OK_F64, ph[..., None, None] * chi)
    want = ph[..., None, None] * (symbol_matrix(k, c) @ chi)
    assert rel(got, want) < 1e-13


# --- full size: 20^3 x 64, plaquette ~ 0.6 ------------------------------------------
@pytest.fixture(scope="module")
def big():
    ok = lib()
    dims = (20, 20, 20, 64)
    cfg = I.make_config("batched_20x20x20x64")
    L = Lattice(dims, cfg["U"], cfg["coeffs"])
    L.precompute(ok.OK_F32)
    L.precompute(ok.OK_F64)
    return L


@pytest.mark.parametrize("prec", [0, 1, 2, 0x100, 0x101, 0x102, 0x200, 0x201],
                         ids=["f64", "f32", "bf16", "f64-saved", "f32-saved", "bf16-saved", "f64-sigma",
                              "f32-sigma"])
def test_full_size_sampled_sites(big, prec):
    """Sampled sites of M psi at 20^3 x 64 against the oracle evaluated site by site."""
    psi = I.gaussian_sources(big.dims, 1, 31)[0]
    got = big.apply(prec, psi)
    rng = np.random.default_rng(7)
    sites = [(0, 0, 0, 0), (19, 19, 19, 63)] + [tuple(int(v) for v in rng.integers(0, [20, 20, 20, 64]))
                                                for _ in range(6)]
    ref = apply_at_sites(big.U, psi, big.c, sites)
    gs = np.stack([got[t, z, y, x] for (x, y, z, t) in sites])
    assert rel(gs, ref) <= TOL_APPLY[prec & 3]


@pytest.mark.parametrize("prec,inner", [(1, False), (2, False), (1 | SITE, False), (2 | SITE, False),
                                        (1 | SITE, True), (2 | SITE, True), (1 | 0x200, True)],
                         ids=["f32", "bf16", "f32-site", "bf16-site", "f32-site-inner", "bf16-site-inner",
                              "f32-sigma-inner"])
def test_full_size_batched_sampled_sites(big, prec, inner):
    """12 right-hand sides through the MFMA kernels at 20^3 x 64, sampled sites vs the oracle."""
    psi = I.gaussian_sources(big.dims, 12, 33).astype(np.complex64)
    got = big.apply(prec, psi, rhs_inner=inner)
    big.W.pop(prec, None)
    rng = np.random.default_rng(8)
    sites = [(0, 0, 0, 0), (19, 19, 19, 63)] + [tuple(int(v) for v in rng.integers(0, [20, 20, 20, 64]))
                                                for _ in range(3)]
    for k in (0, 5, 11):
        ref = apply_at_sites(big.U, psi[k].astype(np.complex128), big.c, sites)
        gs = np.stack([got[k, t, z, y, x] for (x, y, z, t) in sites])
        assert rel(gs, ref) <= TOL_APPLY[prec & 3]


def test_full_size_gamma5_hermiticity(big):
    """<phi, g5 M g5 psi> = <M phi, psi> with the GPU operator at 20^3 x 64 (FP64)."""
    ok = lib()
    from oracle.basis import GAMMA5
    phi, psi = I.gaussian_sources(big.dims, 2, 32)
    g5 = lambda f: GAMMA5 @ f
    for prec in (ok.OK_F64, ok.OK_F64 | SIGMA):
        a = np.vdot(phi, g5(big.apply(prec, g5(psi))))
        b = np.vdot(big.apply(prec, phi), psi)
        assert abs(a - b) / abs(b) < 1e-12
