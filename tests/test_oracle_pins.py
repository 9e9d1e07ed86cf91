"""Pins of the FP64 oracle to facts other than itself.

Each test checks the oracle against something the paper or the mathematics fixes:
closed forms (free field, pure gauge), a textbook special case (Wilson-clover),
invariances (gauge covariance, translation, gamma5-hermiticity), the structure
the paper states (27 offsets, nearest-only time hops, zero colour blocks), two
independent derivations of M (operator composition vs. the printed W), the
paper's two printed forms of the sum (Eqs. minFlopForm and FinalForm), and
brute force (dense LU on 4^4).  A few tests plant a plausible mistake in a copy
of the oracle and check that a pin catches it.
"""
import numpy as np
import pytest

from paper_1311_5029_amd import inputs as I
from oracle import basis
from oracle.bicgstab import bicgstab
from oracle.clover import field_strength, magnetic_electric
from oracle.dense import dense_from_W
from oracle.free import (free_eigenvalues, free_point_solution, momenta,
                         pure_gauge_point_solution, symbol_matrix)
from oracle.lattice import cmul, dag, link, norm2, shift, shift_vec, smul, vdot
from oracle.route_a import FORWARD, FWD_OF_BWD, PAIRS, WForm, offsets
from oracle.route_b import OKOperatorB

D4 = (4, 4, 4, 4)
D6 = (6, 6, 6, 6)
DA = (4, 6, 5, 6)   # asymmetric, every direction distinct


def rel(a, b):
    return np.sqrt(norm2(a - b)) / np.sqrt(norm2(b))


@pytest.fixture(scope="module")
def rough():
    U = I.random_su3_links(DA, 0.45, 11)
    return U


def all_on(u0=1.0, m0=0.5, **kw):
    """Every coefficient non-zero (the stand-in set)."""
    return I.standin_coeffs(m0=m0, u0=u0, **kw)


# --- generators -------------------------------------------------------------
def test_links_are_su3():
    U = I.random_su3_links(D4, 0.3, 1001)
    eye = np.eye(3)
    assert np.max(np.abs(U @ dag(U) - eye)) < 1e-14
    assert np.max(np.abs(np.linalg.det(U) - 1.0)) < 1e-14


def test_epsilon_tuning_hits_plaquette():
    eps = I.tune_epsilon(0.6)
    p = I.plaquette(I.random_su3_links((8, 8, 8, 8), eps, 77))
    assert abs(p - 0.6) < 0.005


def test_gauge_field_haar_su3():
    g = I.random_su3_field(D4, 5)
    assert np.max(np.abs(g @ dag(g) - np.eye(3))) < 1e-13
    assert np.max(np.abs(np.linalg.det(g) - 1.0)) < 1e-13


# --- basis ------------------------------------------------------------------
def test_gamma_algebra():
    g = basis.GAMMA
    for m in range(4):
        for n in range(4):
            ac = g[m] @ g[n] + g[n] @ g[m]
            assert np.allclose(ac, 2.0 * (m == n) * np.eye(4))
        assert np.allclose(g[m], g[m].conj().T)
    g5 = basis.GAMMA5
    assert np.allclose(g5, basis.spin4(basis.Z2, -1j * basis.I2, 1j * basis.I2, basis.Z2))
    for m in range(4):
        assert np.allclose(g5 @ g[m], -g[m] @ g5)


def test_gamma5_conj_block_rule():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12))
    A, B, C, D = X[:6, :6], X[:6, 6:], X[6:, :6], X[6:, 6:]
    h = lambda m: m.conj().T
    expect = np.block([[h(D), -h(B)], [-h(C), h(A)]])
    assert np.allclose(basis.gamma5_conj(X), expect)


# --- clover -----------------------------------------------------------------
def _abelian_clover_error(field_strength_fn):
    """Max deviation of F from the closed form on a diagonal (commuting) gauge field.

    For diagonal links each leaf is exp(i * angle of its plaquette), so
    F_{mu nu}(x) = (i/4) sum over the 4 plaquettes around x of sin(angle), minus the trace.
    """
    rng = np.random.default_rng(3)
    shp = I.lattice_shape(DA)
    th = rng.uniform(-0.7, 0.7, shp + (4, 2))
    ang = np.concatenate([th, -th.sum(-1, keepdims=True)], -1)   # (.., 4, 3), sums to 0
    U = np.zeros(shp + (4, 3, 3), complex)
    for a in range(3):
        U[..., a, a] = np.exp(1j * ang[..., a])
    ax = {0: 3, 1: 2, 2: 1, 3: 0}
    roll = lambda f, mu, n: np.roll(f, -n, axis=ax[mu])
    err = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            A = ang[..., mu, :]
            B = ang[..., nu, :]
            plaq = A + roll(B, mu, 1) - roll(A, nu, 1) - B          # plaquette based at x
            s = (np.sin(plaq) + np.sin(roll(plaq, mu, -1)) + np.sin(roll(roll(plaq, mu, -1), nu, -1))
                 + np.sin(roll(plaq, nu, -1)))
            diag = 0.25j * s
            diag = diag - diag.mean(-1, keepdims=True)
            F = field_strength_fn(U, mu, nu)
            err = max(err, np.max(np.abs(F - np.einsum("...a,ab->...ab", diag, np.eye(3)))))
    return err


def test_clover_abelian_field_strength():
    assert _abelian_clover_error(field_strength) < 1e-14


def test_clover_antihermitian_traceless(rough):
    B, E = magnetic_electric(rough)
    for X in list(B) + list(E):
        assert np.max(np.abs(X + dag(X))) < 1e-14
        assert np.max(np.abs(np.trace(X, axis1=-2, axis2=-1))) < 1e-14


# --- P1 free field ------------------------------------------------------------
@pytest.mark.parametrize("u0", [1.0, 0.9])
def test_free_field_plane_waves(u0):
    dims = (6, 4, 5, 8)
    c = all_on(u0=u0)
    op = OKOperatorB(I.unit_links(dims), c)
    rng = np.random.default_rng(1)
    for n in [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 2, 0), (2, 1, 3, 5), (5, 3, 4, 7)]:
        k = [2 * np.pi * n[m] / dims[m] for m in range(4)]
        phase = np.exp(1j * sum(k[m] * idx for m, idx in enumerate(_coords(dims))))
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = phase[..., None, None] * chi
        got = op.apply(psi)
        want = phase[..., None, None] * (symbol_matrix(k, c) @ chi)
        assert rel(got, want) < 1e-13


def _coords(dims):
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return [x, y, z, t]


def test_free_field_zero_momentum_mass():
    """At u0 = 1 and p = 0 the symbol is the bare mass m0 (kappa reading)."""
    c = all_on(u0=1.0, m0=0.37)
    assert np.allclose(symbol_matrix([0, 0, 0, 0], c), 0.37 * np.eye(4))


def test_free_field_dense_spectrum():
    c = all_on(u0=0.93)
    W = WForm(I.unit_links(D4), c)
    M = dense_from_W(W.W, c.mhat, D4, offsets())
    ev = np.linalg.eigvals(M)
    ref = free_eigenvalues(D4, c)
    key = lambda e: np.lexsort((np.round(e.imag, 9), np.round(e.real, 9)))
    a, b = ev[key(ev)], ref[key(ref)]
    assert np.max(np.abs(a - b)) < 1e-12


# --- P2 textbook Wilson-clover ----------------------------------------------
def test_wilson_clover_special_case(rough):
    """zeta = r_s = c_B = c_E = 1, other c = 0, u0 = 1 is the Sheikholeslami-Wohlert operator
    (m0 + 4) - 1/2 sum_mu [(1 - g_mu) U_mu(x) d_{x+mu} + (1 + g_mu) U_mu(x-mu)^dag d_{x-mu}]
    + (i/4) sum_{mu nu} sigma_{mu nu} F_{mu nu}."""
    m0 = 0.13
    c = I.wilson_clover_coeffs(m0)
    U = rough
    psi = I.gaussian_sources(DA, 1, 9)[0]
    want = (m0 + 4.0) * psi
    one = np.eye(4)
    for mu in range(4):
        Uf = link(U, mu)
        Ub = dag(shift(Uf, mu, -1))
        want = want - 0.5 * smul(one - basis.GAMMA[mu], cmul(Uf, shift(psi, mu, 1)))
        want = want - 0.5 * smul(one + basis.GAMMA[mu], cmul(Ub, shift(psi, mu, -1)))
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            F = field_strength(U, min(mu, nu), max(mu, nu)) * (1 if mu < nu else -1)
            want = want + 0.25j * smul(basis.sigma_munu(mu, nu), cmul(F, psi))
    got = OKOperatorB(U, c, m0=m0).apply(psi)
    assert rel(got, want) < 1e-13
    got_a = WForm(U, c).apply(psi)
    assert rel(got_a, want) < 1e-13


# --- P3 route A == route B ----------------------------------------------------
@pytest.mark.parametrize("u0", [1.0, 0.8712])
def test_route_a_equals_route_b(rough, u0):
    c = all_on(u0=u0)
    psi = I.gaussian_sources(DA, 2, 21)
    a = WForm(rough, c).apply(psi)
    b = OKOperatorB(rough, c).apply(psi)
    assert rel(a, b) < 1e-13


@pytest.mark.parametrize("name", ["zeta", "r_s", "c_B", "c_E", "c_EE", "c_1", "c_2", "c_3", "c_4", "c_5"])
def test_route_a_equals_route_b_one_coefficient(rough, name):
    """P13 style: each coefficient alone (0.5, the others zero) at u0 != 1."""
    zero = dict(zeta=0.0, r_s=0.0, c_B=0.0, c_E=0.0, c_EE=0.0, c_1=0.0, c_2=0.0, c_3=0.0, c_4=0.0, c_5=0.0)
    zero[name] = 0.5
    if name in ("r_s", "c_B", "c_E"):
        zero["zeta"] = 1.0
    c = I.standin_coeffs(m0=0.5, u0=0.85, **zero)
    psi = I.gaussian_sources(DA, 1, 22)[0]
    a = WForm(rough, c).apply(psi)
    b = OKOperatorB(rough, c).apply(psi)
    assert rel(a, b) < 1e-13


def test_affine_in_coefficients(rough):
    """M is affine in each coefficient: M(c + t e) = M(c) + t (M(c + e) - M(c))."""
    psi = I.gaussian_sources(DA, 1, 23)[0]
    base = all_on(u0=0.9)
    for name in ["c_1", "c_2", "c_3", "c_EE", "c_4", "c_5"]:
        vals = [getattr(base, name) + t for t in (0.0, 0.5, 1.7)]
        outs = []
        for v in vals:
            c = all_on(u0=0.9, **{name: v})
            outs.append(OKOperatorB(rough, c).apply(psi))
        lin = outs[0] + (1.7 / 0.5) * (outs[1] - outs[0])
        assert rel(outs[2], lin) < 1e-12


def test_linear_in_psi(rough):
    c = all_on(u0=0.9)
    op = OKOperatorB(rough, c)
    a, b = I.gaussian_sources(DA, 2, 24)
    z = 0.3 - 1.1j
    assert rel(op.apply(a + z * b), op.apply(a) + z * op.apply(b)) < 1e-14


# --- P4 gauge covariance ------------------------------------------------------
@pytest.mark.parametrize("route", ["A", "B"])
def test_gauge_covariance(rough, route):
    c = all_on(u0=0.88)
    g = I.random_su3_field(DA, I.SEED_GAUGE)
    U2 = I.gauge_transform_links(rough, g)
    psi = I.gaussian_sources(DA, 1, 25)[0]
    mk = (lambda U: WForm(U, c)) if route == "A" else (lambda U: OKOperatorB(U, c))
    lhs = mk(U2).apply(cmul(g, psi))
    rhs = cmul(g, mk(rough).apply(psi))
    assert rel(lhs, rhs) < 1e-13


# --- P5 gamma5 hermiticity ----------------------------------------------------
def test_gamma5_hermiticity(rough):
    c = all_on(u0=0.88)
    op = OKOperatorB(rough, c)
    phi, psi = I.gaussian_sources(DA, 2, 26)
    g5 = lambda f: smul(basis.GAMMA5, f)
    lhs = vdot(phi, g5(op.apply(g5(psi))))
    rhs = vdot(op.apply(phi), psi)
    assert abs(lhs - rhs) / abs(rhs) < 1e-13


def test_gamma5_hermiticity_dense():
    U = I.random_su3_links(D4, 0.3, 1001)
    c = all_on(u0=I.tadpole_u0(U))
    M = dense_from_W(WForm(U, c).W, c.mhat, D4, offsets())
    G5 = np.kron(np.eye(256), np.kron(basis.GAMMA5, np.eye(3)))
    assert np.max(np.abs(G5 @ M @ G5 - M.conj().T)) < 1e-13


# --- P6 structure -------------------------------------------------------------
def test_offsets_table():
    offs = offsets()
    assert len(offs) == 27 and len(set(offs)) == 27
    assert all(abs(d[3]) <= 1 for d in offs)
    assert all(d[3] == 0 or sum(abs(v) for v in d[:3]) == 0 for d in offs)  # no t-diagonals
    assert (0, 0, 0, 2) not in offs and (0, 0, 0, -2) not in offs
    for kb, kf in FWD_OF_BWD.items():
        assert offs[kb] == tuple(-v for v in offs[kf])
    assert sorted(FORWARD + list(FWD_OF_BWD)) == list(range(27))
    assert 27 * 16 == 432


def test_stencil_support_route_b(rough):
    """A point source at y reaches exactly the sites y - d_k (6^4 lattice: no wrap coincidences)."""
    U = I.random_su3_links(D6, 0.4, 12)
    c = all_on(u0=0.9)
    op = OKOperatorB(U, c)
    y = (2, 3, 1, 4)
    psi = np.zeros(I.lattice_shape(D6) + (4, 3), complex)
    psi[y[3], y[2], y[1], y[0], 1, 2] = 1.0
    out = op.apply(psi)
    mag = np.abs(out).sum(axis=(-1, -2))
    expect = np.zeros_like(mag, dtype=bool)
    for d in offsets():
        x = [(y[m] - d[m]) % 6 for m in range(4)]
        expect[x[3], x[2], x[1], x[0]] = True
    assert np.all(mag[~expect] < 1e-15)
    assert np.all(mag[expect] > 1e-3)


def test_zero_colour_blocks(rough):
    W = WForm(rough, all_on(u0=0.9)).W
    blk = lambda k, r, cc: W[..., k, 6 * r:6 * r + 6, 6 * cc:6 * cc + 6]
    assert np.all(blk(4, 0, 0) == 0)          # W+_4 upper-left
    assert np.all(blk(8, 1, 1) == 0)          # W-_4 lower-right
    for k in list(range(15, 27)):             # W++_ij, W--_ij, W+-_ij: diagonal spin blocks
        assert np.all(blk(k, 0, 0) == 0) and np.all(blk(k, 1, 1) == 0)


def test_printed_opposite_relations(rough):
    """Eq. conjugate and Eq. opp_diag_pre_mat as printed, against the Gamma rule."""
    Wf = WForm(rough, all_on(u0=0.9))
    W = Wf.W
    offs = offsets()
    h = lambda m: dag(m)
    for p, (i, j) in enumerate(PAIRS):
        # W--_ij,x = -W++_ij,x-i-j ^dag
        src = shift_vec(W[..., 15 + p, :, :], [-v for v in offs[15 + p]])
        assert np.max(np.abs(W[..., 18 + p, :, :] + h(src))) < 1e-15
        # W+-_ji,x = -W+-_ij,x-i+j ^dag
        src = shift_vec(W[..., 21 + p, :, :], [-v for v in offs[21 + p]])
        assert np.max(np.abs(W[..., 24 + p, :, :] + h(src))) < 1e-15
    # W-_4 = [[-U4^dag(x-4), -S4^dag], [-S4^dag, 0]]
    W4 = shift(W[..., 4, :, :], 3, -1)
    S4 = W4[..., :6, 6:]
    U4 = -W4[..., 6:, 6:]
    assert np.max(np.abs(W[..., 8, :6, :6] + h(U4))) < 1e-15
    assert np.max(np.abs(W[..., 8, :6, 6:] + h(S4))) < 1e-15
    assert np.max(np.abs(W[..., 8, 6:, :6] + h(S4))) < 1e-15
    # W-_i = [[D^dag, -S^dag], [-S^dag, D^dag]] of W+_i at x - i
    for i in range(3):
        Wi = shift(W[..., 1 + i, :, :], i, -1)
        Dm, S = Wi[..., :6, :6], Wi[..., :6, 6:]
        assert np.max(np.abs(W[..., 5 + i, :6, :6] - h(Dm))) < 1e-15
        assert np.max(np.abs(W[..., 5 + i, :6, 6:] + h(S))) < 1e-15
        assert np.max(np.abs(W[..., 5 + i, 6:, 6:] - h(Dm))) < 1e-15


def test_diag_pm_two_routes(rough):
    """P7: W+-_ji at x from the i != j formula equals the Gamma of W+-_ij at x - i + j."""
    Wf = WForm(rough, all_on(u0=0.9))
    for p, (i, j) in enumerate(PAIRS):
        direct = Wf.diag_pm(j, i)
        assert np.max(np.abs(direct - Wf.W[..., 24 + p, :, :])) < 1e-14
        # W++ is symmetric in i, j
        assert np.max(np.abs(Wf.diag_pp(j, i) - Wf.W[..., 15 + p, :, :])) < 1e-14


def test_at_most_five_links_and_u0_powers(rough):
    """Scaling every link by a phase-free factor lam scales each W term by lam^(number of links);
    the printed W are polynomials of degree <= 5 in the links (Sec. 2.1)."""
    c = all_on(u0=0.9)
    lam = 1.1
    Wa = WForm(rough, c).W
    Wb = WForm(rough * lam, c).W
    # fit W(lam) = sum_n a_n lam^n using 7 scalings and check degree <= 5 (a_6 == 0)
    lams = np.array([0.7, 0.8, 0.9, 1.0, 1.1, 1.2, 1.3])
    samples = np.stack([WForm(rough * l, c).W[0, 0, 0, 0] for l in lams])
    V = np.vander(lams, 7, increasing=True)
    coef = np.linalg.solve(V, samples.reshape(7, -1))
    assert np.max(np.abs(coef[6])) < 1e-8 * np.max(np.abs(coef))
    assert Wa.shape == Wb.shape


# --- P8 minFlopForm == FinalForm -----------------------------------------------
def test_final_form_equals_min_flop_form(rough):
    Wf = WForm(rough, all_on(u0=0.9))
    psi = I.gaussian_sources(DA, 1, 27)[0]
    assert rel(Wf.apply_final_form(psi), Wf.apply(psi)) < 1e-14


# --- P10 translation ------------------------------------------------------------
def test_translation_invariance(rough):
    c = all_on(u0=0.9)
    psi = I.gaussian_sources(DA, 1, 28)[0]
    a = (1, 3, 2, 5)
    tU = np.stack([shift_vec(link(rough, mu), a) for mu in range(4)], axis=-3)
    lhs = OKOperatorB(tU, c).apply(shift_vec(psi, a))
    rhs = shift_vec(OKOperatorB(rough, c).apply(psi), a)
    assert rel(lhs, rhs) < 1e-14


# --- P11 dense brute force ----------------------------------------------------
def test_dense_lu_vs_bicgstab_c1():
    """The 4^4 workload: eps = 0.3, u0 from the plaquette, Gaussian source."""
    U = I.random_su3_links(D4, 0.3, I.SEED_LINKS + 1)
    c = all_on(u0=I.tadpole_u0(U))
    M = dense_from_W(WForm(U, c).W, c.mhat, D4, offsets())
    xi = I.gaussian_sources(D4, 1, I.SEED_SOURCES + 1)[0]
    x_lu = np.linalg.solve(M, xi.ravel())
    op = OKOperatorB(U, c)
    x, info = bicgstab(op.apply, xi, tol=1e-10)
    assert info["true_rel_resid"] <= 1e-10
    sv = np.linalg.svd(M, compute_uv=False)
    kappa = sv[0] / sv[-1]
    assert np.linalg.norm(x.ravel() - x_lu) / np.linalg.norm(x_lu) <= kappa * 1e-10
    # the route-B operator and the dense W assembly agree on the solution
    assert rel(op.apply(x_lu.reshape(xi.shape)), xi) < 1e-12


# --- P12 FFT exact solutions ------------------------------------------------------
def test_free_point_solution_fft():
    dims = (6, 4, 5, 8)
    c = all_on(u0=1.0)
    chi = I.point_sources(dims)[:, 0, 0, 0, 0]       # the 12 unit spin-colour vectors
    psi = free_point_solution(dims, c, chi)
    op = OKOperatorB(I.unit_links(dims), c)
    assert rel(op.apply(psi), I.point_sources(dims)) < 1e-13


def test_pure_gauge_point_solution_fft():
    dims = (6, 4, 5, 8)
    U, g = I.pure_gauge_links(dims, 31)
    c = all_on(u0=1.0)
    chi = I.point_sources(dims)[:, 0, 0, 0, 0]
    psi = pure_gauge_point_solution(dims, c, g, chi)
    op = OKOperatorB(U, c)
    assert rel(op.apply(psi), I.point_sources(dims)) < 1e-13
    # the plaquette of a pure-gauge field is 1
    assert abs(I.plaquette(U) - 1.0) < 1e-13


# --- planted mistakes: the pins above must catch them ----------------------------
def test_planted_wrong_gamma4_sign_is_caught(monkeypatch):
    import oracle.route_b as rb
    bad = rb.GAMMA.copy()
    bad[3] = -bad[3]
    monkeypatch.setattr(rb, "GAMMA", bad)
    dims = (4, 4, 4, 6)
    c = all_on(u0=1.0)
    op = rb.OKOperatorB(I.unit_links(dims), c)
    k = [0, 0, 0, 2 * np.pi / 6]
    t = _coords(dims)[3]
    chi = np.ones((4, 3), complex)
    psi = np.exp(1j * k[3] * t)[..., None, None] * chi
    want = np.exp(1j * k[3] * t)[..., None, None] * (symbol_matrix(k, c) @ chi)
    assert rel(op.apply(psi), want) > 1e-3


def test_planted_missing_gamma5_conjugation_is_caught(monkeypatch, rough):
    import oracle.route_a as ra
    good = WForm(rough, all_on(u0=0.9))
    monkeypatch.setattr(ra, "gamma5_conj", lambda X: X)
    W = ra.WForm(rough, all_on(u0=0.9))
    psi = I.gaussian_sources(DA, 1, 29)[0]
    b = OKOperatorB(rough, all_on(u0=0.9)).apply(psi)
    assert rel(W.apply(psi), b) > 1e-3 and rel(good.apply(psi), b) < 1e-13


def test_planted_clockwise_leaf_is_caught(monkeypatch):
    import oracle.clover as cl
    good_leaves = cl.clover_leaves

    def bad_leaves(U, mu, nu):
        Umu, Unu = link(U, mu), link(U, nu)
        first = Umu @ shift(Unu, mu, 1) @ dag(shift(Umu, nu, 1)) @ dag(Unu)
        return good_leaves(U, mu, nu) - first + dag(first)     # first leaf run clockwise
    monkeypatch.setattr(cl, "clover_leaves", bad_leaves)
    assert _abelian_clover_error(cl.field_strength) > 1e-3


# --- local evaluation used for sampled parity at full lattice size ----------------
def test_local_window_evaluation_matches_global():
    from oracle.local import apply_at_sites
    dims = (10, 9, 11, 6)
    U = I.random_su3_links(dims, 0.45, 41)
    c = all_on(u0=0.88)
    psi = I.gaussian_sources(dims, 1, 42)[0]
    full = OKOperatorB(U, c).apply(psi)
    sites = [(0, 0, 0, 0), (9, 8, 10, 5), (4, 2, 7, 3), (1, 8, 0, 5)]
    loc = apply_at_sites(U, psi, c, sites)
    for n, (x, y, z, t) in enumerate(sites):
        assert np.max(np.abs(loc[n] - full[t, z, y, x])) < 1e-13 * np.max(np.abs(full))


# --- P9 cubic rotations and spatial parity ---------------------------------------
# A lattice symmetry maps site x to R x and acts on spin by S with
# S gamma_nu S^-1 = sum_mu R_{mu nu} gamma_mu (the textbook spinor representation of
# a rotation or reflection of the lattice).  The transformed fields are
# psi'(x) = S psi(R^-1 x) and U'_mu(x) = the link of the original lattice from
# R^-1 x to R^-1 x + R^-1 mu-hat (a daggered backward link when R^-1 mu-hat = -nu-hat).
# An action invariant under the symmetry satisfies M[U'] psi' = (M[U] psi)'.
# Unlike gauge covariance, gamma5-hermiticity or translations, this fixes which
# Pauli matrix goes with which direction in every term (the sigma_i of S_i, the
# sigma_j of the c_5 staple term, sigma_i +- sigma_j on the diagonals) and the
# relative sign of forward and backward paths.

def _r_inverse(kind, a=None, b=None):
    """Coordinates of R^-1 x and the 4x4 matrix R for a 90-degree rotation
    R e_a = e_b, R e_b = -e_a (kind 'rot'), or spatial parity (kind 'par')."""
    R = np.eye(4)
    if kind == "rot":
        R[:, a] = 0.0
        R[:, b] = 0.0
        R[b, a] = 1.0
        R[a, b] = -1.0
    else:
        R[:3, :3] = -np.eye(3)
    Rinv = np.round(np.linalg.inv(R)).astype(int)
    return R, Rinv


def _spin_matrix(kind, a=None, b=None):
    g = basis.GAMMA
    if kind == "rot":
        return (np.eye(4) - g[a] @ g[b]) / np.sqrt(2.0)
    return g[3].copy()


def _transform(dims, kind, a=None, b=None):
    """Returns (links map U -> U', spinor map psi -> psi') of the symmetry."""
    R, Rinv = _r_inverse(kind, a, b)
    xs = _coords(dims)                                   # [x, y, z, t] over (Lt, Lz, Ly, Lx)
    src = [sum(Rinv[m, n] * xs[n] for n in range(4)) for m in range(4)]

    def gather(f, shift_vec=(0, 0, 0, 0)):
        idx = [np.mod(src[m] + shift_vec[m], dims[m]) for m in range(4)]
        return f[idx[3], idx[2], idx[1], idx[0]]

    S = _spin_matrix(kind, a, b)

    def links(U):
        out = np.empty_like(U)
        for mu in range(4):
            d = Rinv[:, mu]                              # R^-1 mu-hat = +-nu-hat
            nu = int(np.flatnonzero(d)[0])
            if d[nu] > 0:
                out[..., mu, :, :] = gather(U[..., nu, :, :])
            else:
                back = [0, 0, 0, 0]
                back[nu] = -1
                out[..., mu, :, :] = dag(gather(U[..., nu, :, :], back))
        return out

    def spinor(psi):
        return smul(S, gather(psi))
    return links, spinor, R, S


SYMMETRIES = [("rot", 0, 1), ("rot", 0, 2), ("rot", 1, 2), ("par", None, None)]
DC = (5, 5, 5, 4)    # Lx = Ly = Lz for the rotations


@pytest.fixture(scope="module")
def rough_cubic():
    return I.random_su3_links(DC, 0.45, 13)


def c5_alone(u0):
    zero = dict(zeta=0.0, r_s=0.0, c_B=0.0, c_E=0.0, c_EE=0.0, c_1=0.0, c_2=0.0, c_3=0.0, c_4=0.0, c_5=0.5)
    return I.standin_coeffs(m0=0.5, u0=u0, **zero)


@pytest.mark.parametrize("kind,a,b", SYMMETRIES)
def test_symmetry_spin_matrix_is_textbook(kind, a, b):
    """S gamma_nu S^-1 = sum_mu R_{mu nu} gamma_mu, S unitary."""
    _, _, R, S = _transform(DC, kind, a, b)
    Si = np.linalg.inv(S)
    assert np.allclose(S @ S.conj().T, np.eye(4), atol=1e-15)
    for nu in range(4):
        want = sum(R[mu, nu] * basis.GAMMA[mu] for mu in range(4))
        assert np.allclose(S @ basis.GAMMA[nu] @ Si, want, atol=1e-15)


def _symmetry_error(mk, U, c, kind, a, b, psi):
    links, spinor, _, _ = _transform(DC, kind, a, b)
    lhs = mk(links(U), c).apply(spinor(psi))
    rhs = spinor(mk(U, c).apply(psi))
    return rel(lhs, rhs)


@pytest.mark.parametrize("kind,a,b", SYMMETRIES)
@pytest.mark.parametrize("route", ["A", "B"])
@pytest.mark.parametrize("coeffs", ["all", "c5"])
def test_cubic_rotation_and_parity(rough_cubic, kind, a, b, route, coeffs):
    """P9 at u0 != 1, where the c_5 staple term T_eps is switched on."""
    u0 = 0.8712
    c = all_on(u0=u0) if coeffs == "all" else c5_alone(u0)
    mk = WForm if route == "A" else OKOperatorB
    psi = I.gaussian_sources(DC, 1, 30)[0]
    assert _symmetry_error(mk, rough_cubic, c, kind, a, b, psi) < 1e-13


def test_plaquette_and_clover_transform(rough_cubic):
    """The transformed links are a relabelling: same plaquette, and B_i, E_i map as
    an axial and a polar vector under parity."""
    links, _, _, _ = _transform(DC, "par")
    U2 = links(rough_cubic)
    assert abs(I.plaquette(U2) - I.plaquette(rough_cubic)) < 1e-14
    B, E = magnetic_electric(rough_cubic)
    B2, E2 = magnetic_electric(U2)
    R, Rinv = _r_inverse("par")
    xs = _coords(DC)
    src = [np.mod(sum(Rinv[m, n] * xs[n] for n in range(4)), DC[m]) for m in range(4)]
    g = lambda f: f[src[3], src[2], src[1], src[0]]
    for i in range(3):
        assert np.max(np.abs(B2[i] - g(B[i]))) < 1e-14       # axial: unchanged
        assert np.max(np.abs(E2[i] + g(E[i]))) < 1e-14       # polar: flips


# planted slips in the c_5 staple term, made in BOTH routes at once, so the
# route A == route B pin cannot see them
def _staple_variant(U, i, variant):
    """Variants of the c_5 staple sum of D+_i as (sigma index, colour field) pairs."""
    from oracle.route_a import _eps
    out = []
    for j in range(3):
        for k in range(3):
            e = _eps(i, j, k)
            if e == 0:
                continue
            Ui, Uk = link(U, i), link(U, k)
            up = Uk @ shift(Ui, k, 1) @ dag(shift(Uk, i, 1))
            dn = dag(shift(Uk, k, -1)) @ shift(Ui, k, -1) @ shift(shift(Uk, k, -1), i, 1)
            if variant == "sigma_k":
                out.append((k, e * (up - dn)))
            elif variant == "plus":
                out.append((j, e * (up + dn)))
    return out


def _planted_ops(variant):
    import oracle.route_a as ra
    import oracle.route_b as rb

    class BadA(ra.WForm):
        def _eps_staple(self, i):
            return sum(ra.kron2(basis.SIGMA[s], X) for s, X in _staple_variant(self.U, i, variant))

    class BadB(rb.OKOperatorB):
        def _eps_block(self, i):
            c = self.c
            pref = 1j * 0.25 * c.c_5 * (c.u0 ** -2 - c.u0 ** -4)
            X = [0.0, 0.0, 0.0]
            for s, C in _staple_variant(self.U, i, variant):
                X[s] = X[s] + pref * C
            return X
    return BadA, BadB


@pytest.mark.parametrize("variant", ["sigma_k", "plus"])
def test_planted_staple_slip_is_caught_by_symmetry(rough_cubic, variant):
    """A slip shared by both routes passes route A == route B, gauge covariance and
    gamma5-hermiticity, and is caught by the rotation/parity pin."""
    BadA, BadB = _planted_ops(variant)
    c = all_on(u0=0.8712)
    U = rough_cubic
    psi, phi = I.gaussian_sources(DC, 2, 31)
    assert rel(BadA(U, c).apply(psi), BadB(U, c).apply(psi)) < 1e-13          # P3 blind
    assert rel(BadB(U, c).apply(psi), OKOperatorB(U, c).apply(psi)) > 1e-5     # it is a real change
    g = I.random_su3_field(DC, I.SEED_GAUGE)
    U2 = I.gauge_transform_links(U, g)
    assert rel(BadB(U2, c).apply(cmul(g, psi)), cmul(g, BadB(U, c).apply(psi))) < 1e-13   # P4 blind
    g5 = lambda f: smul(basis.GAMMA5, f)
    bad = BadB(U, c)
    lhs, rhs = vdot(phi, g5(bad.apply(g5(psi)))), vdot(bad.apply(phi), psi)
    assert abs(lhs - rhs) / abs(rhs) < 1e-13                                   # P5 blind
    worst = {}
    for mk, name in [(BadA, "A"), (BadB, "B")]:
        worst[name] = max(_symmetry_error(mk, U, c, kind, a, b, psi) for kind, a, b in SYMMETRIES)
    assert worst["A"] > 1e-5 and worst["B"] > 1e-5, worst


def test_slab_evaluation_matches_global():
    """M psi evaluated as time slabs in worker processes equals the global operator (the slab
    windows reach every link and spinor a site's result depends on), for one field and a batch."""
    from oracle.local import apply_slabs
    dims = (5, 4, 6, 11)
    U = I.random_su3_links(dims, 0.45, 43)
    c = all_on(u0=0.87)
    psi = I.gaussian_sources(dims, 2, 44)
    op = OKOperatorB(U, c)
    assert np.array_equal(apply_slabs(U, psi[0], c, nproc=4), op.apply(psi[0]))
    assert np.array_equal(apply_slabs(U, psi, c, nproc=3), op.apply(psi))
