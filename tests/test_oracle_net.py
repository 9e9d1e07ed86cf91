"""Pins of the network oracle: finite differences of the loss, the adjoint
identity of a layer, gauge covariance, linearity and the transports' paths."""
import numpy as np
import pytest

from oracle import net
from oracle.lattice import cmul, dag, link, shift, shift_vec
from paper_1311_5029_amd import inputs as I

DIMS = (4, 5, 4, 6)


@pytest.fixture(scope="module")
def setup():
    U = I.random_su3_links(DIMS, 0.4, 81)
    P = net.all_transports(U)
    params = I.net_init_params(3, 0.3, 82, noise=0.05)
    return U, P, params


def test_transport_paths_match_definitions(setup):
    U, P, _ = setup
    # -mu is the dagger of the link from x - mu
    assert np.allclose(P[5], dag(shift(link(U, 0), 0, -1)))
    # -2y is (U_y(x-2y) U_y(x-y))^dag
    Uy = link(U, 1)
    assert np.allclose(P[13], dag(shift(Uy, 1, -2) @ shift(Uy, 1, -1)))
    # -x+y (k = 24) is the average of the two L-paths x -> x-x -> x-x+y and x -> x+y -> x-x+y
    Ux = link(U, 0)
    p1 = dag(shift(Ux, 0, -1)) @ shift(Uy, 0, -1)
    p2 = Uy @ dag(shift(shift(Ux, 0, -1), 1, 1))
    assert np.allclose(P[24], 0.5 * (p1 + p2))


def test_layer_adjoint_identity(setup):
    U, P, params = setup
    a, b = I.gaussian_sources(DIMS, 2, 83)
    A = params[1]
    lhs = np.vdot(b, net.layer(P, A, a))
    rhs = np.vdot(net.layer_adjoint(P, A, b), a)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def test_gauge_covariance(setup):
    U, P, params = setup
    g = I.random_su3_field(DIMS, 84)
    P2 = net.all_transports(I.gauge_transform_links(U, g))
    phi = I.gaussian_sources(DIMS, 1, 85)[0]
    lhs = net.forward(P2, params, cmul(g, phi))[-1]
    rhs = cmul(g, net.forward(P, params, phi)[-1])
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs) < 1e-13


def test_linear_in_input(setup):
    U, P, params = setup
    a, b = I.gaussian_sources(DIMS, 2, 86)
    z = 0.7 + 0.2j
    f = lambda x: net.forward(P, params, x)[-1]
    assert np.linalg.norm(f(a + z * b) - f(a) - z * f(b)) / np.linalg.norm(f(a)) < 1e-13


def test_gradient_finite_differences(setup):
    U, P, params = setup
    xi = I.gaussian_sources(DIMS, 2, 87)
    psi = I.gaussian_sources(DIMS, 2, 88)
    L0, G = net.loss_and_grad(P, params, xi, psi)
    rng = np.random.default_rng(89)
    for _ in range(4):
        E = rng.standard_normal(params.shape) + 1j * rng.standard_normal(params.shape)
        h = 1e-6
        Lp, _ = net.loss_and_grad(P, params + h * E, xi, psi)
        Lm, _ = net.loss_and_grad(P, params - h * E, xi, psi)
        fd = (Lp - Lm) / (2 * h)
        an = 2.0 * np.real(np.vdot(G, E))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_single_weight_gradient_closed_form(setup):
    """One layer with a single non-zero hop: r = A_4 T_4 xi - psi, and dL/dconj(A_k) = r (T_k xi)^dag / ||psi||^2 for every k."""
    U, P, _ = setup
    xi = I.gaussian_sources(DIMS, 1, 90)
    psi = I.gaussian_sources(DIMS, 1, 91)
    A = np.zeros((1, 27, 4, 4), complex)
    A[0, 4] = np.diag([1.0, 2.0, -1.0, 0.5j])
    L, G = net.loss_and_grad(P, A, xi, psi)
    h = net.hop(P, 4, xi[0])
    r = np.einsum("ab,...bc->...ac", A[0, 4], h) - psi[0]
    n2 = np.vdot(psi[0], psi[0]).real
    assert np.isclose(L, np.vdot(r, r).real / n2)
    for k in range(27):
        hk = net.hop(P, k, xi[0]).reshape(-1, 4, 3)
        want = np.einsum("nac,nbc->ab", r.reshape(-1, 4, 3), np.conj(hk)) / n2
        assert np.allclose(G[0, k], want, rtol=1e-12, atol=1e-15)


def test_adam_step_matches_definition():
    p = np.array([1.0 + 2.0j, -0.5 + 0.1j])
    g = np.array([0.2 - 0.4j, 0.0 + 1.0j])
    m = np.zeros(2, complex)
    v = np.zeros(2, complex)
    p2, m2, v2 = net.adam_step(p, g, m, v, 1, 0.01)
    # first step of Adam moves each real coordinate by lr * sign(gradient)
    assert np.allclose(p2, p - 0.01 * (np.sign(g.real) + 1j * np.sign(g.imag)), atol=1e-6)


def test_adam_steps_two_and_three_closed_forms():
    """Adam (Kingma & Ba) on gradient sequences whose moments have closed forms.

    Per real coordinate with real gradient G_t (twice the Wirtinger gradient):
      constant G:           every step moves by lr sign(G) (bias corrections exact);
      G, -G, G:             step 2 moves by -lr (1-b1)/(1+b1) sign(G),
                            step 3 by lr (1-b1+b1^2)/(1+b1+b1^2) sign(G)  (v^ = G^2 exactly);
      G, 3G:                step 2 moves by lr ((3+b1)/(1+b1)) / sqrt((9+b2)/(1+b2)) sign(G).
    Derived by hand from m_t = b1 m + (1-b1) G_t, v_t = b2 v + (1-b2) G_t^2 and the
    bias-corrected ratio, not by rerunning the recurrence."""
    b1, b2, lr = 0.9, 0.999, 0.01
    G = np.array([0.4, -0.7, 0.25, -1.3])
    seq = [np.array([1.0, -1.0, 1.0]), np.array([1.0, 1.0, 1.0]), np.array([1.0, 3.0, 3.0]),
           np.array([1.0, -1.0, 1.0])]
    # coordinates: re/im of two complex parameters
    g_at = lambda t: np.array([G[0] * seq[0][t] + 1j * G[1] * seq[1][t],
                               G[2] * seq[2][t] + 1j * G[3] * seq[3][t]]) / 2.0
    p = np.array([0.3 - 0.2j, -1.0 + 0.5j])
    m = np.zeros(2, complex)
    v = np.zeros(2, complex)
    moves = []
    for t in range(3):
        p2, m, v = net.adam_step(p, g_at(t), m, v, t + 1, lr, b1, b2, 1e-8)
        d = (p - p2) / lr               # update / lr, per real coordinate
        moves.append(np.array([d[0].real, d[0].imag, d[1].real, d[1].imag]))
        p = p2
    sg = np.sign(G)
    alt2 = -(1 - b1) / (1 + b1)
    alt3 = (1 - b1 + b1 ** 2) / (1 + b1 + b1 ** 2)
    grow2 = ((3 + b1) / (1 + b1)) / np.sqrt((9 + b2) / (1 + b2))
    tol = 1e-6
    for t in range(3):
        assert abs(moves[t][1] - sg[1]) < tol                      # constant
    assert abs(moves[1][0] - alt2 * sg[0]) < tol and abs(moves[2][0] - alt3 * sg[0]) < tol
    assert abs(moves[1][3] - alt2 * sg[3]) < tol and abs(moves[2][3] - alt3 * sg[3]) < tol
    assert abs(moves[1][2] - grow2 * sg[2]) < tol
