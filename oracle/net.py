"""The learned preconditioner: a gauge-covariant linear stencil network (FP64 oracle).

A layer maps one spinor field to another over the same 27 hops as the operator
(0, +-mu, +-2i, +-i+-j):

    phi'_x = sum_k A_k (P_k(x) phi_{x + d_k}),

with A_k a 4x4 complex matrix acting on spin only (colour blind) and P_k(x) the
colour transport along the hop: the identity for d = 0, the link for +-mu, the
two-link product for +-2i, and the average of the two L-shaped paths for the
diagonal hops, with P_{-d}(x) = P_d(x - d)^dag.  Every P_k(x) transforms as
g(x) P_k(x) g(x + d)^dag, so the network is gauge covariant and linear in phi.
The network is a chain of such layers; it is trained so that N(xi) approximates
M^{-1} xi on pairs (xi, psi = M^{-1} xi):

    L = (1/B) sum_b ||N(xi_b) - psi_b||^2 / ||psi_b||^2.

Gradients are Wirtinger derivatives dL/d(conj A): for a layer out = sum_k A_k T_k phi
with upstream g = dL/d(conj out),
    dL/d(conj A_k)^{ab} = sum_x sum_colour g_x^a conj((T_k phi)_x^b),
    dL/d(conj phi)      = sum_k T_k^dag (A_k^dag g),  T_k^dag h = P_{-k} h_{x - d_k};
the real parameters Re A and Im A have gradients 2 Re and 2 Im of dL/d(conj A).
"""
import numpy as np

from .lattice import cmul, dag, link, shift, shift_vec, smul
from .route_a import FWD_OF_BWD, PAIRS, offsets

OFFS = offsets()
# index of the hop -d for every hop d
NEG = [OFFS.index(tuple(-v for v in d)) for d in OFFS]


def forward_transports(U):
    """The colour transports of the 13 forward hops, keyed by hop index k."""
    P = {}
    for mu in range(4):
        P[1 + mu] = link(U, mu)
    for i in range(3):
        Ui = link(U, i)
        P[9 + i] = Ui @ shift(Ui, i, 1)
    for p, (i, j) in enumerate(PAIRS):
        Ui, Uj = link(U, i), link(U, j)
        P[15 + p] = 0.5 * (Ui @ shift(Uj, i, 1) + Uj @ shift(Ui, j, 1))
        P[21 + p] = 0.5 * (Ui @ dag(shift(shift(Uj, j, -1), i, 1)) + dag(shift(Uj, j, -1)) @ shift(Ui, j, -1))
    return P


def all_transports(U):
    """P_k(x) for all 27 hops (k = 0 the identity)."""
    P = forward_transports(U)
    shp = U.shape[:4]
    P[0] = np.broadcast_to(np.eye(3, dtype=np.complex128), shp + (3, 3))
    for kb, kf in FWD_OF_BWD.items():
        P[kb] = dag(shift_vec(P[kf], [-v for v in OFFS[kf]]))
    return P


def hop(P, k, phi):
    """(T_k phi)_x = P_k(x) phi_{x + d_k}."""
    return cmul(P[k], shift_vec(phi, OFFS[k]))


def layer(P, A, phi):
    """One layer: sum_k A_k T_k phi.  A has shape (27, 4, 4)."""
    out = 0.0
    for k in range(27):
        out = out + smul(A[k], hop(P, k, phi))
    return out


def layer_adjoint(P, A, g):
    """Adjoint of the layer: sum_k T_k^dag (A_k^dag g), with T_k^dag = T_{-k}."""
    out = 0.0
    for k in range(27):
        out = out + hop(P, NEG[k], smul(np.conj(A[k]).T, g))
    return out


def layer_weight_grad(P, g, phi):
    """dL/d(conj A_k)^{ab} = sum_x sum_colour g^a conj((T_k phi)^b), shape (27, 4, 4)."""
    G = np.zeros((27, 4, 4), dtype=np.complex128)
    gf = g.reshape(-1, 4, 3)
    for k in range(27):
        h = np.broadcast_to(hop(P, k, phi), g.shape).reshape(-1, 4, 3)
        G[k] = np.einsum("nac,nbc->ab", gf, np.conj(h))
    return G


def forward(P, params, phi):
    """The network on phi (any leading batch axes); returns the list of layer inputs and the output."""
    acts = [phi]
    for A in params:
        acts.append(layer(P, A, acts[-1]))
    return acts


def loss_and_grad(P, params, xi, psi):
    """L and dL/d(conj params) for a batch xi, psi shaped (B, Lt, Lz, Ly, Lx, 4, 3)."""
    B = xi.shape[0]
    acts = forward(P, params, xi)
    out = acts[-1]
    norms = np.array([np.vdot(psi[b], psi[b]).real for b in range(B)])
    diff = out - psi
    L = sum(np.vdot(diff[b], diff[b]).real / norms[b] for b in range(B)) / B
    g = diff / (B * norms[:, None, None, None, None, None, None])
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        grads[l] = layer_weight_grad(P, g, acts[l])
        g = layer_adjoint(P, params[l], g)
    return L, np.stack(grads)


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam on the real and imaginary parts: the real gradients are 2 Re g and 2 Im g."""
    gr = 2.0 * g
    m = b1 * m + (1 - b1) * gr
    v = b2 * v + (1 - b2) * (gr.real ** 2 + 1j * gr.imag ** 2)
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    upd = mh.real / (np.sqrt(vh.real) + eps) + 1j * mh.imag / (np.sqrt(vh.imag) + eps)
    return p - lr * upd, m, v
