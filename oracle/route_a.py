"""The precalculation matrices W exactly as printed (Sec. 2.2, Eqs. shifted_W_first..last).

Forward blocks are built from the printed formulas; the backward blocks follow
from one rule, W_{-d, x} = Gamma(W_{+d, x-d}) with Gamma(X) = gamma5 X^dag gamma5,
which reproduces the printed opposite-direction relations (Eqs. conjugate and
opp_diag_pre_mat).  Each W is 12x12 in spin-colour (index 3*alpha + a), a 4x4
array of 3x3 colour blocks; a 2x2 spin block with entries sigma (x) C is the
Kronecker product.

The 27 offsets of Eq. minFlopForm, in storage order k:

  k = 0          d = 0            W0 (without the mass term mhat)
  k = 1..4       d = +mu          W+_mu            (mu = x, y, z, t)
  k = 5..8       d = -mu          W-_mu
  k = 9..11      d = +2i          W++_ii           (i = x, y, z)
  k = 12..14     d = -2i          W--_ii
  k = 15..17     d = +i+j         W++_ij           (ij = xy, xz, yz)
  k = 18..20     d = -i-j         W--_ij
  k = 21..23     d = +i-j         W+-_ij
  k = 24..26     d = -i+j         W+-_ji
"""
import numpy as np

from .basis import I2, SIGMA, Z2, gamma5_conj
from .clover import magnetic_electric
from .lattice import dag, link, shift, shift_vec

PAIRS = [(0, 1), (0, 2), (1, 2)]


def _unit(mu):
    d = [0, 0, 0, 0]
    d[mu] = 1
    return d


def offsets():
    """The 27 offsets d_k (4-vectors, x y z t) in storage order."""
    out = [[0, 0, 0, 0]]
    out += [_unit(mu) for mu in range(4)]
    out += [[-v for v in _unit(mu)] for mu in range(4)]
    out += [[2 * v for v in _unit(i)] for i in range(3)]
    out += [[-2 * v for v in _unit(i)] for i in range(3)]
    for sgn_i, sgn_j in [(1, 1), (-1, -1), (1, -1), (-1, 1)]:
        for i, j in PAIRS:
            d = [0, 0, 0, 0]
            d[i] += sgn_i
            d[j] += sgn_j
            out.append(d)
    return [tuple(d) for d in out]


# backward block k_b comes from forward block k_f at x - d_{k_f}
FWD_OF_BWD = {5 + m: 1 + m for m in range(4)}
FWD_OF_BWD.update({12 + i: 9 + i for i in range(3)})
FWD_OF_BWD.update({18 + p: 15 + p for p in range(3)})
FWD_OF_BWD.update({24 + p: 21 + p for p in range(3)})
FORWARD = [0, 1, 2, 3, 4, 9, 10, 11, 15, 16, 17, 21, 22, 23]


def kron2(s, C):
    """sigma (x) C on the (2 spin x 3 colour) = 6-dim half space; s is 2x2, C is (...,3,3)."""
    out = np.einsum("st,...ab->...satb", s, C)
    return out.reshape(C.shape[:-2] + (6, 6))


def blocks(A, Bm, Cm, Dm):
    """12x12 matrix [[A, B], [C, D]] from 6x6 half-space blocks (zeros allowed as None)."""
    ref = next(x for x in (A, Bm, Cm, Dm) if x is not None)
    z = np.zeros_like(ref)
    A, Bm, Cm, Dm = [z if x is None else x for x in (A, Bm, Cm, Dm)]
    top = np.concatenate([A, Bm], axis=-1)
    bot = np.concatenate([Cm, Dm], axis=-1)
    return np.concatenate([top, bot], axis=-2)


def colour(C):
    """I2 (x) C: colour matrix acting on both spins of a half space."""
    return kron2(I2, C)


class WForm:
    """The 27 precalculation matrices per site for fixed links and coefficients."""

    def __init__(self, U, c):
        self.U = U
        self.c = c
        self.dims = (U.shape[3], U.shape[2], U.shape[1], U.shape[0])
        B, E = magnetic_electric(U)
        self.Bf, self.Ef = B, E
        # barred spin fields (Sec. 2.2): E^S = sum_i sigma_i E_i, B^D = i sum_i sigma_i B_i
        self.ES = sum(kron2(SIGMA[i], E[i]) for i in range(3))
        self.BD = sum(kron2(1j * SIGMA[i], B[i]) for i in range(3))
        self.fwd = self._forward()
        self.W = self._all27()

    # forward blocks ------------------------------------------------------
    def _forward(self):
        c, U = self.c, self.U
        u0 = c.u0
        ES, BD = self.ES, self.BD
        W = {}
        # W0 without mhat
        D0 = -(c.c_B * c.zeta + 16.0 * c.c_5) / (2.0 * u0 ** 3) * BD
        S0 = -(c.c_E * c.zeta) / (2.0 * u0 ** 3) * ES
        W[0] = blocks(D0, S0, -S0, D0)
        # W+_4 (time)
        U4 = colour(link(U, 3))
        S4 = c.c_EE / (2.0 * u0 ** 4) * (U4 @ shift(ES, 3, 1) - ES @ U4)
        W[4] = blocks(None, S4, S4, -U4)
        # W+_i
        for i in range(3):
            Ui = link(U, i)
            Uc = colour(Ui)
            si = kron2(SIGMA[i], np.broadcast_to(np.eye(3), Ui.shape))
            Bi = self.Bf[i]
            S = 0.5 * (c.zeta - 2.0 * c.c_1 - 12.0 * c.c_2) * kron2(SIGMA[i], Ui)
            S = S + c.c_3 / (2.0 * u0 ** 4) * (Uc @ si @ shift(BD, i, 1) - si @ BD @ Uc
                                               + colour(2j * Bi @ Ui))
            Dm = -0.5 * (c.r_s * c.zeta + 8.0 * c.c_4) * Uc
            Dm = Dm + 1j * c.c_5 / 4.0 * (u0 ** -2 - u0 ** -4) * self._eps_staple(i)
            Dm = Dm + c.c_5 / u0 ** 4 * (Uc @ shift(BD, i, 1) + BD @ Uc
                                         - 1j * kron2(SIGMA[i], Ui @ shift(Bi, i, 1) + Bi @ Ui))
            W[1 + i] = blocks(Dm, S, S, Dm)
        # W++_ii
        for i in range(3):
            Ui = link(U, i)
            UU = Ui @ shift(Ui, i, 1)
            Dd = c.c_4 / u0 * colour(UU)
            Sd = (c.c_1 + 2.0 * c.c_2) / (2.0 * u0) * kron2(SIGMA[i], UU)
            W[9 + i] = blocks(Dd, Sd, Sd, Dd)
        # W++_ij and W+-_ij, i < j
        for p, (i, j) in enumerate(PAIRS):
            W[15 + p] = self.diag_pp(i, j)
            W[21 + p] = self.diag_pm(i, j)
        return W

    def _eps_staple(self, i):
        """sum_{jk} eps_ijk sigma_j (x) (U_k(x) U_i(x+k) U_k(x+i)^dag - U_k(x-k)^dag U_i(x-k) U_k(x-k+i)),
        the staple sum inside the c_5 part of D_i (Sec. 2.2, W+_i), as a 6x6 half-space block."""
        U = self.U
        Ui = link(U, i)
        stap = 0.0
        for j in range(3):
            for k in range(3):
                e = _eps(i, j, k)
                if e == 0:
                    continue
                Uk = link(U, k)
                up = Uk @ shift(Ui, k, 1) @ dag(shift(Uk, i, 1))
                dn = dag(shift(Uk, k, -1)) @ shift(Ui, k, -1) @ shift(shift(Uk, k, -1), i, 1)
                stap = stap + e * kron2(SIGMA[j], up - dn)
        return stap

    def diag_pp(self, i, j):
        """W++_ij = [[0, S], [S, 0]], S = c2/(2u0) (s_i + s_j)(U_i(x) U_j(x+i) + U_j(x) U_i(x+j))."""
        c, U = self.c, self.U
        Ui, Uj = link(U, i), link(U, j)
        P = Ui @ shift(Uj, i, 1) + Uj @ shift(Ui, j, 1)
        S = c.c_2 / (2.0 * c.u0) * kron2(SIGMA[i] + SIGMA[j], P)
        return blocks(None, S, S, None)

    def diag_pm(self, i, j):
        """W+-_ij = [[0, S'], [S', 0]], S' = c2/(2u0)(s_i - s_j)(U_i(x) U_j(x-j+i)^dag + U_j(x-j)^dag U_i(x-j))."""
        c, U = self.c, self.U
        Ui, Uj = link(U, i), link(U, j)
        P = Ui @ dag(shift(shift(Uj, j, -1), i, 1)) + dag(shift(Uj, j, -1)) @ shift(Ui, j, -1)
        S = c.c_2 / (2.0 * c.u0) * kron2(SIGMA[i] - SIGMA[j], P)
        return blocks(None, S, S, None)

    def _all27(self):
        offs = offsets()
        shp = self.fwd[0].shape[:-2]
        W = np.zeros(shp + (27, 12, 12), dtype=np.complex128)
        for k, blk in self.fwd.items():
            W[..., k, :, :] = blk
        for kb, kf in FWD_OF_BWD.items():
            d = offs[kf]
            W[..., kb, :, :] = gamma5_conj(shift_vec(self.fwd[kf], [-v for v in d]))
        return W

    # application ---------------------------------------------------------
    def apply(self, psi, mhat=None):
        """Eq. minFlopForm: (M psi)_x = mhat psi_x + sum_k W_{k,x} psi_{x+d_k}."""
        mhat = self.c.mhat if mhat is None else mhat
        shp = psi.shape
        out = mhat * psi.reshape(shp[:-2] + (12,))
        for k, d in enumerate(offsets()):
            nb = shift_vec(psi, d).reshape(shp[:-2] + (12, 1))
            out = out + (self.W[..., k, :, :] @ nb)[..., 0]
        return out.reshape(shp)

    def saved_set(self):
        """The shifted set saved per site (Sec. 2.2): W0_x, W+_mu,x, W++_ii,x-i,
        W++_ij,x-j and W+-_ij,x+j (i < j)."""
        S = {"W0": self.fwd[0]}
        for mu in range(4):
            S[("P", mu)] = self.fwd[1 + mu]
        for i in range(3):
            S[("PP", i)] = shift(self.fwd[9 + i], i, -1)
        for p, (i, j) in enumerate(PAIRS):
            S[("PPij", p)] = shift(self.fwd[15 + p], j, -1)
            S[("PMij", p)] = shift(self.fwd[21 + p], j, 1)
        return S

    def apply_final_form(self, psi, mhat=None):
        """Eq. FinalForm: the same operator from the 14 saved blocks with pre- and
        post-multiplication translations t_{+-mu} of product fields."""
        mhat = self.c.mhat if mhat is None else mhat
        S = self.saved_set()
        shp = psi.shape
        v = lambda f: f.reshape(shp[:-2] + (12, 1))
        mv = lambda W, f: (W @ v(f))[..., 0].reshape(shp)
        G = gamma5_conj
        out = mhat * psi + mv(S["W0"], psi)
        for mu in range(4):
            out = out + mv(S[("P", mu)], shift(psi, mu, 1))
            # t_{-mu}[ W-_{mu,x+mu} psi_x ],  W-_{mu,x+mu} = Gamma(W+_{mu,x})
            out = out + shift(mv(G(S[("P", mu)]), psi), mu, -1)
        for i in range(3):
            out = out + shift(mv(S[("PP", i)], shift(psi, i, 1)), i, 1)
            # W--_{ii,x+i} = Gamma(W++_{ii,x-i})
            out = out + shift(mv(G(S[("PP", i)]), shift(psi, i, -1)), i, -1)
        for p, (i, j) in enumerate(PAIRS):
            Wpp = S[("PPij", p)]
            Wpm = S[("PMij", p)]
            out = out + shift(mv(Wpp, shift(psi, i, 1)), j, 1)
            out = out - shift(mv(dag(Wpp), shift(psi, j, -1)), i, -1)
            out = out + shift(mv(Wpm, shift(psi, i, 1)), j, -1)
            out = out - shift(mv(dag(Wpm), shift(psi, j, 1)), i, -1)
        return out


def _eps(i, j, k):
    if (i, j, k) in [(0, 1, 2), (1, 2, 0), (2, 0, 1)]:
        return 1
    if (i, j, k) in [(0, 2, 1), (2, 1, 0), (1, 0, 2)]:
        return -1
    return 0
