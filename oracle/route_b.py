"""M applied term by term from the gauge links (operator composition).

The paper defines M only through its precalculated matrices W; the operator
they collect is the tree-level, tadpole-improved OK action (Sec. 1): the
Fermilab action plus the third-order bilinears.  Reading each printed W back
into covariant lattice operators gives, with V = U/u0,

  T+_mu f_x = V_mu(x) f_{x+mu},   T-_mu f_x = V_mu(x-mu)^dag f_{x-mu},
  D_mu = (T+_mu - T-_mu)/2,       Delta_mu = T+_mu + T-_mu - 2,

  M_B[V] = m0 + g4 D4 - Delta4/2 + zeta g.D - (r_s zeta/2) Delta3
           - (c_B zeta/2) i Sigma.B - (c_E zeta/2) alpha.E
           + c_1 sum_i g_i D_i Delta_i + c_2 {g.D, Delta3} + c_3 {g.D, i Sigma.B}
           + c_EE {g4 D4, alpha.E} + c_4 sum_i Delta_i^2
           + c_5 sum_i sum_{j != i} {i Sigma_i B_i, Delta_j}

with B, E the clover fields of V, and

  M(U) = u0 M_B[U/u0] + T_eps + (mhat - u0 d_B) 1,
  d_B  = m0 + 1 + 3 r_s zeta + c_4 sum_i (4 + 2/u0^2)   (identity part of M_B).

T_eps is the c_5 staple term of D+_i in Eq. shifted_W_first..last (weight
(u0^-2 - u0^-4)) together with its backward partner; it vanishes at u0 = 1.
The identity coefficient of M is mhat = u0/(2 kappa), which the paper applies
separately from W0 (footnote of Sec. 2.2).

Nothing here uses the precalculated W; the W-form is in route_a.
"""
import numpy as np

from .basis import ALPHA, BIGSIGMA, EPS3, GAMMA, GAMMA5
from .clover import magnetic_electric
from .lattice import cmul, dag, link, shift, smul


class OKOperatorB:
    """Route-B operator for fixed links and coefficients; call apply(psi)."""

    def __init__(self, U, c, m0=0.5):
        self.U = U
        self.c = c
        self.m0 = m0
        u0 = c.u0
        B, E = magnetic_electric(U)
        self.B = B / u0 ** 4          # clover of V = U/u0 (four links per leaf)
        self.E = E / u0 ** 4
        self.Vf = [link(U, mu) / u0 for mu in range(4)]
        self.Vb = [dag(shift(link(U, mu), mu, -1)) / u0 for mu in range(4)]
        self.eps_fwd = [self._eps_block(i) for i in range(3)]

    # elementary covariant operators ------------------------------------
    def Tp(self, mu, f):
        return cmul(self.Vf[mu], shift(f, mu, 1))

    def Tm(self, mu, f):
        return cmul(self.Vb[mu], shift(f, mu, -1))

    def D(self, mu, f):
        return 0.5 * (self.Tp(mu, f) - self.Tm(mu, f))

    def Lap(self, mu, f):
        return self.Tp(mu, f) + self.Tm(mu, f) - 2.0 * f

    def gD(self, f):
        """gamma.D over the three spatial directions."""
        return sum(smul(GAMMA[i], self.D(i, f)) for i in range(3))

    def Lap3(self, f):
        return sum(self.Lap(i, f) for i in range(3))

    def iSigB(self, f):
        return sum(smul(1j * BIGSIGMA[k], cmul(self.B[k], f)) for k in range(3))

    def alphaE(self, f):
        return sum(smul(ALPHA[k], cmul(self.E[k], f)) for k in range(3))

    # the operator ------------------------------------------------------
    def apply_MB(self, f):
        """M_B[V] f (the untadpoled operator of V = U/u0, with identity part m0 + ...)."""
        c = self.c
        out = self.m0 * f
        out = out + smul(GAMMA[3], self.D(3, f)) - 0.5 * self.Lap(3, f)
        out = out + c.zeta * self.gD(f) - 0.5 * c.r_s * c.zeta * self.Lap3(f)
        out = out - 0.5 * c.c_B * c.zeta * self.iSigB(f) - 0.5 * c.c_E * c.zeta * self.alphaE(f)
        if c.c_1:
            out = out + c.c_1 * sum(smul(GAMMA[i], self.D(i, self.Lap(i, f))) for i in range(3))
        if c.c_2:
            out = out + c.c_2 * (self.gD(self.Lap3(f)) + self.Lap3(self.gD(f)))
        if c.c_3:
            out = out + c.c_3 * (self.gD(self.iSigB(f)) + self.iSigB(self.gD(f)))
        if c.c_EE:
            g4D4 = lambda h: smul(GAMMA[3], self.D(3, h))
            out = out + c.c_EE * (g4D4(self.alphaE(f)) + self.alphaE(g4D4(f)))
        if c.c_4:
            out = out + c.c_4 * sum(self.Lap(i, self.Lap(i, f)) for i in range(3))
        if c.c_5:
            acc = 0.0
            for i in range(3):
                Bi = lambda h, i=i: smul(1j * BIGSIGMA[i], cmul(self.B[i], h))
                for j in range(3):
                    if j != i:
                        acc = acc + Bi(self.Lap(j, f)) + self.Lap(j, Bi(f))
            out = out + c.c_5 * acc
        return out

    def identity_part(self):
        """d_B: coefficient of the unit operator inside M_B (T+T- = T-T+ = 1/u0^2)."""
        c = self.c
        return self.m0 + 1.0 + 3.0 * c.r_s * c.zeta + c.c_4 * 3.0 * (4.0 + 2.0 / c.u0 ** 2)

    def _eps_block(self, i):
        """Colour fields X_j(x) (j = 0..2) of the staple term of D+_i:

        i (c_5/4)(u0^-2 - u0^-4) sum_{jk} eps_ijk sigma_j
            (U_k(x) U_i(x+k) U_k(x+i)^dag - U_k(x-k)^dag U_i(x-k) U_k(x-k+i)).
        """
        c, U = self.c, self.U
        pref = 1j * 0.25 * c.c_5 * (c.u0 ** -2 - c.u0 ** -4)
        X = [0.0, 0.0, 0.0]
        for j in range(3):
            for k in range(3):
                e = EPS3[i, j, k]
                if e == 0.0:
                    continue
                Uk, Ui = link(U, k), link(U, i)
                up = Uk @ shift(Ui, k, 1) @ dag(shift(Uk, i, 1))
                Ukm = shift(Uk, k, -1)
                dn = dag(Ukm) @ shift(Ui, k, -1) @ shift(shift(Uk, k, -1), i, 1)
                X[j] = X[j] + e * pref * (up - dn)
        return X

    def apply_Teps(self, f):
        """T_eps f: forward part on x+i with Sigma_j (x) X_j, backward part its gamma5 partner."""
        if self.c.c_5 == 0.0 or self.c.u0 == 1.0:
            return np.zeros_like(f)
        out = np.zeros_like(f)
        for i in range(3):
            X = self.eps_fwd[i]
            fp = shift(f, i, 1)
            fm = shift(f, i, -1)
            for j in range(3):
                if np.isscalar(X[j]):
                    continue          # eps_ijk = 0 for j = i
                # forward: Sigma_j X_j(x) f_{x+i}
                out = out + smul(BIGSIGMA[j], cmul(X[j], fp))
                # backward: gamma5 (Sigma_j X_j(x-i))^dag gamma5 f_{x-i}
                Xm = dag(shift(X[j], i, -1))
                S = GAMMA5 @ BIGSIGMA[j].conj().T @ GAMMA5
                out = out + smul(S, cmul(Xm, fm))
        return out

    def apply(self, f):
        """M(U) f = u0 M_B[U/u0] f + T_eps f + (mhat - u0 d_B) f."""
        c = self.c
        out = c.u0 * self.apply_MB(f) + self.apply_Teps(f)
        return out + (c.mhat - c.u0 * self.identity_part()) * f
