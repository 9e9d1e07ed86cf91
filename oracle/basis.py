"""Spin basis of the precalculation matrices (Sec. 2.2, Eqs. shifted_W_first..last).

The paper writes every W as a 2x2 array of 2x2-spin blocks [[A, B], [C, D]]
acting on spin pairs (0,1) | (2,3), with Pauli matrices sigma_i inside the
blocks.  The Dirac matrices are not printed (they are those of the Fermilab
action's reference); the reading used here is the one the printed W fix:

* W+_4 has the pure link -U_4 in its lower-right block and zero upper-left block,
  i.e. the forward time hop is -(1/2)(1 - gamma_4) U_4 with gamma_4 = diag(1, 1, -1, -1);
* W+_i has sigma_i U_i in its off-diagonal blocks, i.e. gamma_i = [[0, s_i], [s_i, 0]].

Then gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 = [[0, -i], [i, 0]], Sigma_k =
diag(s_k, s_k) and alpha_k = gamma_4 gamma_k = [[0, s_k], [-s_k, 0]].
"""
import numpy as np

I2 = np.eye(2, dtype=np.complex128)
Z2 = np.zeros((2, 2), dtype=np.complex128)
SIGMA = np.array([
    [[0, 1], [1, 0]],
    [[0, -1j], [1j, 0]],
    [[1, 0], [0, -1]],
], dtype=np.complex128)


def spin4(a, b, c, d):
    """4x4 spin matrix from 2x2 blocks [[a, b], [c, d]]."""
    return np.block([[a, b], [c, d]])


GAMMA = np.array([spin4(Z2, SIGMA[k], SIGMA[k], Z2) for k in range(3)]
                 + [spin4(I2, Z2, Z2, -I2)])
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
BIGSIGMA = np.array([spin4(SIGMA[k], Z2, Z2, SIGMA[k]) for k in range(3)])
ALPHA = np.array([GAMMA[3] @ GAMMA[k] for k in range(3)])
ID4 = np.eye(4, dtype=np.complex128)


def sigma_munu(mu, nu):
    """sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] (textbook clover normalisation)."""
    g = GAMMA
    return 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])


def gamma5_conj(X):
    """Gamma(X) = gamma_5 X^dag gamma_5 on 12x12 spin-colour matrices (index 3*alpha + a).

    The dagger is taken in spin and colour together (Sec. 2.2); with the basis
    above Gamma([[A, B], [C, D]]) = [[D^dag, -B^dag], [-C^dag, A^dag]].
    """
    g5 = np.kron(GAMMA5, np.eye(3))
    Xd = np.conj(np.swapaxes(X, -1, -2))
    return g5 @ Xd @ g5


EPS3 = np.zeros((3, 3, 3))
for _i, _j, _k in [(0, 1, 2), (1, 2, 0), (2, 0, 1)]:
    EPS3[_i, _j, _k] = 1.0
    EPS3[_i, _k, _j] = -1.0
