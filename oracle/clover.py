"""Clover field strength and the chromo-electric/magnetic fields B_i, E_i.

The paper uses B_i and E_i inside W (Eqs. shifted_W_first..last) without
defining them; the reading taken here is the standard clover one:

* Q_{mu nu}(x) is the sum of the four plaquette leaves in the (mu, nu) plane that
  start and end at x, each traversed counter-clockwise (first step along +mu or
  the leaf's own first edge, then +nu, ...);
* F_{mu nu} = (Q - Q^dag)/8 with its trace removed (anti-Hermitian, traceless);
* B_i = (1/2) eps_{ijk} F_{jk},  E_i = F_{4i}  (paper's mu = 4 is index 3 here).
"""
import numpy as np

from .lattice import dag, link, shift


def clover_leaves(U, mu, nu):
    """Q_{mu nu}(x): the four counter-clockwise leaves in the (mu, nu) plane at x."""
    Umu = link(U, mu)
    Unu = link(U, nu)
    # leaf 1: x -> x+mu -> x+mu+nu -> x+nu -> x
    q = Umu @ shift(Unu, mu, 1) @ dag(shift(Umu, nu, 1)) @ dag(Unu)
    # leaf 2: x -> x+nu -> x+nu-mu -> x-mu -> x
    q = q + Unu @ dag(shift(shift(Umu, mu, -1), nu, 1)) @ dag(shift(Unu, mu, -1)) @ shift(Umu, mu, -1)
    # leaf 3: x -> x-mu -> x-mu-nu -> x-nu -> x
    q = q + (dag(shift(Umu, mu, -1)) @ dag(shift(shift(Unu, mu, -1), nu, -1))
             @ shift(shift(Umu, mu, -1), nu, -1) @ shift(Unu, nu, -1))
    # leaf 4: x -> x-nu -> x-nu+mu -> x+mu -> x
    q = q + dag(shift(Unu, nu, -1)) @ shift(Umu, nu, -1) @ shift(shift(Unu, nu, -1), mu, 1) @ dag(Umu)
    return q


def field_strength(U, mu, nu):
    """F_{mu nu} = traceless part of (Q_{mu nu} - Q_{mu nu}^dag)/8."""
    q = clover_leaves(U, mu, nu)
    f = (q - dag(q)) / 8.0
    tr = np.trace(f, axis1=-2, axis2=-1) / 3.0
    return f - tr[..., None, None] * np.eye(3)


def magnetic_electric(U):
    """(B, E) as arrays shaped (3, Lt, Lz, Ly, Lx, 3, 3): B_i = 1/2 eps_ijk F_jk, E_i = F_{4i}."""
    F = {}
    for mu in range(4):
        for nu in range(mu + 1, 4):
            F[(mu, nu)] = field_strength(U, mu, nu)
    B = np.stack([F[(1, 2)], -F[(0, 2)], F[(0, 1)]])
    E = np.stack([-F[(0, 3)], -F[(1, 3)], -F[(2, 3)]])
    return B, E
