"""Periodic lattice fields as NumPy arrays.

Fields carry the site axes (Lt, Lz, Ly, Lx) followed by exactly two trailing
axes: (4, 3) spin-colour for spinors, (3, 3) colour for link-like fields and
(12, 12) for precalculation matrices; any number of leading batch axes is
allowed.  Direction mu = 0, 1, 2, 3 is x, y, z, t.
"""
import numpy as np

_AXIS = {0: -3, 1: -4, 2: -5, 3: -6}


def shift(f, mu, n=1):
    """Translation t_{n mu}: returns the field g with g_x = f_{x + n*mu-hat} (periodic)."""
    if n == 0:
        return f
    return np.roll(f, -n, axis=_AXIS[mu])


def shift_vec(f, d):
    """g_x = f_{x + d} for a 4-vector offset d = (dx, dy, dz, dt)."""
    for mu in range(4):
        if d[mu]:
            f = shift(f, mu, d[mu])
    return f


def dag(m):
    """Hermitian conjugate of the trailing 2 axes."""
    return np.conj(np.swapaxes(m, -1, -2))


def cmul(C, psi):
    """Colour multiplication (C psi)_x^{alpha a} = sum_b C_x^{ab} psi_x^{alpha b}."""
    return psi @ np.swapaxes(C, -1, -2)


def smul(S, psi):
    """Spin multiplication (S psi)^{alpha a} = sum_beta S^{alpha beta} psi^{beta a}."""
    return S @ psi


def link(U, mu):
    return U[..., mu, :, :]


def vdot(a, b):
    """<a, b> = sum conj(a) b over all sites and components."""
    return np.vdot(a.ravel(), b.ravel())


def norm2(a):
    return float(np.vdot(a.ravel(), a.ravel()).real)
