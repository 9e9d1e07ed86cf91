"""Closed forms of the operator on trivial gauge fields.

Free field (U = 1): B = E = 0 and every staple is the identity, so M is diagonal
in momentum.  Summing the printed W over the 27 offsets with e^{ip.d} gives

  M~(p) = A(p) + i sum_mu gamma_mu K_mu(p),
  A   = mhat - cos p4 - (r_s zeta + 8 c4) sum_i cos p_i + (2 c4/u0) sum_i cos 2p_i,
  K_4 = sin p4,
  K_i = (zeta - 2c1 - 12c2) sin p_i + ((c1 + 2c2)/u0) sin 2p_i
        + (4 c2/u0) sin p_i sum_{j != i} cos p_j,

whose eigenvalues are A +- i|K|, each six-fold; M~^{-1} = (A - i gamma.K)/(A^2 + |K|^2).
A point source at the origin is solved exactly by an inverse FFT of M~^{-1}.  A
pure-gauge field U_mu(x) = g(x) g(x+mu)^dag is the free field conjugated by g.
"""
import numpy as np

from .basis import GAMMA


def momenta(dims):
    """Lattice momenta p_mu = 2 pi n_mu / L_mu on the (Lt, Lz, Ly, Lx) grid, as 4 arrays (x,y,z,t)."""
    lx, ly, lz, lt = dims
    pt, pz, py, px = np.meshgrid(*(2 * np.pi * np.fft.fftfreq(n) for n in (lt, lz, ly, lx)),
                                 indexing="ij")
    return [px, py, pz, pt]


def symbol_AK(p, c):
    """(A, K) of the free-field symbol at momenta p = [px, py, pz, pt] (arrays or scalars)."""
    u0 = c.u0
    ps = p[:3]
    A = c.mhat - np.cos(p[3]) - (c.r_s * c.zeta + 8.0 * c.c_4) * sum(np.cos(q) for q in ps) \
        + (2.0 * c.c_4 / u0) * sum(np.cos(2 * q) for q in ps)
    K = []
    for i in range(3):
        others = sum(np.cos(ps[j]) for j in range(3) if j != i)
        K.append((c.zeta - 2 * c.c_1 - 12 * c.c_2) * np.sin(ps[i])
                 + ((c.c_1 + 2 * c.c_2) / u0) * np.sin(2 * ps[i])
                 + (4 * c.c_2 / u0) * np.sin(ps[i]) * others)
    K.append(np.sin(p[3]))
    return A, K


def symbol_matrix(p, c):
    """The 4x4 spin matrix M~(p) (colour blind) for scalar momenta p."""
    A, K = symbol_AK(p, c)
    return A * np.eye(4) + 1j * sum(K[mu] * GAMMA[mu] for mu in range(4))


def free_eigenvalues(dims, c):
    """All 12 V eigenvalues of M on the free field: A +- i|K| six-fold per momentum."""
    A, K = symbol_AK(momenta(dims), c)
    kn = np.sqrt(sum(k ** 2 for k in K))
    ev = np.concatenate([np.repeat((A + 1j * kn).ravel(), 6), np.repeat((A - 1j * kn).ravel(), 6)])
    return ev


def free_point_solution(dims, c, chi):
    """psi with M[U=1] psi = delta_{x,0} chi for spin-colour vectors chi shaped (n, 4, 3)."""
    A, K = symbol_AK(momenta(dims), c)
    den = A ** 2 + sum(k ** 2 for k in K)
    # Minv(p) = (A - i gamma.K)/den, shape (Lt, Lz, Ly, Lx, 4, 4)
    Minv = A[..., None, None] * np.eye(4) - 1j * sum(K[mu][..., None, None] * GAMMA[mu] for mu in range(4))
    Minv = Minv / den[..., None, None]
    out = []
    for ch in chi:
        phat = Minv @ ch  # (Lt, Lz, Ly, Lx, 4, 3): FT of delta_{x,0} chi is chi at every p
        out.append(np.fft.ifftn(phat, axes=(0, 1, 2, 3)))
    return np.stack(out)


def pure_gauge_point_solution(dims, c, g, chi):
    """Solution of M[U] psi = delta_{x,0} chi for U_mu(x) = g(x) g(x+mu)^dag.

    M[U] = G M[1] G^dag with (G f)_x = g(x) f_x, so psi = G M[1]^{-1} G^dag xi.
    """
    g0d = np.conj(g[0, 0, 0, 0]).T
    chi2 = np.stack([ch @ g0d.T for ch in chi])   # colour rotation g(0)^dag on each spin row
    free = free_point_solution(dims, c, chi2)
    return free @ np.swapaxes(g, -1, -2)          # (g(x) psi_x) per spin row
