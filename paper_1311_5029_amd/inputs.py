"""Seeded synthetic inputs for the OK-action operator and its solver.

This module is shared by the CPU oracle and the GPU path and therefore holds
none of the operator's arithmetic: it only draws gauge fields, sources, gauge
transformations, coefficient sets and the preconditioner network's initial
parameters, all on the host with NumPy's PCG64.

Array conventions (shared by both sides):

* lattice dimensions ``dims = (Lx, Ly, Lz, Lt)``; direction mu = 0, 1, 2, 3 is
  x, y, z, t (the paper's mu = 1..4 with mu = 4 the time direction, Sec. 2.1);
* site index ``s = x + Lx*(y + Ly*(z + Lz*t))``, i.e. NumPy arrays are shaped
  ``(Lt, Lz, Ly, Lx, ...)`` in C order;
* gauge links ``U[t, z, y, x, mu, a, b]`` complex128, the link from x to
  x + mu-hat (it multiplies the neighbour spinor psi_{x+mu});
* spinors ``psi[..., t, z, y, x, alpha, a]`` complex, spin alpha = 0..3,
  colour a = 0..2; the spin-colour index is ``3*alpha + a``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Seeds of the synthetic workloads (one stream per purpose).
SEED_LINKS = 1000
SEED_SOURCES = 2000
SEED_TRAIN = 3000
SEED_EVAL = 4000
SEED_GAUGE = 5000
SEED_NET = 6000


def lattice_shape(dims):
    """NumPy shape (Lt, Lz, Ly, Lx) of a lattice with dims (Lx, Ly, Lz, Lt)."""
    lx, ly, lz, lt = dims
    return (lt, lz, ly, lx)


def volume(dims):
    return int(np.prod(dims))


def _random_traceless_hermitian(rng, shape):
    """H = (A + A^dag)/2 - tr/3 with A_ab = g1 + i g2, g ~ N(0, 1)."""
    a = rng.standard_normal(shape + (3, 3)) + 1j * rng.standard_normal(shape + (3, 3))
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[..., None, None] * np.eye(3)
    return h


def _expi(h, eps):
    """exp(i*eps*H) for Hermitian H via its eigendecomposition."""
    lam, vec = np.linalg.eigh(h)
    ph = np.exp(1j * eps * lam)
    return np.einsum("...ak,...k,...bk->...ab", vec, ph, np.conj(vec))


def random_su3_links(dims, eps, seed, chunk=1 << 18):
    """Random links U = exp(i*eps*H), one independent H per (site, mu).

    Returns complex128 of shape (Lt, Lz, Ly, Lx, 4, 3, 3).  Drawn in chunks of
    sites so that the 20^3x64 and 32^3x64 fields do not need large temporaries;
    the stream of normals is the same as one full draw would give.
    """
    rng = np.random.default_rng(seed)
    shp = lattice_shape(dims)
    n = volume(dims) * 4
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        h = _random_traceless_hermitian(rng, (hi - lo,))
        out[lo:hi] = _expi(h, eps)
    return out.reshape(shp + (4, 3, 3))


def _roll_site(f, mu, n):
    """f_{x + n*mu} for a field shaped (Lt, Lz, Ly, Lx, ...) with 2 trailing axes."""
    axis = {0: -3, 1: -4, 2: -5, 3: -6}[mu]
    return np.roll(f, -n, axis=axis)


def plaquette(U):
    """Average of (1/3) Re tr U_P over all sites and the 6 planes mu < nu."""
    tot = 0.0
    cnt = 0
    dag = lambda m: np.conj(np.swapaxes(m, -1, -2))
    for mu in range(4):
        for nu in range(mu + 1, 4):
            umu = U[..., mu, :, :]
            unu = U[..., nu, :, :]
            p = umu @ _roll_site(unu, mu, 1) @ dag(_roll_site(umu, nu, 1)) @ dag(unu)
            tot += np.trace(p, axis1=-2, axis2=-1).real.sum() / 3.0
            cnt += p.shape[0] * p.shape[1] * p.shape[2] * p.shape[3]
    return tot / cnt


def tadpole_u0(U):
    """u0 = <plaquette>^(1/4) (tadpole improvement)."""
    return plaquette(U) ** 0.25


def tune_epsilon(target=0.6, seed=SEED_LINKS, dims=(8, 8, 8, 8), tol=2e-4):
    """Bisect eps so that random_su3_links on an 8^4 lattice has plaquette ~ target.

    The plaquette of independent random links is intensive and decreases
    monotonically with eps on [0, 1.2], so a bisection on a small lattice
    transfers to the production volumes to within statistical noise.
    """
    lo, hi = 0.0, 1.2
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        p = plaquette(random_su3_links(dims, mid, seed))
        if abs(p - target) < tol:
            return mid
        if p > target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def gaussian_sources(dims, nrhs, seed):
    """nrhs Gaussian complex sources, each component (N(0,1) + i N(0,1))/sqrt(2).

    Shape (nrhs, Lt, Lz, Ly, Lx, 4, 3) complex128.
    """
    rng = np.random.default_rng(seed)
    shp = (nrhs,) + lattice_shape(dims) + (4, 3)
    return (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) / math.sqrt(2.0)


def gaussian_source_batches(dims, n, seed, batch):
    """The same distribution as gaussian_sources, drawn in batches of at most `batch` sources
    so that large sets never sit on the host at once: batch j comes from the generator
    seeded with (seed, j).  Yields arrays (nb, Lt, Lz, Ly, Lx, 4, 3) complex128."""
    for j, k0 in enumerate(range(0, n, batch)):
        rng = np.random.default_rng([seed, j])
        shp = (min(batch, n - k0),) + lattice_shape(dims) + (4, 3)
        yield (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) / math.sqrt(2.0)


def point_sources(dims, origin=(0, 0, 0, 0)):
    """The 12 spin-colour point sources xi^(beta,b)_x = delta_{x,origin} delta_{alpha beta} delta_{ab}.

    Source number 3*beta + b.  Shape (12, Lt, Lz, Ly, Lx, 4, 3) complex128.
    """
    out = np.zeros((12,) + lattice_shape(dims) + (4, 3), dtype=np.complex128)
    x, y, z, t = origin
    for beta in range(4):
        for b in range(3):
            out[3 * beta + b, t, z, y, x, beta, b] = 1.0
    return out


def random_su3_field(dims, seed):
    """Haar-random SU(3) matrix per site (QR of a complex Gaussian, phases fixed, det set to 1)."""
    rng = np.random.default_rng(seed)
    shp = lattice_shape(dims)
    z = (rng.standard_normal(shp + (3, 3)) + 1j * rng.standard_normal(shp + (3, 3))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[..., None, None]
    return q


def gauge_transform_links(U, g):
    """U'_mu(x) = g(x) U_mu(x) g^dag(x + mu)."""
    out = np.empty_like(U)
    for mu in range(4):
        gp = _roll_site(g, mu, 1)
        out[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(gp, -1, -2))
    return out


def unit_links(dims):
    shp = lattice_shape(dims)
    out = np.zeros(shp + (4, 3, 3), dtype=np.complex128)
    for a in range(3):
        out[..., a, a] = 1.0
    return out


def pure_gauge_links(dims, seed):
    """U_mu(x) = g(x) g^dag(x + mu): gauge equivalent to the free field (plaquette 1)."""
    g = random_su3_field(dims, seed)
    return gauge_transform_links(unit_links(dims), g), g


@dataclasses.dataclass
class OKCoeffs:
    """Coefficients of the tree-level tadpole-improved OK operator.

    ``mhat`` is the identity coefficient u0/(2 kappa) of W0 (Eq. shifted_W_first),
    applied separately from the stored W0 blocks.
    """

    mhat: float
    u0: float = 1.0
    zeta: float = 1.0
    r_s: float = 1.0
    c_B: float = 1.0
    c_E: float = 1.0
    c_EE: float = 0.1
    c_1: float = -0.1
    c_2: float = 0.02
    c_3: float = 0.05
    c_4: float = 0.03
    c_5: float = 0.02

    def as_tuple(self):
        return tuple(getattr(self, f.name) for f in dataclasses.fields(self))


def standin_coeffs(m0=0.5, u0=1.0, **over):
    """The stand-in coefficient set (not the OK tree-level values) at bare mass m0.

    kappa is read from 1/(2 kappa) = 1 + m0 + 3 r_s zeta + 18 c_4, so that the
    free field at u0 = 1 has M(p = 0) = m0; mhat = u0/(2 kappa).
    """
    c = OKCoeffs(mhat=0.0, u0=u0, **over)
    inv2k = 1.0 + m0 + 3.0 * c.r_s * c.zeta + 18.0 * c.c_4
    c.mhat = u0 * inv2k
    return c


def wilson_clover_coeffs(m0=0.1):
    """Coefficients that reduce the OK operator to the Wilson-clover (SW) operator."""
    return standin_coeffs(m0=m0, u0=1.0, zeta=1.0, r_s=1.0, c_B=1.0, c_E=1.0,
                          c_EE=0.0, c_1=0.0, c_2=0.0, c_3=0.0, c_4=0.0, c_5=0.0)


# The five synthetic workloads: lattice, link roughness, sources; `seed` picks the link
# stream (1000 + seed) and the source stream (2000 + seed).
CONFIGS = {
    "dense_4x4x4x4": dict(seed=1, dims=(4, 4, 4, 4), eps=0.3, nrhs=1, sources="gaussian"),
    "mixed_16x16x16x32": dict(seed=2, dims=(16, 16, 16, 32), eps="plaq0.6", nrhs=1, sources="gaussian"),
    "batched_20x20x20x64": dict(seed=3, dims=(20, 20, 20, 64), eps="plaq0.6", nrhs=12, sources="point"),
    "learned_24x24x24x64": dict(seed=4, dims=(24, 24, 24, 64), eps="plaq0.6", nrhs=64, sources="gaussian"),
    "learned_batched_32x32x32x64": dict(seed=5, dims=(32, 32, 32, 64), eps="plaq0.6", nrhs=12,
                                        sources="point"),
}

_EPS_CACHE = {}


def config_epsilon(spec):
    if isinstance(spec, float):
        return spec
    if spec not in _EPS_CACHE:
        _EPS_CACHE[spec] = tune_epsilon(float(spec[len("plaq"):]))
    return _EPS_CACHE[spec]


def make_config(name, dims=None, with_sources=True):
    """Links, u0, coefficients and sources (None unless with_sources) of a named workload
    (optionally at other dims)."""
    cfg = CONFIGS[name]
    d = tuple(dims) if dims is not None else cfg["dims"]
    num = cfg["seed"]
    eps = config_epsilon(cfg["eps"])
    U = random_su3_links(d, eps, SEED_LINKS + num)
    u0 = tadpole_u0(U)
    coeffs = standin_coeffs(m0=0.5, u0=u0)
    if not with_sources:
        xi = None
    elif cfg["sources"] == "point":
        xi = point_sources(d)
    else:
        xi = gaussian_sources(d, cfg["nrhs"], SEED_SOURCES + num)
    return dict(dims=d, eps=eps, U=U, u0=u0, coeffs=coeffs, xi=xi)


def net_init_params(n_layers, scale, seed=SEED_NET, noise=1e-3):
    """Initial parameters of the preconditioner network, complex128 (n_layers, 27, 4, 4)
    (hop k, spin out, spin in): the first layer scale * 1 on the on-site hop, later layers
    the identity, plus complex Gaussian noise of size `noise` on every weight."""
    rng = np.random.default_rng(seed)
    shape = (n_layers, 27, 4, 4)
    p = noise * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
    p[0, 0] += scale * np.eye(4)
    for l in range(1, n_layers):
        p[l, 0] += np.eye(4)
    return p
