"""Route-B M evaluated on parts of a large lattice.

(M psi)_x depends only on psi within 2 lattice spacings in space and 1 in
time of x, and on links within 3 in space and 2 in time (the clover fields at
x + i and x + t reach one step further than the hops).  Cutting a periodic
window of at least 2*3 + 1 = 7 sites in each spatial direction and 5 in time,
centred on x, therefore reproduces (M psi)_x exactly; the window is evaluated
with the global route-B operator.

The same argument gives M psi on a whole lattice slab by slab: the sites with
t0 <= t < t1 need only the time slices t0 - 2 .. t1 + 1 (all of space), so
route B on that periodic window is exact on its interior.  apply_slabs runs
the slabs in separate worker processes (started fresh, not forked, so that
they hold nothing of the calling process) and concatenates them: the same
operator as OKOperatorB(U, c).apply(psi), only faster on a many-core host.
"""
import multiprocessing

import numpy as np

from .route_b import OKOperatorB

WINDOW = (9, 9, 9, 5)


def _take(f, centre, dims, win):
    """Periodic window of a (Lt, Lz, Ly, Lx, ...) field centred on centre = (x, y, z, t)."""
    idx = []
    for mu in (3, 2, 1, 0):
        h = win[mu] // 2
        idx.append((np.arange(-h, win[mu] - h) + centre[mu]) % dims[mu])
    return f[np.ix_(*idx)]


def apply_at_sites(U, psi, c, sites, m0=0.5, window=WINDOW):
    """(M psi)_x for each x in sites (list of (x, y, z, t)); returns (n, 4, 3) complex."""
    dims = (U.shape[3], U.shape[2], U.shape[1], U.shape[0])
    win = [min(window[mu], dims[mu]) for mu in range(4)]
    out = []
    for s in sites:
        if any(win[mu] < window[mu] for mu in range(4)):
            raise ValueError("lattice smaller than the evaluation window")
        Uw = _take(U, s, dims, win)
        pw = _take(psi, s, dims, win)
        yw = OKOperatorB(Uw, c, m0=m0).apply(pw)
        ct = [win[mu] // 2 for mu in range(4)]
        out.append(yw[ct[3], ct[2], ct[1], ct[0]])
    return np.stack(out)


HALO_T = 2


def _slab(args):
    U, psi, c, m0, t_len = args
    y = OKOperatorB(U, c, m0=m0).apply(psi)
    return np.take(y, np.arange(HALO_T, HALO_T + t_len), axis=-6)


def apply_slabs(U, psi, c, m0=0.5, nproc=8):
    """M psi for psi shaped (..., Lt, Lz, Ly, Lx, 4, 3), evaluated as nproc time slabs."""
    lt = U.shape[0]
    n = max(1, min(nproc, lt // 2))
    bounds = np.linspace(0, lt, n + 1).astype(int)
    jobs = []
    for t0, t1 in zip(bounds[:-1], bounds[1:]):
        idx = np.arange(t0 - HALO_T, t1 + HALO_T) % lt
        jobs.append((U[idx], np.take(psi, idx, axis=-6), c, m0, int(t1 - t0)))
    if n == 1:
        return _slab(jobs[0])
    with multiprocessing.get_context("spawn").Pool(n) as pool:
        parts = pool.map(_slab, jobs)
    return np.concatenate(parts, axis=-6)
