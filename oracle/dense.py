"""Dense assembly of M on tiny lattices (brute force).

Row/column index = 12 * s + 3 * alpha + a with s = x + Lx (y + Ly (z + Lz t)),
which is the C-order flattening of the (Lt, Lz, Ly, Lx, 4, 3) field layout.
"""
import numpy as np


def dense_from_operator(apply, dims, batch=256):
    """M as a dense (12V, 12V) matrix: column n is apply(e_n)."""
    lx, ly, lz, lt = dims
    n = 12 * lx * ly * lz * lt
    M = np.zeros((n, n), dtype=np.complex128)
    for lo in range(0, n, batch):
        hi = min(n, lo + batch)
        e = np.zeros((hi - lo, n), dtype=np.complex128)
        e[np.arange(hi - lo), np.arange(lo, hi)] = 1.0
        cols = apply(e.reshape((hi - lo, lt, lz, ly, lx, 4, 3)))
        M[:, lo:hi] = cols.reshape(hi - lo, n).T
    return M


def dense_from_W(W, mhat, dims, offs):
    """M as a dense matrix from the 27 blocks per site: row block x, column block
    x + d_k receives W_{k,x} (blocks landing on the same column add, as for L = 4)."""
    lx, ly, lz, lt = dims
    V = lx * ly * lz * lt
    M = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    Wf = W.reshape(V, 27, 12, 12)
    for s in range(V):
        x, y, z, t = s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)
        M[12 * s:12 * s + 12, 12 * s:12 * s + 12] += mhat * np.eye(12)
        for k, d in enumerate(offs):
            xs = ((x + d[0]) % lx, (y + d[1]) % ly, (z + d[2]) % lz, (t + d[3]) % lt)
            n = xs[0] + lx * (xs[1] + ly * (xs[2] + lz * xs[3]))
            M[12 * s:12 * s + 12, 12 * n:12 * n + 12] += Wf[s, k]
    return M
