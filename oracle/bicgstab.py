"""Plain FP64 BiCGStab (the paper's "bi-stabilized CG", Sec. 2.3).

The paper names the algorithm but prints none of its details; the reading is the
standard unpreconditioned method: x0 = 0 (or a given guess), shadow vector
r^ = r0, <a, b> = sum conj(a) b, and the true residual ||xi - M x|| / ||xi|| as
the stopping criterion.  On a (near) breakdown the recurrence restarts from the
current iterate with r^ = r.
"""
import numpy as np

from .lattice import norm2, vdot


def bicgstab(apply, xi, tol=1e-10, max_iter=10000, x0=None, max_restarts=5):
    """Solve M x = xi.  Returns (x, info) with info = dict(iters, true_rel_resid, history)."""
    xn = np.sqrt(norm2(xi))
    x = np.zeros_like(xi) if x0 is None else x0.copy()
    if xn == 0.0:
        return np.zeros_like(xi), dict(iters=0, true_rel_resid=0.0, history=[], restarts=0)
    r = xi - apply(x) if x0 is not None else xi.copy()
    hist = []
    it = 0
    restarts = 0
    while True:
        rhat = r.copy()
        rho_old = alpha = omega = 1.0
        v = np.zeros_like(xi)
        p = np.zeros_like(xi)
        broke = False
        while it < max_iter:
            rho = vdot(rhat, r)
            if abs(rho) < 1e-30 * norm2(r) or omega == 0.0:
                broke = True
                break
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
            v = apply(p)
            rv = vdot(rhat, v)
            if rv == 0.0:
                broke = True
                break
            alpha = rho / rv
            s = r - alpha * v
            t = apply(s)
            tt = norm2(t)
            omega = vdot(t, s) / tt if tt > 0 else 0.0
            x = x + alpha * p + omega * s
            r = s - omega * t
            rho_old = rho
            it += 1
            rel = np.sqrt(norm2(r)) / xn
            hist.append(rel)
            if rel <= tol:
                break
        true = np.sqrt(norm2(xi - apply(x))) / xn
        if true <= tol or it >= max_iter or restarts >= max_restarts:
            return x, dict(iters=it, true_rel_resid=true, history=hist, restarts=restarts)
        # recurrence drifted or broke down: restart from the true residual
        restarts += 1
        r = xi - apply(x)
