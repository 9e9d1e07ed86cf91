"""Training the learned preconditioner on the GPU, through the C-ABI.

Pairs (xi, psi = M^-1 xi) come from ok_bicgstab (FP64 true residual <= tol) and
are cast to the network's FP32 fields by ok_cast_f64_to_f32; every training
step (forward, loss, backward, Adam) is one ok_net_train_step.  This module
only sequences the calls and owns the device buffers (torch allocations).
"""
from __future__ import annotations

import time

import numpy as np

from . import inputs as I
from . import okinv as ok


def solve_pairs(dims, c, W64, Wlo, Wlo_prec, n, seed, group=16, tol=1e-10, stream=None, log=None, w64_layout=0):
    """n Gaussian sources (gaussian_source_batches of `seed`, `group` at a time) and their
    solutions; w64_layout is the layout flag of W64.  Returns (xi32, psi32, info): FP32 device
    fields [n][V][4][3] complex as flat float tensors, and totals of the solves."""
    import torch
    V = I.volume(dims)
    xi32 = torch.empty(n * V * 24, dtype=torch.float32, device="cuda")
    psi32 = torch.empty_like(xi32)
    work = ok.empty_bytes(ok.ok_bicgstab_workspace_bytes(dims, group, Wlo_prec))
    info = {"sources": n, "iterations": 0, "seconds": 0.0, "max_true_rel_resid": 0.0}
    k0 = 0
    for xi in I.gaussian_source_batches(dims, n, seed, group):
        nb = xi.shape[0]
        d_xi = ok.to_device_complex(xi)
        psi = torch.zeros_like(d_xi)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, st = ok.ok_bicgstab(dims, c, ok.SolverParams(tol=tol, W64_layout=w64_layout), W64, Wlo, Wlo_prec, d_xi,
                                psi, nb, work, stream)
        torch.cuda.synchronize()
        info["seconds"] += time.perf_counter() - t
        if rc != ok.OK_SUCCESS:
            raise RuntimeError("training-pair solve failed: %s" % st)
        info["iterations"] += sum(s["iterations"] for s in st)
        info["max_true_rel_resid"] = max(info["max_true_rel_resid"], max(s["true_rel_resid"] for s in st))
        off = k0 * V * 24
        ok.ok_cast_f64_to_f32(d_xi, xi32[off:off + nb * V * 24], nb * V * 24, stream)
        ok.ok_cast_f64_to_f32(psi, psi32[off:off + nb * V * 24], nb * V * 24, stream)
        k0 += nb
        if log:
            log("pairs %d/%d (%.1fs of solves)" % (k0, n, info["seconds"]))
    torch.cuda.synchronize()
    return xi32, psi32, info


def train(dims, T, xi32, psi32, n_pairs, scale, n_layers=4, steps=400, batch=16, lr=3e-3, seed=I.SEED_NET,
          log_every=50, stream=None, log=None):
    """Adam on the network parameters over mini-batches of `batch` consecutive pairs, cycled in
    order; the learning rate drops to lr/3 for the second half.  The first layer starts as
    scale * 1 (e.g. 1/mhat), later layers as the identity.  Returns (okinv.Net, history) with
    history a list of (step, mini-batch loss)."""
    import torch
    V = I.volume(dims)
    p0 = I.net_init_params(n_layers, scale, seed)
    d_p = ok.to_device_complex(p0, dtype="float32")
    d_m, d_v = torch.zeros_like(d_p), torch.zeros_like(d_p)
    grad = torch.empty_like(d_p)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    work = ok.empty_bytes(ok.ok_net_workspace_bytes(dims, n_layers, batch, 1))
    nb = max(1, n_pairs // batch)
    fb = batch * V * 24 * 4   # bytes per mini-batch
    hist = []
    for step in range(1, steps + 1):
        i = (step - 1) % nb
        cfg = ok.adam_cfg(lr=lr if 2 * step <= steps else lr / 3)
        ok.ok_net_train_step(dims, n_layers, d_p, d_m, d_v, T, xi32.data_ptr() + i * fb, psi32.data_ptr() + i * fb,
                             batch, 0, cfg, step, loss, grad, work, stream)
        if step % log_every == 0 or step == 1 or step == steps:
            torch.cuda.synchronize()
            hist.append((step, float(loss.item())))
            if log:
                log("train step %d loss %.4f" % hist[-1])
    torch.cuda.synchronize()
    if not np.isfinite(hist[-1][1]):
        raise RuntimeError("training diverged: %s" % hist[-5:])
    return ok.Net(n_layers, d_p, T), hist
