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


def solve_pairs(dims, c, W64, Wlo, Wlo_prec, n, seed, group=16, tol=1e-10, stream=None, log=None, w64_layout=0,
                delta=0.1):
    """n Gaussian sources (gaussian_source_batches of `seed`, `group` at a time) and their
    solutions; w64_layout is the layout flag of W64, delta the reliable-update threshold.  Returns (xi32, psi32, info): FP32 device
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
        rc, st = ok.ok_bicgstab(dims, c, ok.SolverParams(tol=tol, delta=delta, W64_layout=w64_layout), W64, Wlo, Wlo_prec, d_xi,
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


CHECKPOINT_KEYS = ("params", "adam_m", "adam_v", "step", "n_layers", "steps", "batch", "lr", "history")


def save_checkpoint(path, params, adam_m, adam_v, step, n_layers, steps, batch, lr, history):
    """Write the training state (FP32 parameters and Adam moments as flat host arrays, the last
    completed step and the schedule) to an .npz file; the file is written under a temporary name
    and renamed, so an interrupted save leaves the previous checkpoint intact."""
    import os
    tmp = path + ".tmp.npz"
    np.savez(tmp, params=np.asarray(params, dtype=np.float32), adam_m=np.asarray(adam_m, dtype=np.float32),
             adam_v=np.asarray(adam_v, dtype=np.float32), step=np.int64(step), n_layers=np.int64(n_layers),
             steps=np.int64(steps), batch=np.int64(batch), lr=np.float64(lr),
             history=np.asarray(history, dtype=np.float64).reshape(-1, 2))
    os.replace(tmp, path)


def load_checkpoint(path):
    """The training state written by save_checkpoint (no pickled objects are read)."""
    with np.load(path, allow_pickle=False) as f:
        missing = [k for k in CHECKPOINT_KEYS if k not in f.files]
        if missing:
            raise ValueError("%s is not a training checkpoint (missing %s)" % (path, missing))
        st = {k: f[k] for k in CHECKPOINT_KEYS}
    for k in ("step", "n_layers", "steps", "batch"):
        st[k] = int(st[k])
    st["lr"] = float(st["lr"])
    st["history"] = [(int(a), float(b)) for a, b in st["history"]]
    return st


def train(dims, T, xi32, psi32, n_pairs, scale, n_layers=4, steps=400, batch=16, lr=3e-3, seed=I.SEED_NET,
          log_every=50, stream=None, log=None, checkpoint=None, checkpoint_every=0, resume=None, stop_after=None):
    """Adam on the network parameters over mini-batches of `batch` consecutive pairs, cycled in
    order; the learning rate drops to lr/3 for the second half.  The first layer starts as
    scale * 1 (e.g. 1/mhat), later layers as the identity.  Returns (okinv.Net, history) with
    history a list of (step, mini-batch loss).

    checkpoint: path of an .npz file written every `checkpoint_every` steps and at the end
    (parameters, Adam moments, step, schedule); resume: such a file to continue from (its
    n_layers, steps, batch and lr must match).  The mini-batch order and the learning rate are
    functions of the step and the gradient reductions are in a fixed order, so a resumed run
    repeats the uninterrupted one bit for bit.  stop_after: end after that step (an
    interrupted run, for checkpoint tests)."""
    import torch
    V = I.volume(dims)
    first = 1
    hist = []
    if resume is not None:
        st = load_checkpoint(resume)
        if (st["n_layers"], st["steps"], st["batch"], st["lr"]) != (n_layers, steps, batch, lr):
            raise ValueError("checkpoint %s is for n_layers, steps, batch, lr = %s, not %s"
                             % (resume, (st["n_layers"], st["steps"], st["batch"], st["lr"]),
                                (n_layers, steps, batch, lr)))
        d_p = torch.from_numpy(st["params"]).to("cuda")
        d_m = torch.from_numpy(st["adam_m"]).to("cuda")
        d_v = torch.from_numpy(st["adam_v"]).to("cuda")
        if d_p.numel() != ok.ok_net_param_count(n_layers):
            raise ValueError("checkpoint %s holds %d parameters, not %d"
                             % (resume, d_p.numel(), ok.ok_net_param_count(n_layers)))
        first = st["step"] + 1
        hist = list(st["history"])
    else:
        p0 = I.net_init_params(n_layers, scale, seed)
        d_p = ok.to_device_complex(p0, dtype="float32")
        d_m, d_v = torch.zeros_like(d_p), torch.zeros_like(d_p)
    grad = torch.empty_like(d_p)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    work = ok.empty_bytes(ok.ok_net_workspace_bytes(dims, n_layers, batch, 1))
    nb = max(1, n_pairs // batch)
    fb = batch * V * 24 * 4   # bytes per mini-batch

    def save(step):
        torch.cuda.synchronize()
        save_checkpoint(checkpoint, d_p.cpu().numpy(), d_m.cpu().numpy(), d_v.cpu().numpy(), step, n_layers, steps,
                        batch, lr, hist)

    last = steps if stop_after is None else min(steps, stop_after)
    for step in range(first, last + 1):
        i = (step - 1) % nb
        cfg = ok.adam_cfg(lr=lr if 2 * step <= steps else lr / 3)
        ok.ok_net_train_step(dims, n_layers, d_p, d_m, d_v, T, xi32.data_ptr() + i * fb, psi32.data_ptr() + i * fb,
                             batch, 0, cfg, step, loss, grad, work, stream)
        if step % log_every == 0 or step == 1 or step == steps:
            torch.cuda.synchronize()
            hist.append((step, float(loss.item())))
            if log:
                log("train step %d loss %.4f" % hist[-1])
        if checkpoint and checkpoint_every and step % checkpoint_every == 0 and step != last:
            save(step)
    if checkpoint and last >= first:
        save(last)
    torch.cuda.synchronize()
    if not np.isfinite(hist[-1][1]):
        raise RuntimeError("training diverged: %s" % hist[-5:])
    return ok.Net(n_layers, d_p, T), hist
