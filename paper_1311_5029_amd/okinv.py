"""ctypes binding of libokinv (the C-ABI in include/okinv.h), same names as the C calls.

Argument marshalling only: every step of the operator and the solver runs in
the HIP library.  Device buffers are torch CUDA (HIP) tensors, passed by
``data_ptr()``; the stream is torch's current stream unless given.  A negative
status raises OkError with the library's message.  Importing this module fails
loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

# torch first: the library then binds to the HIP runtime torch has loaded.  Loaded the other way
# round, the process holds two HIP and two HSA runtimes (the system's for the library, torch's
# own for torch), and the second to open the device finds none (HIP error 100 at the library's
# first launch).
import torch  # noqa: F401,E402

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libokinv.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("libokinv.so is not built (%s); build it with python -m paper_1311_5029_amd.build" % LIB_PATH)
_lib = C.CDLL(LIB_PATH)

OK_F64, OK_F32, OK_BF16 = 0, 1, 2
OK_LAYOUT_SITE = 0x10
OK_LAYOUT_SAVED = 0x100
OK_LAYOUT_SIGMA = 0x200
OK_SPINOR_RHS_INNER = 0x20
OK_NET_ADJOINT = 0x40
OK_NET_MAX_LAYERS = 16
OK_SUCCESS, OK_NOT_CONVERGED, OK_BREAKDOWN = 0, 1, 2
OK_EINVAL, OK_ESIZE, OK_EALIGN, OK_EDEVICE, OK_ENONFINITE = -1, -2, -3, -4, -5
STATUS_NAMES = {0: "OK_SUCCESS", 1: "OK_NOT_CONVERGED", 2: "OK_BREAKDOWN", -1: "OK_EINVAL",
                -2: "OK_ESIZE", -3: "OK_EALIGN", -4: "OK_EDEVICE", -5: "OK_ENONFINITE"}


class ok_geom(C.Structure):
    _fields_ = [("L", C.c_int32 * 4)]


class ok_coeffs(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("mhat", "u0", "zeta", "r_s", "c_B", "c_E", "c_EE", "c_1", "c_2", "c_3", "c_4", "c_5")]


class ok_solver_params(C.Structure):
    _fields_ = [("tol", C.c_double), ("delta", C.c_double), ("max_iter", C.c_int32),
                ("max_restarts", C.c_int32), ("zero_guess", C.c_int32), ("verbose", C.c_int32),
                ("stall_window", C.c_int32), ("W64_layout", C.c_int32)]


class ok_solver_stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("matvec_hi", C.c_int32),
                ("matvec_lo", C.c_int32), ("reliable_updates", C.c_int32), ("restarts", C.c_int32),
                ("net_applies", C.c_int32), ("fallbacks", C.c_int32),
                ("true_rel_resid", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class ok_net(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("reserved", C.c_int32), ("d_params", C.c_void_p), ("d_T", C.c_void_p)]


class ok_adam_cfg(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double)]


_P = C.c_void_p
_NET = C.POINTER(ok_net)
_sig = {
    "ok_abi_version": ([], C.c_int),
    "ok_last_error": ([], C.c_char_p),
    "ok_W_bytes": ([C.POINTER(ok_geom), C.c_int, C.POINTER(C.c_size_t)], C.c_int),
    "ok_precompute_scratch_bytes": ([C.POINTER(ok_geom), C.POINTER(C.c_size_t)], C.c_int),
    "ok_precompute_W": ([C.POINTER(ok_geom), C.POINTER(ok_coeffs), _P, C.c_int, _P, C.c_size_t, _P,
                         C.c_size_t, _P], C.c_int),
    "ok_apply_M": ([C.POINTER(ok_geom), C.POINTER(ok_coeffs), _P, C.c_int, _P, _P, C.c_int, C.c_int, _P],
                   C.c_int),
    "ok_W_to_dense": ([C.POINTER(ok_geom), _P, C.c_int, _P, _P], C.c_int),
    "ok_bicgstab_workspace_bytes": ([C.POINTER(ok_geom), C.c_int, C.c_int, _NET, C.POINTER(C.c_size_t)], C.c_int),
    "ok_bicgstab": ([C.POINTER(ok_geom), C.POINTER(ok_coeffs), C.POINTER(ok_solver_params), _P, _P, C.c_int, _NET,
                     _P, _P, C.c_int, _P, C.c_size_t, C.POINTER(ok_solver_stats), _P], C.c_int),
    "ok_bicgstab_static": ([C.POINTER(ok_geom), C.POINTER(ok_coeffs), C.POINTER(ok_solver_params), _P, _P, C.c_int,
                            _NET, _P, _P, C.c_int, C.POINTER(ok_solver_stats), _P], C.c_int),
    "ok_bicgstab_static_max_bytes": ([], C.c_size_t),
    "ok_cgnr_workspace_bytes": ([C.POINTER(ok_geom), C.c_int, C.POINTER(C.c_size_t)], C.c_int),
    "ok_cgnr": ([C.POINTER(ok_geom), C.POINTER(ok_coeffs), C.POINTER(ok_solver_params), _P, _P, _P, C.c_int, _P,
                 C.c_size_t, C.POINTER(ok_solver_stats), _P], C.c_int),
    "ok_net_param_count": ([C.c_int, C.POINTER(C.c_size_t)], C.c_int),
    "ok_net_transports_bytes": ([C.POINTER(ok_geom), C.POINTER(C.c_size_t)], C.c_int),
    "ok_net_transports": ([C.POINTER(ok_geom), _P, _P, C.c_size_t, _P], C.c_int),
    "ok_net_layer": ([C.POINTER(ok_geom), _P, _P, _P, _P, C.c_int, C.c_int, _P], C.c_int),
    "ok_net_workspace_bytes": ([C.POINTER(ok_geom), C.c_int, C.c_int, C.c_int, C.POINTER(C.c_size_t)], C.c_int),
    "ok_net_apply": ([C.POINTER(ok_geom), _NET, _P, _P, C.c_int, C.c_int, _P, C.c_size_t, _P], C.c_int),
    "ok_net_layer_wgrad": ([C.POINTER(ok_geom), _P, _P, _P, _P, C.c_int, C.c_int, _P, C.c_size_t, _P], C.c_int),
    "ok_net_loss_grad": ([C.POINTER(ok_geom), _P, _P, _P, _P, C.c_int, C.c_int, _P, C.c_size_t, _P], C.c_int),
    "ok_net_loss_and_grad": ([C.POINTER(ok_geom), _NET, _P, _P, C.c_int, C.c_int, _P, _P, _P, C.c_size_t, _P],
                             C.c_int),
    "ok_cast_f64_to_f32": ([_P, _P, C.c_size_t, _P], C.c_int),
    "ok_adam_step": ([_P, _P, _P, _P, C.c_size_t, C.POINTER(ok_adam_cfg), C.c_int, _P], C.c_int),
    "ok_net_train_step": ([C.POINTER(ok_geom), C.c_int, _P, _P, _P, _P, _P, _P, C.c_int, C.c_int,
                           C.POINTER(ok_adam_cfg), C.c_int, _P, _P, _P, C.c_size_t, _P], C.c_int),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_sig)


class OkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def _check(rc):
    if rc < 0:
        raise OkError(rc, ok_last_error())
    return rc


def geom(dims):
    g = ok_geom()
    for i in range(4):
        g.L[i] = int(dims[i])
    return g


def coeffs(c):
    """ok_coeffs from any object with the attributes mhat, u0, zeta, ... (e.g. inputs.OKCoeffs)."""
    out = ok_coeffs()
    for n, _ in ok_coeffs._fields_:
        setattr(out, n, float(getattr(c, n)))
    return out


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _nbytes(t):
    return t.numel() * t.element_size()


def _stream(stream):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def ok_abi_version():
    return _lib.ok_abi_version()


def ok_last_error():
    return _lib.ok_last_error().decode()


def ok_W_bytes(dims, prec):
    n = C.c_size_t()
    _check(_lib.ok_W_bytes(C.byref(geom(dims)), prec, C.byref(n)))
    return n.value


def ok_precompute_scratch_bytes(dims):
    n = C.c_size_t()
    _check(_lib.ok_precompute_scratch_bytes(C.byref(geom(dims)), C.byref(n)))
    return n.value


def ok_precompute_W(dims, c, d_links, prec, d_W, d_scratch, stream=None):
    return _check(_lib.ok_precompute_W(C.byref(geom(dims)), C.byref(coeffs(c)), _ptr(d_links), prec,
                                       _ptr(d_W), _nbytes(d_W), _ptr(d_scratch), _nbytes(d_scratch),
                                       _stream(stream)))


def ok_apply_M(dims, c, d_W, W_prec, d_psi, d_out, spinor_prec, nrhs=1, stream=None):
    return _check(_lib.ok_apply_M(C.byref(geom(dims)), C.byref(coeffs(c)), _ptr(d_W), W_prec, _ptr(d_psi),
                                  _ptr(d_out), spinor_prec, nrhs, _stream(stream)))


def ok_W_to_dense(dims, d_W, prec, d_dense, stream=None):
    return _check(_lib.ok_W_to_dense(C.byref(geom(dims)), _ptr(d_W), prec, _ptr(d_dense), _stream(stream)))


def ok_bicgstab_workspace_bytes(dims, nrhs, Wlo_prec=-1, net=None):
    n = C.c_size_t()
    _check(_lib.ok_bicgstab_workspace_bytes(C.byref(geom(dims)), nrhs, Wlo_prec, _netp(net), C.byref(n)))
    return n.value


@dataclasses.dataclass
class SolverParams:
    tol: float = 1e-10
    delta: float = 0.1
    max_iter: int = 10000
    max_restarts: int = 5
    zero_guess: int = 1
    verbose: int = 0
    stall_window: int = 0
    W64_layout: int = 0

    def c(self):
        return ok_solver_params(self.tol, self.delta, self.max_iter, self.max_restarts,
                                self.zero_guess, self.verbose, self.stall_window, self.W64_layout)


def ok_bicgstab(dims, c, params, d_W64, d_Wlo, Wlo_prec, d_xi, d_psi, nrhs, d_work, stream=None, net=None):
    """Returns (status, [stats dict per right-hand side]).  net: Net or None."""
    stats = (ok_solver_stats * nrhs)()
    p = params.c() if isinstance(params, SolverParams) else params
    rc = _lib.ok_bicgstab(C.byref(geom(dims)), C.byref(coeffs(c)), C.byref(p), _ptr(d_W64), _ptr(d_Wlo),
                          Wlo_prec, _netp(net), _ptr(d_xi), _ptr(d_psi), nrhs, _ptr(d_work), _nbytes(d_work),
                          stats, _stream(stream))
    _check(rc)
    return rc, [s.as_dict() for s in stats]


def ok_bicgstab_static(dims, c, params, d_W64, d_Wlo, Wlo_prec, d_xi, d_psi, nrhs, stream=None, net=None):
    """ok_bicgstab on the library's fixed per-GPU workspace (no device allocation)."""
    stats = (ok_solver_stats * nrhs)()
    p = params.c() if isinstance(params, SolverParams) else params
    rc = _lib.ok_bicgstab_static(C.byref(geom(dims)), C.byref(coeffs(c)), C.byref(p), _ptr(d_W64), _ptr(d_Wlo),
                                 Wlo_prec, _netp(net), _ptr(d_xi), _ptr(d_psi), nrhs, stats, _stream(stream))
    _check(rc)
    return rc, [s.as_dict() for s in stats]


def ok_bicgstab_static_max_bytes():
    return _lib.ok_bicgstab_static_max_bytes()


def ok_cgnr_workspace_bytes(dims, nrhs):
    n = C.c_size_t()
    _check(_lib.ok_cgnr_workspace_bytes(C.byref(geom(dims)), nrhs, C.byref(n)))
    return n.value


def ok_cgnr(dims, c, params, d_W64, d_xi, d_psi, nrhs, d_work, stream=None):
    """CG on M^dag M (FP64); returns (status, [stats dict per right-hand side])."""
    stats = (ok_solver_stats * nrhs)()
    p = params.c() if isinstance(params, SolverParams) else params
    rc = _lib.ok_cgnr(C.byref(geom(dims)), C.byref(coeffs(c)), C.byref(p), _ptr(d_W64), _ptr(d_xi), _ptr(d_psi),
                      nrhs, _ptr(d_work), _nbytes(d_work), stats, _stream(stream))
    _check(rc)
    return rc, [s.as_dict() for s in stats]


# --------------------------------------------------------------------------- learned preconditioner
@dataclasses.dataclass
class Net:
    """n_layers and the device tensors of its parameters and transports (kept alive by this object)."""
    n_layers: int
    params: object
    T: object

    def c(self):
        return ok_net(self.n_layers, 0, _ptr(self.params), _ptr(self.T))


def _netp(net):
    if net is None:
        return None
    n = net.c() if isinstance(net, Net) else net
    return C.pointer(n)


def ok_net_param_count(n_layers):
    n = C.c_size_t()
    _check(_lib.ok_net_param_count(n_layers, C.byref(n)))
    return n.value


def ok_net_transports_bytes(dims):
    n = C.c_size_t()
    _check(_lib.ok_net_transports_bytes(C.byref(geom(dims)), C.byref(n)))
    return n.value


def ok_net_transports(dims, d_links, d_T, stream=None):
    return _check(_lib.ok_net_transports(C.byref(geom(dims)), _ptr(d_links), _ptr(d_T), _nbytes(d_T),
                                         _stream(stream)))


def ok_net_layer(dims, d_A, d_T, d_in, d_out, nfields, flags=0, stream=None):
    return _check(_lib.ok_net_layer(C.byref(geom(dims)), _ptr(d_A), _ptr(d_T), _ptr(d_in), _ptr(d_out), nfields,
                                    flags, _stream(stream)))


def ok_net_workspace_bytes(dims, n_layers, nfields, training):
    n = C.c_size_t()
    _check(_lib.ok_net_workspace_bytes(C.byref(geom(dims)), n_layers, nfields, training, C.byref(n)))
    return n.value


def ok_net_apply(dims, net, d_in, d_out, nfields, flags, d_work, stream=None):
    return _check(_lib.ok_net_apply(C.byref(geom(dims)), _netp(net), _ptr(d_in), _ptr(d_out), nfields, flags,
                                    _ptr(d_work), _nbytes(d_work) if d_work is not None else 0, _stream(stream)))


def ok_net_layer_wgrad(dims, d_T, d_gout, d_in, d_gA, nfields, flags, d_work, stream=None):
    return _check(_lib.ok_net_layer_wgrad(C.byref(geom(dims)), _ptr(d_T), _ptr(d_gout), _ptr(d_in), _ptr(d_gA),
                                          nfields, flags, _ptr(d_work), _nbytes(d_work), _stream(stream)))


def ok_net_loss_grad(dims, d_out, d_psi, d_gout, d_loss, nfields, flags, d_work, stream=None):
    return _check(_lib.ok_net_loss_grad(C.byref(geom(dims)), _ptr(d_out), _ptr(d_psi), _ptr(d_gout),
                                        _ptr(d_loss), nfields, flags, _ptr(d_work), _nbytes(d_work),
                                        _stream(stream)))


def ok_net_loss_and_grad(dims, net, d_xi, d_psi, nfields, flags, d_loss, d_grad, d_work, stream=None):
    return _check(_lib.ok_net_loss_and_grad(C.byref(geom(dims)), _netp(net), _ptr(d_xi), _ptr(d_psi), nfields,
                                            flags, _ptr(d_loss), _ptr(d_grad), _ptr(d_work), _nbytes(d_work),
                                            _stream(stream)))


def ok_cast_f64_to_f32(d_in, d_out, n, stream=None):
    return _check(_lib.ok_cast_f64_to_f32(_ptr(d_in), _ptr(d_out), n, _stream(stream)))


def adam_cfg(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    return ok_adam_cfg(lr, beta1, beta2, eps)


def ok_adam_step(d_p, d_g, d_m, d_v, n, cfg, step, stream=None):
    return _check(_lib.ok_adam_step(_ptr(d_p), _ptr(d_g), _ptr(d_m), _ptr(d_v), n, C.byref(cfg), step,
                                    _stream(stream)))


def ok_net_train_step(dims, n_layers, d_params, d_m, d_v, d_T, d_xi, d_psi, nfields, flags, cfg, step, d_loss,
                      d_grad, d_work, stream=None):
    return _check(_lib.ok_net_train_step(C.byref(geom(dims)), n_layers, _ptr(d_params), _ptr(d_m), _ptr(d_v),
                                         _ptr(d_T), _ptr(d_xi), _ptr(d_psi), nfields, flags, C.byref(cfg), step,
                                         _ptr(d_loss), _ptr(d_grad), _ptr(d_work), _nbytes(d_work),
                                         _stream(stream)))


# --------------------------------------------------------------------------- plumbing
def to_device_complex(a, dtype="float64", device="cuda"):
    """NumPy complex array -> contiguous torch tensor of interleaved (re, im) reals on the device."""
    import torch
    a = np.ascontiguousarray(a)
    real = np.ascontiguousarray(a.view(np.float64) if a.dtype == np.complex128
                                else a.astype(np.complex128).view(np.float64))
    t = torch.from_numpy(real)
    if dtype == "float32":
        t = t.to(torch.float32)
    return t.to(device)


def to_host_complex(t, shape=None):
    """torch tensor of interleaved (re, im) -> NumPy complex128 (optionally reshaped)."""
    a = t.detach().to("cpu").double().numpy()
    z = a.reshape(-1, 2)
    out = z[:, 0] + 1j * z[:, 1]
    return out.reshape(shape) if shape is not None else out


def empty_bytes(n, device="cuda"):
    """A device buffer of n bytes (256-byte granularity), as a uint8 tensor."""
    import torch
    return torch.empty(max(256, (n + 255) // 256 * 256), dtype=torch.uint8, device=device)
