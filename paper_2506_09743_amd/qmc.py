"""Python binding of libqmc's C ABI (``include/qmc.h``).

Argument marshalling only: tensors become device pointers, the current torch
stream becomes the ``hipStream_t``, and every status code other than QMC_OK
raises.  All arithmetic runs in the HIP kernels; there is no fallback, so a
missing ``libqmc.so`` is an error, not a slower path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqmc.so")

QMC_OK, QMC_EINVAL, QMC_ENOMEM, QMC_EDEVICE, QMC_EUNSUPPORTED, QMC_ENONFINITE = 0, -1, -2, -3, -4, -5
QMC_FP64, QMC_MIXED_FP32, QMC_MIXED_BF16, QMC_MIXED_BF16_X1, QMC_FP64_EXPLICIT = 0, 1, 2, 3, 4
QMC_STO, QMC_GTO = 0, 1
PRECISIONS = {"fp64": QMC_FP64, "fp32": QMC_MIXED_FP32, "bf16": QMC_MIXED_BF16,
              "bf16x1": QMC_MIXED_BF16_X1, "fp64_explicit": QMC_FP64_EXPLICIT}

# every symbol include/qmc.h declares
EXPORTS = ("qmc_system_create", "qmc_system_destroy", "qmc_eval_psi_eloc", "qmc_metropolis_block",
           "qmc_grad", "qmc_eval_eloc_fd", "qmc_param_count", "qmc_bytes_per_walker",
           "qmc_reduce_accumulators", "qmc_status_string")
# columns of the Metropolis accumulators [W][ACC_COLS]: sum E_L, sum E_L^2,
# accepted steps, steps whose state had no finite log|Psi| or E_L
ACC_COLS = 4

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class QmcError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status_string(status)} ({status})")
        self.status = status


class qmc_system_desc(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int32), ("Z", _dp), ("R", _dp),
        ("n_up", C.c_int32), ("n_dn", C.c_int32), ("basis", C.c_int32),
        ("n_shells", C.c_int32), ("shell_atom", _ip), ("shell_l", _ip), ("shell_kn", _ip),
        ("shell_nprim", _ip), ("prim_exp", _dp), ("prim_coef", _dp), ("normalize", C.c_int32),
        ("n_mo", C.c_int32), ("mo_coef", _dp), ("n_det", C.c_int32), ("occ_up", _ip),
        ("occ_dn", _ip), ("ci", _dp), ("jas_a_par", C.c_double), ("jas_a_anti", C.c_double),
        ("jas_b", C.c_double), ("jas_en", _dp), ("jas_een_n", C.c_int32), ("jas_een", _dp),
        ("bf_omega", C.c_double),
    ]


_lib = None


def lib():
    """Loads libqmc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2506_09743_amd.build` (there is no fallback)")
        L = C.CDLL(LIB_PATH)
        L.qmc_system_create.argtypes = [C.POINTER(qmc_system_desc), C.c_int32, C.POINTER(C.c_void_p)]
        L.qmc_system_create.restype = C.c_int
        L.qmc_system_destroy.argtypes = [C.c_void_p]
        L.qmc_system_destroy.restype = None
        L.qmc_eval_psi_eloc.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p]
        L.qmc_eval_psi_eloc.restype = C.c_int
        L.qmc_metropolis_block.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_uint64,
                                           C.c_uint64, C.c_uint32, C.c_void_p, C.c_void_p]
        L.qmc_metropolis_block.restype = C.c_int
        L.qmc_grad.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p]
        L.qmc_grad.restype = C.c_int
        L.qmc_eval_eloc_fd.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_void_p,
                                       C.c_void_p, C.c_void_p]
        L.qmc_eval_eloc_fd.restype = C.c_int
        L.qmc_param_count.argtypes = [C.c_void_p]
        L.qmc_param_count.restype = C.c_int64
        L.qmc_bytes_per_walker.argtypes = [C.c_void_p, C.c_int32]
        L.qmc_bytes_per_walker.restype = C.c_size_t
        L.qmc_reduce_accumulators.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.qmc_reduce_accumulators.restype = C.c_int
        L.qmc_status_string.argtypes = [C.c_int]
        L.qmc_status_string.restype = C.c_char_p
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().qmc_status_string(int(status)).decode()


def _check(status: int, where: str):
    if status != QMC_OK:
        raise QmcError(status, where)


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def make_desc(sysd: dict):
    """qmc_system_desc from a system dict; returns (desc, keep-alive arrays)."""
    keep = {}

    def f64(k):
        keep[k] = np.ascontiguousarray(np.asarray(sysd[k], dtype=np.float64))
        return _ptr(keep[k], _dp)

    def i32(k):
        keep[k] = np.ascontiguousarray(np.asarray(sysd[k], dtype=np.int32))
        return _ptr(keep[k], _ip)

    d = qmc_system_desc()
    d.n_atoms = len(sysd["Z"])
    d.Z, d.R = f64("Z"), f64("R")
    d.n_up, d.n_dn = int(sysd["n_up"]), int(sysd["n_dn"])
    d.basis = QMC_STO if sysd["basis"] == "sto" else QMC_GTO
    d.n_shells = len(sysd["shell_l"])
    d.shell_atom, d.shell_l, d.shell_kn, d.shell_nprim = (
        i32("shell_atom"), i32("shell_l"), i32("shell_kn"), i32("shell_nprim"))
    d.prim_exp, d.prim_coef = f64("prim_exp"), f64("prim_coef")
    d.normalize = int(sysd.get("normalize", 1))
    d.n_mo = int(np.asarray(sysd["mo_coef"]).shape[1])
    d.mo_coef = f64("mo_coef")
    d.n_det = len(sysd["ci"])
    d.occ_up = i32("occ_up") if d.n_up > 0 else None
    d.occ_dn = i32("occ_dn") if d.n_dn > 0 else None
    d.ci = f64("ci")
    d.jas_a_par = float(sysd.get("jas_a_par", 0.25))
    d.jas_a_anti = float(sysd.get("jas_a_anti", 0.5))
    d.jas_b = float(sysd.get("jas_b", 1.0))
    if sysd.get("jas_en") is not None:
        d.jas_en = f64("jas_en")
    een = sysd.get("jas_een")
    if een is not None and len(een) > 0:
        d.jas_een_n = int(np.asarray(een).shape[0])
        d.jas_een = f64("jas_een")
    d.bf_omega = float(sysd.get("bf_omega") or 0.0)
    return d, keep


# ---- same-named wrappers of the C entry points ------------------------------------

def qmc_system_create(sysd: dict, device: int = 0) -> C.c_void_p:
    desc, _keep = make_desc(sysd)
    h = C.c_void_p()
    _check(lib().qmc_system_create(C.byref(desc), int(device), C.byref(h)), "qmc_system_create")
    return h


def qmc_system_destroy(handle) -> None:
    lib().qmc_system_destroy(handle)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, name, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


def qmc_eval_psi_eloc(handle, precision: int, X, logpsi, sign, eloc) -> None:
    W = X.shape[0]
    _check(lib().qmc_eval_psi_eloc(handle, int(precision), _dev_ptr(X, "X"), W,
                                   _dev_ptr(logpsi, "logpsi", (W,)), _dev_ptr(sign, "sign", (W,)),
                                   _dev_ptr(eloc, "eloc", (W,)), _stream()), "qmc_eval_psi_eloc")


def qmc_metropolis_block(handle, precision: int, X, logpsi, sign, eloc, n_steps: int, sigma: float,
                         seed: int, step0: int, walker_offset: int, acc) -> None:
    W = X.shape[0]
    _check(lib().qmc_metropolis_block(handle, int(precision), _dev_ptr(X, "X"),
                                      _dev_ptr(logpsi, "logpsi", (W,)), _dev_ptr(sign, "sign", (W,)),
                                      _dev_ptr(eloc, "eloc", (W,)), W, int(n_steps), float(sigma),
                                      C.c_uint64(seed), C.c_uint64(step0), C.c_uint32(walker_offset),
                                      _dev_ptr(acc, "acc", (W, ACC_COLS)), _stream()), "qmc_metropolis_block")


def qmc_eval_eloc_fd(handle, X, h: float, logpsi, eloc) -> None:
    W = X.shape[0]
    _check(lib().qmc_eval_eloc_fd(handle, _dev_ptr(X, "X"), W, float(h), _dev_ptr(logpsi, "logpsi", (W,)),
                                  _dev_ptr(eloc, "eloc", (W,)), _stream()), "qmc_eval_eloc_fd")


def qmc_grad(handle, X, dlogpsi=None, deloc_dtheta=None, dlogpsi_dR=None, deloc_dR=None,
             precision: int = QMC_FP64) -> None:
    W = X.shape[0]

    def opt(t, name):
        return _dev_ptr(t, name) if t is not None else None

    _check(lib().qmc_grad(handle, precision, _dev_ptr(X, "X"), W, opt(dlogpsi, "dlogpsi"),
                          opt(deloc_dtheta, "deloc_dtheta"), opt(dlogpsi_dR, "dlogpsi_dR"),
                          opt(deloc_dR, "deloc_dR"), _stream()), "qmc_grad")


def qmc_param_count(handle) -> int:
    return int(lib().qmc_param_count(handle))


def qmc_bytes_per_walker(handle, precision: int = QMC_FP64) -> int:
    return int(lib().qmc_bytes_per_walker(handle, int(precision)))


def qmc_reduce_accumulators(acc, out) -> None:
    """out[5] (device) = column sums of acc [W][4] and the number of walkers
    with non-finite steps, in an order fixed by W."""
    W = acc.shape[0]
    _check(lib().qmc_reduce_accumulators(_dev_ptr(acc, "acc", (W, ACC_COLS)), W, _dev_ptr(out, "out", (5,)),
                                         _stream()), "qmc_reduce_accumulators")


# ---- convenience object ------------------------------------------------------------

class System:
    """Device-resident system; thin owner of a qmc_system handle."""

    def __init__(self, sysd: dict, device: int = 0):
        self.sysd = sysd
        self.device = device
        self.n_elec = int(sysd["n_up"]) + int(sysd["n_dn"])
        self.n_atoms = len(sysd["Z"])
        self.handle = qmc_system_create(sysd, device)

    def close(self):
        if getattr(self, "handle", None) is not None:
            qmc_system_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def param_count(self) -> int:
        return qmc_param_count(self.handle)

    def bytes_per_walker(self, precision="fp64") -> int:
        return qmc_bytes_per_walker(self.handle, PRECISIONS[precision])

    def _walkers(self, X):
        """X must be [W][N_e][3]: the kernels read N_e * 3 doubles per walker."""
        if X.dim() != 3 or X.shape[1] != self.n_elec or X.shape[2] != 3:
            raise ValueError(f"X has shape {tuple(X.shape)}, expected (W, {self.n_elec}, 3)")
        return X.shape[0]

    def eval(self, X, precision="fp64"):
        import torch
        W = self._walkers(X)
        out = [torch.empty(W, dtype=torch.float64, device=X.device) for _ in range(3)]
        qmc_eval_psi_eloc(self.handle, PRECISIONS[precision], X, *out)
        return tuple(out)

    def eval_fd(self, X, h: float = 1e-3):
        """log|Psi| and E_L with the kinetic energy from central differences of
        Psi (step h); returns (logpsi, eloc)."""
        import torch
        out = [torch.empty(self._walkers(X), dtype=torch.float64, device=X.device) for _ in range(2)]
        qmc_eval_eloc_fd(self.handle, X, h, *out)
        return tuple(out)

    def grad(self, X, precision="fp64"):
        """(d log|Psi|/d theta [W,P], d E_L/d theta [W,P], d log|Psi|/d R [W,A,3],
        d E_L/d R [W,A,3]), FP64 outputs; precision "fp64" or "fp32" (the
        forward evaluation's AO values and MO value contraction in FP32)."""
        import torch
        W, P, A = self._walkers(X), self.param_count, self.n_atoms
        out = [torch.empty((W, P), dtype=torch.float64, device=X.device),
               torch.empty((W, P), dtype=torch.float64, device=X.device),
               torch.empty((W, A, 3), dtype=torch.float64, device=X.device),
               torch.empty((W, A, 3), dtype=torch.float64, device=X.device)]
        qmc_grad(self.handle, X, *out, precision=PRECISIONS[precision])
        return tuple(out)

    def metropolis(self, X, logpsi, sign, eloc, n_steps, sigma, seed, step0=0, walker_offset=0,
                   acc=None, precision="fp64"):
        """In place on X, logpsi, sign, eloc, acc; returns acc."""
        import torch
        self._walkers(X)
        if acc is None:
            acc = torch.zeros((X.shape[0], ACC_COLS), dtype=torch.float64, device=X.device)
        qmc_metropolis_block(self.handle, PRECISIONS[precision], X, logpsi, sign, eloc, n_steps,
                             sigma, seed, step0, walker_offset, acc)
        return acc
