"""ctypes binding of the FP64 CPU oracle (``oracle/oracle.c``).

Test infrastructure only: the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it; the product path (the HIP library and its binding)
never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "oracle.c")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def compile_library(src: str, out: str) -> str:
    """gcc, OpenMP, no fast-math, no FMA contraction."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-I", _HERE, "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB_PATH):
        compile_library(SRC, LIB_PATH)
    return LIB_PATH


class _System(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int), ("Z", _dp), ("R", _dp),
        ("n_up", C.c_int), ("n_dn", C.c_int), ("basis", C.c_int),
        ("n_shells", C.c_int), ("shell_atom", _ip), ("shell_l", _ip), ("shell_kn", _ip),
        ("shell_nprim", _ip), ("prim_exp", _dp), ("prim_coef", _dp), ("normalize", C.c_int),
        ("n_mo", C.c_int), ("mo_coef", _dp), ("n_det", C.c_int), ("occ_up", _ip), ("occ_dn", _ip),
        ("ci", _dp), ("a_par", C.c_double), ("a_anti", C.c_double), ("b", C.c_double),
        ("en", _dp), ("een_n", C.c_int), ("een", _dp), ("bf_omega", C.c_double),
    ]


class _Detail(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("logpsi", "sign", "eloc", "e_kin", "e_pot", "jastrow", "log_sigma")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
            build()
        _lib = load_library(LIB_PATH)
    return _lib


def load_library(path: str):
    """Load an oracle build (the default one, or a test's variant)."""
    L = C.CDLL(path)
    L.or_n_ao.restype = C.c_int
    L.or_nuclear_repulsion.restype = C.c_double
    L.or_max_threads.restype = C.c_int
    L.or_ao.argtypes = [C.c_void_p, _dp, _dp]
    L.or_mo.argtypes = [C.c_void_p, _dp, _dp]
    L.or_ao_hessian.argtypes = [C.c_void_p, _dp, _dp]
    L.or_backflow.argtypes = [C.c_void_p, _dp, _dp]
    L.or_eval_one.argtypes = [C.c_void_p, _dp, C.c_void_p, _dp]
    L.or_eval.argtypes = [C.c_void_p, _dp, C.c_int64, _dp, _dp, _dp, C.c_int]
    L.or_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                   C.POINTER(C.c_uint32)]
    L.or_proposal.argtypes = [C.c_int, C.c_uint64, C.c_uint32, C.c_uint64, _dp, _dp]
    L.or_metropolis.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, C.c_int64, C.c_int,
                                C.c_double, C.c_uint64, C.c_uint64, C.c_uint32, _dp,
                                C.POINTER(C.c_uint8), C.c_int]
    return L


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


class OracleSystem:
    """Holds the C descriptor and keeps its arrays alive."""

    def __init__(self, sysd: dict, L=None):
        self.L = lib() if L is None else L
        self.d = sysd
        keep = {}

        def f64(k):
            keep[k] = np.ascontiguousarray(np.asarray(sysd[k], dtype=np.float64))
            return _p(keep[k])

        def i32(k):
            keep[k] = np.ascontiguousarray(np.asarray(sysd[k], dtype=np.int32))
            return _p(keep[k], _ip)

        s = _System()
        s.n_atoms = len(sysd["Z"])
        s.Z = f64("Z")
        s.R = f64("R")
        s.n_up = int(sysd["n_up"])
        s.n_dn = int(sysd["n_dn"])
        s.basis = 0 if sysd["basis"] == "sto" else 1
        s.n_shells = len(sysd["shell_l"])
        s.shell_atom, s.shell_l, s.shell_kn, s.shell_nprim = (
            i32("shell_atom"), i32("shell_l"), i32("shell_kn"), i32("shell_nprim"))
        s.prim_exp = f64("prim_exp")
        s.prim_coef = f64("prim_coef")
        s.normalize = int(sysd.get("normalize", 1))
        s.n_mo = int(np.asarray(sysd["mo_coef"]).shape[1])
        s.mo_coef = f64("mo_coef")
        s.n_det = len(sysd["ci"])
        s.occ_up = i32("occ_up")
        s.occ_dn = i32("occ_dn")
        s.ci = f64("ci")
        s.a_par = float(sysd.get("jas_a_par", 0.25))
        s.a_anti = float(sysd.get("jas_a_anti", 0.5))
        s.b = float(sysd.get("jas_b", 1.0))
        if sysd.get("jas_en") is not None:
            s.en = f64("jas_en")
        een = sysd.get("jas_een")
        if een is not None and len(een) > 0:
            s.een_n = int(np.asarray(een).shape[0])
            s.een = f64("jas_een")
        s.bf_omega = float(sysd.get("bf_omega") or 0.0)
        self._keep = keep
        self.s = s
        self.ref = C.byref(s)
        self.n_elec = s.n_up + s.n_dn
        self.n_ao = self.L.or_n_ao(self.ref)
        self.n_mo = s.n_mo

    # --- single-point helpers -------------------------------------------------
    def ao(self, r) -> np.ndarray:
        r = np.ascontiguousarray(np.asarray(r, dtype=np.float64).reshape(3))
        out = np.zeros((self.n_ao, 5))
        self.L.or_ao(self.ref, _p(r), _p(out))
        return out

    def ao_hessian(self, r) -> np.ndarray:
        """[n_ao][10]: value, dx, dy, dz, xx, xy, xz, yy, yz, zz."""
        r = np.ascontiguousarray(np.asarray(r, dtype=np.float64).reshape(3))
        out = np.zeros((self.n_ao, 10))
        self.L.or_ao_hessian(self.ref, _p(r), _p(out))
        return out

    def backflow(self, x) -> np.ndarray:
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(self.n_elec, 3))
        out = np.zeros((self.n_elec, 3))
        self.L.or_backflow(self.ref, _p(x), _p(out))
        return out

    def mo(self, x) -> np.ndarray:
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(self.n_elec, 3))
        out = np.zeros((self.n_elec, 5, self.n_mo))
        self.L.or_mo(self.ref, _p(x), _p(out))
        return out

    def eval_one(self, x, want_grad: bool = False):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(self.n_elec, 3))
        d = _Detail()
        g = np.zeros((self.n_elec, 3)) if want_grad else None
        self.L.or_eval_one(self.ref, _p(x), C.byref(d), _p(g) if want_grad else None)
        out = {k: getattr(d, k) for k, _ in _Detail._fields_}
        if want_grad:
            out["grad"] = g
        return out

    def nuclear_repulsion(self) -> float:
        return self.L.or_nuclear_repulsion(self.ref)

    # --- batch ----------------------------------------------------------------
    def eval(self, X, nthreads: int = 0):
        X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
        W = X.shape[0]
        lp, sg, el = np.zeros(W), np.zeros(W), np.zeros(W)
        self.L.or_eval(self.ref, _p(X), W, _p(lp), _p(sg), _p(el), nthreads)
        return lp, sg, el

    def metropolis(self, X, logpsi, sign, eloc, n_steps, sigma, seed, step0=0,
                   walker_offset=0, acc=None, want_log=False, nthreads: int = 0):
        """Runs in place on copies; returns (X, logpsi, sign, eloc, acc, log)."""
        X = np.array(X, dtype=np.float64, order="C", copy=True)
        lp = np.array(logpsi, dtype=np.float64, copy=True)
        sg = np.array(sign, dtype=np.float64, copy=True)
        el = np.array(eloc, dtype=np.float64, copy=True)
        W = X.shape[0]
        acc = np.zeros((W, 4)) if acc is None else np.array(acc, dtype=np.float64, copy=True)
        log = np.zeros((n_steps, W), dtype=np.uint8) if want_log else None
        self.L.or_metropolis(self.ref, _p(X), _p(lp), _p(sg), _p(el), W, int(n_steps),
                            float(sigma), C.c_uint64(seed), C.c_uint64(step0),
                            C.c_uint32(walker_offset), _p(acc),
                            _p(log, C.POINTER(C.c_uint8)) if want_log else None, nthreads)
        return X, lp, sg, el, acc, log


def philox(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def proposal(n_elec: int, seed: int, walker_id: int, step: int):
    z = np.zeros((n_elec, 3))
    u = C.c_double()
    lib().or_proposal(n_elec, C.c_uint64(seed), C.c_uint32(walker_id), C.c_uint64(step),
                      _p(z), C.byref(u))
    return z, u.value


def max_threads() -> int:
    return lib().or_max_threads()
