"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (a dropped
factor, a wrong sign, a transposed index, a wrong constant), builds that copy
on the CPU, and checks that a named pin rejects it while the real oracle
passes the same pin.  Nothing here touches the HIP path.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2506_09743_amd import synth

SRC = open(oracle.SRC).read()
rng = np.random.default_rng(5)


def _sys(L, d):
    return oracle.OracleSystem(d, L=L)


def pin_he_closed_form(L):
    Z, zeta, a, b = 2.0, 1.7, 0.5, 0.8
    o = _sys(L, synth.single_atom(Z, zeta, n_up=1, n_dn=1, a_par=0.25, a_anti=a, b=b))
    for _ in range(8):
        x = rng.standard_normal((2, 3))
        r1, r2 = np.linalg.norm(x[0]), np.linalg.norm(x[1])
        d = x[0] - x[1]
        r12 = np.linalg.norm(d)
        k1 = a / (1 + b * r12) ** 2
        k2 = -2 * a * b / (1 + b * r12) ** 3
        ref = (-zeta ** 2 + (zeta - Z) * (1 / r1 + 1 / r2) - k2 - 2 * k1 / r12 - k1 ** 2
               + zeta * k1 * np.dot(x[0] / r1 - x[1] / r2, d / r12) + 1 / r12)
        if abs(o.eval_one(x)["eloc"] - ref) > 1e-10 * max(1, abs(ref)):
            return False
    return True


def pin_hydrogenic(L):
    for Z in (1.0, 3.0):
        o = _sys(L, synth.single_atom(Z, Z))
        for p in rng.standard_normal((8, 3)):
            if abs(o.eval_one(p)["eloc"] + 0.5 * Z * Z) > 1e-11 * Z * Z:
                return False
    return True


def pin_2p_and_gaussian(L):
    for basis, e, l, ref_fn in (("sto", 0.5, 1, lambda r: -0.125),
                                ("gto", 0.9, 0, lambda r: 3 * 0.9 - 2 * 0.81 * r * r - 1 / r)):
        col = np.zeros((synth.n_cart(l), 1))
        col[0] = 1
        d = dict(name="t", Z=[1.0], R=[[0, 0, 0]], n_up=1, n_dn=0, basis=basis, shell_atom=[0],
                 shell_l=[l], shell_kn=[0], shell_nprim=[1], prim_exp=[e], prim_coef=[1.0],
                 mo_coef=col, occ_up=[[0]], occ_dn=np.zeros((1, 0), dtype=np.int32), ci=[1.0])
        o = _sys(L, synth._finish(d))
        for p in rng.standard_normal((8, 3)) * 2:
            ref = ref_fn(np.linalg.norm(p))
            if abs(o.eval_one(p)["eloc"] - ref) > 1e-10 * max(1, abs(ref)):
                return False
    return True


def pin_h2_closed_form(L):
    """H2 E_L from the closed-form Laplacian of exp(-z rA) + exp(-z rB),
    including the nuclear repulsion 1/1.4."""
    sysd = synth.make_h2()
    o = _sys(L, sysd)
    zeta, a, b = 1.24, 0.5, 1.0
    R = sysd["R"]
    for _ in range(6):
        x = rng.standard_normal((2, 3)) + R
        d = x[0] - x[1]
        r12 = np.linalg.norm(d)
        k1 = a / (1 + b * r12) ** 2
        k2 = -2 * a * b / (1 + b * r12) ** 3
        gJ = [k1 * d / r12, -k1 * d / r12]
        tot, V = 0.0, 1 / r12 + 1 / 1.4
        for i in range(2):
            ph, gph, lph = 0.0, np.zeros(3), 0.0
            for C in R:
                v = x[i] - C
                rc = np.linalg.norm(v)
                ph += math.exp(-zeta * rc)
                gph += -zeta * v / rc * math.exp(-zeta * rc)
                lph += (zeta ** 2 - 2 * zeta / rc) * math.exp(-zeta * rc)
                V -= 1 / rc
            tot += lph / ph + k2 + 2 * k1 / r12 + 2 * np.dot(gph / ph, gJ[i]) + np.dot(gJ[i], gJ[i])
        ref = -0.5 * tot + V
        if abs(o.eval_one(x)["eloc"] - ref) > 1e-10 * max(1, abs(ref)):
            return False
    return True


def pin_fd_gradient(L):
    sysd = synth.make_system("LiH")
    o = _sys(L, sysd)
    x = synth.init_walkers(sysd, 1, 21)[0]
    g = o.eval_one(x, want_grad=True)["grad"]
    h = 1e-5
    for i in range(x.shape[0]):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            fd = (o.eval_one(xp)["logpsi"] - o.eval_one(xm)["logpsi"]) / (2 * h)
            if abs(fd - g[i, c]) > 1e-5 * max(1, abs(fd)):
                return False
    return True


def pin_swap_sign(L):
    sysd = synth.make_system("CO")
    o = _sys(L, sysd)
    for x in synth.init_walkers(sysd, 6, 8):
        y = x.copy()
        y[[0, 1]] = y[[1, 0]]
        if o.eval_one(y)["sign"] != -o.eval_one(x)["sign"]:
            return False
    return True


def pin_sto_norm(L):
    d = dict(name="t", Z=[1.0], R=[[0, 0, 0]], n_up=1, n_dn=0, basis="sto", shell_atom=[0],
             shell_l=[0], shell_kn=[1], shell_nprim=[1], prim_exp=[1.3], prim_coef=[1.0],
             mo_coef=np.ones((1, 1)), occ_up=[[0]], occ_dn=np.zeros((1, 0), dtype=np.int32), ci=[1.0])
    o = _sys(L, synth._finish(d))
    xs, wr = np.polynomial.laguerre.laggauss(40)
    s = 1 / 2.6
    tot = sum(w * math.exp(x) * s * (x * s) ** 2 * 4 * math.pi * o.ao([x * s, 0, 0])[0, 0] ** 2
              for x, w in zip(xs, wr))
    return abs(tot - 1) < 1e-9


def pin_box_muller(L):
    zs = []
    for w in range(4000):
        z = np.zeros((2, 3))
        u = oracle.C.c_double()
        L.or_proposal(2, oracle.C.c_uint64(1), oracle.C.c_uint32(w), oracle.C.c_uint64(0),
                      oracle._p(z), oracle.C.byref(u))
        zs.append(z)
    f = np.concatenate(zs).reshape(-1, 3)
    c = np.corrcoef(f.T)
    return np.max(np.abs(c - np.eye(3))) < 5 / math.sqrt(f.shape[0]) and \
        stats.kstest(f[:, 1], "norm").pvalue > 1e-4


def pin_h_energy(L):
    zeta = 1.25
    sysd = synth.single_atom(1.0, zeta)
    o = _sys(L, sysd)
    X = synth.init_walkers(sysd, 1500, 4)
    lp, sg, el = o.eval(X)
    X, lp, sg, el, _, _ = o.metropolis(X, lp, sg, el, 150, 0.5, 9)
    _, _, _, _, acc, _ = o.metropolis(X, lp, sg, el, 200, 0.5, 9, step0=150)
    m = acc[:, 0] / 200
    return abs(m.mean() - (0.5 * zeta * zeta - zeta)) < 4 * m.std(ddof=1) / math.sqrt(m.size)


def pin_philox_first_words(L):
    """The oracle's Philox against values the real oracle produced after it
    matched rocRAND (tests/test_oracle_sampler.py)."""
    ref = oracle.philox([1, 2, 3, 4], [5, 6])
    c = (oracle.C.c_uint32 * 4)(1, 2, 3, 4)
    k = (oracle.C.c_uint32 * 2)(5, 6)
    o = (oracle.C.c_uint32 * 4)()
    L.or_philox4x32_10(c, k, o)
    return list(o) == [int(v) for v in ref]


MUTANTS = [
    ("kinetic cross term halved", "2.0 * gJ[q] * gS[q]", "gJ[q] * gS[q]", pin_he_closed_form),
    ("Jastrow K'' sign", "const double k2 = -2.0 * a * bb", "const double k2 = 2.0 * a * bb",
     pin_he_closed_form),
    ("Jastrow spin pairing ignored", "const int same = (i < nu) == (j < nu);",
     "const int same = 1;", pin_he_closed_form),
    ("e-n attraction without Z", "ven -= s->Z[a] /", "ven -= 1.0 /", pin_hydrogenic),
    ("STO radial Laplacian factor", "(2.0 * l + 2.0) * g / rr", "(2.0 * l + 1.0) * g / rr",
     pin_2p_and_gaussian),
    ("GTO radial Laplacian factor", "- (2.0 * l + 2.0) * 2.0 * e", "- (2.0 * l) * 2.0 * e",
     pin_2p_and_gaussian),
    ("nuclear repulsion dropped", "vee + ven + or_nuclear_repulsion(s)", "vee + ven",
     pin_h2_closed_form),
    ("Jacobi trace transposed", "t += inv[k * n + i] * phi", "t += inv[i * n + k] * phi",
     pin_fd_gradient),
    ("pivot sign ignored", "*perm_sign = -*perm_sign;", ";", pin_swap_sign),
    ("STO normalisation power", "pow(2.0 * e, 2 * n + 1)", "pow(2.0 * e, 2 * n)", pin_sto_norm),
    ("Box-Muller sine replaced", "z[3 * e + 1] = r0 * sin(", "z[3 * e + 1] = r0 * cos(",
     pin_box_muller),
    ("accept on |Psi| not |Psi|^2", "u < exp(2.0 * (d.logpsi", "u < exp(1.0 * (d.logpsi",
     pin_h_energy),
    ("Philox multiplier", "0xD2511F53u", "0xD2511F55u", pin_philox_first_words),
]


@pytest.fixture(scope="module")
def real_lib():
    return oracle.lib()


@pytest.mark.parametrize("name,old,new,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_mutant(tmp_path, real_lib, name, old, new, pin):
    assert SRC.count(old) == 1, f"mutation site for '{name}' not unique"
    src = tmp_path / "oracle_mutant.c"
    src.write_text(SRC.replace(old, new))
    so = oracle.compile_library(str(src), str(tmp_path / "liboracle_mutant.so"))
    L = oracle.load_library(so)
    assert pin(real_lib), f"real oracle fails pin {pin.__name__}"
    assert not pin(L), f"pin {pin.__name__} misses mutant '{name}'"
    os.remove(so)
