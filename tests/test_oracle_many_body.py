"""Oracle pins for the many-body Jastrow terms of eq. jastrow (appendix on
the many-body Jastrow factor): the e-n kernel (w0 r + w1 r^2) / (1 + w2 r)
and the e-e-n kernel sum_mu c_mu f1(r_ai) f2(r_aj) f3(r_ij) over nuclei and
ordered pairs i > j, f(a, b; r) = a r / (1 + b r).

* One electron in a Slater 1s orbital with the e-n kernel: E_L in closed
  form, E_L = -1/2 (u'' + 2 u'/r + u'^2) - Z/r with u = -zeta r + K(r), where
  K' and K'' come from polynomial quotient-rule arithmetic (numpy), not from
  the oracle's formulas.
* Kato cusp: for a Gaussian orbital (zero slope at the nucleus) times the e-n
  factor, r E_L -> -(w0 + Z) as r -> 0, so the e-n slope enters exactly once.
* The e-e-n value against a brute-force triple sum over nuclei, ordered
  pairs and terms (tiny system, asymmetric parameters, so the i > j order
  matters).
* grad log|Psi| and lap Psi / Psi against central differences of Psi with
  both terms present (amplified parameters, so a dropped term is visible).
* Same-spin exchange with symmetric e-e-n parameters flips the sign of Psi
  and keeps |Psi| and E_L.
* Mutants: each pin rejects a copy of the oracle with one planted mistake.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2506_09743_amd import synth

P = np.polynomial.polynomial
rng = np.random.default_rng(17)
SRC = open(oracle.SRC).read()


def _rational(num, den, r):
    """(K, K', K'') of K = num / den at r by the quotient rule applied to
    coefficient arrays (lowest order first)."""
    n1, d1 = P.polyder(num), P.polyder(den)
    # K' = (n1 den - num d1) / den^2
    kn = P.polysub(P.polymul(n1, den), P.polymul(num, d1))
    kd = P.polymul(den, den)
    kn1, kd1 = P.polyder(kn), P.polyder(kd)
    k2n = P.polysub(P.polymul(kn1, kd), P.polymul(kn, kd1))
    k2d = P.polymul(kd, kd)
    return (P.polyval(r, num) / P.polyval(r, den), P.polyval(r, kn) / P.polyval(r, kd),
            P.polyval(r, k2n) / P.polyval(r, k2d))


def _one_electron(Z, zeta, basis, w):
    d = synth.single_atom(Z, zeta, basis=basis)
    d["jas_en"] = np.array([w], dtype=np.float64)
    return d


def _amplified(sysd, seed, symmetric):
    d = synth.with_many_body_jastrow(sysd, seed, symmetric=symmetric)
    d["jas_een"] = d["jas_een"].copy()
    d["jas_een"][:, 0] *= 10.0
    d["jas_en"] = d["jas_en"] * np.array([3.0, 3.0, 1.0])
    return d


# ---- pins (take a loaded oracle library, return True when the pin holds) ----

def pin_en_closed_form(L):
    for Z, zeta, w in ((1.0, 1.1, (-0.3, -0.04, 0.9)), (3.0, 2.6, (0.25, -0.02, 1.7))):
        o = oracle.OracleSystem(_one_electron(Z, zeta, "sto", w), L=L)
        for p in rng.standard_normal((8, 3)) * 1.3:
            r = np.linalg.norm(p)
            K, K1, K2 = _rational([0.0, w[0], w[1]], [1.0, w[2]], r)
            u1, u2 = -zeta + K1, K2
            ref = -0.5 * (u2 + 2.0 * u1 / r + u1 * u1) - Z / r
            if abs(o.eval_one(p)["eloc"] - ref) > 1e-10 * max(1.0, abs(ref)):
                return False
    return True


def pin_en_cusp(L):
    Z = 2.0
    for w0 in (-Z, -0.3, 0.4):
        o = oracle.OracleSystem(_one_electron(Z, 0.8, "gto", (w0, -0.01, 1.2)), L=L)
        for r in (1e-6, 3e-7):
            p = np.array([0.6, -0.48, 0.64]) * r
            if abs(r * o.eval_one(p)["eloc"] + (w0 + Z)) > 1e-4:
                return False
    return True


def _een_brute(sysd, x):
    R = np.asarray(sysd["R"])
    tot = 0.0
    for a in range(len(R)):
        for i in range(len(x)):
            for j in range(i):
                ri = np.linalg.norm(x[i] - R[a])
                rj = np.linalg.norm(x[j] - R[a])
                rij = np.linalg.norm(x[i] - x[j])
                for c, a1, b1, a2, b2, a3, b3 in sysd["jas_een"]:
                    tot += c * (a1 * ri / (1 + b1 * ri)) * (a2 * rj / (1 + b2 * rj)) * (a3 * rij / (1 + b3 * rij))
    return tot


def pin_een_brute_force(L):
    base = synth.make_system("LiH")
    d = _amplified(base, 7, symmetric=False)
    d["jas_en"] = None
    d["jas_a_par"] = d["jas_a_anti"] = 0.0
    o = oracle.OracleSystem(d, L=L)
    for x in synth.init_walkers(d, 5, 3):
        ref = _een_brute(d, x)
        if abs(o.eval_one(x)["jastrow"] - ref) > 1e-13 * max(1.0, abs(ref)):
            return False
    return True


def _fd_psi(o, x, h1=1e-5, h2=3e-4):
    """Central differences of Psi / Psi(x): grad Psi / Psi and lap Psi / Psi."""
    d0 = o.eval_one(x)
    l0, s0 = d0["logpsi"], d0["sign"]

    def ratio(y):
        d = o.eval_one(y)
        return d["sign"] * s0 * np.exp(d["logpsi"] - l0)

    g = np.zeros_like(x)
    lap = 0.0
    for i in range(x.shape[0]):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h1
            xm[i, c] -= h1
            g[i, c] = (ratio(xp) - ratio(xm)) / (2 * h1)
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h2
            xm[i, c] -= h2
            lap += (ratio(xp) - 2.0 + ratio(xm)) / h2 ** 2
    return g, lap


def _smooth(sysd, n, seed, min_dist=0.3):
    R = np.asarray(sysd["R"])
    out = []
    for x in synth.init_walkers(sysd, 50 * n, seed):
        den = np.linalg.norm(x[:, None] - R[None], axis=-1).min()
        dee = np.linalg.norm(x[:, None] - x[None], axis=-1) + 9 * np.eye(len(x))
        if den > min_dist and dee.min() > min_dist:
            out.append(x)
        if len(out) == n:
            break
    return out


def _fd_ok(L, name, seed, symmetric):
    d = _amplified(synth.make_system(name), seed, symmetric)
    o = oracle.OracleSystem(d, L=L)
    for x in _smooth(d, 2, seed):
        det = o.eval_one(x, want_grad=True)
        g_fd, lap_fd = _fd_psi(o, x)
        if np.max(np.abs(det["grad"] - g_fd)) > 1e-6 * max(1.0, np.max(np.abs(g_fd))):
            return False
        lap = -2.0 * det["e_kin"]
        if abs(lap - lap_fd) > 2e-5 * max(1.0, abs(lap)):
            return False
    return True


def pin_fd_many_body(L):
    return _fd_ok(L, "LiH", 31, symmetric=False)


# ---- tests on the real oracle ---------------------------------------------------

def test_en_closed_form(oracle_mod):
    assert pin_en_closed_form(oracle_mod.lib())


def test_en_cusp(oracle_mod):
    assert pin_en_cusp(oracle_mod.lib())


def test_een_brute_force(oracle_mod):
    assert pin_een_brute_force(oracle_mod.lib())


@pytest.mark.parametrize("name,symmetric", [("H2", False), ("LiH", False), ("Li2", True), ("CO", True)])
def test_many_body_fd(oracle_mod, name, symmetric):
    assert _fd_ok(oracle_mod.lib(), name, 41, symmetric)


def test_absent_terms_change_nothing(oracle_mod):
    """Zero e-n parameters and zero e-e-n weights reproduce the Pade-only
    wavefunction bit for bit."""
    base = synth.make_system("Li2")
    d = synth.with_many_body_jastrow(base, 3)
    d["jas_en"] = np.zeros_like(d["jas_en"])
    d["jas_een"] = d["jas_een"].copy()
    d["jas_een"][:, 0] = 0.0
    X = synth.init_walkers(base, 16, 4)
    a = oracle_mod.OracleSystem(base).eval(X)
    b = oracle_mod.OracleSystem(d).eval(X)
    for u, v in zip(a, b):
        assert np.array_equal(u, v, equal_nan=True)


@pytest.mark.parametrize("name", ["LiH", "CO"])
def test_symmetric_exchange(oracle_mod, name):
    d = synth.with_many_body_jastrow(synth.make_system(name), 5, symmetric=True)
    o = oracle_mod.OracleSystem(d)
    nu = d["n_up"]
    for x in synth.init_walkers(d, 4, 6):
        y = x.copy()
        y[[0, nu - 1]] = y[[nu - 1, 0]]
        a, b = o.eval_one(x), o.eval_one(y)
        assert b["sign"] == -a["sign"]
        assert abs(a["logpsi"] - b["logpsi"]) < 1e-12 * max(1, abs(a["logpsi"]))
        assert abs(a["eloc"] - b["eloc"]) < 1e-9 * max(1, abs(a["eloc"]))


def test_asymmetric_order_matters(oracle_mod):
    """With a1 != a2 the kernel is not symmetric: exchanging two electrons
    changes J, as the ordered sum i > j of eq. jastrow prescribes."""
    d = _amplified(synth.make_system("LiH"), 8, symmetric=False)
    o = oracle_mod.OracleSystem(d)
    x = synth.init_walkers(d, 1, 2)[0]
    y = x.copy()
    y[[0, 1]] = y[[1, 0]]
    assert abs(o.eval_one(x)["jastrow"] - o.eval_one(y)["jastrow"]) > 1e-6


# ---- planted mistakes ---------------------------------------------------------------

MUTANTS = [
    ("e-n K' second term sign", "const double K1 = N1 / D - N * w2 / (D * D);",
     "const double K1 = N1 / D + N * w2 / (D * D);", pin_en_closed_form),
    ("e-n K'' middle factor", "- 2.0 * N1 * w2 / (D * D) +", "- 1.0 * N1 * w2 / (D * D) +",
     pin_en_closed_form),
    ("e-n 2K'/r dropped", "lapJ += K2 + 2.0 * K1 / r;", "lapJ += K2;", pin_en_cusp),
    ("e-e-n order reversed", "for (int j = 0; j < i; ++j) {\n                double u[3]",
     "for (int j = i + 1; j < ne; ++j) {\n                double u[3]", pin_een_brute_force),
    ("e-e-n f1 uses b as numerator", "f1 = q[1] * ru / D;", "f1 = q[2] * ru / D;", pin_een_brute_force),
    ("e-e-n cross term dropped", " + 2.0 * d1 * d3 * uw + f1 * lap3", " + f1 * lap3", pin_fd_many_body),
    ("e-e-n j gradient sign", "f1 * d2 * v[k] * f3 - f1 * f2 * d3 * w[k]",
     "f1 * d2 * v[k] * f3 + f1 * f2 * d3 * w[k]", pin_fd_many_body),
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
