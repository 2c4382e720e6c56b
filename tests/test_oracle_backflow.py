"""Oracle pins for the inverse backflow transformation (Methods, backflow
paragraph; kernel omega / r_ij of the Results section) and the local energy
of the backflow-transformed determinants (eqs. nabla_d, nabla_sigma and
delta_sigma of the appendix on backflow local energies).

* Closed form: two electrons of opposite spin in one Gaussian s orbital
  exp(-alpha |q|^2) and no Jastrow.  Since q_1 = r_1 + omega u / r and
  q_2 = r_2 - omega u / r (u = r_1 - r_2, r = |u|), |q_1|^2 + |q_2|^2 =
  |r_1|^2 + |r_2|^2 + 2 omega r + 2 omega^2, so log Psi, its gradient and its
  Laplacian follow by hand; the cross term of eq. delta_sigma is the whole
  difference between the two spins' blocks here.
* grad log|Psi| and lap Psi / Psi against central differences of Psi with
  omega != 0, on all four molecules and on a singles-and-doubles expansion.
* omega -> 0 through the backflow code equals the oracle without backflow;
  one electron has no pair, so backflow changes nothing.
* AO Hessians against central differences of the oracle's AO gradient, and
  their trace against its Laplacian (STO with kn > 0, GTO with l = 2).
* Exchange of two same-spin electrons flips the sign and keeps |Psi| and
  E_L (the map is permutation-equivariant).
* Mutants: each pin rejects a copy of the oracle with one planted mistake.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2506_09743_amd import synth
from test_oracle_many_body import _fd_psi, _smooth

SRC = open(oracle.SRC).read()
OMEGA = 0.35


def _bf(sysd, omega=OMEGA):
    d = dict(sysd)
    d["bf_omega"] = omega
    return d


# ---- pins (take a loaded oracle library, return True when the pin holds) ----

def pin_gaussian_pair_closed_form(L):
    rng = np.random.default_rng(5)
    for alpha, omega, Z in ((0.7, 0.3, 2.0), (1.3, -0.15, 1.0), (0.45, 0.8, 3.0)):
        d = synth.single_atom(Z, alpha, n_up=1, n_dn=1, basis="gto", a_par=0.0, a_anti=0.0)
        d["bf_omega"] = omega
        o = oracle.OracleSystem(d, L=L)
        for _ in range(6):
            x = rng.standard_normal((2, 3)) * 0.9
            u = x[0] - x[1]
            r = np.linalg.norm(u)
            uh = u / r
            log_ref = -alpha * (x[0] @ x[0] + x[1] @ x[1] + 2 * omega * r + 2 * omega ** 2)
            g = np.stack([-2 * alpha * (x[0] + omega * uh), -2 * alpha * (x[1] - omega * uh)])
            lap_log = -alpha * (12.0 + 8.0 * omega / r)
            ekin = -0.5 * (lap_log + np.sum(g * g))
            epot = -Z / np.linalg.norm(x[0]) - Z / np.linalg.norm(x[1]) + 1.0 / r
            det = o.eval_one(x, want_grad=True)
            lnorm = 2 * np.log(np.sqrt(2.0 * alpha / np.pi) ** 1.5)  # normalised primitive
            if abs(det["logpsi"] - lnorm - log_ref) > 1e-12 * max(1.0, abs(log_ref)):
                return False
            if np.max(np.abs(det["grad"] - g)) > 1e-12 * max(1.0, np.max(np.abs(g))):
                return False
            if abs(det["e_kin"] - ekin) > 1e-11 * max(1.0, abs(ekin)):
                return False
            if abs(det["eloc"] - ekin - epot) > 1e-11 * max(1.0, abs(ekin + epot)):
                return False
    return True


def _fd_ok(L, sysd, seed, n=2):
    o = oracle.OracleSystem(sysd, L=L)
    for x in _smooth(sysd, n, seed):
        det = o.eval_one(x, want_grad=True)
        g_fd, lap_fd = _fd_psi(o, x)
        if np.max(np.abs(det["grad"] - g_fd)) > 1e-6 * max(1.0, np.max(np.abs(g_fd))):
            return False
        lap = -2.0 * det["e_kin"]
        if abs(lap - lap_fd) > 2e-5 * max(1.0, abs(lap)):
            return False
    return True


def pin_fd_backflow(L):
    return _fd_ok(L, _bf(synth.make_system("Li2"), 0.5), 7)


def pin_fd_p_orbitals(L):
    """LiH's p shells and STO kn = 1 shells, with a larger omega."""
    return _fd_ok(L, _bf(synth.make_system("LiH"), 0.6), 13)


def _ao_points(d, n, seed):
    rng = np.random.default_rng(seed)
    R = np.asarray(d["R"])
    return [R[i % len(R)] + rng.standard_normal(3) * 0.8 for i in range(n)]


def pin_ao_hessian(L, h=1e-5):
    for d in (synth.make_system("LiH"), synth.make_system("CO")):
        o = oracle.OracleSystem(d, L=L)
        for p in _ao_points(d, 6, 3):
            H = o.ao_hessian(p)
            A = o.ao(p)
            if np.max(np.abs(H[:, :4] - A[:, :4])) > 1e-12 * max(1.0, np.max(np.abs(A))):
                return False
            if np.max(np.abs(H[:, 4] + H[:, 7] + H[:, 9] - A[:, 4])) > 1e-10 * max(1.0, np.max(np.abs(A[:, 4]))):
                return False
            fd = np.zeros((A.shape[0], 3, 3))
            for c in range(3):
                e = np.zeros(3)
                e[c] = h
                fd[:, c, :] = (o.ao(p + e)[:, 1:4] - o.ao(p - e)[:, 1:4]) / (2 * h)
            full = np.empty_like(fd)
            for t, (a, b) in enumerate(((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))):
                full[:, a, b] = full[:, b, a] = H[:, 4 + t]
            if np.max(np.abs(full - fd)) > 1e-6 * max(1.0, np.max(np.abs(fd))):
                return False
    return True


# ---- tests on the real oracle ---------------------------------------------------

def test_gaussian_pair_closed_form(oracle_mod):
    assert pin_gaussian_pair_closed_form(oracle_mod.lib())


@pytest.mark.parametrize("name,omega", [("H2", 0.35), ("LiH", 0.35), ("Li2", -0.2), ("CO", 0.25)])
def test_backflow_fd(oracle_mod, name, omega):
    assert _fd_ok(oracle_mod.lib(), _bf(synth.make_system(name), omega), 21)


def test_backflow_fd_sd_expansion(oracle_mod):
    """SD(4,4) on Li2: many determinants sharing both spins' electrons."""
    d = _bf(synth.with_sd_expansion(synth.make_system("Li2"), 4, 3), 0.4)
    assert _fd_ok(oracle_mod.lib(), d, 23, n=1)


def test_backflow_fd_many_body(oracle_mod):
    """Backflow with the many-body Jastrow terms on the bare positions."""
    d = _bf(synth.with_many_body_jastrow(synth.make_system("LiH"), 3, symmetric=False), 0.3)
    assert _fd_ok(oracle_mod.lib(), d, 29, n=1)


def test_ao_hessian(oracle_mod):
    assert pin_ao_hessian(oracle_mod.lib())


def test_small_omega_equals_no_backflow(oracle_mod):
    for name in ("LiH", "CO"):
        base = synth.make_system(name)
        a = oracle_mod.OracleSystem(base)
        b = oracle_mod.OracleSystem(_bf(base, 1e-300))
        for x in synth.init_walkers(base, 4, 2):
            u, v = a.eval_one(x), b.eval_one(x)
            assert u["sign"] == v["sign"]
            for k in ("logpsi", "eloc", "e_kin"):
                assert abs(u[k] - v[k]) < 1e-11 * max(1.0, abs(u[k])), k


def test_one_electron_unchanged(oracle_mod):
    base = synth.single_atom(2.0, 1.3, basis="sto", l=1, kn=1)
    a = oracle_mod.OracleSystem(base)
    b = oracle_mod.OracleSystem(_bf(base, 0.7))
    for p in np.random.default_rng(1).standard_normal((5, 1, 3)):
        assert np.array_equal(b.backflow(p), p)
        u, v = a.eval_one(p), b.eval_one(p)
        for k in ("logpsi", "eloc"):
            assert abs(u[k] - v[k]) < 1e-12 * max(1.0, abs(u[k])), k


def test_backflow_map_equivariant(oracle_mod):
    """q is permutation-equivariant and moves with a rigid translation."""
    d = _bf(synth.make_system("Li2"))
    o = oracle_mod.OracleSystem(d)
    x = synth.init_walkers(d, 1, 4)[0]
    perm = np.random.default_rng(0).permutation(len(x))
    assert np.allclose(o.backflow(x[perm]), o.backflow(x)[perm], rtol=0, atol=1e-14)
    shift = np.array([0.3, -1.1, 2.0])
    assert np.allclose(o.backflow(x + shift), o.backflow(x) + shift, rtol=0, atol=1e-13)


@pytest.mark.parametrize("name", ["LiH", "CO"])
def test_same_spin_exchange(oracle_mod, name):
    d = _bf(synth.make_system(name))
    o = oracle_mod.OracleSystem(d)
    nu = d["n_up"]
    for x in synth.init_walkers(d, 4, 6):
        y = x.copy()
        y[[0, nu - 1]] = y[[nu - 1, 0]]
        a, b = o.eval_one(x), o.eval_one(y)
        assert b["sign"] == -a["sign"]
        assert abs(a["logpsi"] - b["logpsi"]) < 1e-12 * max(1, abs(a["logpsi"]))
        assert abs(a["eloc"] - b["eloc"]) < 1e-9 * max(1, abs(a["eloc"]))


# ---- planted mistakes ---------------------------------------------------------------

MUTANTS = [
    ("cross term of delta_sigma dropped", "g[3 * ne] += 2.0 * gu[a] * gw[a];", "(void)gw;",
     pin_gaussian_pair_closed_form),
    ("third trace sign", "L += t1 + t2 * t2 - t3;", "L += t1 + t2 * t2 + t3;", pin_fd_backflow),
    ("second-derivative map dropped", "v2 += ph[(1 + bb) * nmo] * Kr[bb][a];", "(void)Kr;",
     pin_gaussian_pair_closed_form),
    ("partner column sign", "Jm[row * n3 + 3 * k + aa] -= d1;", "Jm[row * n3 + 3 * k + aa] += d1;",
     pin_gaussian_pair_closed_form),
    ("eta'' factor", "e2 = 2.0 * om / (r * r * r);", "e2 = 1.0 * om / (r * r * r);",
     pin_gaussian_pair_closed_form),
    ("off-diagonal Hessian weight", "(ia[t] == ib[t] ? 1.0 : 2.0)", "(ia[t] == ib[t] ? 1.0 : 1.0)",
     pin_fd_backflow),
    ("Hessian mixed product term", "q * (dP[x1] * d[x2] + dP[x2] * d[x1])", "q * (dP[x1] * d[x2])",
     pin_ao_hessian),
    ("STO R'' kn term", "R2 += c * f * (g * g - kn / (rr * rr));", "R2 += c * f * (g * g);",
     pin_ao_hessian),
    ("q for the partner", "q[3 * i + c] += s->bf_omega / r * u[c];", "q[3 * i + c] += s->bf_omega * u[c];",
     pin_gaussian_pair_closed_form),
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
