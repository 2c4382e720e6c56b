"""Oracle pins: closed forms of hydrogenic, He-like and H2 wavefunctions,
Gaussian orbitals, normalisation integrals and nuclear repulsion.

Each expected value below is derived from the Hamiltonian of the paper's
Introduction (eq. Hmol) applied to a wavefunction whose Laplacian is known in
closed form, independently of the oracle's orbital tables and determinants.
"""
import math

import numpy as np
import pytest
from scipy.special import roots_genlaguerre

from paper_2506_09743_amd import synth

rng = np.random.default_rng(7)


def _points(n, scale=2.0):
    return rng.standard_normal((n, 3)) * scale


def test_hydrogen_1s_exact(oracle_mod):
    """Exact 1s of H (zeta = 1): E_L = -1/2 Ha everywhere, zero variance."""
    o = oracle_mod.OracleSystem(synth.single_atom(1.0, 1.0))
    e = np.array([o.eval_one(p)["eloc"] for p in _points(64)])
    assert np.max(np.abs(e + 0.5)) < 1e-13
    assert np.std(e) < 1e-13


@pytest.mark.parametrize("Z", [2.0, 3.0, 6.0])
def test_hydrogenic_ion(oracle_mod, Z):
    """One electron, 1s with zeta = Z: E_L = -Z^2/2."""
    o = oracle_mod.OracleSystem(synth.single_atom(Z, Z))
    e = np.array([o.eval_one(p)["eloc"] for p in _points(32, 1.0 / Z)])
    assert np.max(np.abs(e + 0.5 * Z * Z)) < 1e-12 * Z * Z


@pytest.mark.parametrize("zeta", [0.7, 1.3])
def test_hydrogen_1s_off_eigen(oracle_mod, zeta):
    """H with a 1s of exponent zeta: E_L = -zeta^2/2 + (zeta - 1)/r."""
    o = oracle_mod.OracleSystem(synth.single_atom(1.0, zeta))
    for p in _points(32):
        r = np.linalg.norm(p)
        assert abs(o.eval_one(p)["eloc"] - (-0.5 * zeta * zeta + (zeta - 1.0) / r)) < 1e-12


def _ao_mo_system(Z, shells, mo_col, normalize=1, basis="sto"):
    """One nucleus, several one-primitive shells, one MO = mo_col."""
    d = dict(name="t", Z=[Z], R=[[0.0, 0.0, 0.0]], n_up=1, n_dn=0, basis=basis,
             shell_atom=[0] * len(shells), shell_l=[s[0] for s in shells],
             shell_kn=[s[1] for s in shells], shell_nprim=[1] * len(shells),
             prim_exp=[s[2] for s in shells], prim_coef=[1.0] * len(shells),
             normalize=normalize, mo_coef=np.asarray(mo_col, dtype=float).reshape(-1, 1),
             occ_up=[[0]], occ_dn=np.zeros((1, 0), dtype=np.int32), ci=[1.0])
    return synth._finish(d)


def test_hydrogen_2p_exact(oracle_mod):
    """2p_x, 2p_y, 2p_z = {x,y,z} exp(-r/2): E_L = -1/8 (n = 2)."""
    for comp in range(3):
        col = np.zeros(3)
        col[comp] = 1.0
        o = oracle_mod.OracleSystem(_ao_mo_system(1.0, [(1, 0, 0.5)], col))
        e = np.array([o.eval_one(p)["eloc"] for p in _points(32, 3.0)])
        assert np.max(np.abs(e + 0.125)) < 1e-11


def test_hydrogen_2s_exact(oracle_mod):
    """2s = (1 - r/2) exp(-r/2) from an r^0 and an r^1 Slater function at
    zeta = 1/2 combined through the MO coefficients: E_L = -1/8.  Exercises
    the r^kn radial power."""
    o = oracle_mod.OracleSystem(_ao_mo_system(1.0, [(0, 0, 0.5), (0, 1, 0.5)], [1.0, -0.5],
                                              normalize=0))
    e = np.array([o.eval_one(p)["eloc"] for p in _points(32, 3.0)])
    assert np.max(np.abs(e + 0.125)) < 1e-10


def test_hydrogen_3d_exact(oracle_mod):
    """3d_xy, 3d_xz, 3d_yz = xy, xz, yz exp(-r/3): E_L = -1/18 (n = 3)."""
    for comp in (1, 2, 4):  # xy, xz, yz in the xx,xy,xz,yy,yz,zz order
        col = np.zeros(6)
        col[comp] = 1.0
        o = oracle_mod.OracleSystem(_ao_mo_system(1.0, [(2, 0, 1.0 / 3.0)], col))
        e = np.array([o.eval_one(p)["eloc"] for p in _points(16, 4.0)])
        assert np.max(np.abs(e + 1.0 / 18.0)) < 1e-10


def test_hydrogen_3d_x2_minus_y2(oracle_mod):
    """(x^2 - y^2) exp(-r/3) is a 3d eigenfunction built from two Cartesian
    components; with unit-normalised primitives both share one factor."""
    col = np.zeros(6)
    col[0], col[3] = 1.0, -1.0
    o = oracle_mod.OracleSystem(_ao_mo_system(1.0, [(2, 0, 1.0 / 3.0)], col))
    e = np.array([o.eval_one(p)["eloc"] for p in _points(16, 4.0)])
    assert np.max(np.abs(e + 1.0 / 18.0)) < 1e-10


@pytest.mark.parametrize("alpha", [0.3, 1.7])
def test_gaussian_s_hydrogen(oracle_mod, alpha):
    """H with exp(-alpha r^2): E_L = 3 alpha - 2 alpha^2 r^2 - 1/r."""
    o = oracle_mod.OracleSystem(_ao_mo_system(1.0, [(0, 0, alpha)], [1.0], basis="gto"))
    for p in _points(16):
        r = np.linalg.norm(p)
        ref = 3 * alpha - 2 * alpha * alpha * r * r - 1.0 / r
        assert abs(o.eval_one(p)["eloc"] - ref) < 1e-11 * max(1, abs(ref))


def test_gaussian_p_hydrogen(oracle_mod):
    """x exp(-alpha r^2): lap / phi = 4 alpha^2 r^2 - 10 alpha."""
    alpha = 0.8
    o = oracle_mod.OracleSystem(_ao_mo_system(1.0, [(1, 0, alpha)], [1.0, 0, 0], basis="gto"))
    for p in _points(16):
        r = np.linalg.norm(p)
        ref = -0.5 * (4 * alpha * alpha * r * r - 10 * alpha) - 1.0 / r
        assert abs(o.eval_one(p)["eloc"] - ref) < 1e-11 * max(1, abs(ref))


def _he_like(Z, zeta, a, b):
    return synth.single_atom(Z, zeta, n_up=1, n_dn=1, a_par=0.25, a_anti=a, b=b)


@pytest.mark.parametrize("Z,zeta,a,b", [(2.0, 27 / 16, 0.5, 1.0), (3.0, 2.5, 0.5, 0.7),
                                        (2.0, 1.8, 0.0, 1.0), (2.0, 1.6, 0.5, 0.0)])
def test_he_like_pade_closed_form(oracle_mod, Z, zeta, a, b):
    """Two opposite-spin electrons in a 1s of exponent zeta with the Pade
    factor exp(a r12 / (1 + b r12)):
      E_L = -zeta^2 + (zeta - Z)(1/r1 + 1/r2) - K'' - 2 K'/r12 - K'^2
            + zeta K' (r1_hat - r2_hat) . r12_hat + 1/r12,
    K' = a/(1 + b r)^2, K'' = -2ab/(1 + b r)^3."""
    o = oracle_mod.OracleSystem(_he_like(Z, zeta, a, b))
    for _ in range(16):
        x = rng.standard_normal((2, 3))
        r1, r2 = np.linalg.norm(x[0]), np.linalg.norm(x[1])
        d = x[0] - x[1]
        r12 = np.linalg.norm(d)
        k1 = a / (1 + b * r12) ** 2
        k2 = -2 * a * b / (1 + b * r12) ** 3
        ref = (-zeta ** 2 + (zeta - Z) * (1 / r1 + 1 / r2) - k2 - 2 * k1 / r12 - k1 ** 2
               + zeta * k1 * np.dot(x[0] / r1 - x[1] / r2, d / r12) + 1 / r12)
        got = o.eval_one(x)
        assert abs(got["eloc"] - ref) < 1e-11 * max(1, abs(ref))
        ref_logpsi = -zeta * (r1 + r2) + a * r12 / (1 + b * r12) + 2 * math.log(zeta ** 1.5 / math.sqrt(math.pi))
        assert abs(got["logpsi"] - ref_logpsi) < 1e-12 * max(1, abs(ref_logpsi))


def test_he_cusp_bounded(oracle_mod):
    """With the antiparallel cusp a = 1/2 the e-e singularity cancels
    (Kato's condition, the cusp values of the neural-Jastrow appendix): E_L
    stays bounded as r12 -> 0; with a = 0.3 it diverges like (1 - 2a)/r12."""
    ok = oracle_mod.OracleSystem(_he_like(2.0, 1.7, 0.5, 1.0))
    bad = oracle_mod.OracleSystem(_he_like(2.0, 1.7, 0.3, 1.0))
    base = np.array([0.4, -0.3, 0.5])
    e_ok, e_bad = [], []
    for eps in (1e-2, 1e-4, 1e-6):
        x = np.stack([base, base + eps * np.array([0.6, 0.0, 0.8])])
        e_ok.append(ok.eval_one(x)["eloc"])
        e_bad.append(bad.eval_one(x)["eloc"] * eps)
    assert max(e_ok) - min(e_ok) < 0.05
    assert abs(e_bad[-1] - (1 - 2 * 0.3)) < 1e-3


def test_h2_closed_form(oracle_mod):
    """H2 with phi = exp(-zeta rA) + exp(-zeta rB) for both electrons and the
    antiparallel Pade factor: E_L from the closed-form Laplacian of phi,
    sum_C (zeta^2 - 2 zeta / r_C) exp(-zeta r_C)."""
    sysd = synth.make_h2()
    o = oracle_mod.OracleSystem(sysd)
    zeta, a, b = 1.24, 0.5, float(sysd["jas_b"])
    R = sysd["R"]
    for _ in range(16):
        x = rng.standard_normal((2, 3)) + R[[0, 1]]
        tot = 0.0
        d = x[0] - x[1]
        r12 = np.linalg.norm(d)
        k1 = a / (1 + b * r12) ** 2
        k2 = -2 * a * b / (1 + b * r12) ** 3
        gJ = [k1 * d / r12, -k1 * d / r12]
        for i in range(2):
            ph, gph, lph = 0.0, np.zeros(3), 0.0
            for C in R:
                v = x[i] - C
                rc = np.linalg.norm(v)
                ex = math.exp(-zeta * rc)
                ph += ex
                gph += -zeta * v / rc * ex
                lph += (zeta ** 2 - 2 * zeta / rc) * ex
            tot += lph / ph + (k2 + 2 * k1 / r12) + 2 * np.dot(gph / ph, gJ[i]) + np.dot(gJ[i], gJ[i])
        V = 1 / r12 + 1 / np.linalg.norm(R[0] - R[1])
        for i in range(2):
            for C in R:
                V -= 1.0 / np.linalg.norm(x[i] - C)
        ref = -0.5 * tot + V
        got = o.eval_one(x)["eloc"]
        assert abs(got - ref) < 1e-11 * max(1, abs(ref))


@pytest.mark.parametrize("name,ref", [("H2", 0.714285714286), ("LiH", 0.995024875622),
                                      ("Li2", 1.781825381113), ("CO", 22.514071294559)])
def test_nuclear_repulsion(oracle_mod, name, ref):
    o = oracle_mod.OracleSystem(synth.make_system(name))
    assert abs(o.nuclear_repulsion() - ref) < 1e-11


def _angular_grid(n=14):
    ct, wt = np.polynomial.legendre.leggauss(n)
    ph = 2 * np.pi * np.arange(2 * n) / (2 * n)
    dirs, w = [], []
    for c, wc in zip(ct, wt):
        s = math.sqrt(1 - c * c)
        for p in ph:
            dirs.append([s * math.cos(p), s * math.sin(p), c])
            w.append(wc * 2 * np.pi / (2 * n))
    return np.array(dirs), np.array(w)


@pytest.mark.parametrize("basis,l,kn,e", [("sto", 0, 0, 1.3), ("sto", 1, 0, 0.9), ("sto", 0, 1, 1.1),
                                          ("sto", 2, 0, 1.7), ("sto", 2, 1, 2.2), ("gto", 0, 0, 0.6),
                                          ("gto", 1, 0, 2.5), ("gto", 2, 0, 0.4), ("gto", 3, 0, 1.0)])
def test_ao_normalisation_quadrature(oracle_mod, basis, l, kn, e):
    """Every unit-normalised primitive integrates |chi|^2 to 1 over R^3
    (Gauss-Legendre x trapezoid angular grid, exact for these degrees;
    Gauss-Laguerre radial grid in the variable r * decay)."""
    sysd = _ao_mo_system(1.0, [(l, kn, e)], np.eye(synth.n_cart(l))[:, 0], basis=basis)
    o = oracle_mod.OracleSystem(sysd)
    dirs, wang = _angular_grid()
    norms = np.zeros(synth.n_cart(l))
    if basis == "sto":
        # x = 2 zeta r: |chi|^2 r^2 dr = poly(x) exp(-x) dx
        xs, wr = np.polynomial.laguerre.laggauss(60)
        scale = 1.0 / (2 * e)
        rs = xs * scale
        wrads = wr * np.exp(xs) * scale * rs * rs
    else:
        # x = 2 alpha r^2: |chi|^2 r^2 dr = poly(x) sqrt(x) exp(-x) dx
        xs, wr = roots_genlaguerre(40, 0.5)
        scale = 1.0 / math.sqrt(2 * e)
        rs = np.sqrt(xs) * scale
        wrads = wr * np.exp(xs) * scale ** 3 * 0.5
    for r, wrad in zip(rs, wrads):
        for dvec, wa in zip(dirs, wang):
            v = o.ao(r * dvec)[:, 0]
            norms += wrad * wa * v * v
    assert np.max(np.abs(norms - 1.0)) < 1e-9, norms
