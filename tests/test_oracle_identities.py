"""Oracle pins: finite differences, symmetries and special cases.

* AO gradients and Laplacians, and the full grad log|Psi| and lap Psi / Psi,
  against central finite differences (h = 1e-5 for gradients, 1e-4 and
  3e-4 for second derivatives).
* Antisymmetry of Psi under exchange of two same-spin electrons (Methods,
  statement after eq. psimol) and its vanishing when two same-spin electrons
  coincide (LiH/Li2 profile appendix).
* Translation invariance of log|Psi| and E_L.
* A CI vector (1, 0, ..., 0) reduces to the single reference determinant;
  reordering the determinant list changes nothing beyond rounding.
* The low-rank excited-determinant identities of the paper's appendix (the
  determinant ratio as a k x k minor and eq. table) hold, read with rows =
  electrons and columns = orbital slots; the HIP path relies on them.
"""
import numpy as np
import pytest

from paper_2506_09743_amd import synth

rng = np.random.default_rng(11)


def _fd_psi(o, x, h1=1e-5, h2=3e-4):
    """Central differences of Psi / Psi(x) (not of log|Psi|, whose curvature
    diverges at the nodes): returns grad Psi / Psi and lap Psi / Psi."""
    ne = x.shape[0]
    d0 = o.eval_one(x)
    l0, s0 = d0["logpsi"], d0["sign"]

    def ratio(y):
        d = o.eval_one(y)
        return d["sign"] * s0 * np.exp(d["logpsi"] - l0)

    g = np.zeros((ne, 3))
    lap = 0.0
    for i in range(ne):
        for d in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, d] += h1
            xm[i, d] -= h1
            g[i, d] = (ratio(xp) - ratio(xm)) / (2 * h1)
            xp, xm = x.copy(), x.copy()
            xp[i, d] += h2
            xm[i, d] -= h2
            lap += (ratio(xp) - 2.0 + ratio(xm)) / h2 ** 2
    return g, lap


def _smooth_walkers(sysd, n, min_dist=0.3):
    """Walkers whose electrons keep min_dist from every nucleus and from each
    other, where log|Psi| is smooth on the finite-difference stencil (the
    Slater e-n cusp and the e-e Jastrow cusp sit at zero distance)."""
    out = []
    X = synth.init_walkers(sysd, 50 * n, 5)
    R = np.asarray(sysd["R"])
    for x in X:
        den = np.linalg.norm(x[:, None, :] - R[None], axis=-1).min()
        dee = np.linalg.norm(x[:, None, :] - x[None], axis=-1) + np.eye(len(x)) * 9
        if den > min_dist and dee.min() > min_dist:
            out.append(x)
        if len(out) == n:
            break
    return out


@pytest.mark.parametrize("name", ["H2", "LiH", "Li2", "CO"])
def test_gradient_and_laplacian_fd(oracle_mod, name):
    """grad log|Psi| and lap Psi / Psi = -2 E_kin against central
    differences of Psi."""
    sysd = synth.make_system(name)
    o = oracle_mod.OracleSystem(sysd)
    for x in _smooth_walkers(sysd, 3):
        d = o.eval_one(x, want_grad=True)
        g_fd, lap_fd = _fd_psi(o, x)
        scale = max(1.0, np.max(np.abs(g_fd)))
        assert np.max(np.abs(d["grad"] - g_fd)) < 1e-6 * scale
        lap_psi = -2.0 * d["e_kin"]
        assert abs(lap_psi - lap_fd) < 2e-5 * max(1.0, abs(lap_psi))


@pytest.mark.parametrize("basis,shells", [
    ("sto", [(0, 0, 1.3), (0, 2, 0.8), (1, 0, 1.1), (1, 1, 0.7), (2, 0, 1.6), (2, 1, 0.9), (3, 0, 1.2)]),
    ("gto", [(0, 0, 0.4), (1, 0, 1.2), (2, 0, 0.7), (3, 0, 0.5)]),
])
def test_ao_derivatives_fd(oracle_mod, basis, shells):
    """Closed-form AO gradient and Laplacian vs central differences, for
    s/p/d/f Cartesian shells, r^kn powers and both radial kinds."""
    nao = sum(synth.n_cart(l) for l, _, _ in shells)
    d = dict(name="ao", Z=[1.0], R=[[0.1, -0.2, 0.3]], n_up=1, n_dn=0, basis=basis,
             shell_atom=[0] * len(shells), shell_l=[s[0] for s in shells],
             shell_kn=[s[1] for s in shells], shell_nprim=[1] * len(shells),
             prim_exp=[s[2] for s in shells], prim_coef=[1.0] * len(shells),
             mo_coef=np.ones((nao, 1)), occ_up=[[0]], occ_dn=np.zeros((1, 0), dtype=np.int32),
             ci=[1.0])
    o = oracle_mod.OracleSystem(synth._finish(d))
    h1, h2 = 1e-5, 1e-4
    for _ in range(6):
        p = rng.standard_normal(3) * 1.2
        a = o.ao(p)
        lap = np.zeros(nao)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h1
            g_fd = (o.ao(p + e)[:, 0] - o.ao(p - e)[:, 0]) / (2 * h1)
            assert np.allclose(a[:, 1 + k], g_fd, rtol=1e-6, atol=1e-8)
            e[k] = h2
            lap += (o.ao(p + e)[:, 0] - 2 * a[:, 0] + o.ao(p - e)[:, 0]) / h2 ** 2
        assert np.allclose(a[:, 4], lap, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("name", ["LiH", "Li2", "CO"])
def test_same_spin_swap_antisymmetry(oracle_mod, name):
    """Psi changes sign, |Psi| and E_L are unchanged, when two same-spin
    electrons are exchanged."""
    sysd = synth.make_system(name)
    o = oracle_mod.OracleSystem(sysd)
    nu, nd = sysd["n_up"], sysd["n_dn"]
    for x in synth.init_walkers(sysd, 4, 9):
        a = o.eval_one(x)
        for i, j in ((0, 1), (nu, nu + 1)):
            if j >= (nu if i < nu else nu + nd):
                continue
            y = x.copy()
            y[[i, j]] = y[[j, i]]
            b = o.eval_one(y)
            assert b["sign"] == -a["sign"]
            assert abs(b["logpsi"] - a["logpsi"]) < 1e-12 * max(1, abs(a["logpsi"]))
            assert abs(b["eloc"] - a["eloc"]) < 1e-9 * max(1, abs(a["eloc"]))


@pytest.mark.parametrize("name", ["LiH", "Li2", "CO"])
def test_pauli_zero(oracle_mod, name):
    """Two same-spin electrons at one point: every determinant vanishes and
    log|Psi| = -inf."""
    sysd = synth.make_system(name)
    o = oracle_mod.OracleSystem(sysd)
    x = synth.init_walkers(sysd, 1, 3)[0]
    x[1] = x[0]
    d = o.eval_one(x)
    assert d["logpsi"] == -np.inf and d["sign"] == 0.0


@pytest.mark.parametrize("name", ["H2", "LiH", "CO"])
def test_translation_invariance(oracle_mod, name):
    sysd = synth.make_system(name)
    o = oracle_mod.OracleSystem(sysd)
    shift = np.array([0.37, -1.21, 0.58])
    moved = dict(sysd)
    moved["R"] = sysd["R"] + shift
    o2 = oracle_mod.OracleSystem(moved)
    for x in synth.init_walkers(sysd, 4, 2):
        a, b = o.eval_one(x), o2.eval_one(x + shift)
        assert abs(a["logpsi"] - b["logpsi"]) < 1e-11 * max(1, abs(a["logpsi"]))
        assert abs(a["eloc"] - b["eloc"]) < 1e-9 * max(1, abs(a["eloc"]))


@pytest.mark.parametrize("name", ["LiH", "CO"])
def test_ci_reference_only(oracle_mod, name):
    """CI = (1, 0, ..., 0) is the single reference determinant."""
    sysd = synth.make_system(name)
    one = dict(sysd)
    one["ci"] = np.zeros_like(sysd["ci"])
    one["ci"][0] = 1.0
    ref = dict(sysd)
    ref["ci"] = np.array([1.0])
    ref["occ_up"] = sysd["occ_up"][:1]
    ref["occ_dn"] = sysd["occ_dn"][:1]
    a, b = oracle_mod.OracleSystem(one), oracle_mod.OracleSystem(ref)
    X = synth.init_walkers(sysd, 8, 4)
    la, sa, ea = a.eval(X)
    lb, sb, eb = b.eval(X)
    assert np.array_equal(sa, sb)
    assert np.max(np.abs(la - lb)) < 1e-13 * np.max(np.abs(la))
    assert np.max(np.abs(ea - eb)) < 1e-10 * np.max(np.abs(ea))


def test_det_list_permutation(oracle_mod):
    sysd = synth.make_system("CO")
    perm = rng.permutation(len(sysd["ci"]))
    p = dict(sysd)
    p["ci"], p["occ_up"], p["occ_dn"] = sysd["ci"][perm], sysd["occ_up"][perm], sysd["occ_dn"][perm]
    X = synth.init_walkers(sysd, 8, 4)
    la, sa, ea = oracle_mod.OracleSystem(sysd).eval(X)
    lb, sb, eb = oracle_mod.OracleSystem(p).eval(X)
    assert np.array_equal(sa, sb)
    assert np.max(np.abs(la - lb)) < 1e-12 * np.max(np.abs(la))
    assert np.max(np.abs(ea - eb)) < 1e-9 * np.max(np.abs(ea))


def test_single_electron_spin_blocks(oracle_mod):
    """A spin block of size zero contributes a unit determinant: the H atom
    with its electron labelled spin-down equals the spin-up one."""
    up = synth.single_atom(1.0, 1.3, n_up=1, n_dn=0)
    dn = synth.single_atom(1.0, 1.3, n_up=0, n_dn=1)
    a, b = oracle_mod.OracleSystem(up), oracle_mod.OracleSystem(dn)
    for p in rng.standard_normal((4, 3)):
        assert a.eval_one(p)["eloc"] == b.eval_one(p)["eloc"]


def test_excited_determinant_identities():
    """Reading of the appendix on excited determinants (eq. table): with
    A0[i,k] = phi_{occ0[k]}(r_i), T = A0^-1 Phi and an excitation that puts
    particle MOs P in hole slots H, det A_X / det A0 = det T[H,P], and for
    any one-body operator B,
      Tr(A_X^-1 B_X) = Tr(A0^-1 B0) + Tr(T[H,P]^-1 Y[H,P]),
      Y = A0^-1 B_full - (A0^-1 B0) T."""
    n, nmo = 5, 11
    for _ in range(20):
        Phi = rng.standard_normal((n, nmo))
        Bf = rng.standard_normal((n, nmo))
        occ0 = list(range(n))
        A0 = Phi[:, occ0]
        B0 = Bf[:, occ0]
        T = np.linalg.solve(A0, Phi)
        Y = np.linalg.solve(A0, Bf) - np.linalg.solve(A0, B0) @ T
        for k in (1, 2, 3):
            H = sorted(rng.choice(n, size=k, replace=False))
            P = sorted(rng.choice(range(n, nmo), size=k, replace=False))
            occ = list(occ0)
            for h, p in zip(H, P):
                occ[h] = p
            AX, BX = Phi[:, occ], Bf[:, occ]
            THP = T[np.ix_(H, P)]
            assert np.isclose(np.linalg.det(AX) / np.linalg.det(A0), np.linalg.det(THP), rtol=1e-10)
            lhs = np.trace(np.linalg.solve(AX, BX))
            rhs = np.trace(np.linalg.solve(A0, B0)) + np.trace(np.linalg.solve(THP, Y[np.ix_(H, P)]))
            assert np.isclose(lhs, rhs, rtol=1e-9, atol=1e-9)


def test_backflow_low_rank_row_update():
    """The update the low-rank backflow path relies on (eq. table applied to
    the backflow rows): with rows electrons, A0 = Phi[:, :n], T = A0^-1 Phi,
    an excitation putting particles P in hole slots H (A_X = Phi[:, occ]),
    R = T[H, P] and any per-electron row matrix B (one row per electron,
    one column per MO, e.g. the orbital gradients at the transformed
    positions):
      B_X A_X^-1 = B0 A0^-1 + Z[:, P] R^-1 A0^-1[H, :],   Z = B - B0 T,
    so the Mt rows of every configuration and its first trace
    Tr(A_X^-1 Psi_X) = Tr(A0^-1 Psi0) + Tr(Zpsi[:, P] R^-1 A0^-1[H, :])
    come from the reference's; Z vanishes on the reference columns."""
    n, nmo = 6, 13
    for _ in range(20):
        Phi = rng.standard_normal((n, nmo))
        B = rng.standard_normal((n, nmo))
        A0 = Phi[:, :n]
        A0i = np.linalg.inv(A0)
        T = A0i @ Phi
        Z = B - B[:, :n] @ T
        assert np.max(np.abs(Z[:, :n])) < 1e-12
        for k in (1, 2):
            H = sorted(rng.choice(n, size=k, replace=False))
            P = sorted(rng.choice(range(n, nmo), size=k, replace=False))
            occ = list(range(n))
            for h, p in zip(H, P):
                occ[h] = p
            AX, BX = Phi[:, occ], B[:, occ]
            R = T[np.ix_(H, P)]
            lhs = BX @ np.linalg.inv(AX)
            rhs = B[:, :n] @ A0i + Z[:, P] @ np.linalg.inv(R) @ A0i[H, :]
            assert np.allclose(lhs, rhs, rtol=1e-9, atol=1e-9)
            assert np.isclose(np.trace(np.linalg.solve(AX, BX)),
                              np.trace(A0i @ B[:, :n]) + np.trace(Z[:, P] @ np.linalg.inv(R) @ A0i[H, :]),
                              rtol=1e-9, atol=1e-9)

