"""Oracle pins for the sampler: Philox4x32-10 against rocRAND's independent
host implementation, Box-Muller and accept-uniform statistics, and the
Metropolis chain against exact expectation values (H atom, He without
Jastrow) and the exact H 1s radial density."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from paper_2506_09743_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND host reference")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "helpers", "philox_rocrand_ref.cpp")],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(oracle_mod, rocrand_ref):
    rng = np.random.default_rng(3)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF)]
    for _ in range(200):
        k = rng.integers(0, 2 ** 32, size=2)
        c = rng.integers(0, 2 ** 32, size=4)
        c[1] %= 2 ** 30  # the reference takes the offset in units of words
        cases.append((*k, *c))
    inp = "\n".join(" ".join(str(int(v)) for v in t) for t in cases) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)
    mine = np.array([oracle_mod.philox(t[2:], t[:2]) for t in cases], dtype=np.uint64)
    assert np.array_equal(ref, mine)


def test_proposal_moments(oracle_mod):
    """Box-Muller normals: mean 0, variance 1, no correlation between the
    three components or with the accept uniform; the accept uniform has the
    moments of U[0,1)."""
    n_e, n = 4, 20000
    z = np.zeros((n, n_e, 3))
    u = np.zeros(n)
    for w in range(n):
        z[w], u[w] = oracle_mod.proposal(n_e, 12345, w, 7)
    flat = z.reshape(-1, 3)
    se = 1.0 / np.sqrt(flat.shape[0])
    assert np.all(np.abs(flat.mean(0)) < 5 * se)
    assert np.all(np.abs(flat.var(0) - 1.0) < 5 * np.sqrt(2) * se)
    c = np.corrcoef(np.c_[flat, np.repeat(u, n_e)].T)
    assert np.max(np.abs(c - np.eye(4))) < 5 * se
    assert abs(u.mean() - 0.5) < 5 / np.sqrt(12 * n)
    assert np.all((u >= 0) & (u < 1))
    assert stats.kstest(flat[:, 2], "norm").pvalue > 1e-4
    assert stats.kstest(u, "uniform").pvalue > 1e-4


def test_proposal_depends_on_every_counter_word(oracle_mod):
    base, ub = oracle_mod.proposal(3, 99, 5, 11)
    for args in ((98, 5, 11), (99, 6, 11), (99, 5, 12), (99, 5, 11 + (1 << 32))):
        z, u = oracle_mod.proposal(3, *args)
        assert not np.array_equal(z, base) and u != ub


def _walker_means(o, sysd, W, burn, steps, sigma, seed):
    X = synth.init_walkers(sysd, W, seed)
    lp, sg, el = o.eval(X)
    X, lp, sg, el, _, _ = o.metropolis(X, lp, sg, el, burn, sigma, seed)
    X, lp, sg, el, acc, _ = o.metropolis(X, lp, sg, el, steps, sigma, seed, step0=burn)
    return X, acc[:, 0] / steps, acc[:, 2] / steps


@pytest.mark.parametrize("zeta", [0.8, 1.25])
def test_hydrogen_variational_energy(oracle_mod, zeta):
    """H with a 1s of exponent zeta: <E> = zeta^2/2 - zeta (variational
    energy, eq. Ev, estimated by the Monte Carlo mean over |Psi|^2 samples).
    Walkers are independent chains, so the walker means give the error bar."""
    sysd = synth.single_atom(1.0, zeta)
    o = oracle_mod.OracleSystem(sysd)
    X, m, acc = _walker_means(o, sysd, 2000, 200, 300, 0.6 / zeta, 17)
    exact = 0.5 * zeta * zeta - zeta
    se = m.std(ddof=1) / np.sqrt(m.size)
    assert abs(m.mean() - exact) < 4 * se, (m.mean(), exact, se)
    assert 0.2 < acc.mean() < 0.9
    # Final positions are independent draws from |Psi|^2: the radial density
    # 4 zeta^3 r^2 exp(-2 zeta r) is Gamma(3, scale 1/(2 zeta)).
    r = np.linalg.norm(X[:, 0, :], axis=1)
    assert stats.kstest(r, stats.gamma(3, scale=1.0 / (2 * zeta)).cdf).pvalue > 1e-3


def test_helium_no_jastrow_energy(oracle_mod):
    """He, both electrons in 1s with zeta = 27/16, no Jastrow:
    <E> = zeta^2 - 2 Z zeta + 5 zeta / 8 = -2.84765625 Ha."""
    zeta = 27.0 / 16.0
    sysd = synth.single_atom(2.0, zeta, n_up=1, n_dn=1, a_par=0.0, a_anti=0.0)
    o = oracle_mod.OracleSystem(sysd)
    _, m, _ = _walker_means(o, sysd, 2000, 200, 300, 0.35, 23)
    se = m.std(ddof=1) / np.sqrt(m.size)
    assert abs(m.mean() - (-2.84765625)) < 4 * se, (m.mean(), se)


def test_metropolis_accept_rule(oracle_mod):
    """Replaying one step by hand: the chain accepts exactly when
    u < exp(2 (log|Psi'| - log|Psi|)) with the same Philox proposal."""
    sysd = synth.make_system("LiH")
    o = oracle_mod.OracleSystem(sysd)
    X = synth.init_walkers(sysd, 64, 2)
    lp, sg, el = o.eval(X)
    sigma, seed, step = 0.2, 777, 41
    X1, lp1, _, el1, acc, log = o.metropolis(X, lp, sg, el, 1, sigma, seed, step0=step,
                                             walker_offset=100, want_log=True)
    for w in range(64):
        z, u = oracle_mod.proposal(4, seed, 100 + w, step)
        d = o.eval_one(X[w] + sigma * z)
        acc_ref = np.isfinite(d["logpsi"]) and u < np.exp(2 * (d["logpsi"] - lp[w]))
        assert bool(log[0, w]) == bool(acc_ref)
        want = X[w] + sigma * z if acc_ref else X[w]
        assert np.array_equal(X1[w], want)
        assert acc[w, 0] == el1[w] and acc[w, 2] == float(acc_ref)


def test_metropolis_resume_bitwise(oracle_mod):
    """Counter-based stream: a block split in two equals one block."""
    sysd = synth.make_system("H2")
    o = oracle_mod.OracleSystem(sysd)
    X = synth.init_walkers(sysd, 32, 1)
    lp, sg, el = o.eval(X)
    a = o.metropolis(X, lp, sg, el, 20, 0.2, 5)
    b1 = o.metropolis(X, lp, sg, el, 8, 0.2, 5)
    b2 = o.metropolis(*b1[:4], 12, 0.2, 5, step0=8, acc=b1[4])
    for u, v in zip(a[:5], b2[:5]):
        assert np.array_equal(u, v)


def test_metropolis_counts_non_finite_states(oracle_mod):
    """The Monte Carlo mean of eq. Ev runs over states with a finite E_L: a
    state without a finite log|Psi| or E_L (NaN positions, or two same-spin
    electrons at one point, where every determinant vanishes) adds to the
    fourth accumulator column and to neither sum.  A finite walker's sums
    are the plain sums of its post-decision E_L over the steps."""
    sysd = synth.make_system("LiH")
    o = oracle_mod.OracleSystem(sysd)
    X = synth.init_walkers(sysd, 3, 5)
    X[1] = np.nan
    X[2, 1] = X[2, 0]  # spin-up electrons 0 and 1 coincide
    lp, sg, el = o.eval(X)
    assert np.isfinite(el[0]) and not np.isfinite(lp[1]) and lp[2] == -np.inf
    steps = 6
    # sigma = 0: every proposal is the current state, so nothing can recover
    _, _, _, _, acc0, _ = o.metropolis(X, lp, sg, el, steps, 0.0, 11)
    assert acc0[0, 3] == 0 and acc0[1, 3] == steps and acc0[2, 3] == steps
    assert acc0[1, 0] == 0 and acc0[1, 1] == 0 and acc0[2, 0] == 0
    assert acc0[1, 2] == 0 and acc0[2, 2] == 0
    # sigma > 0: the coincident walker's first proposal separates the
    # electrons and is always accepted (|Psi| = 0 before it); the NaN walker
    # never moves
    Xs, lps, _, els, acc, _ = o.metropolis(X, lp, sg, el, steps, 0.2, 11)
    assert acc[1, 3] == steps and acc[1, 2] == 0 and np.all(np.isnan(Xs[1]))
    assert acc[2, 3] == 0 and acc[2, 2] >= 1 and np.isfinite(acc[2, 0])
    # the finite walker: its sums replayed one step at a time
    state = [X[:1], lp[:1], sg[:1], el[:1]]
    s1 = s2 = 0.0
    for t in range(steps):
        Xn, lpn, sgn, eln, _, _ = o.metropolis(*state, 1, 0.2, 11, step0=t)
        state = [Xn, lpn, sgn, eln]
        s1 += eln[0]
        s2 += eln[0] * eln[0]
    assert acc[0, 3] == 0
    assert abs(acc[0, 0] - s1) <= 1e-12 * max(1.0, abs(s1))
    assert abs(acc[0, 1] - s2) <= 1e-12 * max(1.0, abs(s2))
