"""qmc_grad (hand-written adjoint) against central finite differences of the
FP64 oracle, h = 1e-5, for every variational parameter (primitive exponents,
MO coefficients, Pade b, and with the many-body Jastrow every e-n and e-e-n
parameter) and every nuclear coordinate:

  d log|Psi| / d theta,  d E_L / d theta,  d log|Psi| / d R,  d E_L / d R.

Walkers are drawn where finite differences are well conditioned: electrons
at least 0.3 bohr from nuclei and from each other, reference matrices with
condition number < 1e3 and a CI sum that cancels by less than 10x.  The
bound |analytic - FD| <= 2e-6 max(1, |FD|, scale) covers the O(h^2)
truncation and the O(eps/h) rounding of the differences.
"""
import numpy as np
import pytest

from paper_2506_09743_amd import synth
from parity_helpers import good_walkers as _good_walkers

pytestmark = pytest.mark.gpu

H = 1e-5


def _perturbed(sysd, kind, idx, h):
    d = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in sysd.items()}
    if kind == "exp":
        d["prim_exp"][idx] += h
    elif kind == "mo":
        d["mo_coef"][idx] += h
    elif kind == "b":
        d["jas_b"] = sysd["jas_b"] + h
    elif kind == "R":
        d["R"][idx] += h
    elif kind in ("jas_en", "jas_een"):
        d[kind][idx] += h
    return d


def _fd(oracle_mod, sysd, X, kind, idx):
    lp_p, _, el_p = oracle_mod.OracleSystem(_perturbed(sysd, kind, idx, H)).eval(X, nthreads=1)
    lp_m, _, el_m = oracle_mod.OracleSystem(_perturbed(sysd, kind, idx, -H)).eval(X, nthreads=1)
    return (lp_p - lp_m) / (2 * H), (el_p - el_m) / (2 * H)


def _check(name, ana, fd, what):
    scale = np.maximum(1.0, np.max(np.abs(fd), axis=-1, keepdims=True))
    err = np.abs(ana - fd) / np.maximum(scale, np.abs(fd))
    worst = float(err.max())
    print(f"{name} {what}: max scaled |analytic - FD| = {worst:.2e}")
    assert worst < 2e-6, f"{name} {what}: {worst}"


@pytest.mark.parametrize("name,nw,mbj", [("Li2", 4, False), ("LiH", 4, False), ("CO", 2, False), ("H2", 4, False),
                                         ("Li2", 3, True), ("LiH", 3, True), ("CO", 2, True)])
def test_grad_vs_oracle_fd(oracle_mod, name, nw, mbj):
    import torch
    from paper_2506_09743_amd import qmc
    sysd = synth.make_system(name)
    if mbj:
        # many-body terms with amplified e-e-n weights so their derivatives matter
        sysd = synth.with_many_body_jastrow(sysd, synth.MBJ_SEED[name], symmetric=False)
        sysd["jas_een"][:, 0] *= 10.0
    o = oracle_mod.OracleSystem(sysd)
    X = _good_walkers(o, sysd, nw, 11)
    s = qmc.System(sysd)
    dl, de, dlR, deR = [t.cpu().numpy() for t in s.grad(torch.from_numpy(X).cuda())]
    n_prim = sysd["prim_exp"].size
    nao, nmo = sysd["mo_coef"].shape
    p_b = n_prim + nao * nmo
    n_en = sysd["jas_en"].size if mbj else 0
    n_een = sysd["jas_een"].size if mbj else 0
    assert dl.shape[1] == p_b + 1 + n_en + n_een == s.param_count
    rng = np.random.default_rng(0)
    # every exponent, b, every many-body parameter and a sample of MO
    # coefficients (all of them for small systems)
    cols = list(range(n_prim)) + list(range(p_b, p_b + 1 + n_en + n_een))
    mo_idx = np.arange(nao * nmo)
    if nao * nmo > 120:
        mo_idx = rng.choice(mo_idx, 120 if not mbj else 40, replace=False)
    cols += [n_prim + int(q) for q in mo_idx]
    fd_l = np.zeros((nw, len(cols)))
    fd_e = np.zeros((nw, len(cols)))
    for j, c in enumerate(cols):
        if c < n_prim:
            kind, idx = "exp", c
        elif c == p_b:
            kind, idx = "b", None
        elif c > p_b and c <= p_b + n_en:
            kind, idx = "jas_en", np.unravel_index(c - p_b - 1, sysd["jas_en"].shape)
        elif c > p_b + n_en:
            kind, idx = "jas_een", np.unravel_index(c - p_b - 1 - n_en, sysd["jas_een"].shape)
        else:
            q = c - n_prim
            kind, idx = "mo", (q // nmo, q % nmo)
        fd_l[:, j], fd_e[:, j] = _fd(oracle_mod, sysd, X, kind, idx)
    tag = name + (" + many-body" if mbj else "")
    _check(tag, dl[:, cols], fd_l, "dlog|Psi|/dtheta")
    _check(tag, de[:, cols], fd_e, "dE_L/dtheta")
    na = len(sysd["Z"])
    fl = np.zeros((nw, na * 3))
    fe = np.zeros((nw, na * 3))
    for a in range(na):
        for k in range(3):
            fl[:, 3 * a + k], fe[:, 3 * a + k] = _fd(oracle_mod, sysd, X, "R", (a, k))
    _check(tag, dlR.reshape(nw, -1), fl, "dlog|Psi|/dR")
    _check(tag, deR.reshape(nw, -1), fe, "dE_L/dR")
    s.close()


def test_grad_batch_and_null_outputs(oracle_mod):
    """Outputs do not depend on the batch; NULL outputs are skipped."""
    import torch
    from paper_2506_09743_amd import qmc
    sysd = synth.make_system("Li2")
    s = qmc.System(sysd)
    X = torch.from_numpy(synth.init_walkers(sysd, 70, 2)).cuda()
    full = [t.cpu().numpy() for t in s.grad(X)]
    part = [t.cpu().numpy() for t in s.grad(X[9:40].contiguous())]
    for a, b in zip(full, part):
        assert np.array_equal(a[9:40], b, equal_nan=True)
    only = torch.full((70, 2, 3), 7.0, dtype=torch.float64, device="cuda")
    qmc.qmc_grad(s.handle, X, None, None, None, only)
    assert np.array_equal(only.cpu().numpy(), full[3], equal_nan=True)
    s.close()


def test_force_estimator_on_gpu_outputs(oracle_mod):
    """eq. force assembled from the adjoint outputs is finite and its two
    terms have the expected shapes; eq. nabla_loss likewise."""
    import torch
    from paper_2506_09743_amd import qmc
    sysd = synth.make_system("Li2")
    s = qmc.System(sysd)
    X = torch.from_numpy(synth.init_walkers(sysd, 512, 3)).cuda()
    lp, sg, el = s.eval(X)
    s.metropolis(X, lp, sg, el, 50, 0.2, 3)
    dl, de, dlR, deR = s.grad(X)
    ok = torch.isfinite(el)
    Ev = el[ok].mean()
    F = -(deR[ok] + (el[ok] - Ev)[:, None, None] * 2 * dlR[ok]).mean(0)
    g = (2 * dl[ok] * (el[ok] - Ev)[:, None]).mean(0)
    assert torch.isfinite(F).all() and torch.isfinite(g).all()
    assert F.shape == (2, 3) and g.shape == (s.param_count,)
    s.close()


@pytest.mark.parametrize("name,nw,mbj", [("Li2", 4, False), ("Li2", 3, True)])
def test_grad_mixed_fp32_vs_oracle_fd(oracle_mod, name, nw, mbj):
    """The mixed FP32 form of qmc_grad (forward AO values and MO value
    contraction in FP32, every derivative pass FP64) on Li2 against the same
    FP64 oracle central differences, h = 1e-5: within 1e-4 of the scale
    (FP32 orbital rounding, about 1e-7 relative, amplified by the Slater
    inverse and the kinetic terms; measured 1.3e-5 and 1.6e-5), and within
    1e-4 of the FP64 form's own outputs."""
    import torch
    from paper_2506_09743_amd import qmc
    sysd = synth.make_system(name)
    if mbj:
        sysd = synth.with_many_body_jastrow(sysd, synth.MBJ_SEED[name], symmetric=False)
        sysd["jas_een"][:, 0] *= 10.0
    o = oracle_mod.OracleSystem(sysd)
    X = _good_walkers(o, sysd, nw, 12)
    s = qmc.System(sysd)
    tX = torch.from_numpy(X).cuda()
    dl, de, dlR, deR = [t.cpu().numpy() for t in s.grad(tX, precision="fp32")]
    g64 = [t.cpu().numpy() for t in s.grad(tX)]
    n_prim = sysd["prim_exp"].size
    nao, nmo = sysd["mo_coef"].shape
    p_b = n_prim + nao * nmo
    cols = list(range(n_prim)) + list(range(p_b, s.param_count))
    cols += list(n_prim + np.random.default_rng(1).choice(nao * nmo, 24, replace=False))
    n_en = sysd["jas_en"].size if mbj else 0
    worst = 0.0
    for c in cols:
        c = int(c)
        if c < n_prim:
            kind, idx = "exp", c
        elif c == p_b:
            kind, idx = "b", None
        elif c > p_b + n_en:
            kind, idx = "jas_een", np.unravel_index(c - p_b - 1 - n_en, sysd["jas_een"].shape)
        elif c > p_b:
            kind, idx = "jas_en", np.unravel_index(c - p_b - 1, sysd["jas_en"].shape)
        else:
            kind, idx = "mo", ((c - n_prim) // nmo, (c - n_prim) % nmo)
        fl, fe = _fd(oracle_mod, sysd, X, kind, idx)
        for ana, fd in ((dl[:, c], fl), (de[:, c], fe)):
            worst = max(worst, float(np.max(np.abs(ana - fd) / np.maximum(1.0, np.abs(fd)))))
    for a, b in zip((dl, de, dlR, deR), g64):
        scale = np.maximum(1.0, np.abs(b))
        worst = max(worst, float(np.max(np.abs(a - b) / scale)))
    print(f"{name}{' many-body' if mbj else ''} FP32 grad: max scaled error {worst:.2e}")
    assert worst < 1e-4
    s.close()
