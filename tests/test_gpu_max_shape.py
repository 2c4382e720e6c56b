"""The kernels at the largest shape they are compiled for: 8 + 8 electrons
(16-lane walkers), 32 MOs (the widest column bucket) and 32 AOs (the
matrix-core limit), with d shells and contracted Gaussians.  FP64 and
explicit-method parity against the oracle, the mixed forms' errors,
Metropolis decisions step by step (also with backflow, where a block of
steps must equal single steps), and the adjoint against oracle finite
differences for a sample of parameters."""
import numpy as np
import pytest

from paper_2506_09743_amd import synth
from parity_helpers import LOG_TOL, _compare, _one_step_margin, good_walkers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def max_system():
    from paper_2506_09743_amd import qmc
    sysd = synth.make_max_shape()
    s = qmc.System(sysd)
    yield sysd, s
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp64_explicit"])
def test_max_shape_eval_parity(torch_cuda, oracle_mod, max_system, precision):
    torch = torch_cuda
    sysd, s = max_system
    X = synth.init_walkers(sysd, 257, 81)
    lp, sg, el = [t.cpu().numpy() for t in s.eval(torch.from_numpy(X).cuda(), precision=precision)]
    _compare(oracle_mod.OracleSystem(sysd), sysd, X, lp, sg, el, f"max shape {precision}")


@pytest.mark.parametrize("precision,med_tol", [("fp32", 1e-3), ("bf16", 1e-2)])
def test_max_shape_mixed_error(torch_cuda, oracle_mod, max_system, precision, med_tol):
    torch = torch_cuda
    sysd, s = max_system
    X = synth.init_walkers(sysd, 128, 82)
    el = s.eval(torch.from_numpy(X).cuda(), precision=precision)[2].cpu().numpy()
    rel = oracle_mod.OracleSystem(sysd).eval(X)[2]
    ok = np.isfinite(el) & np.isfinite(rel)
    err = np.abs(el[ok] - rel[ok]) / np.maximum(1.0, np.abs(rel[ok]))
    print(f"max shape {precision}: median relative |dE_L| {np.median(err):.2e}")
    assert np.median(err) < med_tol


def test_max_shape_metropolis_stepwise(torch_cuda, oracle_mod, max_system):
    torch = torch_cuda
    sysd, s = max_system
    o = oracle_mod.OracleSystem(sysd)
    seed, sigma = 0x2506097400FF, 0.1
    X = synth.init_walkers(sysd, 40, 83)
    lp, sg, el = o.eval(X)
    for t in range(4):
        Xo, lpo, sgo, elo, _, log = o.metropolis(X, lp, sg, el, 1, sigma, seed, step0=t, want_log=True)
        tX = torch.from_numpy(X.copy()).cuda()
        tl, ts, te = (torch.from_numpy(v.copy()).cuda() for v in (lp, sg, el))
        acc = s.metropolis(tX, tl, ts, te, 1, sigma, seed, step0=t)
        torch.cuda.synchronize()
        mism = acc.cpu().numpy()[:, 2] != log[0]
        if mism.any():
            margin = _one_step_margin(o, sysd, X, lp, seed, t, sigma, oracle_mod)
            assert np.all(margin[mism] < 1e-9)
        same = ~mism
        assert np.max(np.abs(tX.cpu().numpy()[same] - Xo[same])) < 1e-12
        glp = tl.cpu().numpy()
        ok = same & np.isfinite(lpo)
        assert np.max(np.abs(glp[ok] - lpo[ok]) / np.maximum(1, np.abs(lpo[ok]))) < LOG_TOL
        X, lp, sg, el = Xo, lpo, sgo, elo


def test_max_shape_grad_fd(torch_cuda, oracle_mod, max_system):
    """A sample of exponents and MO coefficients, b, and every nuclear
    coordinate, by central differences (h = 1e-5) of the oracle."""
    torch = torch_cuda
    sysd, s = max_system
    H = 1e-5
    X = good_walkers(oracle_mod.OracleSystem(sysd), sysd, 1, 84)
    dl, de, dlR, deR = [t.cpu().numpy()[0] for t in s.grad(torch.from_numpy(X.copy()).cuda())]
    n_prim = sysd["prim_exp"].size
    nao, nmo = sysd["mo_coef"].shape
    rng = np.random.default_rng(4)

    def fd(mutate):
        out = []
        for h in (H, -H):
            d = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in sysd.items()}
            mutate(d, h)
            lp, _, el = oracle_mod.OracleSystem(d).eval(X, nthreads=1)
            out.append((lp[0], el[0]))
        return (out[0][0] - out[1][0]) / (2 * H), (out[0][1] - out[1][1]) / (2 * H)

    checks = []
    for p in rng.choice(n_prim, 6, replace=False):
        checks.append((int(p), lambda d, h, p=p: d["prim_exp"].__setitem__(p, d["prim_exp"][p] + h)))
    for q in rng.choice(nao * nmo, 10, replace=False):
        mu, m = divmod(int(q), nmo)
        checks.append((n_prim + int(q), lambda d, h, mu=mu, m=m: d["mo_coef"].__setitem__((mu, m), d["mo_coef"][mu, m] + h)))
    checks.append((dl.size - 1, lambda d, h: d.__setitem__("jas_b", d["jas_b"] + h)))
    for col, mut in checks:
        gl, ge = fd(mut)
        assert abs(dl[col] - gl) <= 2e-6 * max(1.0, abs(gl)), (col, dl[col], gl)
        assert abs(de[col] - ge) <= 2e-6 * max(1.0, abs(ge), np.max(np.abs(de))), (col, de[col], ge)
    for a in range(2):
        for k in range(3):
            gl, ge = fd(lambda d, h, a=a, k=k: d["R"].__setitem__((a, k), d["R"][a, k] + h))
            assert abs(dlR[a, k] - gl) <= 2e-6 * max(1.0, abs(gl))
            assert abs(deR[a, k] - ge) <= 2e-6 * max(1.0, abs(ge), np.max(np.abs(deR)))


@pytest.mark.parametrize("precision", ["fp64", "fp64_explicit"])
def test_max_shape_backflow_parity(torch_cuda, oracle_mod, precision):
    """Both backflow methods at 8 + 8 electrons and 32 MOs (the widest
    private MO tables and reference rows), several waves and a ragged tail."""
    from paper_2506_09743_amd import qmc
    torch = torch_cuda
    sysd = dict(synth.make_max_shape())
    sysd["bf_omega"] = 0.2
    X = synth.init_walkers(sysd, 69, 85)
    s = qmc.System(sysd)
    lp, sg, el = [t.cpu().numpy() for t in s.eval(torch.from_numpy(X).cuda(), precision=precision)]
    _compare(oracle_mod.OracleSystem(sysd), sysd, X, lp, sg, el, f"max shape backflow {precision}")
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp64_explicit"])
def test_max_shape_backflow_metropolis(torch_cuda, oracle_mod, precision):
    """Backflow Metropolis at 8 + 8 electrons and 32 MOs: a 3-step block
    (one kernel per step) equals three chained one-step calls exactly, and
    each step's decisions and states match the oracle's, ties aside."""
    from paper_2506_09743_amd import qmc
    torch = torch_cuda
    sysd = dict(synth.make_max_shape())
    sysd["bf_omega"] = 0.2
    s = qmc.System(sysd)
    o = oracle_mod.OracleSystem(sysd)
    seed, sigma, W = 0x2506097400FE, 0.1, 40
    X = synth.init_walkers(sysd, W, 86)
    lp, sg, el = o.eval(X)
    print(f"max shape backflow Metropolis {precision}", flush=True)

    def state(*vals):
        return [torch.from_numpy(np.array(v, copy=True)).cuda() for v in vals]

    blk = state(X, lp, sg, el)
    acc_blk = s.metropolis(*blk, 3, sigma, seed, step0=0, precision=precision)
    one = state(X, lp, sg, el)
    acc_one = torch.zeros((W, 4), dtype=torch.float64, device="cuda")
    for t in range(3):
        s.metropolis(*one, 1, sigma, seed, step0=t, acc=acc_one, precision=precision)
    torch.cuda.synchronize()
    for u, v in zip(blk + [acc_blk], one + [acc_one]):
        assert torch.equal(u, v)
    for t in range(3):
        Xo, lpo, sgo, elo, _, log = o.metropolis(X, lp, sg, el, 1, sigma, seed, step0=t, want_log=True)
        tX, tl, ts, te = state(X, lp, sg, el)
        acc = s.metropolis(tX, tl, ts, te, 1, sigma, seed, step0=t, precision=precision)
        torch.cuda.synchronize()
        mism = acc.cpu().numpy()[:, 2] != log[0]
        if mism.any():
            margin = _one_step_margin(o, sysd, X, lp, seed, t, sigma, oracle_mod)
            assert np.all(margin[mism] < 1e-9)
        same = ~mism
        assert np.max(np.abs(tX.cpu().numpy()[same] - Xo[same])) < 1e-12
        glp = tl.cpu().numpy()
        ok = same & np.isfinite(lpo)
        assert np.max(np.abs(glp[ok] - lpo[ok]) / np.maximum(1, np.abs(lpo[ok]))) < LOG_TOL
        X, lp, sg, el = Xo, lpo, sgo, elo
    s.close()


def test_max_shape_fd(torch_cuda, max_system):
    """The finite-difference kinetic energy at the largest shape agrees with
    the trace E_L on well-separated walkers to its O(h^2) error."""
    torch = torch_cuda
    sysd, s = max_system
    import oracle
    o = oracle.OracleSystem(sysd)
    X = torch.from_numpy(good_walkers(o, sysd, 16, 86)).cuda()
    el = s.eval(X)[2].cpu().numpy()
    ef = s.eval_fd(X, 1e-3)[1].cpu().numpy()
    ekin = np.array([abs(o.eval_one(x)["e_kin"]) for x in X.cpu().numpy()])
    d = np.abs(ef - el) / np.maximum(1.0, ekin)
    print(f"max shape FD vs trace: median {np.median(d):.2e}, max {d.max():.2e}")
    assert np.median(d) < 1e-4
