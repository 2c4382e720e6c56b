"""The explicit-determinant method (QMC_FP64_EXPLICIT: every distinct spin
configuration factorised on its own, the evaluation that eq. table
accelerates) against the FP64 oracle, which evaluates determinants the same
way, and against the low-rank path; also on the SD(n, n) expansions of the
determinant-count sweep (4 to 876 determinants for CO)."""
import numpy as np
import pytest

from paper_2506_09743_amd import synth
from parity_helpers import LOG_TOL, _compare, _one_step_margin

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _system(name, sd):
    base = synth.make_system(name)
    return synth.with_sd_expansion(base, sd, 5) if sd else base


@pytest.mark.parametrize("name,sd,W", [("H2", 0, 300), ("LiH", 0, 997), ("Li2", 0, 601), ("CO", 0, 515),
                                       ("CO", 2, 130), ("CO", 6, 130), ("CO", 10, 130)])
def test_explicit_eval_parity(torch_cuda, oracle_mod, name, sd, W):
    from paper_2506_09743_amd import qmc
    torch = torch_cuda
    sysd = _system(name, sd)
    X = synth.init_walkers(sysd, W, 79)
    s = qmc.System(sysd)
    tX = torch.from_numpy(X).cuda()
    lp, sg, el = [t.cpu().numpy() for t in s.eval(tX, precision="fp64_explicit")]
    _compare(oracle_mod.OracleSystem(sysd), sysd, X, lp, sg, el, f"{name} SD({sd}) explicit")
    # the low-rank path on the same walkers
    tl, ts, te = [t.cpu().numpy() for t in s.eval(tX)]
    ok = np.isfinite(tl) & np.isfinite(lp)
    assert np.max(np.abs(tl[ok] - lp[ok]) / np.maximum(1, np.abs(lp[ok]))) <= LOG_TOL
    assert np.array_equal(ts[ok], sg[ok])
    s.close()


def test_explicit_full_size_sampled(torch_cuda, oracle_mod):
    """CO SD(10,10) (876 determinants) at 65536 walkers, sampled."""
    from paper_2506_09743_amd import qmc
    torch = torch_cuda
    sysd = _system("CO", 10)
    X = synth.init_walkers(sysd, 65536, synth.WALKER_SEED["CO"])
    s = qmc.System(sysd)
    lp, sg, el = [t.cpu().numpy() for t in s.eval(torch.from_numpy(X).cuda(), precision="fp64_explicit")]
    idx = np.sort(np.random.default_rng(3).choice(65536, 96, replace=False))
    idx[-1] = 65535
    _compare(oracle_mod.OracleSystem(sysd), sysd, X[idx], lp[idx], sg[idx], el[idx], "CO SD(10) explicit 64k")
    s.close()


def test_explicit_metropolis_stepwise(torch_cuda, oracle_mod):
    from paper_2506_09743_amd import qmc
    torch = torch_cuda
    sysd = _system("LiH", 0)
    o = oracle_mod.OracleSystem(sysd)
    s = qmc.System(sysd)
    seed, sigma = synth.PHILOX_SEED["LiH"], 0.2
    X = synth.init_walkers(sysd, 192, 12)
    lp, sg, el = o.eval(X)
    for t in range(6):
        Xo, lpo, sgo, elo, _, log = o.metropolis(X, lp, sg, el, 1, sigma, seed, step0=t, want_log=True)
        tX = torch.from_numpy(X.copy()).cuda()
        tl, ts, te = (torch.from_numpy(v.copy()).cuda() for v in (lp, sg, el))
        acc = s.metropolis(tX, tl, ts, te, 1, sigma, seed, step0=t, precision="fp64_explicit")
        torch.cuda.synchronize()
        mism = acc.cpu().numpy()[:, 2] != log[0]
        if mism.any():
            margin = _one_step_margin(o, sysd, X, lp, seed, t, sigma, oracle_mod)
            assert np.all(margin[mism] < 1e-9)
        same = ~mism
        assert np.max(np.abs(tX.cpu().numpy()[same] - Xo[same])) < 1e-12
        X, lp, sg, el = Xo, lpo, sgo, elo
    s.close()
