"""Metropolis parity at the workloads' full sizes, in the launch shapes the
benchmark and the configurations use.  Walkers are independent and the
Philox counter holds the walker's own index, so a sampled walker's chain
is replayed by the oracle on its own (walker_offset = its index) and must
take the same accept decisions and end in the same state.

  H2    1024 walkers x 200 steps, every walker
  LiH   16384 walkers x 500 steps in one block, 24 sampled walkers
  Li2   32768 walkers x 100 steps, 16 sampled walkers
  CO    65536 walkers x 500 steps in the benchmark's 10-step launches, 24 sampled
"""
import numpy as np
import pytest

from paper_2506_09743_amd import synth

pytestmark = pytest.mark.gpu

E_TOL = 1e-8


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _run_gpu(torch, sysd, W, n_steps, chunk):
    from paper_2506_09743_amd import qmc
    s = qmc.System(sysd)
    name = sysd["name"]
    X0 = synth.init_walkers(sysd, W, synth.WALKER_SEED[name])
    X = torch.from_numpy(X0.copy()).cuda()
    lp, sg, el = s.eval(X)
    lp0, sg0, el0 = [t.cpu().numpy() for t in (lp, sg, el)]
    acc = torch.zeros((W, 4), dtype=torch.float64, device="cuda")
    for s0 in range(0, n_steps, chunk):
        s.metropolis(X, lp, sg, el, min(chunk, n_steps - s0), synth.CONFIG_SIGMA, synth.PHILOX_SEED[name],
                     step0=s0, acc=acc)
    torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in (X, lp, sg, el, acc)]
    s.close()
    return X0, (lp0, sg0, el0), out


def _check_walkers(oracle_mod, sysd, X0, start, out, idx, n_steps, tag):
    o = oracle_mod.OracleSystem(sysd)
    gX, glp, gsg, gel, gacc = out
    lp0, sg0, el0 = start
    for w in idx:
        sl = slice(w, w + 1)
        Xo, lpo, sgo, elo, acco, _ = o.metropolis(X0[sl], lp0[sl], sg0[sl], el0[sl], n_steps,
                                                   synth.CONFIG_SIGMA, synth.PHILOX_SEED[sysd["name"]],
                                                   walker_offset=int(w), nthreads=1)
        assert gacc[w, 2] == acco[0, 2], f"{tag} walker {w}: accept count {gacc[w, 2]} vs {acco[0, 2]}"
        assert np.max(np.abs(gX[w] - Xo[0])) < 1e-9, f"{tag} walker {w}: positions"
        if np.isfinite(lpo[0]):
            assert abs(glp[w] - lpo[0]) <= 1e-10 * max(1.0, abs(lpo[0])), f"{tag} walker {w}: log|Psi|"
            assert gsg[w] == sgo[0]
        assert abs(gacc[w, 0] - acco[0, 0]) <= n_steps * E_TOL * max(1.0, abs(acco[0, 0]) / n_steps), \
            f"{tag} walker {w}: sum E_L {gacc[w, 0]} vs {acco[0, 0]}"


def test_h2_config_every_walker(torch_cuda, oracle_mod):
    torch = torch_cuda
    sysd = synth.make_system("H2")
    W, n = synth.CONFIG_WALKERS["H2"], synth.CONFIG_STEPS["H2"]
    X0, start, out = _run_gpu(torch, sysd, W, n, n)
    o = oracle_mod.OracleSystem(sysd)
    Xo, lpo, sgo, elo, acco, _ = o.metropolis(X0, *start, n, synth.CONFIG_SIGMA, synth.PHILOX_SEED["H2"])
    gX, glp, gsg, gel, gacc = out
    assert np.array_equal(gacc[:, 2], acco[:, 2])
    assert np.max(np.abs(gX - Xo)) < 1e-9
    assert np.max(np.abs(glp - lpo) / np.maximum(1, np.abs(lpo))) <= 1e-10
    mean_gpu = gacc[:, 0].sum() / (W * n)
    mean_or = acco[:, 0].sum() / (W * n)
    print(f"H2 1024 x 200: mean energy GPU {mean_gpu:.12f} oracle {mean_or:.12f}")
    assert abs(mean_gpu - mean_or) < 1e-10


@pytest.mark.parametrize("name,W,n_steps,chunk,n_sample", [
    ("LiH", 16384, 500, 500, 24), ("Li2", 32768, 100, 100, 16), ("CO", 65536, 500, 10, 24)])
def test_config_sampled_walkers(torch_cuda, oracle_mod, name, W, n_steps, chunk, n_sample):
    torch = torch_cuda
    sysd = synth.make_system(name)
    X0, start, out = _run_gpu(torch, sysd, W, n_steps, chunk)
    idx = np.sort(np.random.default_rng(9).choice(W, n_sample, replace=False))
    idx[-1] = W - 1
    _check_walkers(oracle_mod, sysd, X0, start, out, idx, n_steps, f"{name} {W} x {n_steps}")
