"""Finite-difference kinetic energy (qmc_eval_eloc_fd), the baseline of the
trace-formula ablation: the HIP result equals central differences of the
oracle's own Psi at the same points (same formula, both FP64), converges to
the Jacobi-trace E_L at second order in h on well-conditioned walkers, and
rejects bad steps and backflow systems."""
import numpy as np
import pytest

from paper_2506_09743_amd import synth
from parity_helpers import good_walkers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _oracle_fd(o, x, h):
    d0 = o.eval_one(x)
    lp0, s0 = d0["logpsi"], d0["sign"]
    lap = 0.0
    for e in range(x.shape[0]):
        for c in range(3):
            for step in (h, -h):
                y = x.copy()
                y[e, c] += step
                d = o.eval_one(y)
                lap += d["sign"] * s0 * np.exp(d["logpsi"] - lp0) - 1.0
    return lp0, -0.5 * lap / (h * h) + d0["e_pot"]


@pytest.mark.parametrize("name,W,h", [("H2", 40, 1e-3), ("LiH", 33, 1e-3), ("Li2", 20, 2e-3), ("CO", 12, 1e-3)])
def test_fd_equals_oracle_fd(torch_cuda, oracle_mod, name, W, h):
    from paper_2506_09743_amd import qmc
    torch = torch_cuda
    sysd = synth.make_system(name)
    o = oracle_mod.OracleSystem(sysd)
    X = good_walkers(o, sysd, W, 91)
    s = qmc.System(sysd)
    lp, el = [t.cpu().numpy() for t in s.eval_fd(torch.from_numpy(X).cuda(), h)]
    ref = np.array([_oracle_fd(o, x, h) for x in X])
    ekin = np.array([abs(o.eval_one(x)["e_kin"]) for x in X])
    assert np.max(np.abs(lp - ref[:, 0]) / np.maximum(1, np.abs(ref[:, 0]))) < 1e-10
    d = np.abs(el - ref[:, 1]) / np.maximum(1.0, ekin)
    print(f"{name}: FD vs oracle FD, max |dE_L| / max(1, |E_kin|) {d.max():.2e}")
    # both sides round log|Psi| differences at 1e-14 relative, amplified by 1/h^2
    assert d.max() < 1e-5
    s.close()


@pytest.mark.parametrize("name", ["LiH", "Li2"])
def test_fd_converges_to_trace(torch_cuda, oracle_mod, name):
    from paper_2506_09743_amd import qmc
    torch = torch_cuda
    sysd = synth.make_system(name)
    o = oracle_mod.OracleSystem(sysd)
    X = torch.from_numpy(good_walkers(o, sysd, 64, 92)).cuda()
    s = qmc.System(sysd)
    _, _, el = s.eval(X)
    el = el.cpu().numpy()
    errs = []
    for h in (4e-3, 2e-3):
        _, ef = s.eval_fd(X, h)
        errs.append(np.median(np.abs(ef.cpu().numpy() - el)))
    print(f"{name}: median |FD - trace| at h = 4e-3, 2e-3: {errs[0]:.2e}, {errs[1]:.2e}")
    assert errs[1] < errs[0] / 3.0   # second order: ratio 4
    assert errs[1] < 1e-3
    s.close()


def test_fd_empty_batch(torch_cuda):
    from paper_2506_09743_amd import qmc
    torch = torch_cuda
    s = qmc.System(synth.make_system("LiH"))
    X = torch.empty((0, 4, 3), dtype=torch.float64, device="cuda")
    lp, el = s.eval_fd(X, 1e-3)
    assert lp.numel() == 0 and el.numel() == 0
    s.close()


def test_fd_rejects(torch_cuda):
    from paper_2506_09743_amd import qmc
    torch = torch_cuda
    sysd = synth.make_system("LiH")
    s = qmc.System(sysd)
    X = torch.from_numpy(synth.init_walkers(sysd, 4, 1)).cuda()
    for h, status in ((0.0, qmc.QMC_EINVAL), (-1e-3, qmc.QMC_EINVAL), (float("nan"), qmc.QMC_ENONFINITE),
                      (float("inf"), qmc.QMC_ENONFINITE)):
        with pytest.raises(qmc.QmcError) as e:
            s.eval_fd(X, h)
        assert e.value.status == status
    s.close()
    bf = dict(sysd)
    bf["bf_omega"] = 0.2
    sb = qmc.System(bf)
    with pytest.raises(qmc.QmcError) as e:
        sb.eval_fd(X, 1e-3)
    assert e.value.status == qmc.QMC_EUNSUPPORTED
    sb.close()
