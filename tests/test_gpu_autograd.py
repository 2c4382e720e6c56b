"""The torch.autograd binding of qmc_grad.

* Gradients of a weighted sum of log|Psi| and E_L equal the explicit
  contraction of qmc_grad's per-walker Jacobians.
* An in-place parameter update rebuilds the device system: the forward pass
  then agrees with the FP64 oracle at the new parameters (eq. psimol, eq. Hmol).
* The surrogate of eq. nabla_loss / eq. force differentiates to the estimators
  assembled by hand, and one end-to-end derivative matches central finite
  differences of the oracle (h = 1e-5).
"""
import numpy as np
import pytest

from paper_2506_09743_amd import synth

pytestmark = pytest.mark.gpu


def _walkers(name, W, seed):
    import torch
    from paper_2506_09743_amd import qmc
    sysd = synth.make_system(name)
    s = qmc.System(sysd)
    X = torch.from_numpy(synth.init_walkers(sysd, W, seed)).cuda()
    lp, sg, el = s.eval(X)
    s.metropolis(X, lp, sg, el, 30, 0.2, seed)
    s.close()
    return sysd, X


def test_autograd_matches_jacobians():
    import torch
    from paper_2506_09743_amd import autograd as ag
    sysd, X = _walkers("Li2", 300, 5)
    wf = ag.Wavefunction(sysd)
    lp, sg, el = ag.psi_eloc(wf, X)
    ok = torch.isfinite(el)
    g = torch.Generator().manual_seed(0)
    a = torch.randn(X.shape[0], generator=g, dtype=torch.float64).cuda()
    b = torch.randn(X.shape[0], generator=g, dtype=torch.float64).cuda()
    loss = (a[ok] * lp[ok]).sum() + (b[ok] * el[ok]).sum()
    loss.backward()
    dl, de, dlR, deR = wf.system().grad(X)
    m = ok.double()
    want_t = (a * m) @ torch.nan_to_num(dl) + (b * m) @ torch.nan_to_num(de)
    want_R = ((a * m) @ torch.nan_to_num(dlR.reshape(len(m), -1))
              + (b * m) @ torch.nan_to_num(deR.reshape(len(m), -1))).reshape(-1, 3)
    np.testing.assert_allclose(wf.theta.grad.numpy(), want_t.cpu().numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(wf.R.grad.numpy(), want_R.cpu().numpy(), rtol=1e-12, atol=1e-12)
    assert torch.equal(sg, wf.system().eval(X)[1])
    wf.close()


def test_autograd_parameter_update(oracle_mod):
    import torch
    from paper_2506_09743_amd import autograd as ag
    sysd, X = _walkers("LiH", 256, 6)
    wf = ag.Wavefunction(sysd)
    first = wf.system()
    with torch.no_grad():
        wf.theta[-1] += 0.3
        wf.theta[2] *= 1.1
        wf.R[1, 2] += 0.05
    lp, sg, el = ag.psi_eloc(wf, X)
    assert wf.system() is not first
    d = ag.unpack_theta(sysd, wf.theta.detach().numpy(), wf.R.detach().numpy())
    rlp, rsg, rel = oracle_mod.OracleSystem(d).eval(X.cpu().numpy())
    lp, sg, el = lp.detach().cpu().numpy(), sg.cpu().numpy(), el.detach().cpu().numpy()
    ok = np.isfinite(rel)
    assert np.all(np.abs(lp[ok] - rlp[ok]) <= 1e-10 * np.maximum(1, np.abs(rlp[ok])))
    assert np.array_equal(sg[ok], rsg[ok])
    assert np.median(np.abs(el[ok] - rel[ok])) < 1e-9
    wf.close()


def test_autograd_estimators(oracle_mod):
    """eq. nabla_loss and eq. force through the surrogate, and d/db of the
    surrogate against oracle finite differences on fixed walkers."""
    import torch
    from paper_2506_09743_amd import autograd as ag
    sysd, X = _walkers("H2", 512, 7)
    wf = ag.Wavefunction(sysd)
    lp, sg, el = ag.psi_eloc(wf, X)
    E = el.detach().mean()
    surrogate = el.mean() + 2 * ((el.detach() - E) * lp).mean()
    surrogate.backward()
    dl, de, dlR, deR = wf.system().grad(X)
    W = X.shape[0]
    g_theta = (de.sum(0) + 2 * ((el.detach() - E) @ dl)) / W
    F = -(deR.sum(0) + 2 * torch.einsum("w,wad->ad", el.detach() - E, dlR)) / W
    np.testing.assert_allclose(wf.theta.grad.numpy(), g_theta.cpu().numpy(), rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(wf.R.grad.numpy(), -F.cpu().numpy(), rtol=1e-11, atol=1e-12)

    # end to end: d/db of mean(E_L) + mean(log|Psi|) by oracle FD
    h = 1e-5
    Xn = X.cpu().numpy()

    def L(db):
        th = ag.pack_theta(sysd)
        th[-1] += db
        rlp, _, rel = oracle_mod.OracleSystem(ag.unpack_theta(sysd, th, sysd["R"])).eval(Xn)
        return rel.mean() + rlp.mean()

    wf.theta.grad = None
    lp, _, el = ag.psi_eloc(wf, X)
    (el.mean() + lp.mean()).backward()
    fd = (L(h) - L(-h)) / (2 * h)
    assert abs(wf.theta.grad[-1].item() - fd) <= 2e-6 * max(1.0, abs(fd))
    wf.close()
