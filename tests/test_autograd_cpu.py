"""Host side of the autograd binding: the theta layout of qmc_grad
(exponents | MO coefficients row-major | b) round-trips through the system
dict, and malformed parameter vectors are rejected."""
import numpy as np
import pytest

from paper_2506_09743_amd import synth


@pytest.mark.parametrize("name", ["H2", "LiH", "Li2", "CO"])
def test_theta_round_trip(name):
    from paper_2506_09743_amd import autograd as ag
    sysd = synth.make_system(name)
    th = ag.pack_theta(sysd)
    n_prim = sysd["prim_exp"].size
    nao, nmo = sysd["mo_coef"].shape
    assert th.shape == (n_prim + nao * nmo + 1,)
    # position of MO coefficient (mu, k) is n_prim + mu * n_mo + k
    mu, k = nao - 1, nmo // 2
    assert th[n_prim + mu * nmo + k] == sysd["mo_coef"][mu, k]
    assert th[-1] == sysd["jas_b"]
    th2 = th.copy()
    th2[0] += 0.5
    th2[-1] = 2.0
    R2 = sysd["R"] + 0.1
    d = ag.unpack_theta(sysd, th2, R2)
    assert d["prim_exp"][0] == sysd["prim_exp"][0] + 0.5 and d["jas_b"] == 2.0
    assert np.array_equal(d["R"], R2)
    assert np.array_equal(d["mo_coef"], sysd["mo_coef"])
    assert np.array_equal(ag.pack_theta(d), th2)
    # the base dict is untouched
    assert np.array_equal(ag.pack_theta(sysd), th)


def test_theta_shape_rejected():
    from paper_2506_09743_amd import autograd as ag
    sysd = synth.make_system("LiH")
    with pytest.raises(ValueError):
        ag.unpack_theta(sysd, ag.pack_theta(sysd)[:-1], sysd["R"])
