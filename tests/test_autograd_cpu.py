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


def test_theta_round_trip_many_body():
    """With the many-body Jastrow the layout continues with the e-n
    parameters per nucleus and the e-e-n parameters per term."""
    from paper_2506_09743_amd import autograd as ag
    sysd = synth.with_many_body_jastrow(synth.make_system("Li2"), 3)
    th = ag.pack_theta(sysd)
    n_prim = sysd["prim_exp"].size
    nao, nmo = sysd["mo_coef"].shape
    p_b = n_prim + nao * nmo
    assert th.shape == (p_b + 1 + sysd["jas_en"].size + sysd["jas_een"].size,)
    assert th[p_b] == sysd["jas_b"]
    assert th[p_b + 1 + 3 * 1 + 2] == sysd["jas_en"][1, 2]
    assert th[p_b + 1 + sysd["jas_en"].size + 7 * 2 + 4] == sysd["jas_een"][2, 4]
    th2 = th.copy()
    th2[p_b + 2] += 0.25
    th2[-1] += 0.5
    d = ag.unpack_theta(sysd, th2, sysd["R"])
    assert d["jas_en"][0, 1] == sysd["jas_en"][0, 1] + 0.25
    assert d["jas_een"][-1, -1] == sysd["jas_een"][-1, -1] + 0.5
    assert np.array_equal(ag.pack_theta(d), th2)
