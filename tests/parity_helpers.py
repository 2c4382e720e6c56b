"""Shared element-by-element comparison of the HIP path with the FP64 oracle
(imported by the GPU parity tests; holds no test of its own).

Tolerances (FP64 form): |d log|Psi|| <= 1e-10 max(1, |log|Psi||), sign exact,
|d E_L| <= 1e-8 Ha inside the conditioning window: reference matrices with
condition number <= 1e8, a CI sum that does not cancel by more than 1e3
(sum |d_n D_n| / |sum d_n D_n| <= 1e3) and |E_L|, |E_kin| <= 1e4 Ha.  Walkers
outside it are counted, their worst error is printed, and they must still
satisfy |d E_L| <= 1e-12 kappa_S max(1, |E_kin|).
"""
import numpy as np

from paper_2506_09743_amd import synth

LOG_TOL, E_TOL = 1e-10, 1e-8
COND_MAX, KAPPA_S_MAX, E_MAX = 1e8, 1e3, 1e4


def _conditioning(o, sysd, X):
    """Per walker: largest condition number of the two reference Slater
    matrices (orbitals at the backflow-transformed positions when the system
    has backflow), the cancellation factor of the CI sum, and |E_kin| (from the
    oracle's MO values and plain numpy determinants)."""
    nu = sysd["n_up"]
    cond = np.ones(X.shape[0])
    kap = np.ones(X.shape[0])
    ekin = np.zeros(X.shape[0])
    for w, x in enumerate(X):
        # with backflow the matrices hold the orbitals at the transformed positions
        phi = o.mo(o.backflow(x) if sysd.get("bf_omega") else x)[:, 0, :]
        up, dn = phi[:nu], phi[nu:]
        for M, occ in ((up, sysd["occ_up"][0]), (dn, sysd["occ_dn"][0])):
            if M.size:
                cond[w] = max(cond[w], np.linalg.cond(M[:, occ]))
        terms = np.array([c * (np.linalg.det(up[:, ou]) if nu else 1.0) *
                          (np.linalg.det(dn[:, od]) if dn.size else 1.0)
                          for c, ou, od in zip(sysd["ci"], sysd["occ_up"], sysd["occ_dn"])])
        tot = abs(terms.sum())
        kap[w] = np.abs(terms).sum() / tot if tot > 0 else np.inf
        ekin[w] = abs(o.eval_one(x)["e_kin"])
    return cond, kap, ekin


def _compare(o, sysd, X, lp, sg, el, tag):
    rlp, rsg, rel = o.eval(X)
    good = np.isfinite(rlp)
    assert np.array_equal(np.isfinite(lp), good), tag
    assert np.array_equal(sg[good], rsg[good]), f"{tag}: sign mismatch"
    dlp = np.abs(lp[good] - rlp[good]) / np.maximum(1.0, np.abs(rlp[good]))
    assert dlp.max(initial=0) <= LOG_TOL, f"{tag}: log|Psi| rel err {dlp.max()}"
    cond, kap, ekin = _conditioning(o, sysd, X)
    inside = good & (cond <= COND_MAX) & (kap <= KAPPA_S_MAX) & (np.abs(rel) <= E_MAX) & (ekin <= E_MAX)
    de = np.abs(el - rel)
    assert de[inside].max(initial=0) <= E_TOL, f"{tag}: E_L err {de[inside].max()}"
    out = good & ~inside
    bound = 1e-12 * kap * np.maximum(1.0, ekin)
    assert np.all(de[out] <= bound[out]), f"{tag}: outside-window walker beyond its bound"
    n_out = int(np.sum(out))
    worst = de[out].max(initial=0)
    print(f"{tag}: W={X.shape[0]} max dlog={dlp.max(initial=0):.2e} max dE={de[inside].max(initial=0):.2e} "
          f"outside-window={n_out} (worst dE {worst:.2e})")
    return rlp, rsg, rel


def _one_step_margin(o, sysd, X, lp, seed, step, sigma, oracle_mod, offset=0):
    """|2 (log|Psi'| - log|Psi|) - ln u| per walker for one oracle step."""
    ne = X.shape[1]
    out = np.zeros(X.shape[0])
    for w in range(X.shape[0]):
        z, u = oracle_mod.proposal(ne, seed, offset + w, step)
        d = o.eval_one(X[w] + sigma * z)
        out[w] = abs(2 * (d["logpsi"] - lp[w]) - np.log(u)) if np.isfinite(d["logpsi"]) else np.inf
    return out


def good_walkers(o, sysd, n, seed):
    """Walkers where finite differences are well conditioned: electrons at
    least 0.3 bohr from nuclei and from each other, reference matrices with
    condition number < 1e3, a CI sum that cancels by less than 10x."""
    nu = sysd["n_up"]
    R = np.asarray(sysd["R"])
    out = []
    for x in synth.init_walkers(sysd, 400 * n, seed):
        if np.linalg.norm(x[:, None] - R[None], axis=-1).min() < 0.3:
            continue
        dee = np.linalg.norm(x[:, None] - x[None], axis=-1) + 9 * np.eye(len(x))
        if dee.min() < 0.3:
            continue
        phi = o.mo(x)[:, 0, :]
        up, dn = phi[:nu], phi[nu:]
        if max(np.linalg.cond(up[:, sysd["occ_up"][0]]), np.linalg.cond(dn[:, sysd["occ_dn"][0]])) > 1e3:
            continue
        t = np.array([c * np.linalg.det(up[:, a]) * np.linalg.det(dn[:, b])
                      for c, a, b in zip(sysd["ci"], sysd["occ_up"], sysd["occ_dn"])])
        if np.abs(t).sum() > 10 * abs(t.sum()):
            continue
        out.append(x)
        if len(out) == n:
            break
    assert len(out) == n
    return np.array(out)
