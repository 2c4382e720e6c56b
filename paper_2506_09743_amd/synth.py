"""Seeded synthetic systems and walker initialisations.

This module only *draws inputs*: molecular geometries, basis exponents and
contraction coefficients, orthogonal MO coefficient matrices, excitation lists,
CI weights and initial electron positions.  It holds none of the method's
arithmetic (no orbital, determinant, Jastrow or energy evaluation), so both the
FP64 oracle and the HIP path can consume the same inputs without sharing code.

A system is a plain ``dict``::

    Z, R              nuclear charges [n_atoms], positions [n_atoms, 3] (bohr)
    n_up, n_dn        electrons 0..n_up-1 are spin-up, the rest spin-down
    basis             "sto" or "gto"
    shell_atom, shell_l, shell_kn, shell_nprim      per shell
    prim_exp, prim_coef                             concatenated over shells
    normalize         1: unit-normalised primitives, 0: raw functions
    mo_coef           [n_ao, n_mo] (AO order: shells in order, Cartesian
                      components of a shell lexicographic, x-power first)
    occ_up, occ_dn    [n_det, n_up], [n_det, n_dn] MO index per column slot;
                      determinant 0 is the reference configuration
    ci                [n_det]
    jas_a_par, jas_a_anti, jas_b     Pade e-e Jastrow constants

The molecules follow the paper's test set (H2, LiH, Li2, CO; Results section)
with synthetic bases, MOs and CI vectors, because the paper's DZP/HF inputs
are not available.
"""
from __future__ import annotations

import copy
import itertools
import math

import numpy as np

SEED_BASE = 25060974
EQ_BOND = {"H2": 1.4, "LiH": 3.015, "Li2": 5.051, "CO": 2.132}


def n_cart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def n_ao(sysd: dict) -> int:
    return int(sum(n_cart(int(l)) for l in sysd["shell_l"]))


def n_elec(sysd: dict) -> int:
    return int(sysd["n_up"]) + int(sysd["n_dn"])


def _finish(d: dict) -> dict:
    d["Z"] = np.asarray(d["Z"], dtype=np.float64)
    d["R"] = np.asarray(d["R"], dtype=np.float64).reshape(-1, 3)
    for k in ("shell_atom", "shell_l", "shell_kn", "shell_nprim"):
        d[k] = np.asarray(d[k], dtype=np.int32)
    d["prim_exp"] = np.asarray(d["prim_exp"], dtype=np.float64)
    d["prim_coef"] = np.asarray(d["prim_coef"], dtype=np.float64)
    d["mo_coef"] = np.ascontiguousarray(np.asarray(d["mo_coef"], dtype=np.float64))
    n_det = len(d["ci"])
    d["occ_up"] = np.asarray(d["occ_up"], dtype=np.int32).reshape(n_det, d["n_up"])
    d["occ_dn"] = np.asarray(d["occ_dn"], dtype=np.int32).reshape(n_det, d["n_dn"])
    d["ci"] = np.asarray(d["ci"], dtype=np.float64)
    d.setdefault("normalize", 1)
    d.setdefault("jas_a_par", 0.25)
    d.setdefault("jas_a_anti", 0.5)
    d.setdefault("jas_b", 1.0)
    assert d["mo_coef"].shape[0] == n_ao(d)
    assert int(np.sum(d["shell_nprim"])) == d["prim_exp"].size == d["prim_coef"].size
    return d


def orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Q factor of a Gaussian matrix, sign-fixed so that diag(R) > 0."""
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def excitation_dets(n_up: int, n_dn: int, n_mo_up_window: int, n_det: int) -> tuple:
    """Reference determinant plus single/double excitations.

    Determinant 0 occupies MOs 0..n-1 in each spin.  Excited determinants are
    drawn round-robin from five classes (up single, down single, up double,
    down double, up single x down single), each enumerated in lexicographic
    (holes, particles) order, and the list is cut at ``n_det``.  A particle
    replaces its hole in the hole's column slot.
    """
    vu = list(range(n_up, n_mo_up_window))
    vd = list(range(n_dn, n_mo_up_window))

    def singles(n, v):
        return [((h,), (p,)) for h in range(n) for p in v]

    def doubles(n, v):
        return [(hs, ps) for hs in itertools.combinations(range(n), 2)
                for ps in itertools.combinations(v, 2)]

    classes = [
        [(s, None) for s in singles(n_up, vu)],
        [(None, s) for s in singles(n_dn, vd)],
        [(s, None) for s in doubles(n_up, vu)],
        [(None, s) for s in doubles(n_dn, vd)],
        [(a, b) for a in singles(n_up, vu) for b in singles(n_dn, vd)],
    ]
    ref_up = list(range(n_up))
    ref_dn = list(range(n_dn))
    occ_up = [ref_up]
    occ_dn = [ref_dn]
    iters = [iter(c) for c in classes]
    live = [True] * len(iters)
    while len(occ_up) < n_det and any(live):
        for ci, it in enumerate(iters):
            if not live[ci] or len(occ_up) >= n_det:
                continue
            try:
                eu, ed = next(it)
            except StopIteration:
                live[ci] = False
                continue
            ou = list(ref_up)
            od = list(ref_dn)
            if eu is not None:
                for h, p in zip(*eu):
                    ou[h] = p
            if ed is not None:
                for h, p in zip(*ed):
                    od[h] = p
            occ_up.append(ou)
            occ_dn.append(od)
    if len(occ_up) < n_det:
        raise ValueError("not enough single/double excitations for n_det")
    return (np.asarray(occ_up, dtype=np.int32).reshape(n_det, n_up),
            np.asarray(occ_dn, dtype=np.int32).reshape(n_det, n_dn))


def ci_weights(n_det: int, rng: np.random.Generator) -> np.ndarray:
    g = rng.standard_normal(n_det)
    return g / np.linalg.norm(g)


def _sto_shells(spec, atom):
    """spec: list of (l, kn, zeta)."""
    sa, sl, sk, sn, pe, pc = [], [], [], [], [], []
    for l, kn, z in spec:
        sa.append(atom)
        sl.append(l)
        sk.append(kn)
        sn.append(1)
        pe.append(z)
        pc.append(1.0)
    return sa, sl, sk, sn, pe, pc


def make_h2(bond_scale: float = 1.0, seed: int | None = None) -> dict:
    """H2: H at (0,0,+-0.7) bohr, one 1s STO per atom with zeta 1.24,
    one MO (1,1)/sqrt(2), one determinant, Pade b = 1."""
    half = 0.5 * EQ_BOND["H2"] * bond_scale
    d = dict(name="H2", Z=[1.0, 1.0], R=[[0, 0, -half], [0, 0, half]],
             n_up=1, n_dn=1, basis="sto",
             shell_atom=[0, 1], shell_l=[0, 0], shell_kn=[0, 0], shell_nprim=[1, 1],
             prim_exp=[1.24, 1.24], prim_coef=[1.0, 1.0],
             mo_coef=np.array([[1.0], [1.0]]) / math.sqrt(2.0),
             occ_up=[[0]], occ_dn=[[0]], ci=[1.0], jas_b=1.0)
    return _finish(d)


def make_lih(bond_scale: float = 1.0, seed: int | None = None) -> dict:
    """LiH: 12 STO AOs (Li 1s,1s',2s,2s',2p,2p'; H 1s,1s') with zeta ~ U[0.5,3],
    8 MOs from a sign-fixed QR of a Gaussian 12x12, 20 determinants."""
    rng = np.random.default_rng(SEED_BASE + 1 if seed is None else seed)
    zeta = rng.uniform(0.5, 3.0, size=8)
    li = [(0, 0, zeta[0]), (0, 0, zeta[1]), (0, 1, zeta[2]), (0, 1, zeta[3]),
          (1, 0, zeta[4]), (1, 0, zeta[5])]
    h = [(0, 0, zeta[6]), (0, 0, zeta[7])]
    parts = [_sto_shells(li, 0), _sto_shells(h, 1)]
    sa, sl, sk, sn, pe, pc = [sum((p[i] for p in parts), []) for i in range(6)]
    q = orthogonal(12, rng)[:, :8]
    occ_up, occ_dn = excitation_dets(2, 2, 8, 20)
    ci = ci_weights(20, rng)
    d = dict(name="LiH", Z=[3.0, 1.0], R=[[0, 0, 0], [0, 0, EQ_BOND["LiH"] * bond_scale]],
             n_up=2, n_dn=2, basis="sto", shell_atom=sa, shell_l=sl, shell_kn=sk,
             shell_nprim=sn, prim_exp=pe, prim_coef=pc, mo_coef=q,
             occ_up=occ_up, occ_dn=occ_dn, ci=ci, jas_b=1.0)
    return _finish(d)


def make_li2(bond_scale: float = 1.0, seed: int | None = None) -> dict:
    """Li2: Li at (0,0,+-2.5255), 18 STO AOs (per Li 1s,1s',2s,2p,2p') with
    zeta ~ U[0.5,4], 18 MOs from a sign-fixed QR, 10 determinants."""
    rng = np.random.default_rng(SEED_BASE + 3 if seed is None else seed)
    half = 0.5 * EQ_BOND["Li2"] * bond_scale
    parts = []
    for atom in range(2):
        z = rng.uniform(0.5, 4.0, size=5)
        spec = [(0, 0, z[0]), (0, 0, z[1]), (0, 1, z[2]), (1, 0, z[3]), (1, 0, z[4])]
        parts.append(_sto_shells(spec, atom))
    sa, sl, sk, sn, pe, pc = [sum((p[i] for p in parts), []) for i in range(6)]
    q = orthogonal(18, rng)
    occ_up, occ_dn = excitation_dets(3, 3, 18, 10)
    ci = ci_weights(10, rng)
    d = dict(name="Li2", Z=[3.0, 3.0], R=[[0, 0, -half], [0, 0, half]],
             n_up=3, n_dn=3, basis="sto", shell_atom=sa, shell_l=sl, shell_kn=sk,
             shell_nprim=sn, prim_exp=pe, prim_coef=pc, mo_coef=q,
             occ_up=occ_up, occ_dn=occ_dn, ci=ci, jas_b=1.0)
    return _finish(d)


def make_co(bond_scale: float = 1.0, seed: int | None = None) -> dict:
    """CO: C at the origin, O at (0,0,2.132); per atom two s, two p and one
    Cartesian d shell of contracted GTOs (28 AOs), 3-6 primitives per shell,
    exponents log-uniform in [0.1, 5000], Gaussian contraction coefficients;
    20 MOs (first columns of a sign-fixed 28x28 QR); 100 determinants."""
    rng = np.random.default_rng(SEED_BASE + 2 if seed is None else seed)
    sa, sl, sk, sn, pe, pc = [], [], [], [], [], []
    for atom in range(2):
        for l in (0, 0, 1, 1, 2):
            npr = int(rng.integers(3, 7))
            sa.append(atom)
            sl.append(l)
            sk.append(0)
            sn.append(npr)
            pe.extend(np.exp(rng.uniform(math.log(0.1), math.log(5000.0), size=npr)).tolist())
            pc.extend(rng.standard_normal(npr).tolist())
    q = orthogonal(28, rng)[:, :20]
    occ_up, occ_dn = excitation_dets(7, 7, 20, 100)
    ci = ci_weights(100, rng)
    d = dict(name="CO", Z=[6.0, 8.0], R=[[0, 0, 0], [0, 0, EQ_BOND["CO"] * bond_scale]],
             n_up=7, n_dn=7, basis="gto", shell_atom=sa, shell_l=sl, shell_kn=sk,
             shell_nprim=sn, prim_exp=pe, prim_coef=pc, mo_coef=q,
             occ_up=occ_up, occ_dn=occ_dn, ci=ci, jas_b=1.0)
    return _finish(d)


def make_max_shape(seed: int | None = None) -> dict:
    """A synthetic system at the largest shape the kernels are compiled
    for: two Z = 8 nuclei 2.28 bohr apart, 8 up + 8 down electrons, per atom
    four s, two p and one Cartesian d shell of contracted GTOs (32 AOs, 2-4
    primitives per shell, exponents log-uniform in [0.1, 500]), 32 MOs
    (a sign-fixed 32x32 QR), 60 determinants."""
    rng = np.random.default_rng(SEED_BASE + 7 if seed is None else seed)
    sa, sl, sk, sn, pe, pc = [], [], [], [], [], []
    for atom in range(2):
        for l in (0, 0, 0, 0, 1, 1, 2):
            npr = int(rng.integers(2, 5))
            sa.append(atom)
            sl.append(l)
            sk.append(0)
            sn.append(npr)
            pe.extend(np.exp(rng.uniform(math.log(0.1), math.log(500.0), size=npr)).tolist())
            pc.extend(rng.standard_normal(npr).tolist())
    q = orthogonal(32, rng)
    occ_up, occ_dn = excitation_dets(8, 8, 32, 60)
    ci = ci_weights(60, rng)
    d = dict(name="max-shape", Z=[8.0, 8.0], R=[[0, 0, -1.14], [0, 0, 1.14]],
             n_up=8, n_dn=8, basis="gto", shell_atom=sa, shell_l=sl, shell_kn=sk,
             shell_nprim=sn, prim_exp=pe, prim_coef=pc, mo_coef=q,
             occ_up=occ_up, occ_dn=occ_dn, ci=ci, jas_b=1.0)
    return _finish(d)


MAKERS = {"H2": make_h2, "LiH": make_lih, "Li2": make_li2, "CO": make_co}

# Walker counts and block lengths of the four workloads.
CONFIG_WALKERS = {"H2": 1024, "LiH": 16384, "CO": 65536, "Li2": 32768}
CONFIG_STEPS = {"H2": 200, "LiH": 500, "CO": 500, "Li2": 500}
CONFIG_SIGMA = 0.2
WALKER_SEED = {"H2": 1000, "LiH": 1001, "CO": 1002, "Li2": 1003}
PHILOX_SEED = {"H2": 0x250609740000, "LiH": 0x250609740001,
               "CO": 0x250609740002, "Li2": 0x250609740003}


_BASE_SYSTEMS: dict = {}


def make_system(name: str, bond_scale: float = 1.0, seed: int | None = None) -> dict:
    """A fresh copy of the named system at bond length bond_scale x
    equilibrium.  Only the nuclear positions depend on the bond length (all
    four molecules sit on the z axis with positions proportional to it), so
    the drawn tables are made once per (name, seed) and copied."""
    key = (name, seed)
    if key not in _BASE_SYSTEMS:
        _BASE_SYSTEMS[key] = MAKERS[name](bond_scale=1.0, seed=seed)
    d = copy.deepcopy(_BASE_SYSTEMS[key])
    d["R"] = d["R"] * float(bond_scale)
    return d


def with_sd_expansion(sysd: dict, n_active: int, seed: int) -> dict:
    """A copy of ``sysd`` whose determinant list is SD(n_active, n_active):
    the reference plus every single and double excitation (total rank <= 2
    over both spins) of n_active / 2 electrons per spin from the highest
    occupied orbitals into the n_active / 2 lowest virtual orbitals of that
    spin.  An excitation replaces the hole's orbital in its slot.  CI weights:
    1 for the reference, N(0, 0.05^2) for the others."""
    k = n_active // 2
    if 2 * k != n_active or k < 1:
        raise ValueError("n_active must be a positive even number")
    nu, nd = int(sysd["n_up"]), int(sysd["n_dn"])
    n_mo = np.asarray(sysd["mo_coef"]).shape[1]
    if k > min(nu, nd) or max(nu, nd) + k > n_mo:
        raise ValueError("active space does not fit the orbitals")

    def spin_configs(n):
        ref = list(range(n))
        holes = list(range(n - k, n))
        parts = list(range(n, n + k))
        out = {0: [ref], 1: [], 2: []}
        for h in holes:
            for p in parts:
                c = ref.copy()
                c[h] = p
                out[1].append(c)
        for h1, h2 in itertools.combinations(holes, 2):
            for p1, p2 in itertools.combinations(parts, 2):
                c = ref.copy()
                c[h1], c[h2] = p1, p2
                out[2].append(c)
        return out

    up, dn = spin_configs(nu), spin_configs(nd)
    occ_up, occ_dn = [], []
    for ru in (0, 1, 2):
        for rd in (0, 1, 2):
            if ru + rd > 2:
                continue
            for cu in up[ru]:
                for cd in dn[rd]:
                    occ_up.append(cu)
                    occ_dn.append(cd)
    rng = np.random.default_rng(seed)
    ci = rng.normal(0.0, 0.05, len(occ_up))
    ci[0] = 1.0
    d = dict(sysd)
    d["occ_up"] = np.asarray(occ_up, dtype=np.int32).reshape(len(occ_up), nu)
    d["occ_dn"] = np.asarray(occ_dn, dtype=np.int32).reshape(len(occ_dn), nd)
    d["ci"] = ci
    return d


MBJ_SEED = {"H2": 2000, "LiH": 2001, "CO": 2002, "Li2": 2003}


def with_many_body_jastrow(sysd: dict, seed: int, n_terms: int = 5, symmetric: bool = True) -> dict:
    """A copy of ``sysd`` with the many-body Jastrow terms drawn:
    ``jas_en`` [n_atoms, 3] = (omega0, omega1, omega2) per nucleus with
    omega0 ~ U[-0.2, 0.2], omega1 ~ U[-0.05, 0] (no growth at large r),
    omega2 ~ U[0.5, 2]; ``jas_een`` [n_terms, 7] = (c, a1, b1, a2, b2, a3, b3)
    with c ~ N(0, 0.05^2), a ~ U[0.2, 1], b ~ U[0.5, 2].  ``symmetric``
    draws a2 = a1 and b2 = b1, so exp(J) is symmetric under the exchange of
    any two electrons."""
    rng = np.random.default_rng(seed)
    d = dict(sysd)
    na = len(sysd["Z"])
    en = np.empty((na, 3))
    en[:, 0] = rng.uniform(-0.2, 0.2, na)
    en[:, 1] = rng.uniform(-0.05, 0.0, na)
    en[:, 2] = rng.uniform(0.5, 2.0, na)
    een = np.empty((n_terms, 7))
    een[:, 0] = rng.normal(0.0, 0.05, n_terms)
    for k in (1, 3, 5):
        een[:, k] = rng.uniform(0.2, 1.0, n_terms)
        een[:, k + 1] = rng.uniform(0.5, 2.0, n_terms)
    if symmetric:
        een[:, 3], een[:, 4] = een[:, 1], een[:, 2]
    d["jas_en"] = en
    d["jas_een"] = een
    return d


def electron_atoms(sysd: dict) -> list:
    """Home atom of each electron: atoms filled by nuclear charge in atom
    order, spins alternating up/down; returns the atom index per electron in
    the (all up, then all down) electron order."""
    Z = np.asarray(sysd["Z"])
    seq = []
    for a, z in enumerate(Z):
        seq.extend([a] * int(round(z)))
    n_up, n_dn = int(sysd["n_up"]), int(sysd["n_dn"])
    ups, dns = [], []
    k = 0
    while len(ups) < n_up or len(dns) < n_dn:
        a = seq[k % len(seq)] if seq else 0
        if (k % 2 == 0 and len(ups) < n_up) or len(dns) >= n_dn:
            ups.append(a)
        else:
            dns.append(a)
        k += 1
    return ups + dns


def init_walkers(sysd: dict, n_walkers: int, seed: int) -> np.ndarray:
    """[W, N_e, 3] positions: each electron at its home nucleus + N(0, I)."""
    rng = np.random.default_rng(seed)
    home = np.asarray(sysd["R"])[electron_atoms(sysd)]
    x = rng.standard_normal((n_walkers, n_elec(sysd), 3))
    return np.ascontiguousarray(x + home[None, :, :])


def init_walkers_device(sysd: dict, n_walkers: int, seed: int, device):
    """[W, N_e, 3] positions drawn on a GPU: each electron at its home nucleus
    + N(0, I), from torch's generator seeded with ``seed`` on ``device``
    (a different stream of numbers than init_walkers' for the same seed).
    The draw runs on the current stream, so a request can start without a
    host round trip."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    home = torch.as_tensor(np.asarray(sysd["R"])[electron_atoms(sysd)], dtype=torch.float64, device=device)
    x = torch.randn((n_walkers, n_elec(sysd), 3), generator=g, dtype=torch.float64, device=device)
    return (x + home).contiguous()


def single_atom(Z: float, zeta: float, n_up: int = 1, n_dn: int = 0,
                basis: str = "sto", l: int = 0, kn: int = 0, normalize: int = 1,
                a_par: float = 0.25, a_anti: float = 0.5, b: float = 1.0) -> dict:
    """One nucleus at the origin, one shell (STO or one-primitive GTO),
    every electron of a spin in the shell's first Cartesian component."""
    nc = n_cart(l)
    d = dict(name="atom", Z=[Z], R=[[0.0, 0.0, 0.0]], n_up=n_up, n_dn=n_dn, basis=basis,
             shell_atom=[0], shell_l=[l], shell_kn=[kn], shell_nprim=[1],
             prim_exp=[zeta], prim_coef=[1.0], normalize=normalize,
             mo_coef=np.eye(nc)[:, :1], occ_up=[[0] * n_up], occ_dn=[[0] * n_dn], ci=[1.0],
             jas_a_par=a_par, jas_a_anti=a_anti, jas_b=b)
    return _finish(d)


def serving_request_stream(n_requests: int, seed: int, mix=("H2", "LiH", "Li2", "CO"),
                           w_range=(1000, 32000), steps: int = 500) -> list:
    """Request descriptors for the serving workload: molecule drawn from the
    mix in equal shares, bond length U[0.6, 3.0] x equilibrium, walker count
    log-uniform in ``w_range``, precision alternating FP64/mixed, and an
    exponential inter-arrival gap of unit mean (scaled by the caller)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_requests):
        name = mix[int(rng.integers(len(mix)))]
        scale = float(rng.uniform(0.6, 3.0))
        w = int(round(math.exp(rng.uniform(math.log(w_range[0]), math.log(w_range[1])))))
        prec = "fp64" if rng.random() < 0.5 else "fp32"
        gap = float(rng.exponential(1.0))
        reqs.append(dict(id=i, name=name, bond_scale=scale, walkers=w, steps=steps,
                         precision=prec, gap=gap, walker_seed=int(rng.integers(1 << 31)),
                         philox_seed=int(rng.integers(1 << 62))))
    return reqs
