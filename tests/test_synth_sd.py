"""SD(n, n) determinant expansions used by the determinant-count sweep.

The paper's runtime figure runs CO from SD(2,2) to SD(10,10), i.e. from 4 to
876 determinants (appendix on computational performance).  With k = n/2
active electrons and k active virtual orbitals per spin, singles and doubles
number 1 + 2 k^2 + 2 C(k,2)^2 + k^4.
"""
import math

import numpy as np
import pytest

from paper_2506_09743_amd import synth


def test_counts_match_the_paper_endpoints_and_combinatorics():
    co = synth.make_system("CO")
    counts = [len(synth.with_sd_expansion(co, n, 0)["ci"]) for n in (2, 4, 6, 8, 10)]
    assert counts[0] == 4 and counts[-1] == 876
    for n, c in zip((2, 4, 6, 8, 10), counts):
        k = n // 2
        assert c == 1 + 2 * k * k + 2 * math.comb(k, 2) ** 2 + k ** 4


@pytest.mark.parametrize("n", [2, 6, 10])
def test_excitations_are_singles_and_doubles_in_the_active_space(n):
    co = synth.make_system("CO")
    d = synth.with_sd_expansion(co, n, 1)
    k = n // 2
    ref_u, ref_d = d["occ_up"][0], d["occ_dn"][0]
    seen = set()
    for ou, od in zip(d["occ_up"], d["occ_dn"]):
        key = (tuple(ou), tuple(od))
        assert key not in seen
        seen.add(key)
        ru = int(np.sum(ou != ref_u))
        rd = int(np.sum(od != ref_d))
        assert ru + rd <= 2
        for o, ref, ns in ((ou, ref_u, co["n_up"]), (od, ref_d, co["n_dn"])):
            holes = np.nonzero(o != ref)[0]
            assert np.all(holes >= ns - k)
            assert np.all((o[holes] >= ns) & (o[holes] < ns + k))
    assert d["ci"][0] == 1.0
