"""Serving host logic that needs no GPU: footprint admission refusal, the
fixed-order accumulator reduction and the request stream recipe."""
import math

import numpy as np
import pytest

from paper_2506_09743_amd import serve, synth


def test_oversize_request_is_refused():
    s = serve.Server(hbm_budget_bytes=1 << 20)
    fut = s.submit(serve.Request(id=1, name="CO", bond_scale=1.0, walkers=4096, steps=10))
    with pytest.raises(serve.AdmissionError):
        fut.result(timeout=1)


def test_footprint_matches_walker_state():
    req = serve.Request(id=1, name="LiH", bond_scale=1.3, walkers=1000, steps=10)
    assert serve.Server.footprint(req) == 1000 * (3 * 4 + 6) * 8 + (1 << 20)


def test_reduce_accumulators_fixed_order():
    rng = np.random.default_rng(0)
    acc = np.c_[rng.standard_normal(1000) * 1e6, rng.random(1000) * 1e12, rng.integers(0, 5, 1000)]
    m1 = serve.reduce_accumulators(acc, 5)
    m2 = serve.reduce_accumulators(acc.copy(), 5)
    assert m1 == m2
    assert math.isclose(m1[0], acc[:, 0].sum() / 5000, rel_tol=1e-12)
    assert math.isclose(m1[2], acc[:, 2].sum() / 5000)


def test_request_stream_recipe():
    reqs = synth.serving_request_stream(400, 7)
    names = [r["name"] for r in reqs]
    for n in ("H2", "LiH", "Li2", "CO"):
        assert 60 < names.count(n) < 140
    w = np.array([r["walkers"] for r in reqs])
    assert w.min() >= 1000 and w.max() <= 32000
    sc = np.array([r["bond_scale"] for r in reqs])
    assert sc.min() >= 0.6 and sc.max() <= 3.0
    gaps = np.array([r["gap"] for r in reqs])
    assert 0.8 < gaps.mean() < 1.2
    assert synth.serving_request_stream(400, 7) == reqs
