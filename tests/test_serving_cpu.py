"""Serving host logic that needs no GPU: the block statistics from the
device's accumulator sums and the request stream recipe.  (Footprints come
from qmc_bytes_per_walker, which needs a device handle: the admission tests
run on the GPU.)"""
import math

import numpy as np
import pytest

from paper_2506_09743_amd import serve, synth


def test_block_statistics_from_device_sums():
    """Mean, variance and acceptance from the five sums of
    qmc_reduce_accumulators; non-finite walker-steps leave the mean."""
    rng = np.random.default_rng(0)
    W, steps = 1000, 5
    e = rng.standard_normal((W, steps)) * 3.0 - 10.0
    acc = np.c_[e.sum(1), (e * e).sum(1), rng.integers(0, 6, W), np.zeros(W)]
    sums = [acc[:, 0].sum(), acc[:, 1].sum(), acc[:, 2].sum(), 0.0, 0.0]
    mean, var, accr, bad, bad_w = serve.block_statistics(sums, W, steps)
    assert math.isclose(mean, e.mean(), rel_tol=1e-12)
    assert math.isclose(var, e.var(), rel_tol=1e-9)
    assert math.isclose(accr, acc[:, 2].sum() / (W * steps))
    assert (bad, bad_w) == (0, 0)
    # two walkers with 3 and 5 non-finite steps: their sums hold only the finite steps
    e2 = e.copy()
    e2[7, :3] = np.nan
    e2[9, :] = np.nan
    fin = np.isfinite(e2)
    s = [np.where(fin, e2, 0).sum(), np.where(fin, e2 * e2, 0).sum(), 0.0, float((~fin).sum()), 2.0]
    mean2, var2, _, bad2, bad_w2 = serve.block_statistics(s, W, steps)
    assert (bad2, bad_w2) == (8, 2)
    assert math.isclose(mean2, e2[fin].mean(), rel_tol=1e-12)
    assert math.isclose(var2, e2[fin].var(), rel_tol=1e-9)
    # nothing finite: the mean is undefined, not a division by zero
    m3 = serve.block_statistics([0.0, 0.0, 0.0, float(W * steps), float(W)], W, steps)
    assert math.isnan(m3[0]) and m3[3] == W * steps


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
