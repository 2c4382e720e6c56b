"""Continuous batching on the GPU: a request's result is identical alone and
in a mix of concurrently running requests, admission respects the HBM
budget, and a Poisson stream completes with latency statistics."""
import threading

import numpy as np
import pytest

from paper_2506_09743_amd import serve, synth

pytestmark = pytest.mark.gpu


def _req(i, name, w, steps=40, prec="fp64", scale=1.0):
    return serve.Request(id=i, name=name, bond_scale=scale, walkers=w, steps=steps, precision=prec,
                         walker_seed=100 + i, philox_seed=7000 + i)


def test_same_result_alone_and_in_mix():
    target = _req(0, "LiH", 3000, scale=1.4)
    s1 = serve.Server(chunk_steps=10)
    f = s1.submit(target)
    s1.run()
    alone = f.result()

    s2 = serve.Server(chunk_steps=10, max_active=6)
    others = [_req(1, "CO", 4096), _req(2, "H2", 1500, scale=2.2), _req(3, "Li2", 2500, prec="fp32"),
              _req(4, "CO", 2048, prec="fp32", scale=0.7), _req(5, "LiH", 1000, scale=2.9)]
    futs = [s2.submit(r) for r in others[:2]]
    t2 = _req(0, "LiH", 3000, scale=1.4)
    ft = s2.submit(t2)
    futs += [s2.submit(r) for r in others[2:]]
    s2.run()
    mixed = ft.result()
    assert s2.peak_active >= 4, "requests did not overlap"
    assert np.array_equal(alone.acc, mixed.acc)
    assert alone.mean_energy == mixed.mean_energy
    for f in futs:
        assert np.isfinite(f.result().mean_energy)
    print(f"alone {alone.mean_energy:.10f} mixed {mixed.mean_energy:.10f}, peak active {s2.peak_active}")


def test_admission_respects_budget():
    reqs = [_req(i, "CO", 4000, steps=20) for i in range(5)]
    one = serve.Server.footprint(reqs[0])
    s = serve.Server(hbm_budget_bytes=2 * one + 1000, chunk_steps=10)
    futs = [s.submit(r) for r in reqs]
    big = s.submit(_req(9, "CO", 200000, steps=1))
    s.run()
    assert s.peak_active == 2
    assert all(np.isfinite(f.result().mean_energy) for f in futs)
    with pytest.raises(serve.AdmissionError):
        big.result()
    assert s.used == 0


def test_poisson_stream_completes():
    stream = synth.serving_request_stream(12, 3, w_range=(1000, 4000), steps=60)
    timed = serve.requests_from_stream(stream)
    s = serve.Server(chunk_steps=20)
    import time
    t0 = time.perf_counter()
    prod = serve.poisson_producer(s, timed, rate_hz=200.0)
    res = s.run(producer=prod)
    wall = time.perf_counter() - t0
    assert len(res) == 12
    summ = serve.latency_summary(res, wall)
    assert summ["p99_s"] >= summ["p50_s"] > 0
    print(summ)
