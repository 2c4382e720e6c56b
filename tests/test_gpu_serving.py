"""Continuous batching on the GPU: a request's result is identical alone and
in a mix of concurrently running requests, every served FP64 result equals
the oracle's Metropolis block on the same initial walkers and random stream,
admission waits for HBM (not only for stream slots) within the budget, and
a Poisson stream completes with latency statistics."""
import numpy as np
import pytest

from paper_2506_09743_amd import serve, synth

pytestmark = pytest.mark.gpu


def _req(i, name, w, steps=40, prec="fp64", scale=1.0, keep=False):
    return serve.Request(id=i, name=name, bond_scale=scale, walkers=w, steps=steps, precision=prec,
                         walker_seed=100 + i, philox_seed=7000 + i, keep_walkers=keep)


def test_same_result_alone_and_in_mix():
    target = _req(0, "LiH", 3000, scale=1.4, keep=True)
    s1 = serve.Server(chunk_steps=10)
    f = s1.submit(target)
    s1.run()
    alone = f.result()

    s2 = serve.Server(chunk_steps=10, max_active=6)
    others = [_req(1, "CO", 4096), _req(2, "H2", 1500, scale=2.2), _req(3, "Li2", 2500, prec="fp32"),
              _req(4, "CO", 2048, prec="fp32", scale=0.7), _req(5, "LiH", 1000, scale=2.9)]
    futs = [s2.submit(r) for r in others[:2]]
    t2 = _req(0, "LiH", 3000, scale=1.4, keep=True)
    ft = s2.submit(t2)
    futs += [s2.submit(r) for r in others[2:]]
    s2.run()
    mixed = ft.result()
    assert s2.peak_active >= 4, "requests did not overlap"
    assert np.array_equal(alone.initial_walkers, mixed.initial_walkers)
    assert np.array_equal(alone.acc, mixed.acc)
    assert alone.mean_energy == mixed.mean_energy
    for f in futs:
        assert np.isfinite(f.result().mean_energy)
    print(f"alone {alone.mean_energy:.10f} mixed {mixed.mean_energy:.10f}, peak active {s2.peak_active}")


def test_served_results_match_the_oracle(oracle_mod):
    """Overlapping requests of four molecules (FP64 and mixed FP32) with
    chunks that split each block over step0; every FP64 request's
    per-walker accumulators equal the oracle's Metropolis block started from
    the request's device-drawn walkers with its Philox seed and
    request-local walker ids: accept and non-finite counts exactly, the E_L
    sums within n_steps * 1e-8 (relative above 1 Ha), and the served mean is
    their reduction."""
    reqs = [_req(0, "LiH", 257, steps=30, scale=1.3, keep=True),
            _req(1, "H2", 300, steps=30, scale=2.0, keep=True),
            _req(2, "CO", 64, steps=12, keep=True),
            _req(3, "Li2", 200, steps=30, prec="fp32"),
            _req(4, "CO", 1024, steps=21, prec="fp32", scale=0.8),
            _req(5, "Li2", 129, steps=30, scale=0.8, keep=True)]
    s = serve.Server(chunk_steps=7, max_active=6)
    futs = [s.submit(r) for r in reqs]
    s.run()
    assert s.peak_active >= 3, "requests did not overlap"
    checked = 0
    for r, f in zip(reqs, futs):
        res = f.result()
        if not r.keep_walkers:
            assert np.isfinite(res.mean_energy)
            continue
        o = oracle_mod.OracleSystem(synth.make_system(r.name, bond_scale=r.bond_scale))
        X0 = res.initial_walkers
        lp, sg, el = o.eval(X0)
        _, _, _, _, acco, _ = o.metropolis(X0, lp, sg, el, r.steps, r.sigma, r.philox_seed)
        g = res.acc
        assert np.array_equal(g[:, 2], acco[:, 2]), f"request {r.id}: accept counts"
        assert np.array_equal(g[:, 3], acco[:, 3]), f"request {r.id}: non-finite counts"
        tol = r.steps * 1e-8 * np.maximum(1.0, np.abs(acco[:, 0]) / r.steps)
        assert np.all(np.abs(g[:, 0] - acco[:, 0]) <= tol), f"request {r.id}: E_L sums"
        n = r.walkers * r.steps - acco[:, 3].sum()
        ref = acco[:, 0].sum() / n
        assert abs(res.mean_energy - ref) <= 1e-8 * max(1.0, abs(ref)), f"request {r.id}: mean"
        assert res.nonfinite_steps == int(acco[:, 3].sum())
        checked += 1
        print(f"request {r.id} {r.name} W={r.walkers}: mean {res.mean_energy:.10f} oracle {ref:.10f}")
    assert checked == 4


def test_admission_waits_for_memory():
    """With a budget of two CO requests and eight stream slots, memory and
    not the slots holds the other requests; an oversize request fails."""
    reqs = [_req(i, "CO", 4000, steps=20) for i in range(5)]
    one = serve.Server(chunk_steps=10).footprint(reqs[0])
    s = serve.Server(hbm_budget_bytes=2 * one + 1000, chunk_steps=10, max_active=8)
    futs = [s.submit(r) for r in reqs]
    big = s.submit(_req(9, "CO", 200000, steps=1))
    s.run()
    assert s.peak_active == 2
    assert s.peak_used <= s.budget
    assert s.waits_memory >= 3 and s.waits_slot == 0
    assert sum(f.result().waited_for == "memory" for f in futs) >= 3
    assert all(np.isfinite(f.result().mean_energy) for f in futs)
    with pytest.raises(serve.AdmissionError):
        big.result()
    assert s.used == 0


def test_admission_waits_for_slots_and_budget_is_free_hbm():
    """The default budget is the free HBM at start minus the reserve; with
    two slots the other requests wait for a slot, not for memory."""
    import torch
    free, total = torch.cuda.mem_get_info(0)
    s = serve.Server(chunk_steps=10, max_active=2)
    reserve = max(serve.Server.RESERVE_BYTES, int(serve.Server.RESERVE_FRACTION * total))
    assert abs(s.budget - (free - reserve)) <= 64 << 20
    futs = [s.submit(_req(i, "LiH", 2000, steps=20)) for i in range(5)]
    s.run()
    assert s.peak_active == 2
    assert s.waits_slot >= 3 and s.waits_memory == 0
    assert all(np.isfinite(f.result().mean_energy) for f in futs)


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
