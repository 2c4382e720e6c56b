"""Two-stream launches of the Metropolis block (C ABI through the binding).

Large FP64 blocks run their walkers in two halves on two streams; mixed
blocks run the FP64 refinement on a second stream, one step behind, and
keep the walkers it takes until the call ends.  The results must not
depend on either: the FP64 block equals the same walkers advanced in small
single-stream batches bit for bit, and a mixed block ends with every sign
entry a sign and equals single-step calls.
"""
import numpy as np
import pytest

from paper_2506_09743_amd import synth

pytestmark = pytest.mark.gpu


def _co(torch, qmc, W, seed):
    sysd = synth.make_system("CO")
    s = qmc.System(sysd)
    X0 = torch.from_numpy(synth.init_walkers(sysd, W, seed)).cuda()
    return s, X0


def test_fp64_split_block_equals_batches(torch_cuda, qmc):
    """CO, 65536 walkers (two streams) against 16 batches of 4096 walkers
    (one stream each, walker_offset set): identical state and sums."""
    torch = torch_cuda
    W, B = 65536, 4096
    s, X0 = _co(torch, qmc, W, 21)
    lp0, sg0, el0 = s.eval(X0)
    A = [X0.clone(), lp0.clone(), sg0.clone(), el0.clone()]
    accA = s.metropolis(*A, 3, 0.2, 1234, step0=5)
    parts = []
    for lo in range(0, W, B):
        P = [t[lo:lo + B].clone() for t in (X0, lp0, sg0, el0)]
        acc = s.metropolis(*P, 3, 0.2, 1234, step0=5, walker_offset=lo)
        parts.append(P + [acc])
    torch.cuda.synchronize()
    for k in range(5):
        ref = (A + [accA])[k]
        assert torch.equal(ref, torch.cat([p[k] for p in parts])), k
    s.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_block_signs_and_single_steps(torch_cuda, qmc, prec):
    """CO, 65536 walkers: a 6-step mixed block leaves only signs in the sign
    array, and equals six 1-step calls (same walkers, same counters)."""
    torch = torch_cuda
    W = 65536
    s, X0 = _co(torch, qmc, W, 22)
    lp0, sg0, el0 = s.eval(X0, precision=prec)
    torch.cuda.synchronize()
    assert torch.all((sg0 == 1.0) | (sg0 == -1.0) | (sg0 == 0.0))
    A = [X0.clone(), lp0.clone(), sg0.clone(), el0.clone()]
    accA = s.metropolis(*A, 6, 0.2, 4321, precision=prec)
    B = [X0.clone(), lp0.clone(), sg0.clone(), el0.clone()]
    accB = torch.zeros_like(accA)
    for t in range(6):
        s.metropolis(*B, 1, 0.2, 4321, step0=t, acc=accB, precision=prec)
    torch.cuda.synchronize()
    sgA = A[2]
    assert torch.all((sgA == 1.0) | (sgA == -1.0) | (sgA == 0.0))
    same = [torch.equal(a, b) for a, b in zip(A + [accA], B + [accB])]
    acc_a, acc_b = accA.cpu().numpy(), accB.cpu().numpy()
    print(f"CO {prec} block vs single steps: arrays equal {same}; "
          f"acceptance {acc_a[:, 2].sum():.0f} vs {acc_b[:, 2].sum():.0f}")
    assert all(same)
    s.close()


@pytest.mark.parametrize("prec,B", [("fp64", 4096), ("fp32", 4096), ("bf16", 4096), ("fp32", 16384),
                                    ("bf16", 16384), ("fp64", 6000)])
def test_small_block_loop_equals_large_block(torch_cuda, qmc, prec, B):
    """Blocks of at most 1024 waves run as one looping launch (mixed forms
    refine inside it); larger ones one launch per step, mixed blocks of up
    to 8192 waves refining on the caller's stream after each step, larger
    ones on the second stream.  The first B CO walkers (4096: 1024 waves;
    16384: 4096 waves; 6000: 1500 waves, one stream) advanced alone equal
    the same walkers inside a 65536-walker block, bit for bit."""
    torch = torch_cuda
    W = 65536
    s, X0 = _co(torch, qmc, W, 23)
    lp0, sg0, el0 = s.eval(X0, precision=prec)
    A = [X0.clone(), lp0.clone(), sg0.clone(), el0.clone()]
    accA = s.metropolis(*A, 5, 0.2, 777, step0=3, precision=prec)
    P = [t[:B].clone() for t in (X0, lp0, sg0, el0)]
    accP = s.metropolis(*P, 5, 0.2, 777, step0=3, precision=prec)
    torch.cuda.synchronize()
    for k, (a, b) in enumerate(zip(A + [accA], P + [accP])):
        assert torch.equal(a[:B], b), k
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_two_host_threads_share_a_handle(torch_cuda, qmc, prec):
    """Two host threads run 4-step blocks on one handle at once, each on its
    own stream and walkers (both blocks use the handle's second stream); the
    results equal the same blocks run one after the other."""
    import threading
    torch = torch_cuda
    W = 32768 if prec == "fp64" else 65536
    s, X0 = _co(torch, qmc, W, 24)
    lp0, sg0, el0 = s.eval(X0, precision=prec)
    torch.cuda.synchronize()
    starts = [[t.clone() for t in (X0, lp0, sg0, el0)] for _ in range(2)]
    seeds = (11, 12)
    ref = []
    for k in range(2):
        st = [t.clone() for t in starts[k]]
        acc = s.metropolis(*st, 4, 0.2, seeds[k], precision=prec)
        ref.append(st + [acc])
    torch.cuda.synchronize()
    out = [None, None]
    errors = []

    def run(k):
        try:
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                st = [t.clone() for t in starts[k]]
                acc = s.metropolis(*st, 4, 0.2, seeds[k], precision=prec)
            stream.synchronize()
            out[k] = st + [acc]
        except Exception as e:  # reported below
            errors.append(e)

    th = [threading.Thread(target=run, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for k in range(2):
        for a, b in zip(ref[k], out[k]):
            assert torch.equal(a, b)
    s.close()


def test_backflow_split_block_equals_batches(torch_cuda, qmc):
    """Backflow blocks take the same two-stream split: CO with inverse
    backflow (omega = 0.1), 8192 walkers (2048 waves, two halves) against
    four single-stream batches of 2048 walkers, bit for bit."""
    torch = torch_cuda
    sysd = dict(synth.make_system("CO"))
    sysd["bf_omega"] = 0.1
    s = qmc.System(sysd)
    W, B = 8192, 2048
    X0 = torch.from_numpy(synth.init_walkers(sysd, W, 25)).cuda()
    lp0, sg0, el0 = s.eval(X0)
    A = [X0.clone(), lp0.clone(), sg0.clone(), el0.clone()]
    accA = s.metropolis(*A, 2, 0.2, 99)
    parts = []
    for lo in range(0, W, B):
        P = [t[lo:lo + B].clone() for t in (X0, lp0, sg0, el0)]
        acc = s.metropolis(*P, 2, 0.2, 99, walker_offset=lo)
        parts.append(P + [acc])
    torch.cuda.synchronize()
    for k in range(5):
        assert torch.equal((A + [accA])[k], torch.cat([p[k] for p in parts])), k
    s.close()
