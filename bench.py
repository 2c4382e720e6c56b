"""Throughput of all-electron Metropolis sampling with Psi and E_L on one
MI355X: walker-steps/s for the synthetic CO system at 65536 walkers.

One benchmark step is one all-electron Metropolis step of every walker:
Philox proposal, Psi and E_L at the proposal, accept/reject, accumulation of
E_L.  Steps are launched as blocks of --chunk steps (qmc_metropolis_block);
walker state stays in HBM between blocks.  The timed region starts from an
equilibrated state (burn-in) with all inputs resident on the device.

Prints one JSON line (see the keys below).  The FP64 form is `value`; the
mixed forms are reported beside it with their energy errors against the FP64
oracle over every walker: FP32 (FP32 AOs and MO value contraction on the
vector units) and BF16 (FP32 AOs, MO value contraction as split-BF16
matrix-core products with FP32 accumulation); both keep the proposal, pair
terms, determinants, Jacobi-trace contraction and E_L in FP64.  p50/p99 are
over at least 20 repeated blocks.  The compact per-form summary is the
line's last key, `forms`.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU = 78.6e12   # MI355X FP64 vector FLOP/s
PEAK_FP32_VALU = 157.3e12  # MI355X FP32 vector FLOP/s (published)
PEAK_BF16_MFMA = 2.5e15    # MI355X dense BF16 matrix FLOP/s
PEAK_HBM = 8.0e12          # bytes/s

# Algorithmic work of one CO walker-step (flop), from the hot-path formulas
# at the low-rank determinant method's cost: AO values/gradients/Laplacians
# 22k, the five-channel MO contraction 2 * 5 * 14 * 28 * 20 = 78.4k, LU, T
# and channel products 20k, 100-determinant traces 26k, pairs 3k.  The
# roofline's `achieved` uses this per-unit figure; flops_per_walker_step is
# this build's own term-by-term recount (the kernel reassociates the
# per-determinant traces into one adjoint vector per electron).
CO_FLOPS = {"ao": 22.0e3, "mo": 78.4e3, "lu_channels": 20.0e3, "traces": 26.0e3, "pairs": 3.0e3}
CO_FLOPS_PER_WALKER_STEP = 1.45e5


def mixed_peak(form: str) -> dict:
    """Blended peak of a mixed form on the CO work: AO evaluation and the
    value channel of the MO contraction at the FP32 vector peak (the BF16
    forms' contraction at the BF16 matrix peak), the rest (the four
    derivative channels, which become the FP64 Jacobi-trace contraction, the
    determinant algebra and the pairs) at the FP64 peak."""
    total = CO_FLOPS_PER_WALKER_STEP
    f_ao, f_val = CO_FLOPS["ao"], CO_FLOPS["mo"] / 5
    f64 = total - f_ao - f_val
    t = f64 / PEAK_FP64_VALU + f_ao / PEAK_FP32_VALU
    t += f_val / (PEAK_BF16_MFMA if form.startswith("bf16") else PEAK_FP32_VALU)
    return {"peak_flops": total / t, "fp64_flop": f64, "fp32_flop": f_ao + (0 if form.startswith("bf16") else f_val),
            "bf16_flop": f_val if form.startswith("bf16") else 0.0}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "co_metropolis_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2506_09743_amd", "csrc", f)
                  for f in ("qmc_kernels.h", "qmc_form_fp64.hip", "qmc_walker.h", "qmc_backflow.h",
                            "qmc_device.h", "qmc_api.hip")]


def flops_per_walker_step(sysd) -> dict:
    """Algorithmic FP operations of one walker-step (FMA = 2, add/mul/div = 1,
    exp/log/sqrt/sin/cos = 1), counted from the method's formulas at the cost
    of the low-rank excited-determinant scheme; pairs counted once."""
    from paper_2506_09743_amd import synth
    ne, nu, nd = synth.n_elec(sysd), int(sysd["n_up"]), int(sysd["n_dn"])
    na = len(sysd["Z"])
    nmo = int(np.asarray(sysd["mo_coef"]).shape[1])
    nao = synth.n_ao(sysd)
    ndet = len(sysd["ci"])
    sto = sysd["basis"] == "sto"
    f = {}
    f["proposal"] = ne * (6 + 3 * 2 + 7)                    # x + sigma z, Box-Muller
    per_prim = 17 if sto else 13
    n_prim = int(np.sum(sysd["shell_nprim"]))
    n_sh = len(sysd["shell_l"])
    f["ao"] = ne * (n_sh * 10 + n_prim * per_prim + nao * 10)
    f["mo"] = ne * 2 * 5 * nao * nmo                         # 5 channels
    f["lu"] = sum(2 * n * n * nmo for n in (nu, nd))         # Gauss-Jordan on [A0 | Phi]
    f["dets"] = ndet * 8                                      # k<=2 minors, CI sum
    n_ex = 0
    for occ, n in ((sysd["occ_up"], nu), (sysd["occ_dn"], nd)):
        for row in np.asarray(occ):
            k = int(np.sum(np.asarray(row) >= n))
            n_ex += {0: 0, 1: 1, 2: 4}.get(k, 4)
    f["cofactors"] = n_ex * 6
    f["traces"] = sum(n * (4 * n * (nmo - n) + 8 * nmo) for n in (nu, nd))
    f["pairs"] = (ne * (ne - 1) // 2) * 25 + ne * na * 9
    f["eloc"] = ne * 15 + 10
    f["accept"] = 6
    if sysd.get("jas_en") is not None:
        # per electron-nucleus pair: r, K, K', K'' (one division), gradient, Laplacian
        f["jastrow_en"] = ne * na * 20
    n_een = 0 if sysd.get("jas_een") is None else int(np.asarray(sysd["jas_een"]).shape[0])
    if n_een:
        # per nucleus, pair i > j and term: three factors with first and second
        # derivatives (3 divisions), the value, both electrons' gradients and
        # Laplacians by the product rule
        f["jastrow_een"] = na * (ne * (ne - 1) // 2) * n_een * 65 + ne * na * 12
    f["total"] = sum(f.values())
    return f


def backflow_flops_per_walker_step(sysd, low_rank: bool = True) -> dict:
    """Algorithmic FP operations of one walker-step with the inverse backflow
    (same counting rules): the map q, the Jacobian blocks and their products
    Y_ii' = sum_j J_ij J_i'j, AO values, gradients and contracted Hessians at
    q with the MO contraction of five channels, per configuration its
    determinant algebra (low_rank: the reference rows [A0 | Phi], Mt0 and
    the residual rows Z once, then per configuration the k x k minor and the
    rank-k update of the Mt rows; otherwise a Gauss-Jordan inverse and the Mt
    rows per configuration), the second and third traces of eq. nabla_d and
    the other spin's Y g, per determinant its weight and cross term, and the
    gradient assembly sum_i J_ij g_i.  Both traces and the cross term are
    sums over pairs symmetric in (i, i'), so Y blocks and trace terms count
    once per unordered same-spin pair and once per up-down pair."""
    from paper_2506_09743_amd import synth
    ne, nu, nd = synth.n_elec(sysd), int(sysd["n_up"]), int(sysd["n_dn"])
    na = len(sysd["Z"])
    nmo = int(np.asarray(sysd["mo_coef"]).shape[1])
    nao = synth.n_ao(sysd)
    sto = sysd["basis"] == "sto"
    n_prim = int(np.sum(sysd["shell_nprim"]))
    n_sh = len(sysd["shell_l"])
    ncfg = [len({tuple(r) for r in np.asarray(sysd[k]).reshape(len(sysd["ci"]), -1).tolist()})
            for k in ("occ_up", "occ_dn")]
    f = {}
    f["proposal"] = ne * (6 + 3 * 2 + 7)
    f["pairs"] = (ne * (ne - 1) // 2) * 25 + ne * na * 9
    f["bf_map"] = ne * (ne - 1) * 35
    n_blocks = nu * (nu + 1) // 2 + nd * (nd + 1) // 2 + nu * nd  # Y blocks over unordered pairs
    f["jacobian_products"] = ne * ne * 12 + n_blocks * ne * 54
    f["ao"] = ne * (n_sh * 20 + n_prim * ((17 if sto else 13) + 6) + nao * 40)
    f["mo"] = ne * 2 * 5 * nao * nmo
    cf = 0
    for spin, n, no, nc in (("up", nu, nd, ncfg[0]), ("dn", nd, nu, ncfg[1])):
        if low_rank:
            f["reference_" + spin] = 2 * n * n * nmo + 6 * n ** 3 + 2 * n * n + 8 * n * n * (nmo - n)
            cf += nc * (12 + 2 * n * n * 10 + 2 * n + 24 * n * (n + 1) + 12 * n * no)
        else:
            cf += nc * (2 * n ** 3 + 6 * n ** 3 + 2 * n * n + 24 * n * (n + 1) + 12 * n * no)
    f["configurations"] = cf
    f["determinants"] = len(sysd["ci"]) * (4 + 6 * ne)
    f["gradient"] = ne * ne * 30
    f["eloc"] = ne * 15 + 10
    f["accept"] = 6
    f["total"] = sum(f.values())
    return f


def grad_flops_per_walker(sysd) -> dict:
    """Algorithmic FP operations of one walker's qmc_grad, term by term from
    the adjoint's formulas (same counting rules as flops_per_walker_step;
    a Dual operation counts as the value's and the derivative's flops):
      forward      the evaluation (Psi, E_L) without proposal and accept
      direction_B  B[e][m] = sum_mu C[mu][m] (lap chi + 2 grad J . grad chi):
                   radial sums with second derivatives per primitive, AO
                   gradient and beta per AO, the contraction 2 n_ao n_mo
      fwd_dets     Z = B - B0 T, Tdot = A0^-1 Z, Ainvdot, rho_dot and Sdot per
                   determinant, Cdot per cofactor contribution, adot
      main_pass    per electron and AO: t = C a and tdot = C adot (4 n_mo),
                   grad chi, (Hess chi) . grad J, grad lap chi and the force
                   sums; per primitive the exponent derivatives
      mo_coef      chi (x) a and adot (x) chi + a (x) beta over the electrons
      jastrow_dirs one Dual pass of the Jastrow stage per direction (b, the
                   many-body parameters, the nuclear coordinates when the
                   Jastrow depends on them)"""
    from paper_2506_09743_amd import synth
    fw = flops_per_walker_step(sysd)
    ne, nao = synth.n_elec(sysd), synth.n_ao(sysd)
    nu, nd = int(sysd["n_up"]), int(sysd["n_dn"])
    nmo = int(np.asarray(sysd["mo_coef"]).shape[1])
    n_prim = int(np.asarray(sysd["prim_exp"]).size)
    na = len(sysd["Z"])
    ndet = len(sysd["ci"])
    n_en = 3 * na if sysd.get("jas_en") is not None else 0
    n_een = 0 if sysd.get("jas_een") is None else int(np.asarray(sysd["jas_een"]).shape[0])
    f = {"forward": fw["total"] - fw["proposal"] - fw["accept"]}
    f["direction_B"] = ne * (n_prim * 30 + nao * 30 + 2 * nao * nmo)
    fd = 0
    for n in (nu, nd):
        fd += 2 * n * n * (nmo - n) + 2 * n ** 3 + 2 * n * n * nmo + 8 * n * (nmo - n) * n
    f["fwd_dets"] = fd + ndet * 16 + fw["cofactors"] * 2
    f["main_pass"] = ne * (n_prim * 30 + nao * (4 * nmo + 80) + n_prim * 40)
    f["mo_coef"] = 6 * ne * nao * nmo
    # each direction evaluates only the terms that depend on its entry
    dirs = ne * (ne - 1) * 75                                   # b: the Pade pairs
    dirs += n_en * ne * 60                                      # e-n parameter: one nucleus
    dirs += 7 * n_een * ne * ((ne - 1) * na * 120 + na * 20)    # e-e-n parameter: one term
    if n_en or n_een:                                           # nuclear coordinate: one nucleus
        dirs += 3 * na * ne * ((60 if n_en else 0) + (ne - 1) * n_een * 120 + n_een * 20)
    f["jastrow_dirs"] = dirs
    f["total"] = sum(f.values())
    return f


def hbm_bytes_per_launch(sysd, W: int, steps: int) -> int:
    """Walker state read and written once per step (the FP64 block takes one
    kernel per step): X, log|Psi|, sign, E_L and four accumulators, FP64."""
    from paper_2506_09743_amd import synth
    per = (3 * synth.n_elec(sysd) + 7) * 8
    return 2 * per * W * steps


def kernel_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    or None when the kernel sources changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha") != kernel_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def conditioning_window(o, sysd, X):
    """Per walker: inside the FP64 tolerance window (largest reference Slater
    condition number <= 1e8, CI cancellation sum |d_n D_n| / |sum d_n D_n|
    <= 1e3, |E_L| and |E_kin| <= 1e4 Ha), from the oracle's orbitals and
    plain numpy determinants."""
    nu = int(sysd["n_up"])
    inside = np.zeros(X.shape[0], dtype=bool)
    for w, x in enumerate(X):
        phi = o.mo(x)[:, 0, :]
        up, dn = phi[:nu], phi[nu:]
        cond = max(np.linalg.cond(up[:, sysd["occ_up"][0]]), np.linalg.cond(dn[:, sysd["occ_dn"][0]]))
        terms = np.array([c * np.linalg.det(up[:, ou]) * np.linalg.det(dn[:, od])
                          for c, ou, od in zip(sysd["ci"], sysd["occ_up"], sysd["occ_dn"])])
        tot = abs(terms.sum())
        kap = np.abs(terms).sum() / tot if tot > 0 else np.inf
        d = o.eval_one(x)
        inside[w] = cond <= 1e8 and kap <= 1e3 and abs(d["eloc"]) <= 1e4 and abs(d["e_kin"]) <= 1e4
    return inside


def cpu_baseline(sysd, X_host, lp, sg, el, seed, target_s: float) -> dict:
    """The FP64 oracle's Metropolis block on the host cores, on a bounded
    sample of the same equilibrated walkers."""
    import oracle
    o = oracle.OracleSystem(sysd)
    threads = oracle.max_threads()
    nw = min(4096, X_host.shape[0])
    probe_w, probe_s = min(256, nw), 2
    t0 = time.perf_counter()
    o.metropolis(X_host[:probe_w], lp[:probe_w], sg[:probe_w], el[:probe_w], probe_s, 0.2, seed)
    rate = probe_w * probe_s / max(time.perf_counter() - t0, 1e-9)
    steps = max(1, min(200, int(target_s * rate / nw)))
    t0 = time.perf_counter()
    o.metropolis(X_host[:nw], lp[:nw], sg[:nw], el[:nw], steps, 0.2, seed, step0=10_000_000)
    dt = time.perf_counter() - t0
    return {"value": nw * steps / dt, "unit": "walker-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{nw} of the equilibrated CO walkers x {steps} Metropolis steps "
                      f"({dt:.1f} s, explicit per-determinant LU)"}


def serving_bench(n_requests: int, steps: int, seed: int = 2506, rates=(0.5, 0.8, 1.1)) -> dict:
    """Poisson stream of H2/LiH/Li2/CO requests (bond x U[0.6, 3.0],
    walkers log-uniform in [1k, 32k], FP64 or mixed, one block of `steps`
    steps each).  A closed-loop pass (all requests at t = 0) measures the
    capacity; the same stream then arrives at each fraction of that rate in
    `rates`.  The headline p50/p99 request latency is the 0.8x pass."""
    from paper_2506_09743_amd import serve, synth
    stream = synth.serving_request_stream(n_requests, seed, steps=steps)
    srv = serve.Server(chunk_steps=50)
    t0 = time.perf_counter()
    for _, req in serve.requests_from_stream(stream):
        srv.submit(req)
    srv.run()
    closed_wall = time.perf_counter() - t0
    capacity = n_requests / closed_wall
    sweep = {}
    for f in rates:
        srv = serve.Server(chunk_steps=50)
        t0 = time.perf_counter()
        prod = serve.poisson_producer(srv, serve.requests_from_stream(stream), f * capacity)
        res = srv.run(producer=prod)
        wall = time.perf_counter() - t0
        out = serve.latency_summary(res, wall)
        out.update({"rate_hz": f * capacity, "peak_active": srv.peak_active,
                    "mean_active": srv.overlap_active_sum / max(1, srv.overlap_samples),
                    "admissions_waited_for_memory": srv.waits_memory,
                    "admissions_waited_for_slot": srv.waits_slot,
                    "nonfinite_walker_steps": sum(r.nonfinite_steps for r in res)})
        sweep[f"{f:g}x"] = out
    head = dict(sweep.get("0.8x", next(iter(sweep.values()))))
    # the same stream at 0.8x with the budget cut to 16 MiB: memory, not the
    # stream slots, then holds requests back
    srv = serve.Server(chunk_steps=50, hbm_budget_bytes=16 << 20)
    t0 = time.perf_counter()
    prod = serve.poisson_producer(srv, serve.requests_from_stream(stream), 0.8 * capacity)
    res = srv.run(producer=prod)
    wall = time.perf_counter() - t0
    mem = serve.latency_summary(res, wall)
    mem.update({"budget_bytes": srv.budget, "peak_used_bytes": srv.peak_used, "peak_active": srv.peak_active,
                "admissions_waited_for_memory": srv.waits_memory, "admissions_waited_for_slot": srv.waits_slot})
    head.update({"hbm_budget_bytes": serve.Server(chunk_steps=50).budget, "memory_bound_0.8x": mem,
                 "capacity_req_per_s": capacity,
                 "closed_loop_walker_steps_per_s": sum(r["walkers"] * r["steps"] for r in stream) / closed_wall,
                 "rate_sweep": sweep, "steps_per_request": steps,
                 "mix": "H2/LiH/Li2/CO, bond x U[0.6,3.0], walkers log-U[1k,32k], "
                        "FP64 or mixed FP32 in equal shares"})
    return head


def many_body_bench(sysd, args, dev, seed) -> dict:
    """The same workload with the many-body Jastrow terms (e-n kernel per
    nucleus, 5 e-e-n terms), FP64: throughput, roofline and errors against
    the oracle on sampled walkers."""
    import torch
    import oracle
    from paper_2506_09743_amd import qmc, synth
    sysd_m = synth.with_many_body_jastrow(sysd, synth.MBJ_SEED[args.system])
    W = args.walkers
    system = qmc.System(sysd_m, device=0)
    X = torch.from_numpy(synth.init_walkers(sysd_m, W, synth.WALKER_SEED[args.system])).to(dev)
    lp, sg, el = system.eval(X)
    acc = torch.zeros((W, qmc.ACC_COLS), dtype=torch.float64, device=dev)
    step = 0
    for _ in range(0, args.burnin + args.warmup, args.chunk):
        system.metropolis(X, lp, sg, el, args.chunk, 0.2, seed, step0=step, acc=acc)
        step += args.chunk
    acc.zero_()
    events = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(0, args.steps, args.chunk):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        system.metropolis(X, lp, sg, el, args.chunk, 0.2, seed, step0=step, acc=acc)
        e1.record()
        events.append((e0, e1))
        step += args.chunk
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launch_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    fl = flops_per_walker_step(sysd_m)
    achieved = fl["total"] * W * args.chunk / (launch_ms * 1e-3)
    idx = np.random.default_rng(0).choice(W, size=min(512, W), replace=False)
    Xn = X.cpu().numpy()[idx]
    rlp, _, rel = oracle.OracleSystem(sysd_m).eval(Xn)
    glp, _, gel = [t.cpu().numpy()[idx] for t in system.eval(X)]
    ok = np.isfinite(rel) & np.isfinite(gel)
    system.close()
    return {"value": W * args.steps / dt, "unit": "walker-steps/s", "dtype": "f64",
            "launch_ms_mean": launch_ms, "terms": "e-n per nucleus + 5 e-e-n terms",
            "flops_per_walker_step": fl["total"],
            "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                         "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU},
            "median_abs_dE_L": float(np.median(np.abs(gel[ok] - rel[ok]))),
            "max_rel_dlogpsi": float(np.max(np.abs(glp[ok] - rlp[ok]) / np.maximum(1, np.abs(rlp[ok])))),
            "mean_energy": float(acc[:, 0].sum().item() / (W * args.steps - acc[:, 3].sum().item())),
            "nonfinite_walker_steps": int(acc[:, 3].sum().item())}


def grad_bench(args, dev) -> dict:
    """The hand-written adjoint on the Li2 workload (32768 walkers, all four
    outputs), FP64 and the mixed FP32 form: walker-gradients/s, ms per call,
    roofline of the FP64 call against the FP64 vector peak on the term-by-term
    algorithmic count."""
    import torch
    from paper_2506_09743_amd import qmc, synth
    sysd = synth.make_system("Li2")
    W = synth.CONFIG_WALKERS["Li2"]
    system = qmc.System(sysd, device=0)
    X = torch.from_numpy(synth.init_walkers(sysd, W, synth.WALKER_SEED["Li2"])).to(dev)
    P, A = system.param_count, system.n_atoms
    outs = [torch.empty((W, P), dtype=torch.float64, device=dev),
            torch.empty((W, P), dtype=torch.float64, device=dev),
            torch.empty((W, A, 3), dtype=torch.float64, device=dev),
            torch.empty((W, A, 3), dtype=torch.float64, device=dev)]
    def timed(prec):
        qmc.qmc_grad(system.handle, X, *outs, precision=prec)
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            qmc.qmc_grad(system.handle, X, *outs, precision=prec)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))
    ms_fp32 = timed(qmc.QMC_MIXED_FP32)
    ms = timed(qmc.QMC_FP64)
    fl = grad_flops_per_walker(sysd)
    achieved = fl["total"] * W / (ms * 1e-3)
    out_bytes = W * (2 * P + 2 * 3 * A) * 8 + W * synth.n_elec(sysd) * 3 * 8
    system.close()
    return {"workload": f"Li2, {W} walkers, d log|Psi|/d theta, d E_L/d theta ({P} parameters), "
                        "d log|Psi|/d R, d E_L/d R",
            "ms_per_call": ms, "walker_gradients_per_s": W / (ms * 1e-3), "dtype": "f64",
            "mixed_fp32": {"ms_per_call": ms_fp32, "walker_gradients_per_s": W / (ms_fp32 * 1e-3)},
            "flops_per_walker": fl["total"], "flops_per_walker_terms": fl, "hbm_bytes_per_call": out_bytes,
            "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                         "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU,
                         "hbm_GBps": out_bytes / (ms * 1e-3) / 1e9}}


def sd_sweep_bench(args, dev) -> list:
    """Determinant-count sweep on CO, SD(2,2) .. SD(10,10) (4 .. 876
    determinants): E_L evaluation time of the low-rank method and of the
    explicit per-configuration method at 1000 and at the full walker count,
    and the low-rank Metropolis step time at the full walker count."""
    import torch
    from paper_2506_09743_amd import qmc, synth
    base = synth.make_system("CO")

    def timed(fn, reps=3):
        fn()
        out = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return float(np.median(out))

    rows = []
    for n in (2, 4, 6, 8, 10):
        sysd = synth.with_sd_expansion(base, n, 5)
        system = qmc.System(sysd, device=0)
        row = {"sd": f"SD({n},{n})", "dets": len(sysd["ci"])}
        for W in (1000, args.walkers):
            X = torch.from_numpy(synth.init_walkers(sysd, W, synth.WALKER_SEED["CO"])).to(dev)
            outs = [torch.empty(W, dtype=torch.float64, device=dev) for _ in range(3)]
            t_tab = timed(lambda: qmc.qmc_eval_psi_eloc(system.handle, qmc.QMC_FP64, X, *outs))
            t_exp = timed(lambda: qmc.qmc_eval_psi_eloc(system.handle, qmc.QMC_FP64_EXPLICIT, X, *outs))
            row[f"W{W}"] = {"eval_ms_low_rank": t_tab, "eval_ms_explicit": t_exp,
                            "explicit_over_low_rank": t_exp / t_tab}
            if W == args.walkers:
                lp, sg, el = system.eval(X)
                acc = torch.zeros((W, qmc.ACC_COLS), dtype=torch.float64, device=dev)
                t_mc = timed(lambda: system.metropolis(X, lp, sg, el, args.chunk, 0.2, 1, acc=acc))
                row[f"W{W}"]["metropolis_walker_steps_per_s"] = W * args.chunk / (t_mc * 1e-3)
        rows.append(row)
        system.close()
    return rows


BF_OMEGA = 0.1


def kinetic_ablation_bench(dev) -> list:
    """Jacobi-trace kinetic energy against central finite differences of Psi
    (6 N_e + 1 Psi-only evaluations per walker, h = 1e-3), E_L of 1000
    walkers, for the four molecules with the ground-state determinant only
    (the setting of the paper's Fig. kinetic_bench, whose baseline is
    automatic differentiation) and for CO with its 100 determinants."""
    import torch
    from paper_2506_09743_amd import qmc, synth

    def timed(fn, reps=3):
        fn()
        out = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return float(np.median(out))

    rows = []
    for name, ground in (("H2", True), ("LiH", True), ("Li2", True), ("CO", True), ("CO", False)):
        sysd = dict(synth.make_system(name))
        if ground:
            for k in ("occ_up", "occ_dn", "ci"):
                sysd[k] = np.asarray(sysd[k])[:1]
        system = qmc.System(sysd, device=0)
        X = torch.from_numpy(synth.init_walkers(sysd, 1000, synth.WALKER_SEED[name])).to(dev)
        outs = [torch.empty(1000, dtype=torch.float64, device=dev) for _ in range(3)]
        t_tr = timed(lambda: qmc.qmc_eval_psi_eloc(system.handle, qmc.QMC_FP64, X, *outs))
        t_fd = timed(lambda: qmc.qmc_eval_eloc_fd(system.handle, X, 1e-3, outs[0], outs[2]))
        rows.append({"system": name, "dets": len(sysd["ci"]), "walkers": 1000, "eval_ms_trace": t_tr,
                     "eval_ms_finite_differences": t_fd, "fd_over_trace": t_fd / t_tr})
        system.close()
    return rows


def backflow_bench(args, dev, seed) -> dict:
    """The inverse backflow (omega / r_ij, omega = 0.1) on CO, FP64, with the
    low-rank configuration update (QMC_FP64): Metropolis throughput at the
    full walker count with its roofline, the same for the per-configuration
    factorisation (QMC_FP64_EXPLICIT), errors against the oracle on sampled
    walkers, and the E_L evaluation time of the SD(n, n) expansions at 1000
    walkers with and without backflow."""
    import torch
    import oracle
    from paper_2506_09743_amd import qmc, synth
    base = synth.make_system("CO")
    sysd = dict(base)
    sysd["bf_omega"] = BF_OMEGA
    W = args.walkers
    system = qmc.System(sysd, device=0)
    X = torch.from_numpy(synth.init_walkers(sysd, W, synth.WALKER_SEED["CO"])).to(dev)
    lp, sg, el = system.eval(X)
    acc = torch.zeros((W, qmc.ACC_COLS), dtype=torch.float64, device=dev)
    step = 0
    for _ in range(2):  # burn-in and warm-up
        system.metropolis(X, lp, sg, el, args.chunk, 0.2, seed, step0=step, acc=acc)
        step += args.chunk
    acc.zero_()
    n_launch = 3
    X0, lp0, sg0, el0 = X.clone(), lp.clone(), sg.clone(), el.clone()
    timing = {}
    for prec in ("fp64", "fp64_explicit"):
        st = [X0.clone(), lp0.clone(), sg0.clone(), el0.clone()]
        events = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(n_launch):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            system.metropolis(*st, args.chunk, 0.2, seed, step0=step + k * args.chunk, acc=acc, precision=prec)
            e1.record()
            events.append((e0, e1))
        torch.cuda.synchronize()
        timing[prec] = (time.perf_counter() - t0, float(np.mean([a.elapsed_time(b) for a, b in events])))
        if prec == "fp64":
            X, lp, sg, el = st
    dt, launch_ms = timing["fp64"]
    fl = backflow_flops_per_walker_step(sysd)
    fl_x = backflow_flops_per_walker_step(sysd, low_rank=False)
    achieved = fl["total"] * W * args.chunk / (launch_ms * 1e-3)
    achieved_x = fl_x["total"] * W * args.chunk / (timing["fp64_explicit"][1] * 1e-3)
    idx = np.random.default_rng(0).choice(W, size=min(128, W), replace=False)
    Xn = X.cpu().numpy()[idx]
    rlp, _, rel = oracle.OracleSystem(sysd).eval(Xn)
    glp, _, gel = [t.cpu().numpy()[idx] for t in system.eval(X)]
    ok = np.isfinite(rel) & np.isfinite(gel)
    system.close()

    def timed(fn, reps=3):
        fn()
        out = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return float(np.median(out))

    sweep = []
    for n in (2, 4, 6, 8, 10):
        sd = synth.with_sd_expansion(base, n, 5)
        sdb = dict(sd)
        sdb["bf_omega"] = BF_OMEGA
        a, b = qmc.System(sd, device=0), qmc.System(sdb, device=0)
        Xs = torch.from_numpy(synth.init_walkers(sd, 1000, synth.WALKER_SEED["CO"])).to(dev)
        outs = [torch.empty(1000, dtype=torch.float64, device=dev) for _ in range(3)]
        t_lr = timed(lambda: qmc.qmc_eval_psi_eloc(a.handle, qmc.QMC_FP64, Xs, *outs))
        t_ex = timed(lambda: qmc.qmc_eval_psi_eloc(a.handle, qmc.QMC_FP64_EXPLICIT, Xs, *outs))
        t_bl = timed(lambda: qmc.qmc_eval_psi_eloc(b.handle, qmc.QMC_FP64, Xs, *outs))
        t_bx = timed(lambda: qmc.qmc_eval_psi_eloc(b.handle, qmc.QMC_FP64_EXPLICIT, Xs, *outs))
        sweep.append({"sd": f"SD({n},{n})", "dets": len(sd["ci"]), "eval_ms_low_rank": t_lr,
                      "eval_ms_explicit": t_ex, "eval_ms_backflow_low_rank": t_bl,
                      "eval_ms_backflow_explicit": t_bx,
                      "backflow_explicit_over_low_rank": t_bx / t_bl})
        a.close()
        b.close()
    return {"workload": f"CO, 100 determinants, {W} walkers, inverse backflow omega = {BF_OMEGA}",
            "method": "low-rank configuration update (QMC_FP64)",
            "value": W * args.chunk * n_launch / dt, "unit": "walker-steps/s", "dtype": "f64",
            # one qmc_metropolis_block call of block_steps steps; with backflow
            # the library launches one kernel per step
            "block_ms_mean": launch_ms, "block_steps": args.chunk, "kernel_launches_per_block": args.chunk,
            "flops_per_walker_step": fl["total"],
            "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                         "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU},
            "explicit": {"value": W * args.chunk * n_launch / timing["fp64_explicit"][0],
                         "block_ms_mean": timing["fp64_explicit"][1],
                         "flops_per_walker_step": fl_x["total"],
                         "roofline_frac": achieved_x / PEAK_FP64_VALU},
            "median_abs_dE_L": float(np.median(np.abs(gel[ok] - rel[ok]))),
            "max_abs_dE_L": float(np.max(np.abs(gel[ok] - rel[ok]))),
            "max_rel_dlogpsi": float(np.max(np.abs(glp[ok] - rlp[ok]) / np.maximum(1, np.abs(rlp[ok])))),
            "sd_sweep_1000_walkers": sweep}


def summarize_trace(path: str, kernel_regex: str, skip: int, block: int = 0) -> dict:
    """Durations of one kernel's dispatches in a rocprofv3 kernel-trace CSV,
    leaving out its first `skip` dispatches (burn-in and warm-up launches).
    block > 0: the remaining dispatches, in start order, form consecutive
    groups of `block` (one qmc_metropolis_block call: its step launches, two
    per step when the walkers run in two halves on two streams), and the
    span of each group (first start to last end) is reported too."""
    import csv
    import re
    pat = re.compile(kernel_regex)
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if pat.search(r["Kernel_Name"]):
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    rows.sort()
    rows = rows[skip:]
    d = np.array([e - s for s, e in rows], dtype=np.float64)
    out = {"kernel_regex": kernel_regex, "dispatches_total": len(rows) + skip, "skipped": skip,
           "dispatches": int(d.size), "mean_ns": float(d.mean()), "median_ns": float(np.median(d)),
           "min_ns": float(d.min()), "max_ns": float(d.max())}
    if block > 0:
        spans = [max(e for _, e in rows[i:i + block]) - rows[i][0]
                 for i in range(0, len(rows) - block + 1, block)]
        out.update(dispatches_per_block=block, blocks=len(spans), block_span_mean_ns=float(np.mean(spans)),
                   block_span_median_ns=float(np.median(spans)))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed Metropolis steps (one block)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--chunk", type=int, default=10, help="Metropolis steps per launch")
    ap.add_argument("--walkers", type=int, default=65536)
    ap.add_argument("--burnin", type=int, default=500, help="FP64 equilibration steps")
    ap.add_argument("--system", default="CO")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-many-body", action="store_true",
                    help="skip the many-body Jastrow (e-n + e-e-n) measurement")
    ap.add_argument("--no-sd-sweep", action="store_true",
                    help="skip the determinant-count sweep (low-rank vs explicit)")
    ap.add_argument("--no-grad", action="store_true", help="skip the adjoint (qmc_grad) measurement")
    ap.add_argument("--no-backflow", action="store_true", help="skip the inverse backflow measurement")
    ap.add_argument("--no-kinetic-ablation", action="store_true",
                    help="skip the trace vs finite-difference kinetic energy ablation")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serve-requests", type=int, default=256,
                    help="requests in the serving measurement (0: skip)")
    ap.add_argument("--serve-steps", type=int, default=500)
    ap.add_argument("--pmc-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this size (for counter scaling)")
    ap.add_argument("--summarize-trace", default=None,
                    help="print the dispatch statistics of --trace-kernel in this rocprofv3 "
                         "kernel-trace CSV (no GPU run)")
    ap.add_argument("--trace-kernel", default=r"k_metropolis<20, double, 0, false, 0>")
    ap.add_argument("--trace-skip", type=int, default=0, help="leading dispatches to leave out")
    ap.add_argument("--trace-block", type=int, default=0,
                    help="dispatches per qmc_metropolis_block call (block spans; 0: none)")
    args = ap.parse_args()
    if args.summarize_trace:
        print(json.dumps(summarize_trace(args.summarize_trace, args.trace_kernel, args.trace_skip,
                                         args.trace_block)))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the walkers of a multi-GPU run would be independent "
              "shards with one 32-byte all-reduce per block, which this build does not launch.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import oracle
    from paper_2506_09743_amd import qmc, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    sysd = synth.make_system(args.system)
    W = args.walkers
    seed = synth.PHILOX_SEED[args.system]
    system = qmc.System(sysd, device=0)
    X = torch.from_numpy(synth.init_walkers(sysd, W, synth.WALKER_SEED[args.system])).to(dev)

    def run_steps(state, n, step0, precision, acc, events=None):
        s = 0
        while s < n:
            c = min(args.chunk, n - s)
            if events is not None:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
            system.metropolis(*state, c, 0.2, seed, step0=step0 + s, acc=acc, precision=precision)
            if events is not None:
                e1.record()
                events.append((e0, e1, c))
            s += c
        return step0 + n

    # equilibrate in FP64
    lp, sg, el = system.eval(X)
    state = [X, lp, sg, el]
    acc = torch.zeros((W, qmc.ACC_COLS), dtype=torch.float64, device=dev)
    step = run_steps(state, args.burnin, 0, "fp64", acc)
    torch.cuda.synchronize()
    X_eq = X.clone()
    lp_eq, sg_eq, el_eq = lp.clone(), sg.clone(), el.clone()

    results = {}
    n_lat = max(20, args.steps // args.chunk)
    for form in (["fp64"] if args.no_mixed else ["fp64", "fp32", "bf16"]):
        st = [X_eq.clone(), lp_eq.clone(), sg_eq.clone(), el_eq.clone()]
        if form != "fp64":  # the mixed chain carries its own log|Psi| and E_L
            st[1], st[2], st[3] = system.eval(st[0], precision=form)
        acc = torch.zeros((W, qmc.ACC_COLS), dtype=torch.float64, device=dev)
        s0 = run_steps(st, args.warmup, step, form, acc)
        acc.zero_()
        events = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s1 = run_steps(st, args.steps, s0, form, acc, events)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        launch_ms = np.array([a.elapsed_time(b) for a, b, _ in events])
        sums = torch.empty(5, dtype=torch.float64, device=dev)
        qmc.qmc_reduce_accumulators(acc, sums)
        tot = sums.cpu().numpy()
        # latency: at least 20 repeated blocks of `chunk` steps, each timed
        lat = []
        for k in range(n_lat):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            system.metropolis(*st, args.chunk, 0.2, seed, step0=s1 + k * args.chunk, acc=acc, precision=form)
            e1.record()
            lat.append((e0, e1))
        torch.cuda.synchronize()
        lat_ms = np.array([a.elapsed_time(b) for a, b in lat])
        n_fin = W * args.steps - tot[3]
        results[form] = dict(
            value=W * args.steps / dt, ms_per_step=1e3 * dt / args.steps,
            launch_ms_mean=float(launch_ms.mean()), launch_steps=args.chunk,
            p50_ms=float(np.percentile(lat_ms, 50)), p99_ms=float(np.percentile(lat_ms, 99)),
            latency_blocks=int(n_lat), kernel_ms_per_step=float(launch_ms.mean() / args.chunk),
            mean_energy=float(tot[0] / n_fin) if n_fin else float("nan"),
            acceptance=float(tot[2] / (W * args.steps)),
            nonfinite_walker_steps=int(tot[3]), nonfinite_walkers=int(tot[4]))

    # errors against the oracle on identical (FP64-chain) configurations:
    # every walker, and the conditioning-window split on a sample
    Xn = X_eq.cpu().numpy()
    o = oracle.OracleSystem(sysd)
    t0 = time.perf_counter()
    rlp, rsg, rel = o.eval(Xn)
    oracle_full_eval_s = time.perf_counter() - t0
    g64 = system.eval(X_eq, precision="fp64")[2].cpu().numpy()
    fin = np.isfinite(rel)
    for form in results:
        glp, gsg, gel = [t.cpu().numpy() for t in system.eval(X_eq, precision=form)]
        m = fin & np.isfinite(gel)
        d = gel - rel
        e = dict(walkers_compared=int(m.sum()),
                 max_abs_dE_L=float(np.max(np.abs(d[m]))), median_abs_dE_L=float(np.median(np.abs(d[m]))),
                 p99_abs_dE_L=float(np.quantile(np.abs(d[m]), 0.99)),
                 mean_energy_err_vs_oracle=float(abs(gel[m].mean() - rel[m].mean())),
                 max_rel_dlogpsi=float(np.max(np.abs(glp[m] - rlp[m]) / np.maximum(1, np.abs(rlp[m])))))
        if form != "fp64":
            m2 = np.isfinite(gel) & np.isfinite(g64)
            e["mean_energy_err_vs_fp64_all_walkers"] = float(abs(gel[m2].mean() - g64[m2].mean()))
            e["walkers_refined_in_fp64"] = float(np.mean(gel[m2] == g64[m2]))
        results[form].update(e)
    idx = np.random.default_rng(0).choice(W, size=min(512, W), replace=False)
    inside = conditioning_window(o, sysd, Xn[idx])
    d64 = np.abs(g64[idx] - rel[idx])
    ok = np.isfinite(d64)
    results["fp64"]["tolerance_window"] = {
        "sampled": int(idx.size), "inside": int((inside & ok).sum()), "outside": int((~inside & ok).sum()),
        "max_abs_dE_L_inside": float(d64[inside & ok].max(initial=0.0)),
        "max_abs_dE_L_outside": float(d64[~inside & ok].max(initial=0.0)),
        "window": "kappa(A0) <= 1e8, CI cancellation <= 1e3, |E_L|, |E_kin| <= 1e4 Ha"}

    many_body = None
    if not args.no_many_body:
        many_body = many_body_bench(sysd, args, dev, seed)
    sd_sweep = None
    if not args.no_sd_sweep and args.system == "CO":
        sd_sweep = sd_sweep_bench(args, dev)
    gradient = None if args.no_grad else grad_bench(args, dev)
    backflow = None if args.no_backflow else backflow_bench(args, dev, seed)
    kinetic = None if args.no_kinetic_ablation else kinetic_ablation_bench(dev)

    fl = flops_per_walker_step(sysd)
    per_unit = CO_FLOPS_PER_WALKER_STEP if args.system == "CO" else fl["total"]
    main_form = results["fp64"]
    launch_s = main_form["launch_ms_mean"] * 1e-3
    achieved = per_unit * W * args.chunk / launch_s
    traffic = measured_traffic()
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU, "traffic": traffic,
                "kernel": "k_metropolis<20,double> (qmc_metropolis_block)",
                "launch": (f"one qmc_metropolis_block call of {args.chunk} steps: one k_metropolis dispatch "
                           "per step and half of the walkers, the halves on two streams"),
                "flops_per_walker_step": per_unit, "flops_per_walker_step_recount": fl["total"],
                "walker_steps_per_launch": W * args.chunk,
                "hbm_bytes_per_launch_algorithmic": hbm_bytes_per_launch(sysd, W, args.chunk),
                "launch_ms_mean": main_form["launch_ms_mean"]}
    for form in results:
        if form == "fp64":
            results[form]["roofline_frac"] = roofline["frac"]
            continue
        mp = mixed_peak(form)
        ach = per_unit * W * args.chunk / (results[form]["launch_ms_mean"] * 1e-3)
        results[form]["roofline"] = {"bound": "alu", "achieved": ach / 1e12, "peak": mp["peak_flops"] / 1e12,
                                     "unit": "TFLOP/s", "frac": ach / mp["peak_flops"],
                                     "split_flop": {k: v for k, v in mp.items() if k != "peak_flops"}}
        results[form]["roofline_frac"] = ach / mp["peak_flops"]

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(sysd, Xn, lp_eq.cpu().numpy(), sg_eq.cpu().numpy(), el_eq.cpu().numpy(),
                           seed, args.cpu_seconds)
        cpu["full_evaluation"] = {"walkers": W, "seconds": oracle_full_eval_s,
                                  "walker_evals_per_s": W / oracle_full_eval_s}

    serving = None
    if args.serve_requests > 0:
        serving = serving_bench(args.serve_requests, args.serve_steps)

    if args.pmc_calibration_mib:
        n = args.pmc_calibration_mib * (1 << 20) // 8
        a_ = torch.ones(n, dtype=torch.float64, device=dev)
        b_ = torch.empty_like(a_)
        torch.add(a_, 0.0, out=b_)  # one elementwise kernel: reads and writes n doubles
        torch.cuda.synchronize()

    # compact per-form summary, the line's last key
    summary = {}
    for form, r in results.items():
        summary[form] = {"value": r["value"], "ms_per_step": r["ms_per_step"], "p50_ms": r["p50_ms"],
                         "p99_ms": r["p99_ms"], "mean_E_err_vs_oracle": r["mean_energy_err_vs_oracle"],
                         "mean_E_err_vs_fp64": r.get("mean_energy_err_vs_fp64_all_walkers", 0.0),
                         "median_abs_dE_L": r["median_abs_dE_L"], "roofline_frac": r["roofline_frac"],
                         "speedup_vs_fp64": r["value"] / results["fp64"]["value"]}
        if form != "fp64":
            summary[form]["walkers_refined_in_fp64"] = r["walkers_refined_in_fp64"]
    out = {
        "metric": "walker-steps/s (Psi+E_L) CO 64k walkers, mixed vs FP64 at stated err; p50/p99",
        "value": main_form["value"], "unit": "walker-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_form["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.system} all-electron VMC, {W} walkers, Metropolis sigma 0.2, "
                               f"{args.chunk} steps per launch, after {args.burnin} burn-in steps",
                   "walkers": W, "electrons": synth.n_elec(sysd), "aos": synth.n_ao(sysd),
                   "mos": int(np.asarray(sysd['mo_coef']).shape[1]), "dets": len(sysd["ci"])},
        "p50_ms": main_form["p50_ms"], "p99_ms": main_form["p99_ms"],
        "latency_unit": f"ms per block of {args.chunk} steps x {W} walkers, over {n_lat} blocks",
        "details": results,
        "serving": serving,
        "many_body_jastrow": many_body,
        "determinant_sweep": sd_sweep,
        "gradient": gradient,
        "backflow": backflow,
        "kinetic_ablation": kinetic,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": summary,
    }
    print(json.dumps(out), flush=True)
    system.close()


if __name__ == "__main__":
    main()
