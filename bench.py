"""Benchmark of the APC hot path on one MI355X.

Workload: the overdetermined Gaussian system N = 16384, n = 8192 (A iid
N(0, 1/n), x* iid N(0, 1), b = A x*), m = 64 blocks of p = 256 rows, FP32
projections with FP64 state, Theorem 1's optimal (gamma, eta).

One step = one full solve from inputs resident in HBM: setup (FP64
CholeskyQR2 of every block, min-norm init, Lanczos estimate of mu_min/mu_max,
closed-form gamma*/eta*), then the number of updates that takes x_bar to 1e-6
relative error (counted once during warm-up), then one residual check.

Prints one JSON line.  ``value`` is the algorithmic HBM bandwidth of the APC
iteration (bytes an update must move / measured time of the updates).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1e-6 rel. error & HBM GB/s per APC iteration; batched/BF16 vs plain"
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30
KERNELS = os.path.join(ROOT, "paper_1708_01413_amd", "csrc", "apc_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_tall16k_fp32.md")


def kernel_source_hash(names):
    """sha256 over the source text of the named __global__ functions (brace-matched)."""
    import hashlib
    src = open(KERNELS).read()
    h = hashlib.sha256()
    for name in names:
        i = src.index(f"void {name}(")
        j = src.index("{", i)
        depth = 0
        for e in range(j, len(src)):
            depth += {"{": 1, "}": -1}.get(src[e], 0)
            if depth == 0:
                break
        h.update(src[i:e + 1].encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel_label, fn_name):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter summary, or
    None when the summary is missing or the kernel's source changed since it was taken."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    want_hash = kernel_source_hash([fn_name])
    for ln in lines:
        if ln.startswith("traffic|"):
            _, label, src_hash, nbytes = ln.split("|")[:4]
            if label.strip() == kernel_label and src_hash.strip() == want_hash:
                return float(nbytes)
    return None


def algorithmic_bytes(N, n, m, sq=4, sx=8):
    """Bytes each launch must move (its inputs read once, its outputs written once).

    pass A: C, the differences d_i (projection precision), w.
    pass B: C, w, x_i read and written, x_bar.
    average: x_i, x_bar read and written, d_i written.
    Per update (the hot path's own figure): two streams of C plus the FP64 state
    read in A, read in B and written in B: 2 N n s_Q + 3 m n s_x.
    """
    pass_a = N * n * sq + m * n * sq + N * sq
    pass_b = N * n * sq + N * sq + 2 * m * n * sx + n * sx
    average = m * n * sx + 2 * n * sx + m * n * sq
    per_update = 2 * N * n * sq + 3 * m * n * sx
    return pass_a, pass_b, average, per_update


def algorithmic_bytes_single(N, n, m, ntiles, sq=4, sx=8):
    """Bytes of the single-pass update (each launch's inputs read once, outputs written once).

    single pass: C once, the differences d_i, one partial row (n entries) per row tile.
    combine: the partial rows, x_i read and written, x_bar read and written, d_i written.
    Per update: N n s_Q + 2 m n s_Q + 2 ntiles n s_Q + 2 m n s_x + 2 n s_x.
    """
    single = N * n * sq + m * n * sq + ntiles * n * sq
    combine = ntiles * n * sq + 2 * m * n * sx + 2 * n * sx + m * n * sq
    return single, combine, single + combine


def chunks_per_thread(n, elem):
    """Register chunks (16 bytes) of a row per thread of the single-pass kernel."""
    ldc = -(-n // 64) * 64
    chunks = ldc * elem // 16
    c = 1
    while chunks > 256 * c:
        c *= 2
    return c


def cpu_baseline(S, per_iter_bytes, gamma, eta, updates_to_target, budget_iters=8,
                 single_iters=2):
    """The FP64 oracle, as it stands, on the same system: factor + init once, then a few
    updates on all host threads and a few on one thread; reported in the benchmark's
    unit (the GPU path's bytes per update), with the oracle's time to the target error
    (its setup plus the updates the GPU path needed, with the same gamma and eta)."""
    from oracle import apc_oracle as O
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    Qt, R = O.factor(S.A, S.off)
    x = O.init_local(Qt, R, S.B, S.off)
    xbar = O.initial_average(x)
    t_setup = time.perf_counter() - t0
    t1 = time.perf_counter()
    for _ in range(budget_iters):
        x, xbar = O.apc_step(Qt, x, xbar, gamma, eta)
    t_iter = (time.perf_counter() - t1) / budget_iters
    t_one = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t2 = time.perf_counter()
            for _ in range(single_iters):
                x, xbar = O.apc_step(Qt, x, xbar, gamma, eta)
            t_one = (time.perf_counter() - t2) / single_iters
    return {
        "value": per_iter_bytes / t_iter / 1e9,
        "unit": "GB/s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": (f"FP64 NumPy oracle on the same 16384x8192 m=64 system: QR factor + init "
                   f"({t_setup:.1f} s) then {budget_iters} updates at {t_iter * 1e3:.1f} ms each "
                   f"on {cores} threads and {single_iters} on one thread; value = GPU-path "
                   "algorithmic bytes per update / oracle time per update"),
        "ms_per_iter": t_iter * 1e3,
        "ms_per_iter_1_thread": None if t_one is None else t_one * 1e3,
        "value_1_thread": None if t_one is None else per_iter_bytes / t_one / 1e9,
        "setup_s": t_setup,
        f"time_to_target_s": t_setup + updates_to_target * t_iter,
        "time_to_target_note": (f"oracle setup (QR + init) + {updates_to_target} updates (the "
                                "count the GPU path needed) on all threads; gamma and eta are "
                                "given to it (its dense spectrum, ~30-50 s here, is not timed)"),
    }


def plain_updates_ms(plan, T):
    """T updates timed by two HIP events on the plan's stream and nothing between the
    kernels (whole-update time as a caller sees it)."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(plan.stream)
    plan.iterate(T)
    e1.record(plan.stream)
    e1.synchronize()
    return e0.elapsed_time(e1)


def _err(plan, xs, xs_norm):
    """Relative error of x_bar against x*; with k columns the largest column error (the
    figure the tolerances gate on)."""
    import torch
    x = plan.xbar()
    if x.dim() == 1:
        return float(torch.linalg.norm(x - xs)) / xs_norm
    return float(torch.max(torch.linalg.norm(x - xs, dim=0) / torch.linalg.norm(xs, dim=0)))


MFMA_PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "f64": 78.6}


def time_plain(apc, A, b, off, xs, prec, target, ws, max_updates=400, anchor=None, gamma=None,
               eta=None):
    """Setup + the number of updates that reaches `target` relative error (counted
    in an untimed run), timed end to end with the stream synchronised."""
    import torch
    xs_norm = float(torch.linalg.norm(xs))
    plan = apc.Plan(A, b, off, prec, workspace=ws, anchor_every=anchor, gamma=gamma, eta=eta)
    T, err = 0, _err(plan, xs, xs_norm)
    while err > target and T < max_updates:
        plan.iterate(1)
        T += 1
        err = _err(plan, xs, xs_norm)
    plan.close()
    if err > target:
        # Plain FP32 levels off at its rounding floor: report that, and the time to 10x.
        res = {"reached": False, "updates_tried": T, "floor_err": err}
        if target < 1e-5:
            res["time_to_%.0e" % (10 * target)] = time_plain(apc, A, b, off, xs, prec,
                                                              10 * target, ws, max_updates, anchor,
                                                              gamma, eta)
        return res
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = apc.Plan(A, b, off, prec, workspace=ws, anchor_every=anchor, gamma=gamma, eta=eta)
    t1 = time.perf_counter()
    tot = plain_updates_ms(plan, T)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    err = _err(plan, xs, xs_norm)
    # Per-kernel times: the same number of updates again, each kernel timed by events
    # attached to its own launch (not part of the time to target).
    plan.restart()
    _, pa, pb, pv = plan.iterate_timed(T)
    plan.close()
    return {"reached": True, "updates": T, "err": err, "setup_ms": round((t1 - t0) * 1e3, 2),
            "iterate_ms": round((t2 - t1) * 1e3, 2), "total_ms": round((t2 - t0) * 1e3, 2),
            "us_per_update": round(tot * 1e3 / max(T, 1), 1),
            "pass_a_us": round(pa * 1e3 / max(T, 1), 1), "pass_b_us": round(pb * 1e3 / max(T, 1), 1),
            "epilogue_us": round(pv * 1e3 / max(T, 1), 1)}


def time_refined(apc, A, b, off, xs, rtol, ws, anchor=None):
    """Mixed precision: setup + apc_solve to relative residual rtol."""
    import torch
    xs_norm = float(torch.linalg.norm(xs))
    # The first plan of a shape in a process also times its matrix-core launch
    # shapes (cached afterwards): one untimed plan first, its setup reported apart.
    torch.cuda.synchronize()
    tw = time.perf_counter()
    apc.Plan(A, b, off, "bf16_ir", workspace=ws, anchor_every=anchor).close()
    first_ms = (time.perf_counter() - tw) * 1e3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = apc.Plan(A, b, off, "bf16_ir", workspace=ws, anchor_every=anchor)
    t1 = time.perf_counter()
    x, it, rr, st = plan.solve(rtol, 5000)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    err = float(torch.max(torch.linalg.norm(x - xs, dim=0) / torch.linalg.norm(xs, dim=0)))
    info = plan.info()
    plan.close()
    return {"rtol": rtol, "status": apc.STATUS_NAMES.get(st, st), "err": err, "updates": it,
            "refinements": info["refinements"], "setup_ms": round((t1 - t0) * 1e3, 2),
            "solve_ms": round((t2 - t1) * 1e3, 2), "total_ms": round((t2 - t0) * 1e3, 2),
            "warmup_plan_setup_ms": round(first_ms, 2)}


def krhs_rates(apc, A, b, off, prec, ws, T=16):
    """Per-kernel rates of the k-RHS passes (low-precision updates only, anchor off):
    algorithmic flops 2 N n k per pass, bytes = the streamed factor + V + W/Z."""
    N, n = A.shape
    k = b.shape[1]
    sq = {"f32": 4, "bf16_ir": 2, "f64": 8}[prec]
    plan = apc.Plan(A, b, off, prec, workspace=ws, anchor_every=0 if prec != "f64" else None)
    shapes = plan.launch_shapes()
    tot = plain_updates_ms(plan, T)
    _, pa, pb, pv = plan.iterate_timed(T)
    plan.close()
    name = {"f32": "f32", "bf16_ir": "bf16", "f64": "f64"}[prec]
    flops = 2.0 * N * n * k
    out = {"kernel": f"k_tn<{name}>", "launch_shapes": shapes, "us_per_update": round(tot * 1e3 / T, 1)}
    for tag, ms, rows, K in (("pass_a", pa, N, n), ("pass_b", pb, n, N)):
        t = ms * 1e-3 / T
        byts = rows * K * sq + (K + rows) * k * sq
        out[tag] = {"us": round(t * 1e6, 1), "tflops": round(flops / t / 1e12, 1),
                    "mfma_frac": round(flops / t / 1e12 / MFMA_PEAK_TFLOPS[name], 3),
                    "hbm_GBs": round(byts / t / 1e9, 1),
                    "hbm_frac": round(byts / t / 1e9 / HBM_PEAK_GBS, 3)}
    out["epilogue_us"] = round(pv * 1e3 / T, 1)
    return out


def many_systems(apc, synth, dev, count=256):
    """256 independent square systems (n uniform in [64, 1024], m in {4, 8, 16},
    A = G/sqrt(n) + 2I, one RHS each): one persistent launch per pass for all of them,
    against the same plans iterated one after another."""
    import torch
    systems = synth.many_small_systems(count=count, seed=0)
    stream = torch.cuda.Stream(device=dev)
    t0 = time.perf_counter()
    plans, keep = [], []
    for S in systems:
        A = torch.from_numpy(S.A).to(dev)
        b = torch.from_numpy(S.B).to(dev)
        keep.append((A, b))
        plans.append(apc.Plan(A, b, S.off, "f32", stream=stream))
    setup_s = time.perf_counter() - t0
    batch = apc.Batch(plans)
    single = batch.launch()["items_b"] == 0
    # Bytes an update moves, summed over systems (as the k = 1 FP32 path does:
    # one read of each factor in the single pass, two in the two-pass form).
    two_pass_bytes = sum(2 * S.N * S.n * 4 + 3 * S.m * S.n * 8 for S in systems)
    if single:
        # A batch of k = 1 systems alone cuts every block into row tiles of up
        # to 256 rows, one partial row each (the launch's item count is the
        # number of tiles).
        per_update, ntiles = 0, 0
        for S in systems:
            tiles = int(sum(-(-int(q) // 256) for q in np.diff(S.off)))
            ntiles += tiles
            per_update += algorithmic_bytes_single(S.N, S.n, S.m, tiles)[2]
        if ntiles != batch.launch()["items_a"]:
            raise RuntimeError(f"tile count {ntiles} differs from the batch's "
                               f"{batch.launch()['items_a']} items")
    else:
        per_update = two_pass_bytes
    T = 20

    def timed(fn):
        stream.synchronize()
        t = time.perf_counter()
        fn()
        stream.synchronize()
        return (time.perf_counter() - t) / T

    batch.iterate(T, graph=True)                      # capture + warm
    t_graph = timed(lambda: batch.iterate(T, graph=True))
    t_eager = timed(lambda: batch.iterate(T, graph=False))

    def one_by_one():
        for p in plans:
            p.iterate(T)
    t_seq = timed(one_by_one)
    t_two = None
    if single:
        os.environ["APC_FUSED"] = "0"
        try:
            batch2 = apc.Batch(plans)
        finally:
            del os.environ["APC_FUSED"]
        batch2.iterate(T, graph=True)
        t_two = timed(lambda: batch2.iterate(T, graph=True))
        batch2.close()
    # Fresh start, then per-system stopping at relative residual 1e-6.
    for p in plans:
        p.restart()
    batch.activate()
    stream.synchronize()
    t = time.perf_counter()
    iters, rr, st = batch.solve(1e-6, 400, check_every=8, graph=True)
    stream.synchronize()
    solve_ms = (time.perf_counter() - t) * 1e3
    errs = [float(torch.linalg.norm(p.xbar() - torch.from_numpy(S.xstar).to(dev))
                  / np.linalg.norm(S.xstar)) for p, S in zip(plans, systems)]
    res = {
        "workload": f"{count} systems, n in [64, 1024], m in {{4, 8, 16}}, A = G/sqrt(n)+2I, "
                    "k = 1 each, FP32 projections",
        "sum_n2": int(sum(S.n * S.n for S in systems)),
        "launch": batch.launch(),
        "setup_s_all_plans": round(setup_s, 2),
        "us_per_update_graph": round(t_graph * 1e6, 1),
        "us_per_update_eager": round(t_eager * 1e6, 1),
        "us_per_update_one_plan_at_a_time": round(t_seq * 1e6, 1),
        "form": "single pass over each factor" if single else "two passes over each factor",
        "two_pass_batch_us_per_update": round(t_two * 1e6, 1) if t_two else None,
        "algorithmic_bytes_per_update": per_update,
        "GBs_graph": round(per_update / t_graph / 1e9, 1),
        "solve_to_relres_1e-6": {"status": apc.STATUS_NAMES.get(st, st), "ms": round(solve_ms, 2),
                                 "updates_min": int(iters.min()), "updates_max": int(iters.max()),
                                 "max_rel_err": max(errs)},
    }
    batch.close()
    for p in plans:
        p.close()
    return res


def config3_one_batch(apc, synth, dev):
    """Both parts of the batched workload in ONE batch: N = n = 8192, A = G/sqrt(n) + 2I,
    k = 64, 64 uneven blocks (FP32 products, FP64 anchor every 16 updates) and the 256
    independent k = 1 systems; every update is four launches of one persistent kernel over
    work lists that cover both parts, replayed from a hipGraph."""
    import torch
    big = synth.shifted_uneven_8k(k=64)
    many = synth.many_small_systems(count=256, seed=0)
    stream = torch.cuda.Stream(device=dev)
    plans, keep = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for S in [big] + many:
        A = torch.from_numpy(S.A).to(dev)
        b = torch.from_numpy(np.ascontiguousarray(S.B)).to(dev)
        keep.append((A, b))
        plans.append(apc.Plan(A, b, S.off, "f32", stream=stream))
    stream.synchronize()
    setup_s = time.perf_counter() - t0
    batch = apc.Batch(plans)
    T = 16                                  # one anchor update per replay

    def timed(fn, reps=3):
        stream.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        stream.synchronize()
        return (time.perf_counter() - t) / (reps * T)

    batch.iterate(T, graph=True)            # capture + warm
    t_graph = timed(lambda: batch.iterate(T, graph=True))
    t_eager = timed(lambda: batch.iterate(T, graph=False))
    for p in plans:
        p.restart()
    batch.activate()
    stream.synchronize()
    t = time.perf_counter()
    iters, rr, st = batch.solve(1e-6, 400, check_every=8, graph=True)
    stream.synchronize()
    solve_ms = (time.perf_counter() - t) * 1e3
    with torch.cuda.stream(stream):
        xs = [p.xbar().cpu().numpy() for p in plans]
    stream.synchronize()
    errs = [float(np.max(np.linalg.norm((x - S.xstar).reshape(S.n, -1), axis=0)
                         / np.linalg.norm(S.xstar.reshape(S.n, -1), axis=0)))
            for x, S in zip(xs, [big] + many)]
    res = {
        "workload": "one batch: N=n=8192, A=G/sqrt(n)+2I, k=64, 64 uneven blocks (FP32, FP64 "
                    "anchor every 16) + 256 systems n in [64, 1024], k = 1 (FP32)",
        "launch": batch.launch(),
        "launches_per_update": "4 (+1 y_ref prologue on anchor updates)",
        "setup_s_all_plans": round(setup_s, 2),
        "us_per_update_graph": round(t_graph * 1e6, 1),
        "us_per_update_eager": round(t_eager * 1e6, 1),
        "solve_to_relres_1e-6": {"status": apc.STATUS_NAMES.get(st, st), "ms": round(solve_ms, 2),
                                 "updates_k64_system": int(iters[0]),
                                 "updates_256_systems_min": int(iters[1:].min()),
                                 "updates_256_systems_max": int(iters[1:].max()),
                                 "max_rel_err_k64_system": errs[0],
                                 "max_rel_err_256_systems": max(errs[1:])},
    }
    batch.close()
    for p in plans:
        p.close()
    return res


def adjoint_workload(apc, synth, dev):
    """N = n = 4096, A = G/sqrt(n) + 2I, k = 16, m = 32 blocks of 128, FP32, T = 200,
    checkpoint every 14, L = 1/2 ||x_bar(T) - x_target||^2."""
    import torch
    S = synth.shifted_square(4096, 32, k=16, shift=2.0, seed=70, with_target=True)
    A = torch.from_numpy(S.A).to(dev)
    b = torch.from_numpy(S.B).to(dev)
    xt = torch.from_numpy(S.extra["x_target"]).to(dev)
    plan = apc.Plan(A, b, S.off, "f32")
    plan.iterate(200)
    r = plan.xbar() - xt
    plan.backward(r, 200, 14)                       # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.restart()
    plan.iterate(200)
    r = plan.xbar() - xt
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dB, dg, de = plan.backward(r, 200, 14)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ref = torch.linalg.solve(A.T.contiguous(), r)
    res = {"workload": "N=n=4096, A=G/sqrt(n)+2I, k=16, m=32, FP32, T=200, checkpoint every 14",
           "forward_ms": round((t1 - t0) * 1e3, 2), "backward_ms": round((t2 - t1) * 1e3, 2),
           "dB_vs_A^-T_r_rel": float(torch.linalg.norm(dB - ref) / torch.linalg.norm(ref)),
           "dL_dgamma": dg, "dL_deta": de}
    plan.close()
    return res


def time_hbm(apc, plan, kind, xs, target, max_updates, check_every=8):
    """A heavy-ball comparison run (apc_hbm_*) on a plan: creation (the spectrum
    estimate of the plain kind included), updates to `target` relative error counted
    in an untimed run, then those updates timed by two HIP events."""
    import torch
    xs_norm = float(torch.linalg.norm(xs))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = apc.HeavyBall(plan, kind)
    t1 = time.perf_counter()
    q = h.params()
    T, err = 0, float(torch.linalg.norm(h.x() - xs)) / xs_norm
    while err > target and T < max_updates:
        step = 1 if T < 400 else check_every
        h.iterate(step)
        T += step
        err = float(torch.linalg.norm(h.x() - xs)) / xs_norm
    res = {"kind": ["plain (Sec. 4.3)", "preconditioned (Sec. 6)"][kind],
           "create_ms": round((t1 - t0) * 1e3, 2), "lanczos_steps": q["lanczos_steps"],
           "lam_min": q["lam_min"], "lam_max": q["lam_max"], "rho_predicted": q["rho"],
           "reached": err <= target, "updates": T, "err": err}
    if err <= target:
        h.restart()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(plan.stream)
        h.iterate(T)
        e1.record(plan.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        res.update({"iterate_ms": round(ms, 2), "us_per_update": round(ms * 1e3 / max(T, 1), 1),
                    "create_plus_iterate_ms": round((t1 - t0) * 1e3 + ms, 2)})
    h.close()
    return res


def comparison_methods(apc, synth, dev):
    """The paper's comparison methods on the same GPU passes, each from APC's start
    to 1e-6 relative error: block Cimmino (Sec. 4.5, run as APC with gamma = 1 and
    eta = 2 / (mu_min + mu_max): Prop. 2 with the optimal Cimmino step), D-HBM on the
    blocks [A_i, b_i] (Sec. 4.3) and on Sec. 6's preconditioned blocks; on the benchmark
    system (FP32) and on the same shape with entries of mean 1 (FP64: the plain
    heavy ball's FP32 rounding floor is above 1e-6 there).  The heavy-ball runs check
    the error after every update up to 400 updates, then every 8."""
    import torch
    out = {}
    for name, gen, prec in (("tall16k_fp32", synth.tall_gaussian_16k, "f32"),
                            ("tall16k_mean1_fp64", synth.tall_gaussian_16k_mean1, "f64")):
        S = gen()
        A = torch.from_numpy(S.A).to(dev)
        b = torch.from_numpy(S.B).to(dev)
        xs = torch.from_numpy(S.xstar).to(dev)
        ws = torch.empty(apc.Plan.workspace_bytes(S.N, S.n, S.off, prec), dtype=torch.uint8,
                         device=dev)
        p = apc.Plan(A, b, S.off, prec, workspace=ws)
        prm = p.params()
        p.close()
        eta = 2.0 / (prm["mu_min"] + prm["mu_max"])
        entry = {"workload": f"{S.name}: N={S.N} n={S.n} m={S.m}, {prec.upper()}",
                 "apc_params": prm}
        if name != "tall16k_fp32":       # the main line already times APC on the first system
            entry["apc"] = time_plain(apc, A, b, S.off, xs, prec, 1e-6, ws, max_updates=1000)
        entry["block_cimmino"] = time_plain(apc, A, b, S.off, xs, prec, 1e-6, ws, max_updates=4000,
                                            gamma=1.0, eta=eta)
        p = apc.Plan(A, b, S.off, prec, workspace=ws)
        entry["dhbm_preconditioned"] = time_hbm(apc, p, 1, xs, 1e-6, 4000)
        entry["dhbm_plain"] = time_hbm(apc, p, 0, xs, 1e-6, 4000)
        p.close()
        out[name] = entry
        del A, b, xs, ws, S
        torch.cuda.empty_cache()
    return out


def secondary(apc, synth, dev):
    """Batched and mixed-precision workloads, each against plain FP32 on the same inputs."""
    import torch
    out = {}
    # Square Gaussian N = n = 512, m = 8, FP64, 2000 updates (latency-bound: C is 2 MiB).
    S = synth.square_gaussian_512()
    A = torch.from_numpy(S.A).to(dev)
    b = torch.from_numpy(S.B).to(dev)
    plan = apc.Plan(A, b, S.off, "f64")
    plan.iterate(50)
    tot = plain_updates_ms(plan, 2000)
    plan.iterate(2000)
    err = float(torch.linalg.norm(plan.xbar() - torch.from_numpy(S.xstar).to(dev))) / float(
        np.linalg.norm(S.xstar))
    # The same updates launched one kernel pair per update (iterate_timed always takes
    # that path), for comparison with the single launch of all T updates above.
    tt, pa, pb, pv = plan.iterate_timed(2000)
    single = plan.single_pass_shape()
    kern = ({"single_pass_us": round(pa * 1e3 / 2000, 2), "combine_us": round(pv * 1e3 / 2000, 2),
             "single_pass_shape": single} if single is not None else
            {"pass_a_us": round(pa * 1e3 / 2000, 2), "pass_b_us": round(pb * 1e3 / 2000, 2),
             "average_us": round(pv * 1e3 / 2000, 2)})
    kern["per_update_launches_us_per_update"] = round(tt * 1e3 / 2000, 2)
    resident = plan.resident_shape()
    out["square512_fp64"] = dict({"workload": "N=n=512, A, x* iid N(0,1), m=8 blocks of 64, FP64",
                                  "updates": 2000, "us_per_update": round(tot * 1e3 / 2000, 2),
                                  "path": ("one launch for all updates, factor held in registers "
                                           f"({resident})" if resident else "launches per update"),
                                  "err_after_4050": err, "params": plan.params()}, **kern)
    plan.close()
    del A, b, S
    # Batched: N = n = 8192, A = G/sqrt(n) + 2I, k = 64, 64 blocks of uneven size.
    S = synth.shifted_uneven_8k(k=64)
    A = torch.from_numpy(S.A).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(S.B)).to(dev)
    xs = torch.from_numpy(S.xstar).to(dev)
    ws = torch.empty(apc.Plan.workspace_bytes(S.N, S.n, S.off, "f32", k=64), dtype=torch.uint8,
                     device=dev)
    out["batched_fp32"] = {
        "workload": "N=n=8192, A=G/sqrt(n)+2I, k=64, m=64 uneven p_i in [28, 228]",
        "time_to_1e-6": time_plain(apc, A, b, S.off, xs, "f32", 1e-6, ws),
        "time_to_1e-10": time_plain(apc, A, b, S.off, xs, "f32", 1e-10, ws),
        "plain_fp32_time_to_1e-6": time_plain(apc, A, b, S.off, xs, "f32", 1e-6, ws, anchor=0),
        "kernels": krhs_rates(apc, A, b, S.off, "f32", ws),
        "note": "FP32 projections on matrix cores with an FP64 anchor update every 16 updates "
                "(default); plain_fp32 = every update's products in FP32 (the state y, x_bar "
                "stays FP64 in every mode)",
    }
    del A, b, xs, ws, S
    torch.cuda.empty_cache()
    out["many_systems_fp32"] = many_systems(apc, synth, dev)
    torch.cuda.empty_cache()
    out["batched_one_launch"] = config3_one_batch(apc, synth, dev)
    torch.cuda.empty_cache()
    out["adjoint_fp32"] = adjoint_workload(apc, synth, dev)
    out["comparison_methods"] = comparison_methods(apc, synth, dev)
    torch.cuda.empty_cache()
    # Mixed precision vs plain FP32: N = n = 16384, A = G/sqrt(n) + alpha I, k = 128, m = 64.
    n, k, m = 16384, 128, 64
    rng = np.random.default_rng(0)
    G = torch.from_numpy(rng.standard_normal((n, n)) / np.sqrt(n)).to(dev)
    Xs = torch.from_numpy(rng.standard_normal((n, k))).to(dev)
    off = synth.offsets_from_sizes(synth.even_sizes(n, m))
    ws32 = torch.empty(apc.Plan.workspace_bytes(n, n, off, "f32", k=k), dtype=torch.uint8, device=dev)
    ws16 = torch.empty(apc.Plan.workspace_bytes(n, n, off, "bf16_ir", k=k), dtype=torch.uint8,
                       device=dev)
    mixed = {"workload": "N=n=16384, A=G/sqrt(n)+alpha I, k=128, m=64 blocks of 256",
             "note": "plain_fp32: FP32 products on matrix cores with the state (y, x_bar) kept "
                     "in FP64, no anchor updates; fp32_anchored: the same with an FP64 anchor "
                     "update every 16; bf16_ir: bf16 products inside FP64 iterative refinement; "
                     "errors are the largest column error against X* (B = A X* in FP64)"}
    for alpha in (3.0, 1.5):
        A = G.clone()
        A.diagonal().add_(alpha)
        B = (A @ Xs).contiguous()
        entry = {"plain_fp32_time_to_1e-6": time_plain(apc, A, B, off, Xs, "f32", 1e-6, ws32,
                                                       anchor=0),
                 "fp32_anchored_time_to_1e-6": time_plain(apc, A, B, off, Xs, "f32", 1e-6, ws32),
                 "bf16_ir_time_to_1e-6": time_refined(apc, A, B, off, Xs, 1e-7, ws16),
                 "bf16_ir_time_to_1e-10": time_refined(apc, A, B, off, Xs, 1e-11, ws16)}
        if alpha == 3.0:
            entry["kernels_bf16"] = krhs_rates(apc, A, B, off, "bf16_ir", ws16)
            entry["kernels_fp32"] = krhs_rates(apc, A, B, off, "f32", ws32)
        mixed[f"alpha={alpha}"] = entry
        del A, B
    out["mixed_precision"] = mixed
    del G, Xs, ws32, ws16
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--target", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--main-only", action="store_true",
                    help="skip the batched and mixed-precision comparisons")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--bf16-contraction-only", action="store_true",
                    help="only the mixed-precision system (16384^2, k = 128, alpha = 3): setup and "
                         "8 bf16 updates, for counter runs of the matrix-core contraction")
    ap.add_argument("--f32-contraction-only", action="store_true",
                    help="only the batched system (8192^2, k = 64, uneven blocks): setup and 8 "
                         "FP32 updates without anchors, for counter runs of the FP32 contraction")
    ap.add_argument("--setup-only", action="store_true",
                    help="only the benchmark system's setup (tall Gaussian 16384 x 8192, FP32), "
                         "three times, for counter runs of the setup kernels")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: sharding the blocks over several GPUs (one "
              "all-reduce of sum_i x_i per update) is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1708_01413_amd import apc, synth

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.bf16_contraction_only:
        nn, kk, mm = 16384, 128, 64
        rng = np.random.default_rng(0)
        G = torch.from_numpy(rng.standard_normal((nn, nn)) / np.sqrt(nn)).to(dev)
        G.diagonal().add_(3.0)
        Xs = torch.from_numpy(rng.standard_normal((nn, kk))).to(dev)
        Bm = (G @ Xs).contiguous()
        offm = synth.offsets_from_sizes(synth.even_sizes(nn, mm))
        plan = apc.Plan(G, Bm, offm, "bf16_ir", gamma=1.0, eta=1.0, anchor_every=0)
        plan.iterate(8)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "N=n=16384, A=G/sqrt(n)+3I, k=128, m=64, bf16 contraction",
                          "updates": 8, "launch_shapes": plan.launch_shapes()}), flush=True)
        return
    if args.setup_only:
        S = synth.tall_gaussian_16k()
        A = torch.from_numpy(S.A).to(dev)
        b = torch.from_numpy(S.B).to(dev)
        ws = torch.empty(apc.Plan.workspace_bytes(S.N, S.n, S.off, "f32"), dtype=torch.uint8,
                         device=dev)
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = apc.Plan(A, b, S.off, "f32", workspace=ws)
            torch.cuda.synchronize()
            times.append(round((time.perf_counter() - t0) * 1e3, 3))
            plan.close()
        print(json.dumps({"workload": "tall Gaussian N=16384 n=8192, m=64, FP32 plan setup",
                          "setup_ms": times}), flush=True)
        return
    if args.f32_contraction_only:
        Sb = synth.shifted_uneven_8k(k=64)
        Ab = torch.from_numpy(Sb.A).to(dev)
        Bb = torch.from_numpy(np.ascontiguousarray(Sb.B)).to(dev)
        plan = apc.Plan(Ab, Bb, Sb.off, "f32", gamma=1.0, eta=1.0, anchor_every=0)
        plan.iterate(8)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "N=n=8192, A=G/sqrt(n)+2I, k=64, 64 uneven blocks, FP32 "
                          "contraction", "updates": 8, "launch_shapes": plan.launch_shapes()}),
              flush=True)
        return
    S = synth.tall_gaussian_16k()
    N, n, m = S.N, S.n, S.m
    A = torch.from_numpy(S.A).to(dev)
    b = torch.from_numpy(S.B).to(dev)
    xs = torch.from_numpy(S.xstar).to(dev)
    xs_norm = float(torch.linalg.norm(xs))
    ws = torch.empty(apc.Plan.workspace_bytes(N, n, S.off, args.precision), dtype=torch.uint8,
                     device=dev)
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()

    # Warm-up: also counts the updates needed to reach the target error (from x*).
    iters_needed = {}
    for w in range(max(args.warmup, 1)):
        plan = apc.Plan(A, b, S.off, args.precision, workspace=ws, stream=stream)
        if w == 0:
            for t in range(1, 400):
                plan.iterate(1)
                err = float(torch.linalg.norm(plan.xbar() - xs)) / xs_norm
                for lvl in (1e-5, args.target):
                    if lvl not in iters_needed and err <= lvl:
                        iters_needed[lvl] = t
                if args.target in iters_needed:
                    break
            if args.target not in iters_needed:
                raise SystemExit(f"target {args.target} not reached in 400 updates (err {err:.3e})")
            final_err = err
        else:
            plan.iterate(iters_needed[args.target])
        plan.close()
    T = iters_needed[args.target]
    prm = None

    # Timed steps.
    torch.cuda.synchronize()
    setup_ms, iter_ms, pa_ms, pb_ms, av_ms = [], [], [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        plan = apc.Plan(A, b, S.off, args.precision, workspace=ws, stream=stream)
        setup_ms.append((time.perf_counter() - ts) * 1e3)    # setup synchronises at its end
        iter_ms.append(plain_updates_ms(plan, T))
        relres = plan.residual()
        # Per-kernel launch times (roofline): T more updates with events attached to
        # each kernel's own launch; not part of the time to target.
        _, a_ms, b_ms, v_ms = plan.iterate_timed(T)
        pa_ms.append(a_ms)
        pb_ms.append(b_ms)
        av_ms.append(v_ms)
        prm = plan.params()
        plan_info = plan.info()
        single = plan.single_pass_shape()
        qr = plan.setup_info()
        plan.close()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps

    sq = 4 if args.precision == "f32" else 8
    it_ms = float(np.mean(iter_ms))
    ptype = "float" if args.precision == "f32" else "double"
    if single is not None:
        rows, grp = single["rows_per_wg"], single["rows_per_group"]
        ntiles = int(sum(-(-int(p) // rows) for p in np.diff(S.off)))
        bytes_f, bytes_c, per_iter = algorithmic_bytes_single(N, n, m, ntiles, sq=sq)
        launches = T * args.steps
        avg_f = float(np.sum(pa_ms)) / launches
        avg_c = float(np.sum(av_ms)) / launches
        dom_bytes, dom_ms = bytes_f, avg_f
        dom_label = f"k_fused<{ptype}, {ptype}, {chunks_per_thread(n, sq)}, {grp}>"
        dom_fn = "k_fused"
        iteration = {
            "form": "single pass over C per update, then the x_i update + average launch",
            "single_pass_us_per_launch": round(avg_f * 1e3, 2),
            "combine_us_per_launch": round(avg_c * 1e3, 2),
            "single_pass_GBs": round(bytes_f / (avg_f * 1e-3) / 1e9, 1),
            "combine_GBs": round(bytes_c / (avg_c * 1e-3) / 1e9, 1),
            "rows_per_workgroup": rows, "rows_per_register_group": grp, "tiles": ntiles,
        }
    else:
        plan_groups = plan_info["block_groups"]
        bytes_a, bytes_b, bytes_v, per_iter = algorithmic_bytes(N, n, m, sq=sq)
        # Per-launch averages (a group of blocks is one launch of each pass).
        launches = plan_groups * T * args.steps
        avg_a = float(np.sum(pa_ms)) / launches
        avg_b = float(np.sum(pb_ms)) / launches
        avg_v = float(np.sum(av_ms)) / (T * args.steps)
        bytes_a_l, bytes_b_l = bytes_a / plan_groups, bytes_b / plan_groups
        dom, dom_bytes, dom_ms = (("pass_b", bytes_b_l, avg_b) if avg_b >= avg_a
                                  else ("pass_a", bytes_a_l, avg_a))
        dom_label, dom_fn = {"pass_a": (f"k_rowdot<{ptype}, {ptype}, 8, 2, true>", "k_rowdot"),
                             "pass_b": (f"k_pass_b_rows<{ptype}, true>", "k_pass_b_rows")}[dom]
        iteration = {
            "form": "two passes over C per update, then the average",
            "block_groups": plan_groups,
            "pass_a_us_per_launch": round(avg_a * 1e3, 2),
            "pass_b_us_per_launch": round(avg_b * 1e3, 2),
            "average_us": round(avg_v * 1e3, 2),
            "pass_a_GBs": round(bytes_a_l / (avg_a * 1e-3) / 1e9, 1),
            "pass_b_GBs": round(bytes_b_l / (avg_b * 1e-3) / 1e9, 1),
            "average_GBs": round(bytes_v / (avg_v * 1e-3) / 1e9, 1),
        }
    value = per_iter * T / (it_ms * 1e-3) / 1e9
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    # The same system with two passes over C per update (the form the single pass
    # replaces), for comparison: whole-update time only.
    two_pass = None
    if single is not None:
        os.environ["APC_FUSED"] = "0"
        try:
            p2 = apc.Plan(A, b, S.off, args.precision, workspace=ws, stream=stream)
        finally:
            del os.environ["APC_FUSED"]
        p2.iterate(T)
        t2 = plain_updates_ms(p2, T)
        _, a2, b2, v2 = p2.iterate_timed(T)
        ba, bb, _, per2 = algorithmic_bytes(N, n, m, sq=sq)
        two_pass = {"us_per_update": round(t2 * 1e3 / T, 2),
                    "pass_a_us": round(a2 * 1e3 / T, 2), "pass_b_us": round(b2 * 1e3 / T, 2),
                    "average_us": round(v2 * 1e3 / T, 2),
                    "algorithmic_bytes_per_update": per2,
                    "GBs": round(per2 * T / (t2 * 1e-3) / 1e9, 1)}
        p2.close()

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {
            "workload": f"tall Gaussian N={N} n={n}, m={m} blocks of p={N // m}, k=1, "
                        f"{args.precision.upper()} projections, FP64 state",
            "N": N, "n": n, "m": m, "p": N // m, "k": 1, "seed": 0,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom_label,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dom_label, dom_fn),
            "algorithmic_bytes_per_launch": dom_bytes,
            "avg_launch_us": round(dom_ms * 1e3, 2),
        },
        "iteration": dict({
            "updates_to_1e-5": iters_needed.get(1e-5),
            f"updates_to_{args.target:g}": T,
            "err_at_end_of_warmup": final_err,
            "us_per_update": round(it_ms * 1e3 / T, 2),
            "updates_per_s": round(T / (it_ms * 1e-3), 1),
            "algorithmic_bytes_per_update": per_iter,
            "launch_shape": plan_info,
        }, **iteration),
        "two_pass_same_system": two_pass,
        "time_to_target_ms": {
            "target_rel_err": args.target,
            "setup_ms": round(float(np.mean(setup_ms)), 3),
            "iterate_ms": round(it_ms, 3),
            "total_ms": round(float(np.mean(setup_ms)) + it_ms, 3),
            "qr_passes": qr["qr_passes"],
            "qr_defect_after_first_pass": qr["qr_defect"],
        },
        "params": prm,
        "relres_at_end": relres,
        "paper_context": {
            "note": "context only, not a target: the paper reports optimal convergence times "
                    "T = 1/(-log rho) in iterations (Table 2), not wall-clock figures",
            "table2_row": "standard tall Gaussian 1000 x 500, APC",
            "table2_T_APC": 2.34,
            "T_this_system_from_rho": round(1.0 / -math.log(prm["rho"]), 3),
            "rho_estimated": prm["rho"],
            f"updates_to_{args.target:g}": T,
        },
    }
    if not args.main_only:
        del A, b, xs, ws
        torch.cuda.empty_cache()
        out.update(secondary(apc, synth, dev))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(S, per_iter, prm["gamma"], prm["eta"], T)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
