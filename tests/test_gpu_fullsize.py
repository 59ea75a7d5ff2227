"""GPU parity at the benchmark workloads' full sizes, in the launch configurations
bench.py times (tuned shapes, default anchors, persistent batch launches with a
hipGraph).  Expected values come from tests/golden/make_golden.py, which calls only
the FP64 oracle and the seeded generators; where the oracle cannot run the full
trajectory in reasonable time the test checks properties that hold at any size
(the error against the known solution X*).

Bars: FP64 1e-10 and FP32 1e-5, per right-hand side c, both norm-wise
(||x_gpu[:, c] - x_oracle[:, c]|| / ||x*[:, c]||) and element by element
(|x_gpu[j, c] - x_oracle[j, c]| / max_j |x*[j, c]|), on whole vectors."""

import math
import os
import sys

import numpy as np
import pytest

from paper_1708_01413_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = {"f64": 1e-10, "f32": 1e-5}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _apc():
    from paper_1708_01413_amd import apc
    return apc


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_full_size_batched_8k_k64(prec):
    """N = n = 8192, A = G/sqrt(n) + 2I, 64 uneven blocks, k = 64: the error curve
    t = 0..56 (largest column error, and the Frobenius form) and the whole n x 64 x_bar(t)
    at t = 5, 20, 56, element by element."""
    torch = _torch()
    apc = _apc()
    g = np.load(os.path.join(GOLDEN, "shifted_uneven_8192_k64.npz"), allow_pickle=False)
    S = synth.shifted_uneven_8k(k=64)
    say(f"case: full-size batched 8192 k=64 {prec}")
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(np.ascontiguousarray(S.B)).cuda()
    xs = torch.from_numpy(S.xstar).cuda()
    off = S.off
    del S
    plan = apc.Plan(A, b, off, prec, gamma=float(g["gamma"]), eta=float(g["eta"]))
    check = [int(t) for t in g["check_t"]]
    xn = torch.from_numpy(g["xstar_norm"]).cuda()          # per column
    xmax = g["xstar_max"]                                  # per column
    errs, errs_f, full = [], [], {}
    xs_f = float(torch.linalg.norm(xs))
    for t in range(check[-1] + 1):
        if t:
            plan.iterate(1)
        xb = plan.xbar()
        errs.append(float(torch.max(torch.linalg.norm(xb - xs, dim=0) / xn)))
        errs_f.append(float(torch.linalg.norm(xb - xs)) / xs_f)
        if t in check:
            full[t] = xb.cpu().numpy()
    errs, errs_f = np.array(errs), np.array(errs_f)
    say("err gpu ", " ".join(f"{e:.3e}" for e in errs[[5, 20, 34, 56]]),
        " Frobenius ", " ".join(f"{e:.3e}" for e in errs_f[[5, 20, 34, 56]]))
    say("err orc ", " ".join(f"{e:.3e}" for e in g["err"][[5, 20, 34, 56]]),
        " Frobenius ", " ".join(f"{e:.3e}" for e in g["err_fro"][[5, 20, 34, 56]]))
    assert np.max(np.abs(errs - g["err"])) <= TOL[prec]
    assert np.max(np.abs(errs_f - g["err_fro"])) <= TOL[prec]
    xn_np = g["xstar_norm"]
    for k, t in enumerate(check):
        d = full[t] - g["xbar"][k]
        col = float(np.max(np.linalg.norm(d, axis=0) / xn_np))
        elem = float(np.max(np.abs(d) / xmax))
        say(f"t = {t}: largest column deviation {col:.3e}, element-wise {elem:.3e}")
        assert col <= TOL[prec] and elem <= TOL[prec], (t, col, elem)


def test_full_size_many_systems_batch():
    """256 independent systems (n in [64, 1024], m in {4, 8, 16}), FP32, one persistent
    launch per pass captured in a hipGraph: the whole x_bar of every system after 20
    updates against the oracle's, norm-wise and element by element."""
    torch = _torch()
    apc = _apc()
    g = np.load(os.path.join(GOLDEN, "many_small_systems_256.npz"), allow_pickle=False)
    systems = synth.many_small_systems(count=256, seed=0)
    say("case: full-size 256 systems batch")
    stream = torch.cuda.Stream()
    plans, keep = [], []
    for s, S in enumerate(systems):
        A = torch.from_numpy(S.A).cuda()
        b = torch.from_numpy(S.B).cuda()
        keep.append((A, b))
        plans.append(apc.Plan(A, b, S.off, "f32", gamma=float(g["gamma"][s]),
                              eta=float(g["eta"][s]), stream=stream))
    batch = apc.Batch(plans)
    T = int(g["T"])
    batch.iterate(T, graph=True)
    stream.synchronize()
    worst, worst_e = 0.0, 0.0
    for s, (p, S) in enumerate(zip(plans, systems)):
        xb = p.xbar()                    # enqueued on the plans' stream
        stream.synchronize()
        got = xb.cpu().numpy()
        ref = g["xbar"][g["starts"][s]:g["starts"][s + 1]]
        d = got - ref
        worst = max(worst, float(np.linalg.norm(d) / np.linalg.norm(S.xstar)))
        worst_e = max(worst_e, float(np.max(np.abs(d)) / np.max(np.abs(S.xstar))))
    say(f"worst deviation over 256 systems: norm-wise {worst:.3e}, element-wise {worst_e:.3e}")
    assert worst <= TOL["f32"] and worst_e <= TOL["f32"]
    batch.close()
    for p in plans:
        p.close()


@pytest.mark.parametrize("alpha", [3.0, 1.5])
def test_full_size_mixed_precision(alpha):
    """N = n = 16384, A = G/sqrt(n) + alpha I, k = 128, 64 blocks of 256: the bf16
    refinement mode reaches 1e-10 relative error against X* (B = A X* in FP64, so X*
    is the solution to within kappa(A) eps), and anchored FP32 reaches 1e-6."""
    torch = _torch()
    apc = _apc()
    n, k, m = 16384, 128, 64
    rng = np.random.default_rng(0)
    G = torch.from_numpy(rng.standard_normal((n, n)) / np.sqrt(n)).cuda()
    Xs = torch.from_numpy(rng.standard_normal((n, k))).cuda()
    off = synth.offsets_from_sizes(synth.even_sizes(n, m))
    A = G
    A.diagonal().add_(alpha)
    B = (A @ Xs).contiguous()
    say(f"case: full-size mixed precision alpha={alpha}")
    plan = apc.Plan(A, B, off, "bf16_ir")
    x, it, rr, st = plan.solve(1e-11, 5000)
    err = float(torch.max(torch.linalg.norm(x - Xs, dim=0) / torch.linalg.norm(Xs, dim=0)))
    say(f"bf16 refinement: status {st} updates {it} refinements {plan.info()['refinements']} "
        f"relres {rr:.2e} max column error {err:.2e}")
    assert st == apc.APC_OK and err <= 1e-10
    plan.close()
    del plan
    torch.cuda.empty_cache()
    plan = apc.Plan(A, B, off, "f32")
    x, it, rr, st = plan.solve(1e-7, 2000)
    err = float(torch.linalg.norm(x - Xs) / torch.linalg.norm(Xs))
    say(f"anchored fp32: status {st} updates {it} relres {rr:.2e} error {err:.2e}")
    assert err <= 1e-6
    plan.close()
