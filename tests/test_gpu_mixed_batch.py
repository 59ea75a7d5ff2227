"""Mixed batches: a k-RHS plan (the (y, x_bar) form, FP32 products, FP64 anchor updates)
and many k = 1 systems advanced by the same persistent launches (apc_batch_* with both
kinds of plans), eagerly and from a captured hipGraph.

Bars: FP32 1e-5 against the FP64 oracle, per right-hand side, norm-wise
(||x_gpu - x_oracle|| / ||x*||) and element by element (|x_gpu - x_oracle| / max|x*|);
graph replays bit for bit equal to eager launches."""

import math
import os
import sys

import numpy as np
import pytest

from oracle import apc_oracle as O
from paper_1708_01413_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-5


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


def _devs(got, ref, xstar):
    n = xstar.shape[0]
    got, ref, xs = (np.asarray(v).reshape(n, -1) for v in (got, ref, xstar))
    col = float(np.max(np.linalg.norm(got - ref, axis=0) / np.linalg.norm(xs, axis=0)))
    elem = float(np.max(np.abs(got - ref) / np.max(np.abs(xs), axis=0)))
    return col, elem


def _systems(seed):
    big = synth.gaussian_system(1024, 1024, 8, k=24, seed=seed, scale=1 / math.sqrt(1024),
                                shift=2.0,
                                sizes=synth.renormalised_sizes(np.random.default_rng(seed), 8, 1024,
                                                               64, 200))
    small = synth.many_small_systems(count=5, seed=seed + 1, lo=64, hi=600)
    return [big] + small


def _plans(systems, stream, params=None):
    apc = _apc()
    torch = _torch()
    plans, keep = [], []
    for i, S in enumerate(systems):
        A = torch.from_numpy(S.A).cuda()
        b = torch.from_numpy(np.ascontiguousarray(S.B)).cuda()
        kw = {} if params is None else {"gamma": params[i][0], "eta": params[i][1]}
        plans.append(apc.Plan(A, b, S.off, "f32", stream=stream, **kw))
        keep.append((A, b))
    return plans, keep


def test_mixed_batch_matches_oracle():
    """One k = 24 system (uneven blocks, anchored FP32) and five k = 1 systems: 40 updates
    in one batch (anchor updates at 0, 16, 32), every system against the oracle."""
    apc = _apc()
    torch = _torch()
    systems = _systems(120)
    params = [O.optimal_params(*O.spectrum(S.A, S.off))[:2] for S in systems]
    stream = torch.cuda.Stream()
    plans, keep = _plans(systems, stream, params)
    batch = apc.Batch(plans)
    say(f"case: mixed batch k=24 + 5 systems: launch {batch.launch()}")
    T = 40
    batch.iterate(T)
    stream.synchronize()
    worst = (0.0, 0.0)
    for S, p, (g, e) in zip(systems, plans, params):
        ref = O.apc_run(S.A, S.B, S.off, T, g, e)["xbar"]
        with torch.cuda.stream(stream):
            x = p.xbar()
        stream.synchronize()
        ref = ref[:, 0] if S.B.ndim == 1 else ref
        col, elem = _devs(x.cpu().numpy(), ref, S.xstar)
        worst = (max(worst[0], col), max(worst[1], elem))
        assert p.iterations == T
    say(f"max deviation from the oracle: column {worst[0]:.2e}, element {worst[1]:.2e}")
    assert worst[0] <= TOL and worst[1] <= TOL
    batch.close()


def test_mixed_batch_graph_equals_eager():
    """The captured graph of 5 updates (its anchor phase changes between replays), replayed
    with eager work in between, equals eager launches of the same batch bit for bit."""
    apc = _apc()
    torch = _torch()
    systems = _systems(121)
    stream = torch.cuda.Stream()
    pa, ka = _plans(systems, stream)
    pb, kb = _plans(systems, stream)
    ba, bb = apc.Batch(pa), apc.Batch(pb)
    for rep in range(5):
        ba.iterate(5, graph=True)
        bb.iterate(5, graph=False)
        stream.synchronize()
        junk = float(torch.randn(2048, device="cuda").sum())
        for p, q in zip(pa, pb):
            with torch.cuda.stream(stream):
                same = torch.equal(p.xbar(), q.xbar())
            stream.synchronize()
            assert same, (rep, junk)
    say("case: mixed batch graph replays equal eager launches (25 updates)")
    ba.close()
    bb.close()


def test_mixed_batch_solve_stops_each_system():
    apc = _apc()
    torch = _torch()
    systems = _systems(122)
    stream = torch.cuda.Stream()
    plans, keep = _plans(systems, stream)
    batch = apc.Batch(plans)
    iters, rr, st = batch.solve(1e-6, 600, check_every=4, graph=True)
    say(f"case: mixed batch solve: status {st} updates {iters.tolist()} relres {rr.max():.2e}")
    assert st == apc.APC_OK and np.all(rr <= 1e-6)
    for S, p in zip(systems, plans):
        with torch.cuda.stream(stream):
            x = p.xbar()
        stream.synchronize()
        err = O.rel_error(x.cpu().numpy(), S.xstar)
        assert err <= 1e-4, err
    batch.close()


def test_full_size_config3_one_batch():
    """N = n = 8192, A = G/sqrt(n) + 2I, k = 64, 64 uneven blocks, anchored FP32, and the 256
    independent systems (n in [64, 1024]) in ONE batch, replayed from hipGraphs: after 20
    updates every one of the 256 systems and the k = 64 system against the oracle's stored
    whole vectors, element by element; the k = 64 system again at t = 56."""
    apc = _apc()
    torch = _torch()
    gk = np.load(os.path.join(GOLDEN, "shifted_uneven_8192_k64.npz"), allow_pickle=False)
    gm = np.load(os.path.join(GOLDEN, "many_small_systems_256.npz"), allow_pickle=False)
    big = synth.shifted_uneven_8k(k=64)
    many = synth.many_small_systems(count=256, seed=0)
    stream = torch.cuda.Stream()
    params = [(float(gk["gamma"]), float(gk["eta"]))] + \
        [(float(gm["gamma"][s]), float(gm["eta"][s])) for s in range(256)]
    plans, keep = _plans([big] + many, stream, params)
    batch = apc.Batch(plans)
    say(f"case: config 3 in one batch: launch {batch.launch()}")
    check = [int(t) for t in gk["check_t"]]
    assert check == [5, 20, 56] and int(gm["T"]) == 20
    done = 0
    for t in check:
        batch.iterate(t - done, graph=True)
        done = t
        stream.synchronize()
        with torch.cuda.stream(stream):
            xb = plans[0].xbar()
        stream.synchronize()
        col, elem = _devs(xb.cpu().numpy(), gk["xbar"][check.index(t)], big.xstar)
        say(f"t = {t}: k = 64 system vs oracle: column {col:.2e}, element {elem:.2e}")
        assert col <= TOL and elem <= TOL
        if t == 20:
            worst = (0.0, 0.0)
            for s, (p, S) in enumerate(zip(plans[1:], many)):
                with torch.cuda.stream(stream):
                    x = p.xbar()
                stream.synchronize()
                ref = gm["xbar"][gm["starts"][s]:gm["starts"][s + 1]]
                c, e = _devs(x.cpu().numpy(), ref, S.xstar)
                worst = (max(worst[0], c), max(worst[1], e))
            say(f"t = 20: 256 systems vs oracle: column {worst[0]:.2e}, element {worst[1]:.2e}")
            assert worst[0] <= TOL and worst[1] <= TOL
    batch.close()
