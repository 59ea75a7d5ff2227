"""apc_iterate_graph: T updates of a single plan replayed from a captured HIP graph.

Every replay must give bit for bit the states of the same updates launched eagerly
(apc_iterate) on a twin plan, with eager work and synchronisations between the
replays, and the trajectory must stay within the FP64 / FP32 bar of the oracle."""

import math
import sys

import numpy as np
import pytest

from oracle import apc_oracle as O
from paper_1708_01413_amd import synth

pytestmark = pytest.mark.gpu

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


def _oracle_xbar(S, T, g, e):
    Qt, R = O.factor(S.A, S.off)
    x = O.init_local(Qt, R, S.B, S.off)
    xbar = O.initial_average(x)
    for _ in range(T):
        x, xbar = O.apc_step(Qt, x, xbar, g, e)
    return xbar


CASES = [
    # (name, N, n, m, k, precision, anchor_every, T per replay, replays)
    ("square512-f64", 512, 512, 8, 1, "f64", None, 10, 5),
    ("ragged-f32", 1000, 700, 9, 1, "f32", None, 7, 4),
    ("krhs-f32-anchored", 1024, 768, 8, 12, "f32", 16, 5, 5),
    ("krhs-f64", 600, 400, 6, 5, "f64", None, 6, 3),
]


@pytest.mark.parametrize("name,N,n,m,k,prec,anchor,T,reps", CASES, ids=[c[0] for c in CASES])
def test_graph_replays_equal_eager_updates(name, N, n, m, k, prec, anchor, T, reps):
    apc = _apc()
    torch = _torch()
    S = synth.gaussian_system(N, n, m, k=k, seed=110, scale=1.0 if N == 512 else 1 / math.sqrt(n),
                              shift=0.0 if N == 512 else (1.5 if N == n else 0.0))
    g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(S.B).cuda()
    stream = torch.cuda.Stream()
    kw = {} if anchor is None else {"anchor_every": anchor}
    pg = apc.Plan(A, b, S.off, prec, gamma=g, eta=e, stream=stream, **kw)
    pe = apc.Plan(A, b, S.off, prec, gamma=g, eta=e, stream=stream, **kw)
    say(f"case: graph {name} T={T} x {reps}")
    for rep in range(reps):
        pg.iterate(T, graph=True)
        pe.iterate(T)
        stream.synchronize()
        junk = float(torch.randn(4096, device="cuda").sum())  # eager work between replays
        with torch.cuda.stream(stream):
            same = torch.equal(pg.xbar(), pe.xbar())
        stream.synchronize()
        assert same, (rep, junk)
    assert pg.iterations == pe.iterations == T * reps
    with torch.cuda.stream(stream):
        got = pg.xbar()
    stream.synchronize()
    ref = _oracle_xbar(S, T * reps, g, e)
    ref = ref[:, 0] if k == 1 else ref
    dev = float(np.max(np.linalg.norm((got.cpu().numpy() - ref).reshape(n, -1), axis=0)
                       / np.linalg.norm(S.xstar.reshape(n, -1), axis=0)))
    say(f"after {T * reps} updates: equal to eager launches; dev vs oracle {dev:.2e}")
    assert dev <= TOL[prec]
    pg.close()
    pe.close()


def test_graph_after_set_params_uses_the_new_parameters():
    """The cached graph carries (gamma, eta) by value: apc_set_params must drop it, so the
    next replay runs with the new parameters (compared with eager updates)."""
    apc = _apc()
    torch = _torch()
    S = synth.gaussian_system(700, 500, 7, seed=111, scale=1 / math.sqrt(500))
    g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(S.B).cuda()
    stream = torch.cuda.Stream()
    pg = apc.Plan(A, b, S.off, "f64", gamma=g, eta=e, stream=stream)
    pe = apc.Plan(A, b, S.off, "f64", gamma=g, eta=e, stream=stream)
    pg.iterate(8, graph=True)
    pe.iterate(8)
    for p in (pg, pe):
        p.set_params(0.9 * g, 0.8 * e)
    pg.iterate(8, graph=True)
    pe.iterate(8)
    stream.synchronize()
    with torch.cuda.stream(stream):
        same = torch.equal(pg.xbar(), pe.xbar())
    stream.synchronize()
    say(f"case: graph after set_params: equal {same}")
    assert same


def test_graph_after_refined_solve():
    """bf16 refinement, then graph replays continue it exactly as eager updates do."""
    apc = _apc()
    torch = _torch()
    S = synth.shifted_square(1024, 8, k=4, shift=3.0, seed=112)
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(S.B).cuda()
    stream = torch.cuda.Stream()
    pg = apc.Plan(A, b, S.off, "bf16_ir", stream=stream)
    pe = apc.Plan(A, b, S.off, "bf16_ir", stream=stream)
    for p in (pg, pe):
        with torch.cuda.stream(stream):
            p.solve(1e-9, 2000)
    pg.iterate(10, graph=True)
    pe.iterate(10)
    stream.synchronize()
    with torch.cuda.stream(stream):
        xg, xe = pg.xbar(), pe.xbar()
    stream.synchronize()
    err = float(torch.linalg.norm(xg - torch.from_numpy(S.xstar).cuda())
                / float(np.linalg.norm(S.xstar)))
    say(f"case: graph after refined solve: equal {torch.equal(xg, xe)}, error {err:.2e}")
    assert torch.equal(xg, xe)
    assert err <= 1e-8


def test_graph_needs_a_stream():
    apc = _apc()
    torch = _torch()
    S = synth.shifted_square(256, 4, seed=113)
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(S.B).cuda()
    plan = apc.Plan(A, b, S.off, "f64", stream=torch.cuda.default_stream())
    if torch.cuda.default_stream().cuda_stream != 0:
        pytest.skip("the default stream is not the NULL stream here")
    with pytest.raises(apc.ApcError) as ex:
        plan.iterate(3, graph=True)
    assert ex.value.status == apc.APC_EINVAL
