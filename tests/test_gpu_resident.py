"""The single-launch k = 1 update (FP64, every block in one workgroup's registers, the m
workgroups meeting at a device-wide barrier once per update).

Against the oracle's trajectory element by element (1e-10 of max|x*|), x_bar and every
x_i; handing its state to and from the per-update kernels; graph replays bit for bit
equal to eager launches; the XCD-packed launch equal to the plain one bit for bit; the
eligibility rule; and the bounded wait given up on purpose from the host (a poll limit
of 0), which every workgroup leaves normally and apc_residual reports."""

import math
import os
import sys

import numpy as np
import pytest

from oracle import apc_oracle as O
from paper_1708_01413_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-10


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


class _env:
    """Environment variables read by apc_setup, set only while plans are made."""

    def __init__(self, **kv):
        self.kv = kv

    def __enter__(self):
        self.old = {k: os.environ.get(k) for k in self.kv}
        os.environ.update({k: str(v) for k, v in self.kv.items()})

    def __exit__(self, *exc):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _system(name):
    if name == "square512-m8":
        return synth.square_gaussian_512()
    if name == "ragged-m13":
        # A one-row block, full 64-row blocks and everything between; sum 500.
        sizes = [64, 1, 37, 50, 64, 12, 45, 33, 64, 20, 58, 7, 45]
        return synth.gaussian_system(500, 300, 13, seed=131, scale=1 / math.sqrt(300),
                                     sizes=sizes)
    if name == "n1000-m40":
        return synth.gaussian_system(1000, 1000, 40, seed=132, scale=1 / math.sqrt(1000),
                                     shift=1.5)
    if name == "n90-m3":
        return synth.gaussian_system(90, 90, 3, seed=133, scale=1 / math.sqrt(90), shift=1.0)
    if name == "one-block":
        return synth.gaussian_system(40, 40, 1, seed=134, scale=1 / math.sqrt(40), shift=1.0)
    raise KeyError(name)


# name, block rows and columns one workgroup holds
CASES = [("square512-m8", 64, 512), ("ragged-m13", 64, 512), ("n1000-m40", 32, 1024),
         ("n90-m3", 32, 128), ("one-block", 64, 128)]


def _plan(S, stream, g, e, **env):
    apc = _apc()
    torch = _torch()
    A = torch.from_numpy(np.ascontiguousarray(S.A)).cuda()
    b = torch.from_numpy(S.B).cuda()
    with _env(**env):
        p = apc.Plan(A, b, S.off, "f64", gamma=g, eta=e, stream=stream)
    p._keep = (A, b)
    return p


def _read(p, stream):
    torch = _torch()
    with torch.cuda.stream(stream):
        xb, X = p.xbar(), p.local()
    stream.synchronize()
    return xb.cpu().numpy(), X.cpu().numpy()


@pytest.mark.parametrize("name,rows,cols", CASES, ids=[c[0] for c in CASES])
def test_single_launch_matches_oracle(name, rows, cols):
    """Launches of 1, 9 and 50 updates; after each, x_bar and every x_i against the
    oracle's iteration, element by element."""
    torch = _torch()
    S = _system(name)
    g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    stream = torch.cuda.Stream()
    p = _plan(S, stream, g, e)
    shape = p.resident_shape()
    say(f"case: single launch {name}: A {S.A.shape} m={len(S.off) - 1} shape {shape}")
    assert shape == {"rows_per_wg": rows, "cols_per_wg": cols}
    Qt, _R = O.factor(S.A, S.off)
    x = O.init_local(Qt, _R, S.B, S.off)
    xbar = O.initial_average(x)
    scale = float(np.max(np.abs(S.xstar)))
    done = 0
    for T in (1, 9, 50):
        p.iterate(T)
        for _ in range(T):
            x, xbar = O.apc_step(Qt, x, xbar, g, e)
        done += T
        gb, gX = _read(p, stream)
        db = float(np.max(np.abs(gb - xbar[:, 0]))) / scale
        dX = float(np.max(np.abs(gX - x[:, :, 0]))) / scale
        say(f"t = {done}: x_bar {db:.2e}, x_i {dX:.2e} (of max|x*|)")
        assert db <= TOL and dX <= TOL
    assert p.iterations == 60
    p.close()


def test_state_hands_over_to_per_update_kernels():
    """5 updates in one launch, 4 through the per-update kernels (iterate_timed), 6 in
    one launch again; against the oracle, and against a plan that never uses the
    single launch."""
    torch = _torch()
    S = _system("ragged-m13")
    g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    stream = torch.cuda.Stream()
    p = _plan(S, stream, g, e)
    q = _plan(S, stream, g, e, APC_RESIDENT=0)
    assert p.resident_shape() is not None and q.resident_shape() is None
    p.iterate(5)
    p.iterate_timed(4)
    p.iterate(6)
    q.iterate(15)
    Qt, R = O.factor(S.A, S.off)
    x = O.init_local(Qt, R, S.B, S.off)
    xbar = O.initial_average(x)
    for _ in range(15):
        x, xbar = O.apc_step(Qt, x, xbar, g, e)
    scale = float(np.max(np.abs(S.xstar)))
    (pb, pX), (qb, qX) = _read(p, stream), _read(q, stream)
    dp = max(float(np.max(np.abs(pb - xbar[:, 0]))), float(np.max(np.abs(pX - x[:, :, 0]))))
    dq = float(np.max(np.abs(pb - qb))) / scale
    say(f"case: hand-over: vs oracle {dp / scale:.2e}, vs per-update kernels {dq:.2e}")
    assert dp / scale <= TOL and dq <= TOL


def test_graph_and_xcd_packed_launch_equal_eager():
    """Graph replays of 10 updates (3 replays, eager work between) and the launch that
    keeps every eighth workgroup (one XCD) give the eager single launch's bits."""
    torch = _torch()
    S = _system("square512-m8")
    g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    stream = torch.cuda.Stream()
    pe = _plan(S, stream, g, e)
    pg = _plan(S, stream, g, e)
    px = _plan(S, stream, g, e, APC_RESIDENT_STRIDE=8)
    for rep in range(3):
        pe.iterate(10)
        pg.iterate(10, graph=True)
        px.iterate(10)
        stream.synchronize()
        junk = float(torch.randn(4096, device="cuda").sum())
        eb, gb, xb = (_read(p, stream)[0] for p in (pe, pg, px))
        assert np.array_equal(eb, gb) and np.array_equal(eb, xb), (rep, junk)
    say("case: graph replays and the XCD-packed launch equal eager launches (30 updates)")


def test_solve_stops_at_tolerance():
    apc = _apc()
    torch = _torch()
    S = _system("n1000-m40")
    stream = torch.cuda.Stream()
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(S.B).cuda()
    p = apc.Plan(A, b, S.off, "f64", stream=stream)
    assert p.resident_shape() is not None
    with torch.cuda.stream(stream):
        x, it, rr, st = p.solve(1e-10, 5000)
    stream.synchronize()
    err = float(np.linalg.norm(x.cpu().numpy() - S.xstar) / np.linalg.norm(S.xstar))
    say(f"case: single-launch solve: status {st} updates {it} relres {rr:.2e} error {err:.2e}")
    assert st == apc.APC_OK and rr <= 1e-10 and err <= 1e-8


@pytest.mark.parametrize("what", ["rows65", "n1100", "m300", "f32", "k2"])
def test_eligibility(what):
    """Blocks over 64 rows, rows over 1024 columns, more blocks than CUs, FP32 and k > 1
    plans launch per update."""
    apc = _apc()
    torch = _torch()
    prec, k = "f64", 1
    def gs(N, n, m, **kw):
        return synth.gaussian_system(N, n, m, scale=1 / math.sqrt(n), shift=2.0, **kw)
    if what == "rows65":
        S = gs(130, 100, 2, seed=135)
    elif what == "n1100":
        S = gs(1100, 1100, 40, seed=136)
    elif what == "m300":
        S = gs(600, 600, 300, seed=137)
    elif what == "f32":
        S, prec = gs(512, 512, 8, seed=138), "f32"
    else:
        S, k = gs(512, 512, 8, k=2, seed=139), 2
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(np.ascontiguousarray(S.B)).cuda()
    p = apc.Plan(A, b, S.off, prec, gamma=1.0, eta=1.0)
    say(f"case: eligibility {what}: {p.resident_shape()}")
    assert p.resident_shape() is None
    p.close()


def test_wait_given_up_is_reported():
    """A poll limit of 0 set from the host: the waiting workgroups give up at once and
    every workgroup leaves; x_bar is NaN, apc_residual reports APC_EHIP, the next
    launch stops at once the same way, and a fresh plan is unaffected."""
    apc = _apc()
    torch = _torch()
    S = _system("square512-m8")
    g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    stream = torch.cuda.Stream()
    bad = _plan(S, stream, g, e, APC_RESIDENT_SPIN=0)
    bad.iterate(3)
    stream.synchronize()
    with pytest.raises(apc.ApcError) as ex:
        bad.residual()
    assert ex.value.status == apc.APC_EHIP
    bad.iterate(2)
    xb, _ = _read(bad, stream)
    assert np.all(np.isnan(xb))
    good = _plan(S, stream, g, e)
    good.iterate(3)
    rr = good.residual()
    say(f"case: wait given up: APC_EHIP reported; fresh plan relres {rr:.2e}")
    assert math.isfinite(rr)
