"""GPU parity of the single-pass k = 1 update (one read of the factor per update):
every launch shape against the FP64 oracle and against the two-pass update, on
ragged blocks (tiles and register groups with short tails), row widths that
leave part of a thread's chunks empty, and the widest rows the kernel holds.

Bars: FP64 1e-10 and FP32 1e-5, as ||x_bar_gpu(t) - x_bar_oracle(t)|| / ||x*||."""

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


def oracle_traj(S, T, gamma, eta):
    Qt, R = O.factor(S.A, S.off)
    x = O.init_local(Qt, R, S.B, S.off)
    xbar = O.initial_average(x)
    traj = [xbar[:, 0].copy()]
    for _ in range(T):
        x, xbar = O.apc_step(Qt, x, xbar, gamma, eta)
        traj.append(xbar[:, 0].copy())
    return np.stack(traj)


def gpu_traj(plan, T):
    torch = _torch()
    snaps = [plan.xbar()]
    for _ in range(T):
        plan.iterate(1)
        snaps.append(plan.xbar())
    torch.cuda.synchronize()
    return torch.stack(snaps).cpu().numpy()


def dev(a, b, xstar):
    return float(np.max(np.linalg.norm(a - b, axis=-1)) / np.linalg.norm(xstar))


def make(N, n, m, seed, lo, hi, shift=0.0):
    sizes = synth.renormalised_sizes(np.random.default_rng(seed), m, N, lo, hi)
    return synth.gaussian_system(N, n, m, seed=seed, shift=shift, sizes=sizes,
                                 scale=1.0 / math.sqrt(n))


SHAPES = [("16", "1"), ("16", "4"), ("32", "2"), ("64", "4"), ("128", "1"), ("64", "1")]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("rows,g", SHAPES)
def test_single_pass_shapes_match_oracle(prec, rows, g, monkeypatch):
    """N = n = 1000 (ldc 1024: the last chunk of a row is partly past n), 13 blocks of
    40..120 rows, so every tile height and register group ends in a short tail."""
    apc = _apc()
    torch = _torch()
    S = make(1000, 1000, 13, 2, 40, 120, shift=2.0)
    g_opt, e_opt, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    T = 50
    ref = oracle_traj(S, T, g_opt, e_opt)
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(S.B).cuda()
    monkeypatch.setenv("APC_FUSED_ROWS", rows)
    monkeypatch.setenv("APC_FUSED_G", g)
    plan = apc.Plan(A, b, S.off, prec, gamma=g_opt, eta=e_opt)
    shape = plan.single_pass_shape()
    say(f"case: single pass {prec} sizes={np.diff(S.off).tolist()} shape={shape}")
    assert shape == {"rows_per_wg": int(rows), "rows_per_group": int(g)}
    d = dev(gpu_traj(plan, T), ref, S.xstar)
    say(f"max dev {d:.3e}")
    assert d <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_pass_matches_two_pass(prec, monkeypatch):
    """The same plan arithmetic with one and with two reads of the factor per update."""
    apc = _apc()
    torch = _torch()
    S = make(2048, 1536, 16, 5, 64, 192)
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(S.B).cuda()
    one = apc.Plan(A, b, S.off, prec)
    assert one.single_pass_shape() is not None
    monkeypatch.setenv("APC_FUSED", "0")
    two = apc.Plan(A, b, S.off, prec, gamma=one.params()["gamma"], eta=one.params()["eta"])
    assert two.single_pass_shape() is None
    one.iterate(40)
    two.iterate(40)
    xs = np.linalg.norm(S.xstar)
    d = float(torch.linalg.norm(one.xbar() - two.xbar())) / xs
    err = float(torch.linalg.norm(one.xbar() - torch.from_numpy(S.xstar).cuda())) / xs
    say(f"case: one vs two passes {prec}: dev {d:.3e}, error after 40 updates {err:.3e}")
    assert d <= TOL[prec]


def test_single_pass_widest_fp32_rows():
    """n = 9000 in FP32: 16 chunks per thread (the widest the kernel holds), one row
    per register group; gamma = eta = 1 so no spectrum is needed."""
    apc = _apc()
    torch = _torch()
    N, n, m = 9000, 9000, 36
    S = synth.gaussian_system(N, n, m, seed=11, shift=2.0, scale=1.0 / math.sqrt(n))
    T = 6
    ref = oracle_traj(S, T, 1.0, 1.0)
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(S.B).cuda()
    plan = apc.Plan(A, b, S.off, "f32", gamma=1.0, eta=1.0)
    shape = plan.single_pass_shape()
    say(f"case: widest FP32 rows n={n} shape={shape}")
    assert shape is not None and shape["rows_per_group"] == 1
    d = dev(gpu_traj(plan, T), ref, S.xstar)
    say(f"max dev {d:.3e}")
    assert d <= TOL["f32"]


def test_single_pass_fp64_is_deterministic():
    apc = _apc()
    torch = _torch()
    S = make(1024, 768, 12, 10, 40, 140)
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(S.B).cuda()
    runs = []
    for _ in range(2):
        plan = apc.Plan(A, b, S.off, "f64", gamma=1.05, eta=3.0)
        plan.iterate(30)
        runs.append(plan.xbar().cpu().numpy())
    np.testing.assert_array_equal(runs[0], runs[1])


def test_wide_fp64_rows_take_two_passes():
    """FP64 rows wider than 8192 do not fit the single-pass registers: the plan falls
    back to two passes and still matches the oracle."""
    apc = _apc()
    torch = _torch()
    N, n, m = 8300, 8300, 10
    S = synth.gaussian_system(N, n, m, seed=12, shift=2.0, scale=1.0 / math.sqrt(n))
    T = 4
    ref = oracle_traj(S, T, 1.0, 1.0)
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(S.B).cuda()
    plan = apc.Plan(A, b, S.off, "f64", gamma=1.0, eta=1.0)
    assert plan.single_pass_shape() is None
    d = dev(gpu_traj(plan, T), ref, S.xstar)
    say(f"case: wide FP64 rows n={n}, two passes: max dev {d:.3e}")
    assert d <= TOL["f64"]


def _plans(systems, stream):
    apc = _apc()
    torch = _torch()
    plans, keep = [], []
    for S in systems:
        A = torch.from_numpy(S.A).cuda()
        b = torch.from_numpy(S.B).cuda()
        keep.append((A, b))
        g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
        plans.append(apc.Plan(A, b, S.off, "f32", gamma=g, eta=e, stream=stream))
    return plans, keep


def test_batch_single_pass_matches_two_pass_and_oracle(monkeypatch):
    """A batch of plans that all update in one pass runs one pass over every factor
    (no pass-B items); the same plans batched with APC_FUSED=0 run two passes.  Both
    follow the oracle to the FP32 bar and each other to FP32 rounding."""
    apc = _apc()
    torch = _torch()
    systems = synth.many_small_systems(count=12, seed=84, lo=64, hi=1024)
    stream = torch.cuda.Stream()
    p1, k1 = _plans(systems, stream)
    b1 = apc.Batch(p1)
    monkeypatch.setenv("APC_FUSED", "0")
    p2, k2 = _plans(systems, stream)
    b2 = apc.Batch(p2)
    monkeypatch.delenv("APC_FUSED")
    l1, l2 = b1.launch(), b2.launch()
    say(f"case: batch single pass {l1}, two passes {l2}, n = {[S.n for S in systems]}")
    assert l1["items_b"] == 0 and l2["items_b"] > 0
    T = 30
    b1.iterate(T, graph=True)
    b2.iterate(T)
    stream.synchronize()
    worst_o, worst_2 = 0.0, 0.0
    for S, p, q in zip(systems, p1, p2):
        g, e = p.params()["gamma"], p.params()["eta"]
        ref = O.apc_run(S.A, S.B, S.off, T, g, e)["xbar"][:, 0]
        x = p.xbar().cpu().numpy()
        xs = np.linalg.norm(S.xstar)
        worst_o = max(worst_o, np.linalg.norm(x - ref) / xs)
        worst_2 = max(worst_2, np.linalg.norm(x - q.xbar().cpu().numpy()) / xs)
    say(f"max dev vs oracle {worst_o:.2e}, vs two-pass batch {worst_2:.2e}")
    assert worst_o <= TOL["f32"]
    assert worst_2 <= 1e-6
    b1.close()
    b2.close()


def test_batch_single_pass_blocks_over_several_tiles(monkeypatch):
    """Tall systems whose blocks span several single-pass row tiles (a tile holds up to
    256 rows of one block): blocks of 1, 255, 256, 257, 520 and 700 rows, rows of 700
    and 1024 columns (two and four 16-byte chunks per lane).  The batch's one pass
    follows the oracle to the FP32 bar and the two-pass batch to FP32 rounding."""
    apc = _apc()
    torch = _torch()
    systems = [
        synth.gaussian_system(1400, 700, sizes=[520, 257, 256, 1, 366], seed=91,
                              shift=2.0, scale=1.0 / math.sqrt(700)),
        synth.gaussian_system(1279, 1024, sizes=[700, 324, 255], seed=92,
                              shift=2.0, scale=1.0 / math.sqrt(1024)),
        synth.many_small_systems(count=1, seed=93, lo=300, hi=400)[0],
    ]
    stream = torch.cuda.Stream()
    p1, k1 = _plans(systems, stream)
    b1 = apc.Batch(p1)
    monkeypatch.setenv("APC_FUSED", "0")
    p2, k2 = _plans(systems, stream)
    b2 = apc.Batch(p2)
    monkeypatch.delenv("APC_FUSED")
    l1, l2 = b1.launch(), b2.launch()
    tiles = sum(-(-int(q) // 256) for S in systems for q in np.diff(S.off))
    say(f"case: batch single pass over multi-tile blocks {l1}, two passes {l2}, "
        f"tiles {tiles}")
    assert l1["items_b"] == 0 and l1["items_a"] == tiles and l2["items_b"] > 0
    T = 25
    b1.iterate(T, graph=True)
    b2.iterate(T)
    stream.synchronize()
    worst_o, worst_2 = 0.0, 0.0
    for S, p, q in zip(systems, p1, p2):
        g, e = p.params()["gamma"], p.params()["eta"]
        ref = O.apc_run(S.A, S.B, S.off, T, g, e)["xbar"][:, 0]
        x = p.xbar().cpu().numpy()
        xs = np.max(np.abs(S.xstar))
        # element by element, relative to the largest entry of x*
        worst_o = max(worst_o, np.max(np.abs(x - ref)) / xs)
        worst_2 = max(worst_2, np.max(np.abs(x - q.xbar().cpu().numpy())) / xs)
    say(f"max element dev vs oracle {worst_o:.2e}, vs two-pass batch {worst_2:.2e}")
    assert worst_o <= TOL["f32"]
    assert worst_2 <= 1e-6
    b1.close()
    b2.close()


def test_batch_with_wide_rows_takes_two_passes():
    """A system with rows wider than 1024 puts the whole batch on the two-pass kernels."""
    apc = _apc()
    torch = _torch()
    systems = synth.many_small_systems(count=3, seed=85, lo=64, hi=512)
    systems.append(synth.gaussian_system(1100, 1100, 4, seed=86, shift=2.0,
                                         scale=1.0 / math.sqrt(1100)))
    stream = torch.cuda.Stream()
    plans, keep = _plans(systems, stream)
    batch = apc.Batch(plans)
    launch = batch.launch()
    say(f"case: batch with a 1100-wide system: {launch}")
    assert launch["items_b"] > 0
    T = 20
    batch.iterate(T)
    stream.synchronize()
    for S, p in zip(systems, plans):
        g, e = p.params()["gamma"], p.params()["eta"]
        ref = O.apc_run(S.A, S.B, S.off, T, g, e)["xbar"][:, 0]
        assert np.linalg.norm(p.xbar().cpu().numpy() - ref) / np.linalg.norm(S.xstar) <= TOL["f32"]
    batch.close()


def test_one_row_groups_when_tiles_just_exceed_the_cus():
    """8192^2 FP32 with 64 uneven blocks (sizes drawn from [32, 256]): the single pass's
    tiles outnumber the CUs by less than a second round, and two-row register groups fit
    one workgroup per CU, so the plan takes one-row groups (two workgroups per CU); the
    update still matches the oracle."""
    apc = _apc()
    torch = _torch()
    S = synth.shifted_uneven_8k(seed=5, k=1)
    T = 8
    ref = oracle_traj(S, T, 1.0, 1.0)
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(np.ascontiguousarray(S.B[:, 0])).cuda()
    plan = apc.Plan(A, b, S.off, "f32", gamma=1.0, eta=1.0)
    shape = plan.single_pass_shape()
    tiles = sum(-(-int(p) // shape["rows_per_wg"]) for p in np.diff(S.off))
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    say(f"case: uneven 8192^2 FP32, {tiles} tiles on {cus} CUs, shape {shape}")
    if not cus < tiles <= 2 * cus:
        pytest.skip(f"{tiles} tiles on {cus} CUs: not between one and two per CU")
    assert shape["rows_per_group"] == 1
    d = dev(gpu_traj(plan, T), ref, S.xstar[:, 0])
    say(f"max dev {d:.3e}")
    assert d <= TOL["f32"]
    plan.close()
