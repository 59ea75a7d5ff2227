"""Regression tests for fixed defects (GPU, through the C ABI):

* a batch whose system diverges reports APC_EDIVERGED, and a tolerance check never
  trusts flags left by an earlier check with another tolerance;
* the autograd wrapper differentiates the trajectory of its own forward, also when
  another forward on the same plan ran in between;
* updates after a refined (bf16) solve continue the refinement instead of re-adding
  the last committed correction.
"""

import math
import sys

import numpy as np
import pytest

from oracle import apc_oracle as O
from paper_1708_01413_amd import synth

pytestmark = pytest.mark.gpu


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


def _plans(systems, stream, params):
    apc = _apc()
    torch = _torch()
    plans, keep = [], []
    for S, (g, e) in zip(systems, params):
        A = torch.from_numpy(S.A).cuda()
        b = torch.from_numpy(S.B).cuda()
        plans.append(apc.Plan(A, b, S.off, "f32", gamma=g, eta=e, stream=stream))
        keep.append((A, b))
    return plans, keep


def test_batch_solve_reports_a_diverging_system():
    """Four systems, one with gamma = 1 and eta = 3 / mu_max, which puts the root
    1 - eta mu_max = -2 of its characteristic polynomial (eq. (5)) outside the unit disc:
    its iterates double every update until they overflow.  The batch solve must return
    APC_EDIVERGED (the kernels keep running on the non-finite values and finish)."""
    apc = _apc()
    torch = _torch()
    systems = synth.many_small_systems(count=4, seed=83, lo=64, hi=300)
    params = [O.optimal_params(*O.spectrum(S.A, S.off))[:2] for S in systems]
    _, mx = O.spectrum(systems[2].A, systems[2].off)
    params[2] = (1.0, 3.0 / mx)
    stream = torch.cuda.Stream()
    plans, keep = _plans(systems, stream, params)
    batch = apc.Batch(plans)
    say("case: batch with one diverging system")
    with pytest.raises(apc.ApcError) as ex:
        batch.solve(1e-6, 3000, check_every=8, graph=False)
    assert ex.value.status == apc.APC_EDIVERGED
    rr, _ = batch.residuals()
    say(f"relres after the solve: {rr.tolist()}")
    assert not math.isfinite(rr[2])
    assert all(rr[s] <= 1e-6 for s in (0, 1, 3))
    batch.close()


def test_batch_solve_does_not_trust_stale_flags():
    """A loose check deactivates every system; a later solve with a tight tolerance must
    still iterate them all to it."""
    apc = _apc()
    torch = _torch()
    systems = synth.many_small_systems(count=5, seed=84, lo=64, hi=400)
    params = [O.optimal_params(*O.spectrum(S.A, S.off))[:2] for S in systems]
    stream = torch.cuda.Stream()
    plans, keep = _plans(systems, stream, params)
    batch = apc.Batch(plans)
    rr0, act = batch.residuals(1e3)        # every relative residual is below 1e3
    assert not act.any()
    iters, rr, st = batch.solve(1e-5, 500, check_every=4, graph=True)
    say(f"case: stale flags: relres before {rr0.max():.2e}, after {rr.max():.2e}, "
        f"updates {iters.tolist()}")
    assert st == apc.APC_OK
    assert np.all(rr <= 1e-5) and np.all(iters > 0)
    batch.close()


def test_autograd_with_two_forwards_on_one_plan():
    """Two forwards on one plan with different right-hand sides, then both backwards:
    each gradient is the oracle adjoint of its own trajectory."""
    apc = _apc()
    torch = _torch()
    S = synth.shifted_square(384, 6, k=4, shift=1.5, seed=74, with_target=True)
    A, b1 = torch.from_numpy(S.A).cuda(), torch.from_numpy(S.B).cuda()
    B2 = np.random.default_rng(75).standard_normal(S.B.shape)
    b2 = torch.from_numpy(B2).cuda()
    T = 10
    g0, e0, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    xt_np = S.extra["x_target"]
    xt = torch.from_numpy(xt_np).cuda()
    plan = apc.Plan(A, b1, S.off, "f64")
    leaves, losses = [], []
    for bb in (b1, b2):
        bl = bb.clone().requires_grad_(True)
        gg = torch.tensor(g0, dtype=torch.float64, requires_grad=True)
        ee = torch.tensor(e0, dtype=torch.float64, requires_grad=True)
        x = apc.unrolled_apc(plan, bl, gg, ee, T, ckpt_every=3)
        losses.append(0.5 * torch.sum((x - xt) ** 2))
        leaves.append((bl, gg, ee))
    for L in losses:
        L.backward()
    for (bl, gg, ee), Bn in zip(leaves, (S.B, B2)):
        xr = O.apc_run(S.A, Bn, S.off, T, g0, e0)["xbar"]
        dB_ref, dg_ref, de_ref = O.apc_adjoint(S.A, Bn, S.off, T, g0, e0, xr - xt_np)
        rel = np.linalg.norm(bl.grad.cpu().numpy() - dB_ref) / np.linalg.norm(dB_ref)
        say(f"case: two forwards: dB rel {rel:.2e}, dgamma {float(gg.grad):.6e} vs {dg_ref:.6e}")
        assert rel <= 1e-10
        assert abs(float(gg.grad) - dg_ref) <= 1e-9 * abs(dg_ref)
        assert abs(float(ee.grad) - de_ref) <= 1e-9 * abs(de_ref)


def test_updates_after_a_refined_solve_continue_the_refinement():
    """bf16 refinement to 1e-12, then more updates and a second solve: the error against
    the oracle's converged solution must not grow (before the fix the next updates drove
    x_bar back to the last correction and added it to X a second time)."""
    apc = _apc()
    torch = _torch()
    S = synth.shifted_square(1024, 8, k=4, shift=3.0, seed=91)
    mn, mx = O.spectrum(S.A, S.off)
    g, e, rho = O.optimal_params(mn, mx)
    ref = O.apc_run(S.A, S.B, S.off, T=int(math.log(1e-17) / math.log(rho)) + 60,
                    gamma=g, eta=e)["xbar"]
    A, b = torch.from_numpy(S.A).cuda(), torch.from_numpy(S.B).cuda()
    plan = apc.Plan(A, b, S.off, "bf16_ir")
    x1, it1, rr1, st1 = plan.solve(1e-12, 2000)
    d1 = float(np.max(np.abs(x1.cpu().numpy() - ref)))
    plan.iterate(30)
    d2 = float(np.max(np.abs(plan.xbar().cpu().numpy() - ref)))
    r2 = plan.residual()
    x3, it3, rr3, st3 = plan.solve(1e-12, 2000)
    d3 = float(np.max(np.abs(x3.cpu().numpy() - ref)))
    scale = float(np.max(np.abs(S.xstar)))
    say(f"case: iterate after refined solve: max dev {d1:.2e} -> {d2:.2e} (relres {r2:.2e}) "
        f"-> {d3:.2e}; statuses {st1} {st3}")
    assert st1 == apc.APC_OK and st3 == apc.APC_OK
    assert d2 <= max(2 * d1, 1e-11 * scale)
    assert d3 <= 1e-10 * scale
