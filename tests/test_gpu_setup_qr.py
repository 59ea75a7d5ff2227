"""GPU checks of the thin QR at setup (Sec. 3.1, CholeskyQR): an FP32 or bf16 plan (k = 1
or the k-RHS form) skips the second CholeskyQR pass only when the first pass's rows are
orthonormal far below FP32 rounding, and takes both passes otherwise; either way the
trajectory matches the FP64 oracle (Householder QR) to the FP32 bar 1e-5, and bf16
refinement still reaches the FP64 solution.

The ill-conditioned case mixes each block's rows by a p x p matrix whose singular values
span five orders of magnitude.  That leaves every row space, so every projector P_i and
the whole oracle trajectory, unchanged, while kappa(A_i) grows to ~1e5 and a single
CholeskyQR pass loses orthogonality to ~kappa^2 eps.  (A diagonal row scaling would
not do: Cholesky-based orthogonalisation is insensitive to it.)"""

import math
import sys

import numpy as np
import pytest

from oracle import apc_oracle as O
from paper_1708_01413_amd import synth

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


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


def mixed_rows(S, decades):
    """The same system with block i replaced by M_i [A_i, b_i], M_i = U diag(s) W^T with
    random orthogonal U, W and s spread over `decades` orders of magnitude: each row
    space, so each P_i and the oracle trajectory, is unchanged; kappa(A_i) is not."""
    rng = np.random.default_rng(99)
    A, B = S.A.copy(), S.B.copy()
    for i in range(len(S.off) - 1):
        r0, r1 = S.off[i], S.off[i + 1]
        p = r1 - r0
        U, _ = np.linalg.qr(rng.standard_normal((p, p)))
        W, _ = np.linalg.qr(rng.standard_normal((p, p)))
        M = (U * np.logspace(0, -decades, p)) @ W.T
        A[r0:r1] = M @ S.A[r0:r1]
        B[r0:r1] = M @ S.B[r0:r1]
    return synth.System(A=A, B=B, xstar=S.xstar, off=S.off, name=S.name)


def run(S, prec, T, monkeypatch=None, env=None):
    apc = _apc()
    torch = _torch()
    if env:
        for k, v in env.items():
            monkeypatch.setenv(k, v)
    A = torch.from_numpy(np.ascontiguousarray(S.A)).cuda()
    b = torch.from_numpy(S.B).cuda()
    g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    plan = apc.Plan(A, b, S.off, prec, gamma=g, eta=e)
    return plan, g, e


def test_well_conditioned_fp32_plan_takes_one_pass():
    S = synth.gaussian_system(1536, 1024, 8, seed=61, scale=1 / math.sqrt(1024))
    plan, g, e = run(S, "f32", 0)
    info = plan.setup_info()
    say(f"case: well-conditioned FP32 setup {info}")
    assert info["qr_passes"] == 1
    assert info["qr_defect"] < 1e-13
    T = 40
    d = dev(gpu_traj(plan, T), oracle_traj(S, T, g, e), S.xstar)
    say(f"max dev {d:.3e}")
    assert d <= TOL32


def test_ill_conditioned_fp32_plan_takes_two_passes():
    S = mixed_rows(synth.gaussian_system(1536, 1024, 8, seed=61, scale=1 / math.sqrt(1024)), 5)
    kappa = max(np.linalg.cond(Ai) for Ai in O.blocks(S.A, S.off))
    plan, g, e = run(S, "f32", 0)
    info = plan.setup_info()
    say(f"case: mixed-row FP32 setup (max kappa(A_i) {kappa:.1e}) {info}")
    assert kappa > 1e4
    assert info["qr_passes"] == 2
    assert info["qr_defect"] > 1e-10 / math.sqrt(192)
    T = 40
    d = dev(gpu_traj(plan, T), oracle_traj(S, T, g, e), S.xstar)
    say(f"max dev {d:.3e}")
    assert d <= TOL32


def test_two_passes_forced_and_fp64_plans(monkeypatch):
    S = synth.gaussian_system(1536, 1024, 8, seed=61, scale=1 / math.sqrt(1024))
    p64, _, _ = run(S, "f64", 0)
    i64 = p64.setup_info()
    assert i64["qr_passes"] == 2 and math.isnan(i64["qr_defect"])
    forced, _, _ = run(S, "f32", 0, monkeypatch, {"APC_QR_PASSES": "2"})
    i32 = forced.setup_info()
    assert i32["qr_passes"] == 2 and math.isnan(i32["qr_defect"])
    say(f"case: forced two passes {i32}, FP64 {i64}")


def test_vector_unit_setup_takes_the_same_decisions(monkeypatch):
    """The vector-unit setup (APC_SETUP_MFMA=0: its own Gram and triangular product, the
    start by an expansion pass, the two-pass orthogonality estimate) against the
    matrix-core one (the start and the estimate from the triangular product's row
    sums): the same one-pass / two-pass decisions, estimates of the same order, and both
    trajectories within the FP32 bar of the oracle."""
    good = synth.gaussian_system(1536, 1024, 8, seed=61, scale=1 / math.sqrt(1024))
    bad = mixed_rows(good, 5)
    T = 30
    for S, passes in ((good, 1), (bad, 2)):
        ref = oracle_traj(S, T, *O.optimal_params(*O.spectrum(S.A, S.off))[:2])
        infos = []
        for mfma in ("1", "0"):
            monkeypatch.setenv("APC_SETUP_MFMA", mfma)
            plan, g, e = run(S, "f32", 0)
            info = plan.setup_info()
            d = dev(gpu_traj(plan, T), ref, S.xstar)
            say(f"case: APC_SETUP_MFMA={mfma}, expected passes {passes}: {info}, max dev {d:.3e}")
            assert info["qr_passes"] == passes
            assert d <= TOL32
            infos.append(info["qr_defect"])
        monkeypatch.delenv("APC_SETUP_MFMA")
        if passes == 1:
            assert max(infos) < 1e-13
        else:
            lo, hi = min(infos), max(infos)
            assert lo > 1e-10 / math.sqrt(192) and hi / lo < 200


def test_restart_after_one_pass_setup():
    """apc_restart on a one-pass plan applies only the first inverse factor: a restart
    with new right-hand sides follows a fresh plan's trajectory."""
    apc = _apc()
    torch = _torch()
    S = synth.gaussian_system(1536, 1024, 8, seed=62, scale=1 / math.sqrt(1024))
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(S.B).cuda()
    b2 = torch.from_numpy(np.random.default_rng(63).standard_normal(S.B.shape)).cuda()
    plan = apc.Plan(A, b, S.off, "f32")
    assert plan.setup_info()["qr_passes"] == 1
    g, e = plan.params()["gamma"], plan.params()["eta"]
    plan.iterate(5)
    plan.restart(b2)
    plan.iterate(30)
    fresh = apc.Plan(A, b2, S.off, "f32", gamma=g, eta=e)
    fresh.iterate(30)
    d = float(torch.linalg.norm(plan.xbar() - fresh.xbar()) / torch.linalg.norm(fresh.xbar()))
    say(f"case: restart after one-pass setup, dev {d:.2e}")
    assert d <= 1e-12


# ---------------------------------------------------------------- k right-hand sides


def oracle_traj_k(S, T, gamma, eta):
    Qt, R = O.factor(S.A, S.off)
    x = O.init_local(Qt, R, S.B, S.off)
    xbar = O.initial_average(x)
    traj = [xbar.copy()]
    for _ in range(T):
        x, xbar = O.apc_step(Qt, x, xbar, gamma, eta)
        traj.append(xbar.copy())
    return np.stack(traj)


def gpu_traj_k(plan, T):
    torch = _torch()
    snaps = [plan.xbar()]
    for _ in range(T):
        plan.iterate(1)
        snaps.append(plan.xbar())
    torch.cuda.synchronize()
    return torch.stack(snaps).cpu().numpy()


def dev_k(a, b, xstar):
    """Largest column error over t: max_t max_c ||a_t[:, c] - b_t[:, c]|| / ||x*[:, c]||."""
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(xstar, axis=0)))


def test_krhs_fp32_plan_takes_one_pass_and_keeps_the_anchored_bar():
    """A well-conditioned FP32 plan with k = 12 (the (y, x_bar) form, FP64 anchor every
    16 updates) skips the second pass: its anchored trajectory, whose FP64 anchor
    products run on the one-pass FP64 factor, stays within the FP32 bar of the oracle
    over 40 updates (anchors at 0, 16, 32)."""
    S = synth.gaussian_system(1536, 1024, 8, k=12, seed=64, scale=1 / math.sqrt(1024))
    plan, g, e = run(S, "f32", 0)
    info = plan.setup_info()
    say(f"case: k = 12 FP32 setup {info}")
    assert info["qr_passes"] == 1
    assert info["qr_defect"] <= 1e-10 / math.sqrt(192)
    T = 40
    d = dev_k(gpu_traj_k(plan, T), oracle_traj_k(S, T, g, e), S.xstar)
    say(f"max column dev {d:.3e}")
    assert d <= TOL32


def test_ill_conditioned_krhs_fp32_plan_takes_two_passes():
    S = mixed_rows(synth.gaussian_system(1536, 1024, 8, k=12, seed=65, scale=1 / math.sqrt(1024)), 5)
    plan, g, e = run(S, "f32", 0)
    info = plan.setup_info()
    say(f"case: mixed-row k = 12 FP32 setup {info}")
    assert info["qr_passes"] == 2
    T = 40
    d = dev_k(gpu_traj_k(plan, T), oracle_traj_k(S, T, g, e), S.xstar)
    say(f"max column dev {d:.3e}")
    assert d <= TOL32


@pytest.mark.parametrize("anchor", [0, 4])
def test_bf16_plan_one_pass_refines_to_fp64(anchor):
    """bf16 refinement on a one-pass factor reaches the FP64 solution; with anchor
    updates turned on after setup (the FP64 pass-A factor copy is packed then)."""
    apc = _apc()
    torch = _torch()
    S = synth.shifted_square(1024, 8, k=6, shift=3.0, seed=66)
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(np.ascontiguousarray(S.B)).cuda()
    plan = apc.Plan(A, b, S.off, "bf16_ir", anchor_every=anchor)
    info = plan.setup_info()
    x, it, rr, st = plan.solve(1e-11, 4000)
    ref = np.linalg.solve(S.A, S.B)
    err = float(np.max(np.linalg.norm(x.cpu().numpy() - ref, axis=0) / np.linalg.norm(ref, axis=0)))
    say(f"case: bf16 anchor={anchor} setup {info}: status {st} updates {it} relres {rr:.2e} "
        f"err {err:.2e}")
    assert info["qr_passes"] == 1
    assert st == apc.APC_OK and err <= 1e-9


@pytest.mark.parametrize("n", [2048, 2050])
def test_split_gram_in_both_passes_fp64(n):
    """Rows of 2048 or more columns split the Gram product's K range (partial Grams in
    the factor slice the pass writes next); an FP64 plan takes both CholeskyQR passes,
    so both write their partials there: in place (n = 2048, the first pass reads A
    itself) and through the padded copy (n = 2050).  Mixed rows (kappa(A_i) ~ 1e4) make
    the second pass matter.  FP64 bar 1e-10 against the oracle's trajectory."""
    sizes = synth.renormalised_sizes(np.random.default_rng(62), 9, 2304, 160, 352)
    S = mixed_rows(synth.gaussian_system(2304, n, 9, seed=62, sizes=sizes,
                                         scale=1 / math.sqrt(n)), 4)
    plan, g, e = run(S, "f64", 0)
    info = plan.setup_info()
    say(f"case: split Gram, FP64, n={n}, blocks {np.diff(S.off).tolist()}, {info}")
    assert info["qr_passes"] == 2
    T = 30
    d = dev(gpu_traj(plan, T), oracle_traj(S, T, g, e), S.xstar)
    say(f"max dev {d:.3e}")
    assert d <= 1e-10
    plan.close()
