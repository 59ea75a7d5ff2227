"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (written per test): FP64 mode 1e-10 and FP32 mode 1e-5, as
||x_bar_gpu(t) - x_bar_oracle(t)||_2 / ||x*||_2 at every checked t and, where
stated, element by element as |x_bar_gpu(t)[j] - x_bar_oracle(t)[j]| / max_j |x*[j]|.
"""

import math
import os
import sys

import numpy as np
import pytest

from oracle import apc_oracle as O
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


def upload(S):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(S.A)).cuda(), torch.from_numpy(S.B).cuda()


def oracle_traj(S, T, gamma, eta):
    Qt, R = O.factor(S.A, S.off)
    x = O.init_local(Qt, R, S.B, S.off)
    xbar = O.initial_average(x)
    traj = [xbar[:, 0].copy()]
    for _ in range(T):
        x, xbar = O.apc_step(Qt, x, xbar, gamma, eta)
        traj.append(xbar[:, 0].copy())
    return np.stack(traj), x


def gpu_traj(plan, T):
    torch = _torch()
    snaps = [plan.xbar()]
    for _ in range(T):
        plan.iterate(1)
        snaps.append(plan.xbar())
    torch.cuda.synchronize()
    return torch.stack(snaps).cpu().numpy()


def rel_dev(a, b, xstar):
    return float(np.max(np.linalg.norm(a - b, axis=-1)) / np.linalg.norm(xstar))


def elem_dev(a, b, xstar):
    """max over entries (and over t) of |a - b| / max_j |x*[j]|."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(xstar)))


# ---------------------------------------------------------------- the FP64 workload


def householder_permuted_factor(S, seed):
    """The oracle's own factorisation (LAPACK Householder QR of A_i^T) applied to A_i^T
    with its n coordinates permuted, then permuted back: another valid thin QR of every
    block, with different rounding.  Used only to measure how strongly the oracle's
    trajectory reacts to rounding in its projectors."""
    rng = np.random.default_rng(seed)
    Qt, R = [], []
    for Ai in O.blocks(S.A, S.off):
        pi = rng.permutation(Ai.shape[1])
        Q, Ri = np.linalg.qr(Ai.T[pi], mode="reduced")
        Qf = np.empty_like(Q)
        Qf[pi] = Q
        Qt.append(Qf.T.copy())
        R.append(Ri)
    return Qt, R


@pytest.fixture(scope="module")
def square512():
    S = synth.square_gaussian_512()
    mn, mx = O.spectrum(S.A, S.off)
    g, e, rho = O.optimal_params(mn, mx)
    traj, _ = oracle_traj(S, 2000, g, e)
    # Sensitivity scale s(t): the largest drift of the oracle iteration run on four
    # coordinate-permuted Householder factors from the oracle's own trajectory.
    sens = np.zeros(2001)
    for seed in range(4):
        Qp, Rp = householder_permuted_factor(S, seed)
        x = O.init_local(Qp, Rp, S.B, S.off)
        xbar = O.initial_average(x)
        alt = [xbar[:, 0].copy()]
        for _ in range(2000):
            x, xbar = O.apc_step(Qp, x, xbar, g, e)
            alt.append(xbar[:, 0].copy())
        sens = np.maximum(sens, np.linalg.norm(np.stack(alt) - traj, axis=1)
                          / np.linalg.norm(S.xstar))
    return S, dict(mu_min=mn, mu_max=mx, gamma=g, eta=e, rho=rho), traj, sens


def test_fp64_square512_trajectory_2000(square512):
    """N = n = 512, m = 8, FP64, optimal (gamma, eta) from the oracle, 2000 updates through
    the transient growth (error peaks at ~31 ||x*||).  kappa(X) = 5.5e6 makes this
    trajectory amplify ~1e-16 differences between two valid projectors: the oracle run on
    its own Householder QR of coordinate-permuted blocks drifts from the unpermuted oracle
    by s(t) ~ 6e-11 at t = 300 and ~4e-9 at t = 2000 (largest of four permutations).
    Bar: 1e-10 for t <= 300, and 1e-10 + 2 s(t) for every t, i.e. at most twice the
    spread between two equally valid runs of the oracle itself."""
    apc = _apc()
    S, prm, ref, sens = square512
    say("case: square512 f64 trajectory T=2000")
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, "f64", gamma=prm["gamma"], eta=prm["eta"])
    got = gpu_traj(plan, 2000)
    dev_t = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(S.xstar)
    err = np.linalg.norm(got - S.xstar, axis=1) / np.linalg.norm(S.xstar)
    say(f"dev(300)={dev_t[300]:.3e} dev(2000)={dev_t[-1]:.3e} against the oracle's own "
        f"spread s(300)={sens[300]:.3e} s(2000)={sens[-1]:.3e} (ratio {dev_t[-1] / sens[-1]:.2f}); "
        f"element-wise dev(t<=300) {elem_dev(got[:301], ref[:301], S.xstar):.3e}; "
        f"err(1)={err[1]:.3f} peak={err.max():.2f} err(2000)={err[-1]:.2f}")
    assert dev_t[:301].max() <= TOL["f64"]
    assert elem_dev(got[:301], ref[:301], S.xstar) <= TOL["f64"]
    assert np.all(dev_t <= TOL["f64"] + 2.0 * sens)
    assert plan.iterations == 2000


def test_fp64_square512_invariants(square512):
    """App. A: A_i x_i(t) = b_i at every iterate (checked at t = 0, 700, 1400)."""
    apc = _apc()
    S, prm, _, _ = square512
    say("case: square512 f64 invariants")
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, "f64", gamma=prm["gamma"], eta=prm["eta"])
    for t in (0, 700, 1400):
        if t:
            plan.iterate(700)
        X = plan.local().cpu().numpy()
        for i, (Ai, bi) in enumerate(zip(O.blocks(S.A, S.off), O.blocks(S.B, S.off))):
            r = np.linalg.norm(Ai @ X[i] - bi) / np.linalg.norm(bi)
            assert r < 1e-11, (t, i, r)


def test_fp64_square512_eigen_estimate(square512):
    """Setup's Lanczos estimate of mu_min, mu_max (eq. (4)) and Theorem 1's optimum."""
    apc = _apc()
    S, prm, _, _ = square512
    say("case: square512 eigen estimate")
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, "f64")
    p = plan.params()
    say(p, prm)
    say(plan.info())
    assert prm["mu_max"] * (1 - 1e-12) <= p["mu_max"] <= prm["mu_max"] * (1 + 1e-4)
    assert prm["mu_min"] * (1 - 5e-2) <= p["mu_min"] <= prm["mu_min"] * (1 + 1e-9)
    assert p["gamma"] == pytest.approx(prm["gamma"], rel=1e-2)
    assert p["eta"] == pytest.approx(prm["eta"], rel=2e-2)
    assert prm["rho"] <= p["rho"] <= prm["rho"] + 1e-3


def test_setup_init_and_projectors_match_oracle():
    """Alg. 1 init (min-norm x_i(0), mean x_bar(0)) and P_i = I - Q_i Q_i^T on device:
    compare P_i v with the dense definition, and check P_i^2 = P_i and A_i P_i = 0."""
    apc = _apc()
    torch = _torch()
    S = synth.gaussian_system(300, 200, 7, seed=3,
                              sizes=synth.renormalised_sizes(np.random.default_rng(3), 7, 300, 20, 60))
    say("case: init/projectors N=300 n=200 m=7 uneven", np.diff(S.off))
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, "f64", gamma=1.0, eta=1.0)
    Qt, R = O.factor(S.A, S.off)
    x0 = O.init_local(Qt, R, S.B, S.off)[:, :, 0]
    np.testing.assert_allclose(plan.local().cpu().numpy(), x0, atol=1e-12)
    np.testing.assert_allclose(plan.xbar().cpu().numpy(), O.initial_average(x0[:, :, None])[:, 0],
                               atol=1e-12)
    V = torch.from_numpy(np.random.default_rng(0).standard_normal((7, 200))).cuda()
    PV = plan.project(V)
    PPV = plan.project(PV)
    PVn, PPVn, Vn = PV.cpu().numpy(), PPV.cpu().numpy(), V.cpu().numpy()
    for i, Ai in enumerate(O.blocks(S.A, S.off)):
        np.testing.assert_allclose(PVn[i], O.projector(Ai) @ Vn[i], atol=1e-12)
        np.testing.assert_allclose(PPVn[i], PVn[i], atol=1e-12)
        assert np.abs(Ai @ PVn[i]).max() < 1e-11


# ---------------------------------------------------------------- ragged / edge shapes


RAGGED = [
    # (N, n, m, size range or None, seed, shift)
    (300, 200, 7, (20, 60), 1, 0.0),       # n not a multiple of the tile/slab widths
    (1000, 1000, 13, (40, 120), 2, 2.0),   # several tiles per block, ragged tails
    (517, 333, 5, None, 4, 0.0),           # odd sizes, N mod m != 0
    (2048, 1536, 16, None, 5, 0.0),        # slab count > 1 in both precisions
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("N,n,m,rng_sizes,seed,shift", RAGGED)
def test_ragged_trajectory(prec, N, n, m, rng_sizes, seed, shift):
    apc = _apc()
    sizes = None
    if rng_sizes:
        sizes = synth.renormalised_sizes(np.random.default_rng(seed), m, N, *rng_sizes)
    S = synth.gaussian_system(N, n, m, seed=seed, shift=shift, sizes=sizes,
                              scale=1.0 / math.sqrt(n))
    say(f"case: ragged {prec} N={N} n={n} m={m} sizes={np.diff(S.off).tolist()}")
    g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    T = 60
    ref, _ = oracle_traj(S, T, g, e)
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, prec, gamma=g, eta=e)
    got = gpu_traj(plan, T)
    dev = rel_dev(got, ref, S.xstar)
    say(f"max dev {dev:.3e} (tol {TOL[prec]})")
    assert dev <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_row_blocks(prec):
    """p_i = 1 for every block (m = N = n = 96)."""
    apc = _apc()
    S = synth.gaussian_system(96, 96, 96, seed=7, shift=3.0, scale=1 / math.sqrt(96))
    say(f"case: single-row blocks {prec}")
    g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    ref, _ = oracle_traj(S, 40, g, e)
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, prec, gamma=g, eta=e)
    assert rel_dev(gpu_traj(plan, 40), ref, S.xstar) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("m", [129, 200, 260])
def test_many_blocks_single_pass(prec, m):
    """More blocks than the combine keeps in registers (a lane holds its first
    2 x 4 blocks' new x_i, 16 lanes per column: m <= 128 needs no read-back), so the
    later blocks' differences take the read-back path; blocks of 1 to 4 rows."""
    apc = _apc()
    rng = np.random.default_rng(40 + m)
    sizes = [int(v) for v in rng.integers(1, 5, size=m)]
    N = sum(sizes)
    n = N - 20  # tall: X has full rank
    S = synth.gaussian_system(N, n, sizes=sizes, seed=41 + m, shift=2.0, scale=1 / math.sqrt(n))
    say(f"case: many blocks {prec} m={m} N={N} n={n}")
    g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    ref, _ = oracle_traj(S, 30, g, e)
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, prec, gamma=g, eta=e)
    d = rel_dev(gpu_traj(plan, 30), ref, S.xstar)
    say(f"max dev {d:.3e}")
    assert d <= TOL[prec]


@pytest.mark.parametrize("N,n,m", [(64, 64, 1), (128, 64, 2), (3, 1, 3)])
def test_full_blocks_converge_in_one_step(N, n, m):
    """Every p_i = n: X = I, so gamma* = eta* = 1 and x_bar(1) = x* (Theorem 1).  Also
    runs the on-device eigenvalue estimate on an X with a single distinct eigenvalue."""
    apc = _apc()
    S = synth.gaussian_system(N, n, m, seed=8, shift=2.0 if N == n else 0.0)
    say(f"case: full blocks N={N} n={n} m={m}")
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, "f64")
    p = plan.params()
    assert p["gamma"] == pytest.approx(1.0, abs=1e-6) and p["eta"] == pytest.approx(1.0, abs=1e-6)
    plan.iterate(1)
    x = plan.xbar().cpu().numpy()
    assert np.linalg.norm(x - S.xstar) / np.linalg.norm(S.xstar) < 1e-10


def test_zero_updates_is_a_no_op():
    apc = _apc()
    S = synth.gaussian_system(64, 64, 4, seed=9, shift=2.0)
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, "f64", gamma=1.1, eta=1.5)
    x0 = plan.xbar().cpu().numpy()
    plan.iterate(0)
    np.testing.assert_array_equal(plan.xbar().cpu().numpy(), x0)
    assert plan.iterations == 0


def test_fp64_is_deterministic():
    apc = _apc()
    S = synth.gaussian_system(1024, 768, 12, seed=10, scale=1 / math.sqrt(768))
    say("case: determinism")
    A, b = upload(S)
    outs = []
    for _ in range(2):
        plan = apc.Plan(A, b, S.off, "f64", gamma=1.05, eta=3.0)
        plan.iterate(50)
        outs.append(plan.xbar().cpu().numpy())
        plan.close()
    np.testing.assert_array_equal(outs[0], outs[1])


# ---------------------------------------------------------------- error paths


def test_rank_deficient_block_is_reported():
    apc = _apc()
    S = synth.gaussian_system(64, 64, 4, seed=11)
    S.A[5] = S.A[4]
    say("case: rank-deficient block")
    A, b = upload(S)
    with pytest.raises(apc.ApcError) as ei:
        apc.Plan(A, b, S.off, "f64")
    assert ei.value.status == apc.APC_ERANK


def test_singular_system_is_reported():
    apc = _apc()
    S = synth.gaussian_system(80, 40, 4, seed=12)
    S.A[:, 3] = S.A[:, 4]
    say("case: singular X")
    A, b = upload(S)
    with pytest.raises(apc.ApcError) as ei:
        apc.Plan(A, b, S.off, "f64")
    assert ei.value.status == apc.APC_ESINGULAR


def test_solve_reports_divergence():
    """gamma = 1 and eta * mu_max = 3 put the root 1 - eta*mu_max = -2 of p_i outside the
    unit disc (eq. (6)): the residual blows up and apc_solve returns APC_EDIVERGED."""
    apc = _apc()
    S = synth.gaussian_system(64, 64, 4, seed=13, shift=2.0)
    _, mx = O.spectrum(S.A, S.off)
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, "f64", gamma=1.0, eta=3.0 / mx)
    say("case: divergence")
    with pytest.raises(apc.ApcError) as ei:
        plan.solve(1e-12, 5000)
    assert ei.value.status == apc.APC_EDIVERGED


@pytest.mark.parametrize("prec,rtol,xtol", [("f64", 1e-13, 1e-11), ("f32", 1e-6, 1e-5)])
def test_solve_reaches_direct_solution(prec, rtol, xtol):
    apc = _apc()
    S = synth.shifted_square(1024, 8, seed=14)
    say(f"case: solve {prec}")
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, prec)
    x, it, rr, st = plan.solve(rtol, 500)
    assert st == apc.APC_OK and rr <= rtol
    ref = np.linalg.solve(S.A, S.B)
    assert np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref) < xtol
    assert it == plan.iterations and it % 8 == 0


# ---------------------------------------------------------------- full size


@pytest.fixture(scope="module")
def tall16k():
    torch = _torch()
    g = np.load(os.path.join(GOLDEN, "tall_gauss_16384x8192_m64.npz"), allow_pickle=False)
    S = synth.tall_gaussian_16k()
    A, b = upload(S)
    xs = torch.from_numpy(S.xstar).cuda()
    off = S.off
    del S
    return A, b, xs, off, g


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_full_size_tall16k_trajectory(tall16k, prec):
    """N = 16384, n = 8192, m = 64 (the benchmark workload) in the launch configuration
    the benchmark times: the relative-error curve t = 0..60 and the whole vector x_bar(t)
    at 11 values of t against the oracle's stored values (tests/golden/make_golden.py),
    norm-wise and element by element."""
    torch = _torch()
    apc = _apc()
    A, b, xs, off, g = tall16k
    say(f"case: full-size tall16k {prec}")
    plan = apc.Plan(A, b, off, prec, gamma=float(g["gamma"]), eta=float(g["eta"]))
    check = list(g["check_t"])
    xn, xmax = float(g["xstar_norm"]), float(g["xstar_max"])
    errs, full = [], {}
    for t in range(int(check[-1]) + 1):
        if t:
            plan.iterate(1)
        xb = plan.xbar()
        errs.append(float(torch.linalg.norm(xb - xs)) / xn)
        if t in check:
            full[t] = xb.cpu().numpy()
    errs = np.array(errs)
    ref_err = g["err"]
    say("err gpu ", " ".join(f"{e:.3e}" for e in errs[[10, 20, 30, 40, 60]]))
    say("err orc ", " ".join(f"{e:.3e}" for e in ref_err[[10, 20, 30, 40, 60]]))
    assert np.max(np.abs(errs - ref_err)) <= TOL[prec]
    worst_n, worst_e = 0.0, 0.0
    for k, t in enumerate(check):
        d = full[t] - g["xbar"][k]
        worst_n = max(worst_n, float(np.linalg.norm(d)) / xn)
        worst_e = max(worst_e, float(np.max(np.abs(d))) / xmax)
    say(f"x_bar(t) vs oracle at t = {check}: norm-wise {worst_n:.3e}, element-wise {worst_e:.3e}")
    assert worst_n <= TOL[prec] and worst_e <= TOL[prec]
    first = lambda e, lvl: int(np.argmax(e <= lvl))
    assert abs(first(errs, 1e-5) - first(ref_err, 1e-5)) <= 1
    assert errs[-1] <= (1e-6 if prec == "f32" else 1e-9)


def test_full_size_tall16k_eigen_estimate(tall16k):
    """Setup's eigenvalue estimate in FP32 mode: Lanczos on X v through the FP32 factor the
    iteration uses (FP64 accumulation).  Accuracy contract: an interval that encloses the
    spectrum (FP32 rounding of Q shifts X by ~1e-7 absolute) and is at most 15 % wider at
    the bottom and 5e-3 at the top.  With these parameters the solve must need at most two
    more updates to 1e-5 than with the oracle's exact ones."""
    torch = _torch()
    apc = _apc()
    A, b, xs, off, g = tall16k
    say("case: full-size eigen estimate")
    plan = apc.Plan(A, b, off, "f32")
    p = plan.params()
    say(p, plan.info(), {k: float(g[k]) for k in ("mu_min", "mu_max", "gamma", "eta", "rho")})
    mx, mn = float(g["mu_max"]), float(g["mu_min"])
    assert mx * (1 - 2e-6) <= p["mu_max"] <= mx * (1 + 5e-3)
    assert mn * (1 - 0.15) <= p["mu_min"] <= mn * (1 + 1e-4)
    assert p["gamma"] == pytest.approx(float(g["gamma"]), rel=2e-3)
    assert p["eta"] == pytest.approx(float(g["eta"]), rel=3e-2)
    xn = float(g["xstar_norm"])
    t = 0
    while float(torch.linalg.norm(plan.xbar() - xs)) / xn > 1e-5 and t < 60:
        plan.iterate(1)
        t += 1
    ref_t = int(np.argmax(g["err"] <= 1e-5))
    say(f"updates to 1e-5 with the estimated parameters: {t} (oracle parameters: {ref_t})")
    assert ref_t - 1 <= t <= ref_t + 2


def test_fp64_eigen_estimate_uneven_blocks():
    """FP64 mode on a smaller system with uneven blocks: the estimate against eigvalsh of
    the dense X (oracle): an enclosing interval, at most 20 % wider at the bottom and 5e-3
    at the top."""
    apc = _apc()
    sizes = synth.renormalised_sizes(np.random.default_rng(21), 11, 1500, 40, 200)
    S = synth.gaussian_system(1500, 1200, 11, seed=21, sizes=sizes, scale=1 / math.sqrt(1200))
    mn, mx = O.spectrum(S.A, S.off)
    say("case: f64 eigen estimate uneven", np.diff(S.off).tolist())
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, "f64")
    p = plan.params()
    say(p, plan.info(), mn, mx)
    assert mx * (1 - 1e-12) <= p["mu_max"] <= mx * (1 + 5e-3)
    assert mn * (1 - 0.2) <= p["mu_min"] <= mn * (1 + 1e-9)


# ---------------------------------------------------------------- k right-hand sides


MULTI = [
    # (N, n, m, size range, k, seed)
    (300, 200, 7, (20, 60), 3, 31),        # k padded to 16; n not a multiple of 64
    (1000, 800, 9, (40, 160), 20, 32),      # k padded to 32; 128-row tiles + tails
    (2048, 2048, 16, (64, 192), 64, 33),    # full 64-wide tile, square, shifted
    (512, 512, 4, (96, 160), 130, 35),      # k > 128: two 128-wide column groups
    (301, 201, 5, (40, 80), 8, 42),         # odd n and lda: element-wise operand packing
]


@pytest.mark.parametrize("prec", ["f64", "f32", "f32-plain"])
@pytest.mark.parametrize("N,n,m,rng_sizes,k,seed", MULTI)
def test_multi_rhs_trajectory(prec, N, n, m, rng_sizes, k, seed):
    """k right-hand sides, the (y, x_bar) form on the matrix cores (FP64; FP32 with the
    default FP64 anchors; "f32-plain": every update in FP32), against the literal oracle
    run on the same k columns.  Bar: max over t of ||X_gpu(t) - X_oracle(t)||_F / ||X*||_F."""
    apc = _apc()
    torch = _torch()
    sizes = synth.renormalised_sizes(np.random.default_rng(seed), m, N, *rng_sizes)
    S = synth.gaussian_system(N, n, m, k=k, seed=seed, sizes=sizes, scale=1 / math.sqrt(n),
                              shift=2.0 if N == n else 0.0)
    say(f"case: multi-rhs {prec} N={N} n={n} m={m} k={k} sizes={np.diff(S.off).tolist()}")
    g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    T = 40
    Qt, R = O.factor(S.A, S.off)
    x = O.init_local(Qt, R, S.B, S.off)
    xbar = O.initial_average(x)
    ref = [xbar.copy()]
    for _ in range(T):
        x, xbar = O.apc_step(Qt, x, xbar, g, e)
        ref.append(xbar.copy())
    A, b = upload(S)
    base = prec.split("-")[0]
    plan = apc.Plan(A, b, S.off, base, gamma=g, eta=e,
                    anchor_every=0 if prec.endswith("plain") else None)
    snaps = [plan.xbar()]
    for _ in range(T):
        plan.iterate(1)
        snaps.append(plan.xbar())
    torch.cuda.synchronize()
    got = torch.stack(snaps).cpu().numpy()
    dev = max(np.linalg.norm(got[t] - ref[t]) for t in range(T + 1)) / np.linalg.norm(S.xstar)
    err = np.linalg.norm(got[-1] - S.xstar) / np.linalg.norm(S.xstar)
    say(f"max dev {dev:.3e} (tol {TOL[base]}), err(T) {err:.2e}, shapes {plan.launch_shapes()}")
    assert dev <= TOL[base]
    # the local solutions keep A_i x_i = b_i for every column
    X = plan.local().cpu().numpy()
    for i, (Ai, bi) in enumerate(zip(O.blocks(S.A, S.off), O.blocks(S.B, S.off))):
        r = np.linalg.norm(Ai @ X[i] - bi) / np.linalg.norm(bi)
        assert r < (1e-10 if base == "f64" else 1e-4), (i, r)


def test_fp32_anchor_updates_remove_the_fp32_floor():
    """Plain FP32 products on y level off near eps_32 / mu_min; with FP64 anchor updates
    the FP32 products act on y - y_ref only and the error keeps falling at the FP64 rate."""
    apc = _apc()
    torch = _torch()
    S = synth.shifted_square(2048, 16, k=16, shift=1.5, seed=36)
    A, b = upload(S)
    xs = torch.from_numpy(S.xstar).to(A.device)
    errs = {}
    for every in (0, 16):
        plan = apc.Plan(A, b, S.off, "f32", anchor_every=every)
        plan.iterate(150)
        errs[every] = float(torch.linalg.norm(plan.xbar() - xs) / torch.linalg.norm(xs))
        plan.close()
    ref = apc.Plan(A, b, S.off, "f64")
    ref.iterate(150)
    e64 = float(torch.linalg.norm(ref.xbar() - xs) / torch.linalg.norm(xs))
    say(f"case: anchors; err(150) plain FP32 {errs[0]:.2e}, anchored {errs[16]:.2e}, FP64 {e64:.2e}")
    assert errs[16] <= max(10 * e64, 1e-11)
    assert errs[16] < 1e-2 * errs[0]


def test_anchor_argument_errors():
    apc = _apc()
    S = synth.shifted_square(256, 4, k=2, seed=37)
    A, b = upload(S)
    p64 = apc.Plan(A, b, S.off, "f64")
    with pytest.raises(apc.ApcError) as ex:
        apc.apc_set_anchor(p64.handle, 4)
    assert ex.value.status == apc.APC_EUNSUPPORTED
    p32 = apc.Plan(A, b, S.off, "f32")
    with pytest.raises(apc.ApcError) as ex:
        apc.apc_set_anchor(p32.handle, -1)
    assert ex.value.status == apc.APC_EINVAL
    p32.iterate(1)
    with pytest.raises(apc.ApcError) as ex:
        apc.apc_set_anchor(p32.handle, 4)
    assert ex.value.status == apc.APC_EINVAL


@pytest.mark.parametrize("rt,split", [("1", "8"), ("4", "1"), ("2", "3")])
def test_launch_shapes_change_rounding_only(rt, split, monkeypatch):
    """Every (rows per workgroup, split-K) shape computes the same products: FP64
    trajectories from forced shapes agree with the tuned one to rounding."""
    apc = _apc()
    torch = _torch()
    S = synth.gaussian_system(1500, 1000, 10, k=24, seed=38, scale=1 / math.sqrt(1000))
    A, b = upload(S)
    g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    tuned = apc.Plan(A, b, S.off, "f64", gamma=g, eta=e)
    tuned.iterate(25)
    x_tuned = tuned.xbar()
    monkeypatch.setenv("APC_TN_RT", rt)
    monkeypatch.setenv("APC_TN_SPLIT", split)
    forced = apc.Plan(A, b, S.off, "f64", gamma=g, eta=e)
    shapes = forced.launch_shapes()
    forced.iterate(25)
    dev = float(torch.linalg.norm(forced.xbar() - x_tuned) / torch.linalg.norm(x_tuned))
    say(f"case: forced shapes {shapes['pass_a']} {shapes['pass_b']}: dev {dev:.2e}")
    assert shapes["pass_b"]["splits"] == int(split)
    assert dev <= 1e-12


@pytest.mark.parametrize("rt,pf,nt,split,waves", [("1", "4", "1", "1", "4"), ("2", "3", "1", "2", "4"),
                                                 ("4", "2", "0", "4", "4"), ("2", "1", "1", "8", "4"),
                                                 ("1", "2", "1", "4", "8"), ("2", "1", "1", "2", "8")])
def test_fp32_launch_shapes_match_oracle(rt, pf, nt, split, waves, monkeypatch):
    """FP32 k-RHS plans with forced contraction shapes (row tiles per wave, prefetch depth,
    non-temporal loads, split-K, waves per workgroup), including the deep-prefetch and
    eight-wave ones, against the oracle's trajectory at the FP32 bar (plain FP32 updates,
    no anchors)."""
    apc = _apc()
    torch = _torch()
    S = synth.gaussian_system(1536, 1024, 12, k=24, seed=39, scale=1 / math.sqrt(1024))
    g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    T = 30
    Qt, R = O.factor(S.A, S.off)
    x = O.init_local(Qt, R, S.B, S.off)
    xbar = O.initial_average(x)
    ref = [xbar.copy()]
    for _ in range(T):
        x, xbar = O.apc_step(Qt, x, xbar, g, e)
        ref.append(xbar.copy())
    A, b = upload(S)
    for var, val in (("APC_TN_RT", rt), ("APC_TN_PF", pf), ("APC_TN_NT", nt), ("APC_TN_SPLIT", split),
                     ("APC_TN_WAVES", waves)):
        monkeypatch.setenv(var, val)
    plan = apc.Plan(A, b, S.off, "f32", gamma=g, eta=e, anchor_every=0)
    shapes = plan.launch_shapes()
    assert shapes["pass_a"]["rows_per_wg"] == 16 * int(waves) * int(rt)
    snaps = [plan.xbar()]
    for _ in range(T):
        plan.iterate(1)
        snaps.append(plan.xbar())
    got = torch.stack(snaps).cpu().numpy()
    dev = max(np.linalg.norm(got[t] - ref[t]) for t in range(T + 1)) / np.linalg.norm(S.xstar)
    say(f"case: fp32 forced shape rt={rt} pf={pf} nt={nt} split={split} waves={waves} {shapes['pass_a']}: "
        f"dev {dev:.2e}")
    assert shapes["pass_a"]["splits"] == int(split)
    assert dev <= TOL["f32"]


def test_multi_rhs_solve_and_residual():
    apc = _apc()
    S = synth.shifted_square(1024, 8, k=5, seed=34)
    say("case: multi-rhs solve")
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, "f32")
    x, it, rr, st = plan.solve(1e-6, 400)
    assert st == apc.APC_OK and rr <= 1e-6
    ref = np.linalg.solve(S.A, S.B)
    assert np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-5


# ---------------------------------------------------------------- mixed precision


@pytest.mark.parametrize("alpha,k,anchor", [(3.0, 32, 0), (1.5, 32, 0), (3.0, 1, 0), (1.5, 32, 8)])
def test_bf16_refinement_reaches_fp64_accuracy(alpha, k, anchor):
    """BF16 projections on matrix cores inside FP64 iterative refinement: the solution
    matches x* (b = A x* in FP64; kappa(A) < 10 here) to 1e-10 relative error, the
    bar for the mixed-precision mode against the FP64 oracle's direct solve."""
    apc = _apc()
    S = synth.shifted_square(2048, 8, k=k, shift=alpha, seed=40)
    say(f"case: bf16 refinement alpha={alpha} k={k} anchor={anchor}")
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, "bf16_ir", anchor_every=anchor)
    x, it, rr, st = plan.solve(1e-13, 2000)
    info = plan.info()
    xs = S.xstar
    err = np.linalg.norm(x.cpu().numpy() - xs) / np.linalg.norm(xs)
    ref = np.linalg.solve(S.A, S.B)
    dev = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    say(f"status {st} updates {it} refinements {info['refinements']} relres {rr:.2e} "
        f"err vs x* {err:.2e} vs LAPACK solve {dev:.2e}")
    assert st == apc.APC_OK
    assert err <= 1e-10 and dev <= 1e-10
    assert info["refinements"] >= 2      # the inner bf16 solve alone cannot reach 1e-10


def test_bf16_restart_with_new_rhs_reaches_fp64_accuracy():
    """A refined bf16 solve, then apc_restart with new right-hand sides and a second solve
    (the inner solves start from x_bar(0) formed on the FP32 matrix cores): both
    solutions match the LAPACK solve of their right-hand sides to 1e-10."""
    apc = _apc()
    torch = _torch()
    S = synth.shifted_square(2048, 8, k=16, shift=3.0, seed=45)
    A, b = upload(S)
    b2 = torch.from_numpy(np.random.default_rng(46).standard_normal(S.B.shape)).to(A.device)
    plan = apc.Plan(A, b, S.off, "bf16_ir")
    x1, it1, rr1, st1 = plan.solve(1e-12, 2000)
    ref1 = np.linalg.solve(S.A, S.B)
    d1 = np.linalg.norm(x1.cpu().numpy() - ref1) / np.linalg.norm(ref1)
    plan.restart(b2)
    x2, it2, rr2, st2 = plan.solve(1e-12, 2000)
    ref2 = np.linalg.solve(S.A, b2.cpu().numpy())
    d2 = np.linalg.norm(x2.cpu().numpy() - ref2) / np.linalg.norm(ref2)
    say(f"case: bf16 restart: first solve {it1} updates dev {d1:.2e}, after restart {it2} "
        f"updates dev {d2:.2e}")
    assert st1 == apc.APC_OK and st2 == apc.APC_OK
    assert d1 <= 1e-10 and d2 <= 1e-10
    plan.close()


def test_bf16_inner_solve_contracts():
    """One inner solve on the bf16 factor (no refinement) cuts the residual by > 100x."""
    apc = _apc()
    S = synth.shifted_square(2048, 8, k=16, shift=3.0, seed=41)
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, "bf16_ir")
    r0 = plan.residual()
    plan.iterate(20)
    r1 = plan.residual()
    say(f"case: bf16 inner solve relres {r0:.2e} -> {r1:.2e}")
    assert r1 < 1e-2 * r0


# ---------------------------------------------------------------- differentiation


def test_restart_and_set_params_reproduce_fresh_plans():
    """apc_restart(B2) + apc_set_params(g, e) give the trajectory of a plan set up on B2
    with (g, e): same factor, so FP64 results agree to rounding."""
    apc = _apc()
    torch = _torch()
    S = synth.gaussian_system(600, 400, 6, k=5, seed=50, scale=1 / math.sqrt(400))
    A, b = upload(S)
    b2 = torch.from_numpy(np.random.default_rng(51).standard_normal(S.B.shape)).to(A.device)
    plan = apc.Plan(A, b, S.off, "f64")
    g, e = plan.params()["gamma"] * 0.97, plan.params()["eta"] * 0.9
    plan.iterate(7)
    plan.set_params(g, e)
    plan.restart(b2)
    assert plan.iterations == 0
    plan.iterate(30)
    fresh = apc.Plan(A, b2, S.off, "f64", gamma=g, eta=e)
    fresh.iterate(30)
    dev = float(torch.linalg.norm(plan.xbar() - fresh.xbar()) / torch.linalg.norm(fresh.xbar()))
    say(f"case: restart/set_params dev {dev:.2e}")
    assert dev <= 1e-13


@pytest.mark.parametrize("N,n,m,k,T,ckpt,reduced", [(300, 200, 7, 3, 25, 4, False),
                                                    (256, 256, 4, 1, 20, 5, True),
                                                    (512, 384, 8, 20, 16, 16, False)])
def test_backward_matches_oracle_adjoint(N, n, m, k, T, ckpt, reduced):
    """FP64 plan: dL/dB, dL/dgamma, dL/deta from apc_backward against the oracle's
    literal-form adjoint on the same inputs and (gamma, eta)."""
    apc = _apc()
    torch = _torch()
    S = synth.gaussian_system(N, n, m, k=k, seed=52 + k, scale=1 / math.sqrt(n),
                              shift=1.5 if N == n else 0.0)
    g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    dx = np.random.default_rng(60 + k).standard_normal((n, k) if k > 1 else (n,))
    dB_ref, dg_ref, de_ref = O.apc_adjoint(S.A, S.B, S.off, T, g, e, dx)
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, "f64", gamma=g, eta=e, reduced_form=reduced)
    dB, dg, de = plan.backward(torch.from_numpy(dx).to(A.device), T, ckpt)
    dB = dB.cpu().numpy().reshape(dB_ref.shape)
    rel_b = np.linalg.norm(dB - dB_ref) / np.linalg.norm(dB_ref)
    say(f"case: backward f64 N={N} n={n} k={k} T={T}: dB rel {rel_b:.2e}, dgamma {dg:.6e} vs "
        f"{dg_ref:.6e}, deta {de:.6e} vs {de_ref:.6e}")
    assert rel_b <= 1e-10
    scale = np.linalg.norm(dx) * np.linalg.norm(S.xstar)
    assert abs(dg - dg_ref) <= 1e-9 * max(abs(dg_ref), scale)
    assert abs(de - de_ref) <= 1e-9 * max(abs(de_ref), scale)
    assert plan.iterations == T


def test_backward_fp32_converged_gradient_and_differences():
    """N = n = 4096, A = G/sqrt(n) + 2I, k = 16, m = 32 blocks of 128, FP32, T = 200 with a
    checkpoint every 14 updates, L = 1/2 ||x_bar(T) - x_target||^2.  At T = 200 the
    iteration has converged: dL/dB = A^{-T} (x_bar(T) - x_target) and dL/dgamma, dL/deta
    ~ 0.  At T = 10 (before convergence): the FP64 adjoint against central differences
    of the FP64 forward (h = 1e-5, and h = 1e-3 within that difference's own Richardson
    truncation estimate), the FP32 adjoint against the FP64 one, and dL/dB along a
    direction (exact: L is quadratic in B)."""
    apc = _apc()
    torch = _torch()
    S = synth.shifted_square(4096, 32, k=16, shift=2.0, seed=70, with_target=True)
    A, b = upload(S)
    dev = A.device
    xt = torch.from_numpy(S.extra["x_target"]).to(dev)
    p32 = apc.Plan(A, b, S.off, "f32")
    g, e = p32.params()["gamma"], p32.params()["eta"]
    p32.iterate(200)
    r = p32.xbar() - xt
    dB, dg, de = p32.backward(r, 200, 14)
    ref = torch.linalg.solve(A.T.contiguous(), r)
    rel = float(torch.linalg.norm(dB - ref) / torch.linalg.norm(ref))
    scale = float(torch.linalg.norm(r) * torch.linalg.norm(p32.xbar()))
    say(f"case: adjoint T=200: dB vs A^-T r rel {rel:.2e}; dgamma {dg:.2e}, deta {de:.2e} "
        f"(scale {scale:.2e})")
    assert rel <= 1e-5
    assert abs(dg) <= 1e-6 * scale and abs(de) <= 1e-6 * scale
    # Before convergence: FP64 forward differences.
    T = 10
    p64 = apc.Plan(A, b, S.off, "f64", gamma=g, eta=e)

    def loss(gg, ee, bb=None):
        p64.set_params(gg, ee)
        p64.restart(bb if bb is not None else b)
        p64.iterate(T)
        return 0.5 * float(torch.linalg.norm(p64.xbar() - xt) ** 2)

    p32.set_params(g, e)
    p32.restart(b)
    p32.iterate(T)
    r10 = p32.xbar() - xt
    dB10, dg10, de10 = p32.backward(r10, T, 3)
    p64.set_params(g, e)
    p64.restart(b)
    p64.iterate(T)
    _, dg64, de64 = p64.backward(p64.xbar() - xt, T, 3)
    fd = {}
    for h in (1e-3, 5e-4, 1e-5):
        fd[h] = ((loss(g + h, e) - loss(g - h, e)) / (2 * h),
                 (loss(g, e + h) - loss(g, e - h)) / (2 * h))
    h = 1e-3
    d = torch.from_numpy(np.random.default_rng(71).standard_normal(S.B.shape)).to(dev)
    fd_b = (loss(g, e, b + h * d) - loss(g, e, b - h * d)) / (2 * h)
    dir_b = float(torch.sum(dB10 * d))
    say(f"case: adjoint T=10: dgamma f32 {dg10:.6e} f64 {dg64:.6e} fd(1e-3) {fd[1e-3][0]:.6e} "
        f"fd(1e-5) {fd[1e-5][0]:.6e}; deta f32 {de10:.6e} f64 {de64:.6e} fd(1e-3) "
        f"{fd[1e-3][1]:.6e}; dB.d {dir_b:.6e} fd {fd_b:.6e}")
    for q, (adj64, adj32) in enumerate(((dg64, dg10), (de64, de10))):
        # Central differences are L' + c h^2 + ...; c estimated from h = 1e-3 and h/2
        # bounds the truncation at h = 1e-3 and, scaled by h^2, at h = 1e-5.
        c = (fd[1e-3][q] - fd[5e-4][q]) / (1e-6 - 0.25e-6)
        for h in (1e-3, 1e-5):
            assert abs(adj64 - fd[h][q]) <= 2.0 * abs(c) * h * h + 1e-6 * abs(fd[h][q])
        # FP32 products in the FP32 plan's adjoint.
        assert abs(adj32 - adj64) <= 1e-4 * abs(adj64)
    assert abs(dir_b - fd_b) <= 1e-4 * abs(fd_b)


def test_autograd_function_matches_oracle():
    """torch.autograd through unrolled_apc (FP64 plan) gives the oracle adjoint of
    L = 1/2 ||x_bar(T) - x_target||^2 for b, gamma and eta."""
    apc = _apc()
    torch = _torch()
    S = synth.shifted_square(384, 6, k=4, shift=1.5, seed=72, with_target=True)
    A, b = upload(S)
    T = 12
    g0, e0, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    plan = apc.Plan(A, b, S.off, "f64")
    bb = b.clone().requires_grad_(True)
    gg = torch.tensor(g0, dtype=torch.float64, requires_grad=True)
    ee = torch.tensor(e0, dtype=torch.float64, requires_grad=True)
    x = apc.unrolled_apc(plan, bb, gg, ee, T, ckpt_every=5)
    xt = torch.from_numpy(S.extra["x_target"]).to(A.device)
    loss = 0.5 * torch.sum((x - xt) ** 2)
    loss.backward()
    xr = O.apc_run(S.A, S.B, S.off, T, g0, e0)["xbar"]
    dB_ref, dg_ref, de_ref = O.apc_adjoint(S.A, S.B, S.off, T, g0, e0, xr - S.extra["x_target"])
    rel = np.linalg.norm(bb.grad.cpu().numpy() - dB_ref) / np.linalg.norm(dB_ref)
    say(f"case: autograd: dB rel {rel:.2e}, dgamma {float(gg.grad):.6e} vs {dg_ref:.6e}, "
        f"deta {float(ee.grad):.6e} vs {de_ref:.6e}")
    assert rel <= 1e-10
    assert abs(float(gg.grad) - dg_ref) <= 1e-9 * abs(dg_ref)
    assert abs(float(ee.grad) - de_ref) <= 1e-9 * abs(de_ref)


def test_backward_unsupported_plans():
    apc = _apc()
    torch = _torch()
    S = synth.shifted_square(256, 4, k=1, seed=73)
    A, b = upload(S)
    for prec, kw in (("f64", {}), ("bf16_ir", {})):
        plan = apc.Plan(A, b, S.off, prec, **kw)
        with pytest.raises(apc.ApcError) as ex:
            plan.backward(torch.zeros(256, dtype=torch.float64, device=A.device), 5, 2)
        assert ex.value.status in (apc.APC_EUNSUPPORTED,)


# ---------------------------------------------------------------- many independent systems


def _batch_plans(systems, stream, params=True):
    apc = _apc()
    torch = _torch()
    plans, tensors = [], []
    for S in systems:
        A = torch.from_numpy(S.A).to("cuda")
        b = torch.from_numpy(S.B).to("cuda")
        if params:
            g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
            plans.append(apc.Plan(A, b, S.off, "f32", gamma=g, eta=e, stream=stream))
        else:
            plans.append(apc.Plan(A, b, S.off, "f32", stream=stream))
        tensors.append((A, b))
    return plans, tensors


def test_batch_matches_oracle_and_single_plans():
    """Ten independent systems (n in [64, 700], m in {4, 8, 16}, uneven n) through one
    persistent launch per pass: every x_bar(T) within the FP32 bar of the oracle's, and
    equal to the same plan iterated alone up to FP32 rounding."""
    apc = _apc()
    torch = _torch()
    systems = synth.many_small_systems(count=10, seed=80, lo=64, hi=700)
    stream = torch.cuda.Stream()
    plans, keep = _batch_plans(systems, stream)
    single, keep2 = _batch_plans(systems, stream)
    batch = apc.Batch(plans)
    say(f"case: batch of {len(systems)}: n = {[S.n for S in systems]}, launch {batch.launch()}")
    T = 30
    batch.iterate(T)
    for p in single:
        p.iterate(T)
    stream.synchronize()
    worst_o, worst_s = 0.0, 0.0
    for S, p, q in zip(systems, plans, single):
        g, e = p.params()["gamma"], p.params()["eta"]
        ref = O.apc_run(S.A, S.B, S.off, T, g, e)["xbar"][:, 0]
        x = p.xbar().cpu().numpy()
        worst_o = max(worst_o, np.linalg.norm(x - ref) / np.linalg.norm(S.xstar))
        worst_s = max(worst_s, np.linalg.norm(x - q.xbar().cpu().numpy()) / np.linalg.norm(S.xstar))
        assert p.iterations == T
    say(f"max dev vs oracle {worst_o:.2e}, vs single plans {worst_s:.2e}")
    assert worst_o <= TOL["f32"]
    assert worst_s <= 1e-6
    batch.close()


def test_batch_graph_replays_match_eager_launches():
    """The captured graph of 5 updates, replayed three times with eager work and syncs in
    between, gives bitwise the same states as eager launches, at every replay."""
    apc = _apc()
    torch = _torch()
    systems = synth.many_small_systems(count=6, seed=81, lo=64, hi=400)
    stream = torch.cuda.Stream()
    pa, k1 = _batch_plans(systems, stream)
    pb, k2 = _batch_plans(systems, stream)
    ba, bb = apc.Batch(pa), apc.Batch(pb)
    for rep in range(3):
        ba.iterate(5, graph=True)
        bb.iterate(5, graph=False)
        stream.synchronize()
        junk = torch.randn(1000, device="cuda").sum().item()  # eager work between replays
        ra, _ = ba.residuals()
        for p, q in zip(pa, pb):
            assert torch.equal(p.xbar(), q.xbar()), (rep, junk)
        say(f"case: graph replay {rep}: residuals {ra.max():.2e}")
    ba.close()
    bb.close()


def test_batch_solve_stops_each_system():
    """Per-system stopping: every system reaches rtol, systems converge after different
    numbers of updates, and each x_bar is near its x*."""
    apc = _apc()
    torch = _torch()
    systems = synth.many_small_systems(count=16, seed=82, lo=64, hi=1024)
    stream = torch.cuda.Stream()
    plans, keep = _batch_plans(systems, stream, params=False)
    batch = apc.Batch(plans)
    iters, rr, st = batch.solve(1e-5, 400, check_every=4, graph=True)
    say(f"case: batch solve: status {st}, iterations {iters.tolist()}, max relres {rr.max():.2e}")
    assert st == apc.APC_OK
    assert np.all(rr <= 1e-5)
    assert len(set(iters.tolist())) > 1
    for S, p in zip(systems, plans):
        err = np.linalg.norm(p.xbar().cpu().numpy() - S.xstar) / np.linalg.norm(S.xstar)
        assert err <= 1e-4
    batch.close()
