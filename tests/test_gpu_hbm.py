"""GPU parity of the comparison methods (Sec. 4.3 D-HBM, Sec. 6 preconditioned
D-HBM) through the C ABI, against the FP64 oracle.

Tolerances as for APC: ||x_gpu(t) - x_oracle(t)||_2 / ||x*||_2 <= 1e-10 (FP64
plans) and 1e-5 (FP32 plans) at every checked t, parameters passed from the
oracle."""

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


def hbm_traj(h, T):
    torch = _torch()
    snaps = [h.x()]
    for _ in range(T):
        h.iterate(1)
        snaps.append(h.x())
    torch.cuda.synchronize()
    return torch.stack(snaps).cpu().numpy()


def rel_dev(a, b, xstar):
    return float(np.max(np.linalg.norm(a - b, axis=-1)) / np.linalg.norm(xstar))


CASES = [
    # (N, n, m, size range or None, seed, shift)
    (300, 200, 7, (20, 60), 1, 0.0),
    (1000, 1000, 13, (40, 120), 2, 2.0),
    (517, 333, 5, None, 4, 0.0),
    (2048, 1536, 16, None, 5, 0.0),
]


def make_case(N, n, m, rng_sizes, seed, shift):
    sizes = None
    if rng_sizes:
        sizes = synth.renormalised_sizes(np.random.default_rng(seed), m, N, *rng_sizes)
    return synth.gaussian_system(N, n, m, seed=seed, shift=shift, sizes=sizes,
                                 scale=1.0 / math.sqrt(n))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind", [0, 1], ids=["plain", "preconditioned"])
@pytest.mark.parametrize("N,n,m,rng_sizes,seed,shift", CASES)
def test_hbm_trajectory_matches_oracle(prec, kind, N, n, m, rng_sizes, seed, shift):
    apc = _apc()
    S = make_case(N, n, m, rng_sizes, seed, shift)
    say(f"case: hbm kind={kind} {prec} N={N} n={n} m={m} sizes={np.diff(S.off).tolist()}")
    T = 40
    ref = O.dhbm_run(S.A, S.B, S.off, T, preconditioned=bool(kind), keep_traj=True)
    g, e, _ = O.optimal_params(*O.spectrum(S.A, S.off))
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, prec, gamma=g, eta=e)
    h = apc.HeavyBall(plan, kind, alpha=ref["alpha"], beta=ref["beta"])
    got = hbm_traj(h, T)
    dev = rel_dev(got, ref["traj"][:, :, 0], S.xstar)
    say(f"alpha {ref['alpha']:.6g} beta {ref['beta']:.6g} max dev {dev:.3e} (tol {TOL[prec]})")
    assert dev <= TOL[prec]
    assert h.params()["iters"] == T


def test_hbm_start_is_the_plans_start():
    torch = _torch()
    apc = _apc()
    S = make_case(300, 200, 7, (20, 60), 1, 0.0)
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, "f64", gamma=1.0, eta=1.0)
    x0 = plan.xbar()
    plan.iterate(5)                      # the run starts from x_bar(0) whatever the plan did
    for kind in (0, 1):
        h = apc.HeavyBall(plan, kind, alpha=0.1, beta=0.2)
        d = float(torch.max(torch.abs(h.x() - x0)))
        assert d <= 1e-14 * float(torch.max(torch.abs(x0)))
        h.iterate(3)
        h.restart()
        assert float(torch.max(torch.abs(h.x() - x0))) <= 1e-14 * float(torch.max(torch.abs(x0)))
    assert plan.iterations == 5


def test_preconditioned_hbm_equals_apc_on_the_gpu():
    """Eliminating y from the (y, x_bar) form gives x_bar(t+1) = x_bar(t)
    - gamma eta (X x_bar(t) - x_bar(0)) + (gamma-1)(eta-1)(x_bar(t) - x_bar(t-1)):
    the preconditioned heavy ball with alpha = gamma eta / m, beta = (gamma-1)(eta-1).
    Two different kernel sequences on the GPU, one trajectory (FP64)."""
    apc = _apc()
    S = make_case(1000, 1000, 13, (40, 120), 2, 2.0)
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, "f64")
    p = plan.params()
    g, e, m = p["gamma"], p["eta"], len(S.off) - 1
    h = apc.HeavyBall(plan, 1, alpha=g * e / m, beta=(g - 1) * (e - 1))
    torch = _torch()
    T = 60
    a_tr = [plan.xbar()]
    for _ in range(T):
        plan.iterate(1)
        a_tr.append(plan.xbar())
    got = hbm_traj(h, T)
    ref = torch.stack(a_tr).cpu().numpy()
    dev = rel_dev(got, ref, S.xstar)
    say(f"APC vs preconditioned heavy ball on the GPU: {dev:.3e}")
    assert dev <= 1e-10


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_hbm_default_parameters_and_convergence(prec):
    """Default parameters: the plain kind estimates A^T A's spectrum by the same
    Lanczos procedure (contract: encloses the spectrum, at most 20 % wider at the
    bottom and 5e-3 at the top); the preconditioned kind takes m times the plan's
    enclosure of X's.  Both then converge to x*."""
    torch = _torch()
    apc = _apc()
    S = make_case(1500, 1200, 11, (40, 200), 21, 0.0)
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, prec)
    ev = np.linalg.eigvalsh(S.A.T @ S.A)
    xs = torch.from_numpy(S.xstar).cuda()
    for kind in (0, 1):
        h = apc.HeavyBall(plan, kind)
        q = h.params()
        say(f"case: hbm defaults {prec} kind={kind}", q)
        if kind == 0:
            lo_ok = ev[0] * (1 - 0.2) <= q["lam_min"] <= ev[0] * (1 + (1e-9 if prec == "f64" else 1e-4))
            hi_ok = ev[-1] * (1 - (1e-12 if prec == "f64" else 2e-6)) <= q["lam_max"] <= ev[-1] * (1 + 5e-3)
            assert lo_ok and hi_ok, (ev[0], ev[-1])
            assert q["lanczos_steps"] > 0
        else:
            pp = plan.params()
            m = len(S.off) - 1
            assert q["lam_min"] == pytest.approx(m * pp["mu_min"], rel=1e-14)
            assert q["lam_max"] == pytest.approx(m * pp["mu_max"], rel=1e-14)
            assert q["rho"] == pytest.approx(pp["rho"], rel=1e-12)
        T = int(math.ceil(math.log(1e-9) / math.log(q["rho"]))) + 40
        h.iterate(T)
        err = float(torch.linalg.norm(h.x() - xs) / torch.linalg.norm(xs))
        rr = h.residual()
        say(f"T={T} err {err:.3e} relres {rr:.3e}")
        assert err <= (1e-9 if prec == "f64" else 1e-5)
        assert rr <= (1e-9 if prec == "f64" else 1e-6)
        h.close()


def test_full_size_tall16k_preconditioned_hbm(tmp_path):
    """The benchmark shape (16384 x 8192, m = 64, FP32 plan, the benchmark's launch
    configuration): the preconditioned heavy ball with alpha = gamma eta / m,
    beta = (gamma-1)(eta-1) follows the oracle's stored APC curve (they are one
    sequence), whole vectors included, element by element."""
    torch = _torch()
    apc = _apc()
    g = np.load(os.path.join(GOLDEN, "tall_gauss_16384x8192_m64.npz"), allow_pickle=False)
    S = synth.tall_gaussian_16k()
    A, b = upload(S)
    xs = torch.from_numpy(S.xstar).cuda()
    off = S.off
    del S
    gam, eta = float(g["gamma"]), float(g["eta"])
    plan = apc.Plan(A, b, off, "f32", gamma=gam, eta=eta)
    h = apc.HeavyBall(plan, 1, alpha=gam * eta / 64, beta=(gam - 1) * (eta - 1))
    check = list(g["check_t"])
    xn, xmax = float(g["xstar_norm"]), float(g["xstar_max"])
    errs, full = [], {}
    for t in range(int(check[-1]) + 1):
        if t:
            h.iterate(1)
        x = h.x()
        errs.append(float(torch.linalg.norm(x - xs)) / xn)
        if t in check:
            full[t] = x.cpu().numpy()
    errs = np.array(errs)
    say("err hbm ", " ".join(f"{e:.3e}" for e in errs[[10, 20, 30, 40, 60]]))
    say("err orc ", " ".join(f"{e:.3e}" for e in g["err"][[10, 20, 30, 40, 60]]))
    assert np.max(np.abs(errs - g["err"])) <= TOL["f32"]
    for k, t in enumerate(check):
        d = full[t] - g["xbar"][k]
        assert float(np.linalg.norm(d)) / xn <= TOL["f32"], t
        assert float(np.max(np.abs(d))) / xmax <= TOL["f32"], t


def test_hbm_argument_errors():
    apc = _apc()
    S = make_case(300, 200, 7, (20, 60), 1, 0.0)
    A, b = upload(S)
    plan = apc.Plan(A, b, S.off, "f64", gamma=1.0, eta=1.0)
    assert apc.lib.apc_hbm_workspace_bytes(plan.handle, 7) == 0
    with pytest.raises(apc.ApcError) as ei:
        apc.HeavyBall(plan, 1, alpha=-1.0, beta=0.5)
    assert ei.value.status == apc.APC_EINVAL
    with pytest.raises(apc.ApcError) as ei:
        apc.HeavyBall(plan, 1, alpha=0.1, beta=1.0)
    assert ei.value.status == apc.APC_EINVAL
    nb = apc.lib.apc_hbm_workspace_bytes(plan.handle, 0)
    import ctypes
    torch = _torch()
    ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    wp = (ws.data_ptr() + 255) // 256 * 256
    h = ctypes.c_void_p()
    assert apc.lib.apc_hbm_create(ctypes.byref(h), plan.handle, 0, 0.1, 0.5, wp, nb - 1) == apc.APC_EINVAL
    assert apc.lib.apc_hbm_create(ctypes.byref(h), plan.handle, 0, 0.1, 0.5, wp + 8, nb) == apc.APC_EINVAL
    Bk = torch.from_numpy(np.ascontiguousarray(np.stack([S.B, S.B], 1))).cuda()
    plan2 = apc.Plan(A, Bk, S.off, "f64", gamma=1.0, eta=1.0)
    assert apc.lib.apc_hbm_workspace_bytes(plan2.handle, 1) == 0
    with pytest.raises(apc.ApcError) as ei:
        apc.HeavyBall(plan2, 1)
    assert ei.value.status == apc.APC_EUNSUPPORTED
