"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, rejects invalid arguments on the host before any HIP call,
and its host-only helpers agree with the oracle."""

import math
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import apc_oracle as O
from paper_1708_01413_amd import apc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(apc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("apc_workspace_bytes", "apc_setup", "apc_iterate", "apc_solve",
                     "apc_get_xbar", "apc_get_params", "apc_destroy", "apc_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", apc.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (apc_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    assert set(apc.EXPORTED) == set(declared_functions())


def test_library_is_built_for_gfx950():
    """The offload bundle of our own build names the gfx950 target."""
    sections = subprocess.run(["readelf", "-S", apc.LIB_PATH], capture_output=True, text=True,
                              check=True).stdout
    assert ".hip_fatbin" in sections
    blob = open(apc.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def _setup_status(N=64, n=64, off=None, m=4, k=1, prec=0, lda=None, ldb=1, A=0x1000, B=0x1000,
                  ws=0x100000, ws_bytes=1 << 40, gamma=math.nan, eta=math.nan):
    import ctypes
    if off is None:
        off = [i * (N // m) for i in range(m)] + [N]
    h = ctypes.c_void_p(123)
    st = apc.lib.apc_setup(ctypes.byref(h), A, n if lda is None else lda, B, ldb, N, n,
                           apc._off_array(off), m, k, prec, gamma, eta, ws, ws_bytes, None)
    return st, h.value


@pytest.mark.parametrize("kwargs,status", [
    (dict(N=32, n=64), apc.APC_EINVAL),                                  # N < n
    (dict(off=[0, 10, 5, 40, 64]), apc.APC_EINVAL),                      # decreasing offsets
    (dict(off=[0, 16, 32, 48, 63]), apc.APC_EINVAL),                     # off[m] != N
    (dict(off=[1, 16, 32, 48, 64]), apc.APC_EINVAL),                     # off[0] != 0
    (dict(N=128, n=32, m=2, off=[0, 40, 128]), apc.APC_EINVAL),         # p_i > n
    (dict(m=0, off=[0]), apc.APC_EINVAL),
    (dict(k=0), apc.APC_EINVAL),
    (dict(k=2000), apc.APC_EINVAL),
    (dict(prec=7), apc.APC_EINVAL),
    (dict(lda=10), apc.APC_EINVAL),
    (dict(ldb=0), apc.APC_EINVAL),
    (dict(A=0), apc.APC_EINVAL),
    (dict(ws=0), apc.APC_EINVAL),
    (dict(ws=0x100010), apc.APC_EINVAL),                                 # misaligned workspace
    (dict(ws_bytes=16), apc.APC_EINVAL),                                 # workspace too small
    (dict(gamma=math.inf, eta=1.0), apc.APC_EINVAL),
])
def test_setup_rejects_bad_arguments_before_any_hip_call(kwargs, status):
    st, h = _setup_status(**kwargs)
    assert st == status, apc.apc_last_error()
    assert h is None
    assert apc.apc_last_error()


def test_workspace_bytes():
    off = list(range(0, 16385, 256))
    ws64 = apc.apc_workspace_bytes(16384, 8192, off, 64, 1, apc.APC_F64)
    ws32 = apc.apc_workspace_bytes(16384, 8192, off, 64, 1, apc.APC_F32)
    assert ws64 >= 2 * 16384 * 8192 * 8
    # The FP32 plan adds its FP32 factor; the single-pass partials (one row of ldc per
    # 16-row tile) take 8 bytes per entry in FP64 and 4 in FP32.
    partial_rows = 16384 // 16
    assert ws32 - ws64 >= 16384 * 8192 * 4 - 256 - partial_rows * 8192 * 4
    assert apc.apc_workspace_bytes(10, 20, [0, 10], 1, 1, 0) == 0      # N < n
    assert apc.apc_workspace_bytes(5000, 4000, [0, 2500, 5000], 2, 1, 0) == 0  # p_i > 2048


def test_null_plan_is_rejected():
    assert apc.lib.apc_iterate(None, 1) == apc.APC_EINVAL
    assert apc.lib.apc_iterations(None) == -1
    apc.lib.apc_destroy(None)


def test_setup_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, h = _setup_status(ws_bytes=1 << 40)
    assert st == apc.APC_ENODEV and h is None
    assert "device" in apc.apc_last_error()


@pytest.mark.parametrize("seed", range(25))
def test_optimal_params_match_oracle(seed):
    rng = np.random.default_rng(seed)
    lo, hi = np.sort(rng.uniform(1e-9, 1.0, 2))
    if seed == 0:
        lo, hi = 1.0, 1.0
    g, e, r = apc.apc_optimal_params(lo, hi)
    og, oe, orr = O.optimal_params(lo, hi)
    assert g == pytest.approx(og, rel=1e-12, abs=1e-12)
    assert e == pytest.approx(oe, rel=1e-12)
    assert r == pytest.approx(orr, rel=1e-12, abs=1e-15)


def test_optimal_params_rejects_bad_interval():
    with pytest.raises(apc.ApcError):
        apc.apc_optimal_params(0.0, 0.5)
    with pytest.raises(apc.ApcError):
        apc.apc_optimal_params(0.6, 0.5)


@pytest.mark.parametrize("k", [1, 2, 3, 17, 200])
def test_tridiag_extremes_match_eigvalsh(k):
    rng = np.random.default_rng(k)
    a = rng.uniform(0, 1, k)
    b = rng.uniform(0.01, 0.5, k)
    lo, hi, blo, bhi = apc.apc_tridiag_extremes(a, b, with_bounds=True)
    T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    w, v = np.linalg.eigh(T)
    assert lo == pytest.approx(w[0], abs=1e-14)
    assert hi == pytest.approx(w[-1], abs=1e-14)
    # Lanczos residual bounds |beta_k * s_k| for the extreme Ritz pairs
    assert blo == pytest.approx(abs(b[-1] * v[-1, 0]), rel=1e-6, abs=1e-14)
    assert bhi == pytest.approx(abs(b[-1] * v[-1, -1]), rel=1e-6, abs=1e-14)


def test_tridiag_bounds_enclose_true_extremes():
    """Lanczos on a dense symmetric matrix with known spectrum (host NumPy), then the
    library's bounds: [theta_lo - bound_lo, theta_hi + bound_hi] holds the extremes."""
    rng = np.random.default_rng(3)
    n = 60
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    mu = np.sort(rng.uniform(0.01, 0.9, n))
    X = Qm @ np.diag(mu) @ Qm.T
    V = [rng.standard_normal(n)]
    V[0] /= np.linalg.norm(V[0])
    al, be = [], []
    for j in range(20):
        y = X @ V[j]
        for _ in range(2):
            y = y - np.stack(V).T @ (np.stack(V) @ y)
        al.append(V[j] @ X @ V[j])
        be.append(np.linalg.norm(y))
        V.append(y / be[-1])
    lo, hi, blo, bhi = apc.apc_tridiag_extremes(al, be, with_bounds=True)
    assert lo - blo <= mu[0] + 1e-12 and hi + bhi >= mu[-1] - 1e-12
    assert lo >= mu[0] - 1e-12 and hi <= mu[-1] + 1e-12


def test_one_hip_runtime_in_process():
    """torch bundles a HIP runtime with the system runtime's soname; the binding loads
    torch first so libapc binds to the same one."""
    runtimes = apc._hip_runtimes()
    assert len(runtimes) == 1, runtimes


def test_hbm_null_arguments_are_rejected():
    assert apc.lib.apc_hbm_workspace_bytes(None, 0) == 0
    assert apc.lib.apc_hbm_iterate(None, 1) == apc.APC_EINVAL
    assert apc.lib.apc_hbm_restart(None) == apc.APC_EINVAL
    assert apc.lib.apc_hbm_residual(None, None) == apc.APC_EINVAL
    assert apc.lib.apc_hbm_get_params(None, None, None, None, None, None, None, None) == apc.APC_EINVAL
    import ctypes
    h = ctypes.c_void_p()
    assert apc.lib.apc_hbm_create(ctypes.byref(h), None, 0, 0.1, 0.5, None, 0) == apc.APC_EINVAL
    assert h.value is None
    apc.lib.apc_hbm_destroy(None)
