"""Thin Python binding of libapc (``include/apc.h``).

Argument marshalling only: every step of the solver runs in the HIP kernels of
``libapc.so``.  PyTorch supplies device memory and the stream; this module
passes raw pointers through ctypes.  Importing it fails loudly when the
library has not been built.

The functions ``apc_workspace_bytes``, ``apc_setup``, ``apc_iterate``, ... carry
the names and argument order of the C ABI.  ``Plan`` wraps them for torch
tensors.
"""

from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapc.so")

APC_F64, APC_F32, APC_BF16_IR = 0, 1, 2
APC_REDUCED_FORM = 16
PRECISIONS = {"f64": APC_F64, "f32": APC_F32, "bf16_ir": APC_BF16_IR}

STATUS_NAMES = {
    0: "APC_OK", 1: "APC_EINVAL", 2: "APC_ERANK", 3: "APC_ESINGULAR", 4: "APC_EDIVERGED",
    5: "APC_ENOCONV", 6: "APC_ENODEV", 7: "APC_EHIP", 8: "APC_EUNSUPPORTED",
}
APC_OK, APC_EINVAL, APC_ERANK, APC_ESINGULAR, APC_EDIVERGED, APC_ENOCONV, APC_ENODEV, \
    APC_EHIP, APC_EUNSUPPORTED = range(9)

EXPORTED = (
    "apc_workspace_bytes", "apc_setup", "apc_iterate", "apc_iterate_graph", "apc_iterate_timed",
    "apc_residual",
    "apc_solve", "apc_get_xbar", "apc_get_local", "apc_project", "apc_get_params",
    "apc_iterations", "apc_destroy", "apc_last_error", "apc_optimal_params",
    "apc_tridiag_extremes", "apc_get_info", "apc_get_setup", "apc_get_launch", "apc_set_anchor",
    "apc_set_params",
    "apc_restart", "apc_backward_workspace_bytes", "apc_backward", "apc_backward_noalloc",
    "apc_batch_workspace_bytes", "apc_batch_create", "apc_batch_iterate",
    "apc_batch_iterate_graph", "apc_batch_residuals", "apc_batch_activate", "apc_batch_solve",
    "apc_batch_get_launch", "apc_batch_destroy",
    "apc_hbm_workspace_bytes", "apc_hbm_create", "apc_hbm_iterate", "apc_hbm_restart",
    "apc_hbm_get_x", "apc_hbm_residual", "apc_hbm_get_params", "apc_hbm_destroy",
)
APC_HBM_PLAIN, APC_HBM_PRECONDITIONED = 0, 1


class ApcError(RuntimeError):
    """A non-OK status from libapc."""

    def __init__(self, status: int, message: str):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


def _hip_runtimes() -> set:
    """Distinct libamdhip64 files mapped into this process."""
    try:
        with open("/proc/self/maps") as f:
            return {line.split()[-1] for line in f if "libamdhip64" in line}
    except OSError:
        return set()


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "python paper_1708_01413_amd/build.py (hipcc --offload-arch=gfx950); "
                          "there is no fallback path")
    # torch ships its own HIP runtime with the same soname as the system one.
    # Load it first so libapc binds to it: two HIP runtimes in one process
    # cannot share the device (HIP then reports no device to one of them).
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    if len(_hip_runtimes()) > 1:
        raise ImportError(f"two HIP runtimes are loaded: {sorted(_hip_runtimes())}")
    vp, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    P64 = ctypes.POINTER(ctypes.c_int64)
    Pd = ctypes.POINTER(ctypes.c_double)
    Pf = ctypes.POINTER(ctypes.c_float)
    Pi = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "apc_workspace_bytes": (ctypes.c_size_t, [i64, i64, P64, i32, i32, i32]),
        "apc_setup": (i32, [ctypes.POINTER(vp), vp, i64, vp, i64, i64, i64, P64, i32, i32, i32,
                            f64, f64, vp, ctypes.c_size_t, vp]),
        "apc_iterate": (i32, [vp, i32]),
        "apc_iterate_graph": (i32, [vp, i32]),
        "apc_iterate_timed": (i32, [vp, i32, Pf, Pf, Pf, Pf]),
        "apc_residual": (i32, [vp, Pd]),
        "apc_solve": (i32, [vp, f64, i32, vp, i64, Pi, Pd]),
        "apc_get_xbar": (i32, [vp, vp, i64]),
        "apc_get_local": (i32, [vp, vp, i64]),
        "apc_project": (i32, [vp, vp, vp, i64]),
        "apc_get_params": (i32, [vp, Pd, Pd, Pd, Pd, Pd]),
        "apc_iterations": (i64, [vp]),
        "apc_get_info": (i32, [vp, Pi, Pi, Pi, Pi, Pi]),
        "apc_get_setup": (i32, [vp, Pi, Pd]),
        "apc_get_launch": (i32, [vp, i32, Pi, Pi, Pf]),
        "apc_set_anchor": (i32, [vp, i32]),
        "apc_set_params": (i32, [vp, f64, f64]),
        "apc_restart": (i32, [vp, vp, i64]),
        "apc_backward_workspace_bytes": (ctypes.c_size_t, [vp, i32, i32]),
        "apc_backward": (i32, [vp, vp, i64, i32, i32, vp, i64, Pd, Pd, vp, ctypes.c_size_t]),
        "apc_backward_noalloc": (i32, [vp, vp, i64, i32, i32, vp, i64, Pd, Pd]),
        "apc_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(vp), i32]),
        "apc_batch_create": (i32, [ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp, ctypes.c_size_t]),
        "apc_batch_iterate": (i32, [vp, i32]),
        "apc_batch_iterate_graph": (i32, [vp, i32]),
        "apc_batch_residuals": (i32, [vp, f64, Pd, Pi]),
        "apc_batch_activate": (i32, [vp]),
        "apc_batch_solve": (i32, [vp, f64, i32, i32, i32, Pi, Pd]),
        "apc_batch_get_launch": (i32, [vp, Pi, Pi, Pi, Pi, Pf]),
        "apc_batch_destroy": (None, [vp]),
        "apc_hbm_workspace_bytes": (ctypes.c_size_t, [vp, i32]),
        "apc_hbm_create": (i32, [ctypes.POINTER(vp), vp, i32, f64, f64, vp, ctypes.c_size_t]),
        "apc_hbm_iterate": (i32, [vp, i32]),
        "apc_hbm_restart": (i32, [vp]),
        "apc_hbm_get_x": (i32, [vp, vp, i64]),
        "apc_hbm_residual": (i32, [vp, Pd]),
        "apc_hbm_get_params": (i32, [vp, Pd, Pd, Pd, Pd, Pd, Pi, P64]),
        "apc_hbm_destroy": (None, [vp]),
        "apc_optimal_params": (i32, [f64, f64, Pd, Pd, Pd]),
        "apc_tridiag_extremes": (i32, [Pd, Pd, i32, i32, Pd, Pd, Pd, Pd]),
        "apc_destroy": (None, [vp]),
        "apc_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(status: int):
    if status != APC_OK:
        raise ApcError(status, lib.apc_last_error().decode(errors="replace"))


def _off_array(off) -> ctypes.Array:
    off = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    return (ctypes.c_int64 * len(off))(*off.tolist())


# ---------------------------------------------------------------- C-named calls


def apc_workspace_bytes(N: int, n: int, off, m: int, k: int = 1, precision: int = APC_F64) -> int:
    return int(lib.apc_workspace_bytes(N, n, _off_array(off), m, k, precision))


def apc_setup(A: int, lda: int, B: int, ldb: int, N: int, n: int, off, m: int, k: int,
              precision: int, gamma: float, eta: float, workspace: int, ws_bytes: int,
              stream: int) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib.apc_setup(ctypes.byref(h), A, lda, B, ldb, N, n, _off_array(off), m, k,
                         precision, gamma, eta, workspace, ws_bytes, stream))
    return h


def apc_iterate(plan, T: int):
    _check(lib.apc_iterate(plan, T))


def apc_iterate_graph(plan, T: int):
    _check(lib.apc_iterate_graph(plan, T))


def apc_iterate_timed(plan, T: int):
    """Returns (ms_total, ms_pass_a, ms_pass_b, ms_average)."""
    v = [ctypes.c_float() for _ in range(4)]
    _check(lib.apc_iterate_timed(plan, T, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def apc_residual(plan) -> float:
    r = ctypes.c_double()
    _check(lib.apc_residual(plan, ctypes.byref(r)))
    return r.value


def apc_solve(plan, rtol: float, max_iters: int, Xbar: int, ldx: int = 1):
    it, rr = ctypes.c_int32(), ctypes.c_double()
    st = lib.apc_solve(plan, rtol, max_iters, Xbar, ldx, ctypes.byref(it), ctypes.byref(rr))
    return st, it.value, rr.value


def apc_get_xbar(plan, Xbar: int, ldx: int = 1):
    _check(lib.apc_get_xbar(plan, Xbar, ldx))


def apc_get_local(plan, X: int, ldx: int):
    _check(lib.apc_get_local(plan, X, ldx))


def apc_project(plan, V: int, Out: int, ldv: int):
    _check(lib.apc_project(plan, V, Out, ldv))


def apc_get_params(plan) -> dict:
    vals = [ctypes.c_double() for _ in range(5)]
    _check(lib.apc_get_params(plan, *[ctypes.byref(v) for v in vals]))
    return dict(zip(("gamma", "eta", "mu_min", "mu_max", "rho"), (v.value for v in vals)))


def apc_get_info(plan) -> dict:
    vals = [ctypes.c_int32() for _ in range(5)]
    _check(lib.apc_get_info(plan, *[ctypes.byref(v) for v in vals]))
    return dict(zip(("lanczos_steps", "rows_per_tile", "column_splits", "block_groups",
                     "refinements"), (v.value for v in vals)))


def apc_get_setup(plan) -> dict:
    passes, defect = ctypes.c_int32(), ctypes.c_double()
    _check(lib.apc_get_setup(plan, ctypes.byref(passes), ctypes.byref(defect)))
    return {"qr_passes": passes.value, "qr_defect": defect.value}


def apc_get_launch(plan, which: int) -> dict:
    rows, splits, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
    _check(lib.apc_get_launch(plan, which, ctypes.byref(rows), ctypes.byref(splits),
                              ctypes.byref(us)))
    return {"rows_per_wg": rows.value, "splits": splits.value, "tuned_us": us.value}


def apc_set_anchor(plan, every: int):
    _check(lib.apc_set_anchor(plan, every))


def apc_set_params(plan, gamma: float, eta: float):
    _check(lib.apc_set_params(plan, gamma, eta))


def apc_restart(plan, B: int, ldb: int):
    _check(lib.apc_restart(plan, B, ldb))


def apc_backward_workspace_bytes(plan, T: int, ckpt_every: int) -> int:
    return int(lib.apc_backward_workspace_bytes(plan, T, ckpt_every))


def apc_backward(plan, dXbar: int, ldd: int, T: int, ckpt_every: int, dB: int, lddb: int,
                 ws: int, ws_bytes: int):
    dg, de = ctypes.c_double(), ctypes.c_double()
    _check(lib.apc_backward(plan, dXbar, ldd, T, ckpt_every, dB, lddb, ctypes.byref(dg),
                            ctypes.byref(de), ws, ws_bytes))
    return dg.value, de.value


def apc_backward_noalloc(plan, dXbar: int, ldd: int, T: int, ckpt_every: int, dB: int,
                         lddb: int):
    dg, de = ctypes.c_double(), ctypes.c_double()
    _check(lib.apc_backward_noalloc(plan, dXbar, ldd, T, ckpt_every, dB, lddb, ctypes.byref(dg),
                                    ctypes.byref(de)))
    return dg.value, de.value


def apc_iterations(plan) -> int:
    return int(lib.apc_iterations(plan))


def apc_optimal_params(mu_min: float, mu_max: float):
    g, e, r = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib.apc_optimal_params(mu_min, mu_max, ctypes.byref(g), ctypes.byref(e), ctypes.byref(r)))
    return g.value, e.value, r.value


def apc_tridiag_extremes(alpha, beta, with_bounds: bool = False):
    a = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64))
    b = np.ascontiguousarray(np.asarray(beta, dtype=np.float64))
    k = len(a)
    if len(b) < (k if with_bounds else k - 1):
        raise ValueError("beta too short")
    if len(b) == 0:
        b = np.zeros(1)
    Pd = ctypes.POINTER(ctypes.c_double)
    out = [ctypes.c_double() for _ in range(4)]
    _check(lib.apc_tridiag_extremes(a.ctypes.data_as(Pd), b.ctypes.data_as(Pd), k,
                                    1 if with_bounds else 0, *[ctypes.byref(v) for v in out]))
    return tuple(v.value for v in out)


def apc_destroy(plan):
    lib.apc_destroy(plan)


def apc_last_error() -> str:
    return lib.apc_last_error().decode(errors="replace")


# ---------------------------------------------------------------- torch wrapper


class Plan:
    """An APC solver instance on one GPU.

    A: (N, n) float64 CUDA tensor (row stride may exceed n); b: (N,) or (N, k)
    float64 CUDA tensor (row-major); off: m+1 block offsets.  gamma/eta None
    selects Theorem 1's optimum.  The plan keeps references to A, b and its
    workspace.  anchor_every (FP32 / bf16 plans with k > 1 or bf16): FP64
    anchor spacing, see apc_set_anchor (None keeps the library default).
    reduced_form: run k = 1 in the (y, x_bar) form too (needed for backward()).
    """

    def __init__(self, A, b, off, precision: str = "f64", gamma=None, eta=None, stream=None,
                 workspace=None, anchor_every=None, reduced_form=False):
        import torch

        if A.dtype != torch.float64 or b.dtype != torch.float64:
            raise TypeError("A and b must be float64")
        if not (A.is_cuda and b.is_cuda):
            raise TypeError("A and b must be device tensors")
        if A.dim() != 2 or A.stride(1) != 1:
            raise ValueError("A must be a row-major matrix")
        if b.dim() not in (1, 2) or (b.dim() == 2 and b.stride(1) != 1):
            raise ValueError("b must be a vector or a row-major (N, k) matrix")
        self._torch = torch
        self.device = A.device
        self.N, self.n = A.shape
        self.off = np.asarray(off, dtype=np.int64)
        self.m = len(self.off) - 1
        self.k = 1 if b.dim() == 1 else b.shape[1]
        self.precision = PRECISIONS[precision] | (APC_REDUCED_FORM if reduced_form else 0)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ws = apc_workspace_bytes(self.N, self.n, self.off, self.m, self.k, self.precision)
        if ws == 0:
            raise ApcError(APC_EINVAL, apc_last_error())
        self.ws_bytes = ws
        if workspace is None:
            workspace = torch.empty(ws + 256, dtype=torch.uint8, device=self.device)
        elif workspace.numel() < ws + 256 or workspace.dtype != torch.uint8:
            raise ValueError(f"workspace needs {ws + 256} bytes (uint8)")
        self.workspace = workspace
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.A, self.b = A, b
        self._streams_in()
        g = math.nan if gamma is None else float(gamma)
        e = math.nan if eta is None else float(eta)
        self.handle = apc_setup(A.data_ptr(), A.stride(0), b.data_ptr(), b.stride(0), self.N,
                                self.n, self.off, self.m, self.k, self.precision, g, e,
                                self._ws_ptr, ws, self.stream.cuda_stream)
        if anchor_every is not None:
            apc_set_anchor(self.handle, int(anchor_every))

    # -- stream order between torch and the library
    def _streams_in(self):
        """Make the plan's stream wait for what is queued on the caller's current stream:
        the tensors a call reads, and memory the caching allocator just handed out (it
        orders reuse on the current stream only)."""
        cur = self._torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def _streams_out(self):
        """Make the caller's current stream wait for the plan's stream, so that torch work
        on the tensors a call wrote (and later reuse of their memory) comes after it."""
        cur = self._torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.wait_stream(self.stream)

    # -- iteration
    def iterate(self, T: int, graph: bool = False):
        """T updates; graph=True replays a captured HIP graph of them (needs a plan on a
        non-default stream)."""
        (apc_iterate_graph if graph else apc_iterate)(self.handle, T)

    def iterate_timed(self, T: int):
        """(ms_total, ms_pass_a, ms_pass_b, ms_average) of T updates, timed with HIP events."""
        return apc_iterate_timed(self.handle, T)

    @staticmethod
    def workspace_bytes(N, n, off, precision="f64", k=1) -> int:
        """Bytes to pass as a preallocated ``workspace`` (uint8) tensor."""
        off = np.asarray(off, dtype=np.int64)
        return apc_workspace_bytes(N, n, off, len(off) - 1, k, PRECISIONS[precision]) + 256

    def residual(self) -> float:
        return apc_residual(self.handle)

    def _xshape(self):
        return (self.n,) if self.k == 1 else (self.n, self.k)

    def solve(self, rtol: float, max_iters: int):
        x = self._torch.empty(self._xshape(), dtype=self._torch.float64, device=self.device)
        self._streams_in()
        st, it, rr = apc_solve(self.handle, rtol, max_iters, x.data_ptr(), 1 if self.k == 1 else self.k)
        self._streams_out()
        if st not in (APC_OK, APC_ENOCONV):
            _check(st)
        return x, it, rr, st

    def set_params(self, gamma: float, eta: float):
        apc_set_params(self.handle, float(gamma), float(eta))

    def restart(self, b=None):
        """Start Alg. 1 again, optionally from new right-hand sides b (same shape)."""
        if b is None:
            apc_restart(self.handle, None, 1)
            return
        if b.dtype != self._torch.float64 or not b.is_cuda or b.shape != self.b.shape:
            raise ValueError("b must be a float64 CUDA tensor shaped like the plan's b")
        b = b.contiguous()
        self.b = b
        self._streams_in()
        apc_restart(self.handle, b.data_ptr(), 1 if self.k == 1 else self.k)

    def backward(self, dxbar, T: int, ckpt_every: int | None = None):
        """(dL/db, dL/dgamma, dL/deta) for dL/dx_bar(T) = dxbar over T updates from the start."""
        torch = self._torch
        if ckpt_every is None:
            ckpt_every = max(1, int(math.isqrt(max(T, 1))))
        dxbar = dxbar.to(device=self.device, dtype=torch.float64).contiguous()
        if dxbar.shape != tuple(self._xshape()):
            raise ValueError(f"dxbar must have shape {tuple(self._xshape())}")
        nb = apc_backward_workspace_bytes(self.handle, T, ckpt_every)
        if nb == 0:
            raise ApcError(APC_EUNSUPPORTED, "backward needs the (y, x_bar) form: k > 1 or "
                           "reduced_form=True, precision f64 or f32")
        ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        wp = (ws.data_ptr() + 255) // 256 * 256
        dB = torch.empty(self.b.shape, dtype=torch.float64, device=self.device)
        ld = 1 if self.k == 1 else self.k
        self._streams_in()
        dg, de = apc_backward(self.handle, dxbar.data_ptr(), ld, T, ckpt_every, dB.data_ptr(), ld,
                              wp, nb)
        self._streams_out()
        return dB, dg, de

    # -- state access
    def xbar(self):
        x = self._torch.empty(self._xshape(), dtype=self._torch.float64, device=self.device)
        self._streams_in()
        apc_get_xbar(self.handle, x.data_ptr(), 1 if self.k == 1 else self.k)
        self._streams_out()
        return x

    def local(self):
        shape = (self.m, self.n) if self.k == 1 else (self.m, self.n, self.k)
        X = self._torch.empty(shape, dtype=self._torch.float64, device=self.device)
        self._streams_in()
        apc_get_local(self.handle, X.data_ptr(), self.n if self.k == 1 else self.k)
        self._streams_out()
        return X

    def project(self, V):
        if V.shape != (self.m, self.n) or V.dtype != self._torch.float64 or not V.is_contiguous():
            raise ValueError("V must be a contiguous (m, n) float64 tensor")
        out = self._torch.empty_like(V)
        self._streams_in()
        apc_project(self.handle, V.data_ptr(), out.data_ptr(), self.n)
        self._streams_out()
        return out

    def params(self) -> dict:
        return apc_get_params(self.handle)

    def info(self) -> dict:
        return apc_get_info(self.handle)

    def launch_shapes(self) -> dict:
        """Launch shapes of the k-RHS contractions (pass A, pass B, start, residual)."""
        return {name: apc_get_launch(self.handle, w)
                for w, name in enumerate(("pass_a", "pass_b", "start", "residual"))}

    def setup_info(self) -> dict:
        """CholeskyQR passes setup took and the measured orthogonality defect after the
        first (NaN when not measured)."""
        return apc_get_setup(self.handle)

    def single_pass_shape(self):
        """Rows per workgroup and rows per register group of the single-pass k = 1
        update, or None when the plan updates in two passes over C."""
        rows, g, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
        st = lib.apc_get_launch(self.handle, 4, ctypes.byref(rows), ctypes.byref(g),
                                ctypes.byref(us))
        if st == APC_EUNSUPPORTED:
            return None
        _check(st)
        return {"rows_per_wg": rows.value, "rows_per_group": g.value}

    def resident_shape(self):
        """Block rows and columns one workgroup holds in the single-launch k = 1 update
        (T updates in one launch), or None when the plan launches per update."""
        rows, cols, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
        st = lib.apc_get_launch(self.handle, 5, ctypes.byref(rows), ctypes.byref(cols),
                                ctypes.byref(us))
        if st == APC_EUNSUPPORTED:
            return None
        _check(st)
        return {"rows_per_wg": rows.value, "cols_per_wg": cols.value}

    @property
    def iterations(self) -> int:
        return apc_iterations(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.stream.synchronize()
            apc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class UnrolledAPC:
    """torch.autograd.Function wrapper: x_bar(T) = APC_T(b; gamma, eta) on a plan's
    factorisation, differentiable in b, gamma and eta (adjoint with checkpoints)."""

    _fn = None

    @classmethod
    def function(cls):
        if cls._fn is None:
            import torch

            class _F(torch.autograd.Function):
                @staticmethod
                def forward(ctx, b, gamma, eta, plan, T, ckpt_every):
                    plan.set_params(float(gamma), float(eta))
                    plan.restart(b.detach())
                    plan.iterate(T)
                    ctx.plan, ctx.T, ctx.ckpt = plan, T, ckpt_every
                    ctx.params = (float(gamma), float(eta))
                    ctx.b = b.detach().clone()
                    return plan.xbar()

                @staticmethod
                def backward(ctx, gx):
                    # The adjoint re-runs the forward from the plan's last restart;
                    # another forward on the same plan may have restarted it since.
                    plan = ctx.plan
                    plan.set_params(*ctx.params)
                    plan.restart(ctx.b)
                    dB, dg, de = plan.backward(gx, ctx.T, ctx.ckpt)
                    return (dB, torch.tensor(dg, dtype=torch.float64),
                            torch.tensor(de, dtype=torch.float64), None, None, None)

            cls._fn = _F
        return cls._fn


def unrolled_apc(plan, b, gamma, eta, T: int, ckpt_every: int | None = None):
    """x_bar(T) of Alg. 1 with right-hand sides b and parameters (gamma, eta) as tensors;
    gradients flow to every argument that requires them."""
    import torch
    g = gamma if torch.is_tensor(gamma) else torch.tensor(float(gamma), dtype=torch.float64)
    e = eta if torch.is_tensor(eta) else torch.tensor(float(eta), dtype=torch.float64)
    ck = ckpt_every if ckpt_every is not None else max(1, int(math.isqrt(max(T, 1))))
    return UnrolledAPC.function().apply(b, g, e, plan, T, ck)


class Batch:
    """Many independent k = 1 FP32 plans iterated together: one persistent launch per
    pass over a work list covering every system (apc_batch_*).  The plans must share
    one stream and outlive the batch."""

    def __init__(self, plans):
        import torch
        self._torch = torch
        self.plans = list(plans)
        self.count = len(self.plans)
        arr = (ctypes.c_void_p * self.count)(*[p.handle for p in self.plans])
        self._arr = arr
        nb = int(lib.apc_batch_workspace_bytes(arr, self.count))
        if nb == 0:
            raise ApcError(APC_EUNSUPPORTED, lib.apc_last_error().decode(errors="replace"))
        dev = self.plans[0].device
        self.workspace = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        wp = (self.workspace.data_ptr() + 255) // 256 * 256
        self.plans[0]._streams_in()
        h = ctypes.c_void_p()
        _check(lib.apc_batch_create(ctypes.byref(h), arr, self.count, wp, nb))
        self.handle = h.value

    def iterate(self, T: int, graph: bool = False):
        _check((lib.apc_batch_iterate_graph if graph else lib.apc_batch_iterate)(self.handle, T))

    def residuals(self, rtol: float = -1.0):
        rr = (ctypes.c_double * self.count)()
        act = (ctypes.c_int32 * self.count)()
        _check(lib.apc_batch_residuals(self.handle, rtol, rr, act))
        return np.array(rr[:]), np.array(act[:])

    def activate(self):
        _check(lib.apc_batch_activate(self.handle))

    def solve(self, rtol: float, max_iters: int, check_every: int = 8, graph: bool = True):
        it = (ctypes.c_int32 * self.count)()
        rr = (ctypes.c_double * self.count)()
        st = lib.apc_batch_solve(self.handle, rtol, max_iters, check_every, 1 if graph else 0, it, rr)
        if st not in (APC_OK, APC_ENOCONV):
            _check(st)
        return np.array(it[:]), np.array(rr[:]), st

    def launch(self) -> dict:
        g, a, b, v, us = (ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(),
                          ctypes.c_float())
        _check(lib.apc_batch_get_launch(self.handle, ctypes.byref(g), ctypes.byref(a),
                                        ctypes.byref(b), ctypes.byref(v), ctypes.byref(us)))
        return {"grid": g.value, "items_a": a.value, "items_b": b.value, "items_avg": v.value,
                "tuned_us": us.value}

    def close(self):
        if getattr(self, "handle", None) is not None:
            lib.apc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HeavyBall:
    """The distributed heavy-ball method (Sec. 4.3) on a plan's row blocks, plain
    (kind APC_HBM_PLAIN) or on Sec. 6's preconditioned blocks
    (APC_HBM_PRECONDITIONED), through apc_hbm_*.  alpha/beta None: the
    heavy-ball optimum from the estimated spectrum.  The plan must outlive it."""

    def __init__(self, plan, kind: int = APC_HBM_PRECONDITIONED, alpha=None, beta=None):
        import torch
        self._torch = torch
        self.plan = plan
        nb = int(lib.apc_hbm_workspace_bytes(plan.handle, kind))
        if nb == 0:
            raise ApcError(APC_EUNSUPPORTED, lib.apc_last_error().decode(errors="replace"))
        self.workspace = torch.empty(nb + 256, dtype=torch.uint8, device=plan.device)
        wp = (self.workspace.data_ptr() + 255) // 256 * 256
        plan._streams_in()
        nan = float("nan")
        h = ctypes.c_void_p()
        _check(lib.apc_hbm_create(ctypes.byref(h), plan.handle, kind,
                                  nan if alpha is None else float(alpha),
                                  nan if beta is None else float(beta), wp, nb))
        self.handle = h.value

    def iterate(self, T: int):
        _check(lib.apc_hbm_iterate(self.handle, T))

    def restart(self):
        _check(lib.apc_hbm_restart(self.handle))

    def x(self):
        out = self._torch.empty(self.plan.n, dtype=self._torch.float64, device=self.plan.device)
        self.plan._streams_in()
        _check(lib.apc_hbm_get_x(self.handle, out.data_ptr(), 1))
        self.plan._streams_out()
        return out

    def residual(self) -> float:
        r = ctypes.c_double()
        _check(lib.apc_hbm_residual(self.handle, ctypes.byref(r)))
        return r.value

    def params(self) -> dict:
        v = [ctypes.c_double() for _ in range(5)]
        steps, iters = ctypes.c_int32(), ctypes.c_int64()
        _check(lib.apc_hbm_get_params(self.handle, *[ctypes.byref(q) for q in v],
                                      ctypes.byref(steps), ctypes.byref(iters)))
        return {"alpha": v[0].value, "beta": v[1].value, "lam_min": v[2].value,
                "lam_max": v[3].value, "rho": v[4].value, "lanczos_steps": steps.value,
                "iters": iters.value}

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.plan.stream.synchronize()
            lib.apc_hbm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
