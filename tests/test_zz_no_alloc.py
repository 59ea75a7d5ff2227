"""apc_backward_noalloc (the adjoint with the library's fixed device scratch instead of
a caller workspace) against apc_backward on the same plans: two calls in a row, the
second on a smaller problem, each equal to the workspace variant within the FP64 bar
(1e-10 relative; the two run the same kernels on the same data, so they agree
bitwise in practice); an oversized request is rejected on the host."""

import math
import sys

import numpy as np
import pytest

from paper_1708_01413_amd import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _both(plan, dx, T, ckpt):
    """(dB, dgamma, deta) from apc_backward with a caller workspace, then from
    apc_backward_noalloc, both through the C ABI."""
    from paper_1708_01413_amd import apc
    torch = _torch()
    ld = 1 if plan.k == 1 else plan.k
    nb = apc.apc_backward_workspace_bytes(plan.handle, T, ckpt)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=plan.device)
    wp = (ws.data_ptr() + 255) // 256 * 256
    dB_ws = torch.full(plan.b.shape, float("nan"), dtype=torch.float64, device=plan.device)
    g_ws, e_ws = apc.apc_backward(plan.handle, dx.data_ptr(), ld, T, ckpt, dB_ws.data_ptr(), ld,
                                  wp, nb)
    dB_na = torch.full(plan.b.shape, float("nan"), dtype=torch.float64, device=plan.device)
    g_na, e_na = apc.apc_backward_noalloc(plan.handle, dx.data_ptr(), ld, T, ckpt,
                                          dB_na.data_ptr(), ld)
    torch.cuda.synchronize()
    return (dB_ws, g_ws, e_ws), (dB_na, g_na, e_na), nb


def _check(ref, got, label):
    torch = _torch()
    dB_ws, g_ws, e_ws = ref
    dB_na, g_na, e_na = got
    assert bool(torch.isfinite(dB_na).all())
    rel = float(torch.linalg.norm(dB_na - dB_ws) / torch.linalg.norm(dB_ws))
    bitwise = bool(torch.equal(dB_na, dB_ws)) and g_na == g_ws and e_na == e_ws
    say(f"{label}: dB rel {rel:.2e}, dgamma {g_na:.9e} vs {g_ws:.9e}, deta {e_na:.9e} vs "
        f"{e_ws:.9e}, bitwise equal {bitwise}")
    assert rel <= 1e-10
    assert abs(g_na - g_ws) <= 1e-10 * max(abs(g_ws), 1e-300)
    assert abs(e_na - e_ws) <= 1e-10 * max(abs(e_ws), 1e-300)


def test_noalloc_backward_matches_workspace_backward():
    from paper_1708_01413_amd import apc
    torch = _torch()
    # First call: the differentiation workload's shape (N = n = 4096, k = 16, m = 32,
    # FP32, T = 200, checkpoint every 14): ~32 MB of scratch.
    S = synth.shifted_square(4096, 32, k=16, shift=2.0, seed=70, with_target=True)
    A = torch.from_numpy(S.A).cuda()
    b = torch.from_numpy(S.B).cuda()
    plan = apc.Plan(A, b, S.off, "f32")
    dx = torch.from_numpy(np.random.default_rng(1).standard_normal((4096, 16))).cuda()
    say("case: noalloc backward, n=4096 k=16 f32 T=200 ckpt=14")
    ref, got, nb = _both(plan, dx, 200, 14)
    say(f"scratch needed {nb / 2**20:.1f} MiB")
    _check(ref, got, "first call")
    # Second call, smaller: N = 600, n = 400, k = 5, FP64, T = 30, checkpoint every 4.
    S2 = synth.gaussian_system(600, 400, 6, k=5, seed=50, scale=1 / math.sqrt(400))
    A2 = torch.from_numpy(S2.A).cuda()
    b2 = torch.from_numpy(S2.B).cuda()
    plan2 = apc.Plan(A2, b2, S2.off, "f64")
    dx2 = torch.from_numpy(np.random.default_rng(2).standard_normal((400, 5))).cuda()
    say("case: noalloc backward, N=600 n=400 k=5 f64 T=30 ckpt=4")
    ref2, got2, nb2 = _both(plan2, dx2, 30, 4)
    _check(ref2, got2, "second call")
    # An adjoint whose checkpoints do not fit the fixed scratch is refused on the host.
    big = apc.apc_backward_workspace_bytes(plan.handle, 4000, 14)
    assert big > 64 << 20
    dB = torch.empty(S.B.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(apc.ApcError) as ex:
        apc.apc_backward_noalloc(plan.handle, dx.data_ptr(), 16, 4000, 14, dB.data_ptr(), 16)
    assert ex.value.status == apc.APC_EINVAL
    say(f"oversized request ({big / 2**20:.0f} MiB) refused: {ex.value}")
    plan.close()
    plan2.close()
