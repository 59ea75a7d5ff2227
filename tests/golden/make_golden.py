"""Write the oracle's expected values for the full-size parity tests.

Calls only the FP64 oracle and the seeded input generator.  Output:
tests/golden/tall_gauss_16384x8192_m64.npz with the oracle's spectrum
estimate inputs (mu_min, mu_max), Theorem 1's parameters, the relative error
curve err(t) for t = 0..T and x_bar(t) at every 8th coordinate for a few t.

Run:  python tests/golden/make_golden.py      (about a minute, ~3 GB of RAM)
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import apc_oracle as O  # noqa: E402
from paper_1708_01413_amd import synth  # noqa: E402

T = 60
CHECK_T = [0, 1, 2, 5, 10, 20, 30, 33, 40, 50, 60]
STRIDE = 8


def main():
    t0 = time.time()
    S = synth.tall_gaussian_16k()
    Qt, R = O.factor(S.A, S.off)
    x = O.init_local(Qt, R, S.B, S.off)
    xbar = O.initial_average(x)
    print(f"factor+init {time.time() - t0:.1f}s", flush=True)
    mu_min, mu_max = O.spectrum(S.A, S.off)
    g, e, rho = O.optimal_params(mu_min, mu_max)
    print(f"spectrum {time.time() - t0:.1f}s mu=[{mu_min:.6g}, {mu_max:.6g}] gamma={g:.9g} "
          f"eta={e:.9g} rho={rho:.6g}", flush=True)
    idx = np.arange(0, S.n, STRIDE)
    err = [O.rel_error(xbar, S.xstar)]
    samples = {0: xbar[idx, 0].copy()}
    for t in range(1, T + 1):
        x, xbar = O.apc_step(Qt, x, xbar, g, e)
        err.append(O.rel_error(xbar, S.xstar))
        if t in CHECK_T:
            samples[t] = xbar[idx, 0].copy()
    print(f"iterate {time.time() - t0:.1f}s err(T)={err[-1]:.3e}", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tall_gauss_16384x8192_m64.npz")
    np.savez(out, mu_min=mu_min, mu_max=mu_max, gamma=g, eta=e, rho=rho, err=np.array(err),
             check_t=np.array(CHECK_T), idx=idx,
             samples=np.stack([samples[t] for t in CHECK_T]), xstar_norm=np.linalg.norm(S.xstar))
    print("wrote", out)


if __name__ == "__main__":
    main()
