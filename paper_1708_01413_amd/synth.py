"""Seeded synthetic inputs for the APC solver and its checks.

This module builds test and benchmark inputs only: consistent linear systems
A x* = b shaped like the paper's synthetic workloads (square and tall Gaussian
matrices, Sec. 5), scaled up, plus row-block sizes.  It holds none of the
method's arithmetic and imports nothing else from this repository, so both the
HIP path's tests and the independent oracle can consume the same arrays.

Conventions: ``numpy.random.default_rng(seed)``, float64 ``standard_normal``,
row-major; draw order is (block sizes, when random) -> A -> x* -> extra vectors.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class System:
    """A consistent system A X* = B split into row blocks off[i]:off[i+1]."""

    A: np.ndarray            # (N, n) float64
    B: np.ndarray            # (N,) or (N, k) float64
    xstar: np.ndarray        # (n,) or (n, k) float64
    off: np.ndarray          # (m+1,) int64 block boundaries
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]

    @property
    def m(self) -> int:
        return len(self.off) - 1

    @property
    def k(self) -> int:
        return 1 if self.B.ndim == 1 else self.B.shape[1]


def offsets_from_sizes(sizes) -> np.ndarray:
    """Block boundaries [0, p_1, p_1+p_2, ...] from the block sizes."""
    return np.concatenate([[0], np.cumsum(np.asarray(sizes, dtype=np.int64))]).astype(np.int64)


def even_sizes(N: int, m: int) -> np.ndarray:
    """m contiguous blocks of N rows; the first N mod m blocks get one extra row."""
    base, extra = divmod(N, m)
    return np.array([base + (1 if i < extra else 0) for i in range(m)], dtype=np.int64)


def renormalised_sizes(rng, m: int, total: int, lo: int, hi: int) -> np.ndarray:
    """m sizes drawn uniformly from [lo, hi], scaled to sum to ``total``.

    Scaling uses largest-remainder rounding so the sum is exact and every size
    stays >= 1.
    """
    raw = rng.integers(lo, hi + 1, m).astype(np.float64)
    scaled = raw * (total / raw.sum())
    sizes = np.floor(scaled).astype(np.int64)
    short = total - int(sizes.sum())
    order = np.argsort(-(scaled - sizes), kind="stable")
    sizes[order[:short]] += 1
    sizes = np.maximum(sizes, 1)
    while sizes.sum() > total:           # only reachable if a size was clamped to 1
        sizes[np.argmax(sizes)] -= 1
    return sizes


def gaussian_system(N: int, n: int, m: int | None = None, *, k: int = 1, seed: int = 0,
                    scale: float = 1.0, shift: float = 0.0, sizes=None, mean: float = 0.0,
                    name: str = "") -> System:
    """A = scale * (G + mean) (+ shift * I on the leading n x n block), G iid N(0, 1);
    X* iid N(0, 1) with k columns (a vector when k == 1); B = A X*."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, n))
    if mean:
        A += mean
    A *= scale
    if shift:
        A[np.arange(min(N, n)), np.arange(min(N, n))] += shift
    xs = rng.standard_normal((n, k))
    if k == 1:
        xs = xs[:, 0]
    B = A @ xs
    if sizes is None:
        sizes = even_sizes(N, m)
    return System(A=A, B=B, xstar=xs, off=offsets_from_sizes(sizes), name=name)


# ---------------------------------------------------------------------------
# Named workloads (sizes follow the benchmark configurations)
# ---------------------------------------------------------------------------

def tall_gaussian_16k_mean1(seed: int = 0) -> System:
    """The benchmark shape with entries of mean 1: A = (G + 1)/sqrt(n), x* iid N(0, 1),
    m = 64 blocks of 256 rows (the nonzero-mean random systems of the paper's comparison,
    where A^T A has one large outlying eigenvalue)."""
    n = 8192
    return gaussian_system(16384, n, 64, seed=seed, scale=1.0 / np.sqrt(n), mean=1.0,
                           name="tall-gauss-mean1-16384x8192-m64")


def square_gaussian_512(seed: int = 0) -> System:
    """N = n = 512, A and x* iid N(0, 1), m = 8 blocks of 64 rows (FP64 case)."""
    return gaussian_system(512, 512, 8, seed=seed, name="square-gauss-512-m8")


def tall_gaussian_16k(seed: int = 0) -> System:
    """N = 16384, n = 8192, A iid N(0, 1/n), x* iid N(0, 1), m = 64 blocks of 256 rows."""
    n = 8192
    return gaussian_system(16384, n, 64, seed=seed, scale=1.0 / np.sqrt(n),
                           name="tall-gauss-16384x8192-m64")


def shifted_uneven_8k(seed: int = 0, k: int = 64) -> System:
    """N = n = 8192, A = G/sqrt(n) + 2I, k right-hand sides, 64 blocks whose sizes
    are drawn uniformly from [32, 256] and renormalised to sum to 8192."""
    rng = np.random.default_rng(seed)
    n = 8192
    sizes = renormalised_sizes(rng, 64, n, 32, 256)
    A = rng.standard_normal((n, n)) / np.sqrt(n)
    A[np.arange(n), np.arange(n)] += 2.0
    xs = rng.standard_normal((n, k))
    return System(A=A, B=A @ xs, xstar=xs, off=offsets_from_sizes(sizes),
                  name=f"shifted-uneven-8192-k{k}")


def shifted_square(n: int, m: int, k: int = 1, shift: float = 2.0, seed: int = 0,
                   with_target: bool = False) -> System:
    """N = n, A = G/sqrt(n) + shift*I, m even blocks, k RHS; optional x_target."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) / np.sqrt(n)
    A[np.arange(n), np.arange(n)] += shift
    xs = rng.standard_normal((n, k))
    extra = {}
    if with_target:
        extra["x_target"] = rng.standard_normal((n, k))
    if k == 1:
        xs = xs[:, 0]
        if with_target:
            extra["x_target"] = extra["x_target"][:, 0]
    return System(A=A, B=A @ xs, xstar=xs, off=offsets_from_sizes(even_sizes(n, m)),
                  name=f"shifted-{n}-m{m}-k{k}", extra=extra)


def many_small_systems(count: int = 256, seed: int = 0, lo: int = 64, hi: int = 1024):
    """``count`` independent square systems: n_s uniform in [lo, hi], m_s in {4, 8, 16},
    A_s = G/sqrt(n_s) + 2I, one RHS each (drawn in system order)."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        n = int(rng.integers(lo, hi + 1))
        m = int(rng.choice([4, 8, 16]))
        A = rng.standard_normal((n, n)) / np.sqrt(n)
        A[np.arange(n), np.arange(n)] += 2.0
        xs = rng.standard_normal(n)
        out.append(System(A=A, B=A @ xs, xstar=xs, off=offsets_from_sizes(even_sizes(n, m)),
                          name=f"small-{s}"))
    return out
