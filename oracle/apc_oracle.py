"""Plain FP64 CPU oracle for Accelerated Projection-based Consensus (APC).

TEST INFRASTRUCTURE ONLY.  This module exists to check the HIP implementation.
Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import it.  The product path (the C-ABI library and its Python binding)
never imports, calls or links anything here, and this module imports nothing
from the product package.

Everything is NumPy in float64, written for clarity rather than speed: one
Python loop over the row blocks ("machines"), library primitives (QR,
triangular solve, symmetric eigenvalues, matrix products) as single steps, and
no fusion or reordering beyond what the paper writes down.

Paper: Azizan-Ruhi, Lahouti, Avestimehr, Hassibi, "Distributed Solution of
Large-Scale Linear Systems via Accelerated Projection-Based Consensus"
(arXiv 1708.01413).  Citations below name the section / equation / algorithm.

Readings taken where the paper is silent or ambiguous (each is repeated in the
design notes):
  R1 partition   -- the paper assumes m divides N (Sec. 2).  When it does not,
                    the first (N mod m) blocks get one extra row.
  R2 init        -- Alg. 1 lets each machine pick any solution of A_i x = b_i;
                    we take the minimum-norm one A_i^T (A_i A_i^T)^{-1} b_i.
                    Alg. 1 never initialises x_bar; we take the mean of the
                    x_i(0).
  R3 iteration   -- Alg. 1 loops "t = 1 to T" starting from x_i(0); we read it
                    as T updates, with the trajectory indexed by the number of
                    updates applied (t = 0 is the initial average).
  R4 optimum     -- Theorem 1's two equations are symmetric in (gamma, eta);
                    gamma* is the smaller root (it must satisfy |1-gamma| <= rho,
                    from the (m-1)n eigenvalues equal to 1-gamma in App. A, and
                    gamma in [0, 2] from the definition of S, eq. (6)).
  R5 metric      -- relative l2 error ||x_bar - x*|| / ||x*|| (Sec. 5); with k
                    right-hand sides the paper is silent: the error of each
                    column, and the maximum over columns is the figure that
                    tolerances gate on (rel_error); the Frobenius form over all
                    columns (rel_error_fro) is reported beside it.
  R6 rank        -- a block is rank deficient when min|diag R_i| <=
                    n * eps * max|diag R_i| (thin QR of A_i^T).
  R7 singular    -- no unique solution when mu_min <= n * eps (App. A, steady
                    state: the error vanishes iff mu_min != 0).
  R13 D-HBM start -- Sec. 4.3 gives no start for the comparison methods; D-HBM
                    and its preconditioned form start from APC's x_bar(0) with
                    zero momentum, so every method starts from the same point.

Parity note: every function here is pinned by tests that do not reuse its
arithmetic (definitions written differently, brute force, closed forms, the
paper's invariants).
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

EPS = np.finfo(np.float64).eps


class OracleError(ValueError):
    """Raised for inputs the method rejects (rank-deficient block, singular X)."""


# ----------------------------------------------------------------------------
# Sec. 2: the row partition [A_i, b_i]
# ----------------------------------------------------------------------------

def partition(N: int, m: int) -> np.ndarray:
    """Contiguous row blocks, block i = rows off[i]:off[i+1] (Sec. 2).

    p = N/m when m divides N; otherwise reading R1 (first N mod m blocks get
    one extra row).
    """
    if m < 1 or N < m:
        raise OracleError("need 1 <= m <= N")
    base, extra = divmod(N, m)
    sizes = [base + (1 if i < extra else 0) for i in range(m)]
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def blocks(M: np.ndarray, off: np.ndarray) -> list[np.ndarray]:
    """Row blocks M_i = M[off[i]:off[i+1]] (Sec. 2)."""
    return [M[off[i]:off[i + 1]] for i in range(len(off) - 1)]


def _as_cols(B: np.ndarray) -> np.ndarray:
    B = np.asarray(B, dtype=np.float64)
    return B[:, None] if B.ndim == 1 else B


# ----------------------------------------------------------------------------
# Sec. 3.1: projections
# ----------------------------------------------------------------------------

def projector(Ai: np.ndarray) -> np.ndarray:
    """Dense nullspace projector P_i = I - A_i^T (A_i A_i^T)^{-1} A_i (Sec. 3.1).

    Written straight from the definition; used only for small dense checks.
    """
    Ai = np.asarray(Ai, dtype=np.float64)
    n = Ai.shape[1]
    return np.eye(n) - Ai.T @ np.linalg.solve(Ai @ Ai.T, Ai)


def factor(A: np.ndarray, off: np.ndarray):
    """Thin QR of every A_i^T = Q_i R_i (Sec. 3.3, "e.g. using QR").

    Returns (Qt, R): Qt[i] = Q_i^T (p_i x n, orthonormal rows spanning the row
    space of A_i) and R[i] (p_i x p_i, upper triangular).  Then
    P_i v = v - Q_i (Q_i^T v).  Rank check: reading R6.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[1]
    Qt, R = [], []
    for i, Ai in enumerate(blocks(A, off)):
        if Ai.shape[0] > n:
            raise OracleError(f"block {i}: p_i > n")
        Q, Ri = np.linalg.qr(Ai.T, mode="reduced")
        dg = np.abs(np.diag(Ri))
        if dg.min() <= n * EPS * dg.max():
            raise OracleError(f"block {i} is rank deficient")
        Qt.append(Q.T.copy())
        R.append(Ri)
    return Qt, R


def project(Qti: np.ndarray, v: np.ndarray) -> np.ndarray:
    """P_i v = v - Q_i Q_i^T v, the two mat-vecs of Sec. 3.3."""
    return v - Qti.T @ (Qti @ v)


# ----------------------------------------------------------------------------
# Alg. 1, initialisation
# ----------------------------------------------------------------------------

def init_local(Qt, R, B: np.ndarray, off: np.ndarray) -> np.ndarray:
    """x_i(0) = A_i^T (A_i A_i^T)^{-1} b_i for every block (Alg. 1 init, R2).

    With A_i^T = Q_i R_i this is Q_i R_i^{-T} b_i.  Returns (m, n, k).
    """
    B = _as_cols(B)
    xs = []
    for Qti, Ri, bi in zip(Qt, R, blocks(B, off)):
        ci = solve_triangular(Ri, bi, trans="T", lower=False)
        xs.append(Qti.T @ ci)
    return np.stack(xs)


def initial_average(x0: np.ndarray) -> np.ndarray:
    """x_bar(0) = (1/m) sum_i x_i(0) (reading R2)."""
    return x0.mean(axis=0)


# ----------------------------------------------------------------------------
# Sec. 3.2: the matrix X and its spectrum; Theorem 1
# ----------------------------------------------------------------------------

def X_matrix(A: np.ndarray, off: np.ndarray) -> np.ndarray:
    """X = (1/m) sum_i A_i^T (A_i A_i^T)^{-1} A_i, eq. (3), formed densely."""
    A = np.asarray(A, dtype=np.float64)
    m = len(off) - 1
    X = np.zeros((A.shape[1], A.shape[1]))
    for Ai in blocks(A, off):
        X += Ai.T @ np.linalg.solve(Ai @ Ai.T, Ai)
    return X / m


def spectrum(A: np.ndarray, off: np.ndarray):
    """(mu_min, mu_max) of X, eq. (4); raises for a singular X (reading R7)."""
    mu = np.linalg.eigvalsh(X_matrix(A, off))
    n = A.shape[1]
    if mu[0] <= n * EPS:
        raise OracleError("mu_min ~ 0: the system has no unique solution")
    return float(mu[0]), float(mu[-1])


def optimal_params(mu_min: float, mu_max: float):
    """Optimal (gamma*, eta*, rho*) of Theorem 1.

    Theorem 1 fixes gamma, eta by
        mu_max * eta*gamma = (1 + r)^2,   mu_min * eta*gamma = (1 - r)^2,
    with r = sqrt((gamma-1)(eta-1)) = rho.  Taking square roots and adding
    gives s = eta*gamma = 4/(sqrt(mu_max)+sqrt(mu_min))^2; subtracting gives
    r = (sqrt(mu_max)-sqrt(mu_min))/(sqrt(mu_max)+sqrt(mu_min)), which is
    (sqrt(kappa)-1)/(sqrt(kappa)+1), eq. (7).  From s and r,
    gamma + eta = s + 1 - r^2, so gamma and eta are the roots of
    z^2 - (s + 1 - r^2) z + s = 0; gamma is the smaller root (reading R4).
    """
    if not (0.0 < mu_min <= mu_max <= 1.0 + 1e-12):
        raise OracleError("need 0 < mu_min <= mu_max <= 1")
    a, c = np.sqrt(mu_max), np.sqrt(mu_min)
    s = 4.0 / (a + c) ** 2
    r = (a - c) / (a + c)
    tr = s + 1.0 - r * r
    disc = max(tr * tr - 4.0 * s, 0.0)
    gamma = (tr - np.sqrt(disc)) / 2.0
    eta = (tr + np.sqrt(disc)) / 2.0
    return float(gamma), float(eta), float(r)


def char_poly_roots(mu: float, gamma: float, eta: float) -> np.ndarray:
    """Roots of p_i(lambda; gamma, eta), eq. (5)."""
    b1 = -eta * gamma * (1.0 - mu) + gamma - 1.0 + eta - 1.0
    b0 = (gamma - 1.0) * (eta - 1.0)
    return np.roots([1.0, b1, b0])


def predicted_rate(mus: np.ndarray, gamma: float, eta: float) -> float:
    """Spectral radius predicted by App. A: max of |1-gamma| (when m > 1) and
    the magnitudes of the roots of every p_i, eq. (5)."""
    rad = abs(1.0 - gamma)
    for mu in np.atleast_1d(mus):
        rad = max(rad, float(np.max(np.abs(char_poly_roots(mu, gamma, eta)))))
    return rad


# ----------------------------------------------------------------------------
# Eq. (2a)-(2b), Alg. 1: the iteration
# ----------------------------------------------------------------------------

def apc_step(Qt, x: np.ndarray, xbar: np.ndarray, gamma: float, eta: float):
    """One APC update (eq. (2a) for every block, then eq. (2b)).

    x: (m, n, k) local solutions x_i(t); xbar: (n, k).  Block i computes
    d = x_bar - x_i, w = Q_i^T d, x_i <- x_i + gamma (d - Q_i w); the master
    then forms x_bar <- (eta/m) sum_i x_i + (1-eta) x_bar, summing in block
    order.
    """
    m = x.shape[0]
    xn = np.empty_like(x)
    for i in range(m):
        d = xbar - x[i]
        w = Qt[i] @ d
        xn[i] = x[i] + gamma * (d - Qt[i].T @ w)
    acc = np.zeros_like(xbar)
    for i in range(m):
        acc = acc + xn[i]
    xbar_n = (eta / m) * acc + (1.0 - eta) * xbar
    return xn, xbar_n


def rel_error(xbar: np.ndarray, xstar: np.ndarray) -> float:
    """Relative l2 error ||x_bar - x*|| / ||x*|| (Sec. 5).  With k columns:
    the error of every column on its own, and the largest of them (R5)."""
    xb, xs = _as_cols(xbar), _as_cols(xstar)
    per_col = [np.sqrt(np.sum((xb[:, c] - xs[:, c]) ** 2)) / np.sqrt(np.sum(xs[:, c] ** 2))
               for c in range(xs.shape[1])]
    return float(max(per_col))


def rel_error_fro(xbar: np.ndarray, xstar: np.ndarray) -> float:
    """The same error taken over all k columns at once, ||X_bar - X*||_F / ||X*||_F
    (the figure reported beside rel_error, R5).  Equal to rel_error for k = 1."""
    xb, xs = _as_cols(xbar), _as_cols(xstar)
    return float(np.sqrt(np.sum((xb - xs) ** 2)) / np.sqrt(np.sum(xs ** 2)))


def residual(A: np.ndarray, B: np.ndarray, X: np.ndarray) -> float:
    """Relative residual of eq. (1) over all k columns, ||B - A X||_F / ||B||_F
    (the convergence monitor a solver can evaluate without knowing x*)."""
    B = _as_cols(B)
    R = B - np.asarray(A, dtype=np.float64) @ _as_cols(X)
    return float(np.sqrt(np.sum(R ** 2)) / np.sqrt(np.sum(B ** 2)))


def apc_run(A, B, off, T: int, gamma: float | None = None, eta: float | None = None,
            xstar=None, keep_traj: bool = False, keep_state: bool = False):
    """Algorithm 1: factor, initialise, then T updates (reading R3).

    gamma/eta default to Theorem 1's optimum.  Returns a dict with the
    parameters, x_bar(T), the relative-error curve err[t] for t = 0..T when
    x* is given, and optionally the whole x_bar trajectory (T+1, n, k).
    """
    A = np.asarray(A, dtype=np.float64)
    B = _as_cols(B)
    Qt, R = factor(A, off)
    x = init_local(Qt, R, B, off)
    xbar = initial_average(x)
    out = {}
    if gamma is None or eta is None:
        mu_min, mu_max = spectrum(A, off)
        g, e, rho = optimal_params(mu_min, mu_max)
        gamma = g if gamma is None else gamma
        eta = e if eta is None else eta
        out.update(mu_min=mu_min, mu_max=mu_max, rho=rho)
    out.update(gamma=gamma, eta=eta)
    errs, traj = [], []
    if xstar is not None:
        errs.append(rel_error(xbar, xstar))
    if keep_traj:
        traj.append(xbar.copy())
    for _ in range(T):
        x, xbar = apc_step(Qt, x, xbar, gamma, eta)
        if xstar is not None:
            errs.append(rel_error(xbar, xstar))
        if keep_traj:
            traj.append(xbar.copy())
    out["xbar"] = xbar
    out["err"] = np.array(errs)
    if keep_traj:
        out["traj"] = np.stack(traj)
    if keep_state:
        out["x"] = x
        out["Qt"] = Qt
    return out


# ----------------------------------------------------------------------------
# Differentiation of the unrolled iteration (adjoint of Alg. 1)
# ----------------------------------------------------------------------------

def apc_adjoint(A, B, off, T: int, gamma: float, eta: float, dxbar: np.ndarray):
    """Reverse-mode derivative of x_bar(T) from Alg. 1 (R2, R3) with respect to
    b, gamma and eta, for the scalar L with dL/dx_bar(T) = dxbar.

    The forward trajectory (every x_i(t), x_bar(t)) is stored; the reverse pass
    applies the transpose of each step of eqs. (2a)-(2b) in the opposite order.
    With l_i = lambda_i(t+1) + (eta/m) mu(t+1) (the adjoint of x_i(t+1), its
    direct path plus the path through x_bar(t+1)) and P_i symmetric:
        lambda_i(t) = l_i - gamma P_i l_i                  (transpose of eq. (2a) in x_i)
        mu(t)       = (1 - eta) mu(t+1) + gamma sum_i P_i l_i
        dL/dgamma  += sum_i <l_i, P_i (x_bar(t) - x_i(t))>
        dL/deta    += <mu(t+1), (1/m) sum_i x_i(t+1) - x_bar(t)>
    and for the start x_i(0) = Q_i R_i^{-T} b_i, x_bar(0) = mean:
        dL/db_i = R_i^{-1} Q_i^T (lambda_i(0) + mu(0) / m).
    Returns (dB (N, k), dgamma, deta).
    """
    A = np.asarray(A, dtype=np.float64)
    B = _as_cols(B)
    dxbar = _as_cols(dxbar)
    Qt, R = factor(A, off)
    x = init_local(Qt, R, B, off)
    xbar = initial_average(x)
    m = x.shape[0]
    xs, xbars = [x], [xbar]
    for _ in range(T):
        x, xbar = apc_step(Qt, x, xbar, gamma, eta)
        xs.append(x)
        xbars.append(xbar)
    lam = np.zeros_like(xs[0])
    mu = dxbar.copy()
    dgamma = 0.0
    deta = 0.0
    for t in range(T - 1, -1, -1):
        x_t, xb_t, x_next = xs[t], xbars[t], xs[t + 1]
        acc = np.zeros_like(xb_t)
        for i in range(m):
            acc = acc + x_next[i]
        deta += float(np.sum(mu * (acc / m - xb_t)))
        lam_new = np.empty_like(lam)
        push = np.zeros_like(mu)
        for i in range(m):
            li = lam[i] + (eta / m) * mu
            pli = project(Qt[i], li)
            dgamma += float(np.sum(pli * (xb_t - x_t[i])))   # <l_i, P_i d> = <P_i l_i, d>
            lam_new[i] = li - gamma * pli
            push = push + pli
        mu = (1.0 - eta) * mu + gamma * push
        lam = lam_new
    dB = np.zeros_like(B)
    for i, (Qti, Ri) in enumerate(zip(Qt, R)):
        gi = Qti @ (lam[i] + mu / m)
        dB[off[i]:off[i + 1]] = solve_triangular(Ri, gi, lower=False)
    return dB, dgamma, deta


# ----------------------------------------------------------------------------
# Sec. 4.5: block Cimmino (used only to check Proposition 2)
# ----------------------------------------------------------------------------

def cimmino_step(A, B, off, xbar: np.ndarray, nu: float) -> np.ndarray:
    """x_bar <- x_bar + nu sum_i A_i^+ (b_i - A_i x_bar), eqs. (15a)-(15b)."""
    B = _as_cols(B)
    upd = np.zeros_like(xbar)
    for Ai, bi in zip(blocks(np.asarray(A, dtype=np.float64), off), blocks(B, off)):
        upd = upd + Ai.T @ np.linalg.solve(Ai @ Ai.T, bi - Ai @ xbar)
    return xbar + nu * upd


# ----------------------------------------------------------------------------
# Sec. 4.3 (distributed heavy-ball method, D-HBM) and Sec. 6 (distributed
# preconditioning): the comparison methods, run on the same row blocks
# ----------------------------------------------------------------------------

def hbm_optimal_params(lam_min: float, lam_max: float):
    """Optimal heavy-ball step alpha, momentum beta and rate for a quadratic
    whose Hessian spectrum lies in [lam_min, lam_max] (the rate Sec. 4.3
    quotes for D-HBM).

    For one eigenvalue lam the iteration's characteristic polynomial is
    z^2 - (1 + beta - alpha lam) z + beta; its roots are complex with
    |z| = sqrt(beta) exactly when (1 - sqrt(beta))^2 <= alpha lam <=
    (1 + sqrt(beta))^2.  Putting lam_min and lam_max on the two ends gives
    sqrt(alpha) (sqrt(lam_max) + sqrt(lam_min)) = 2 and
    sqrt(alpha) (sqrt(lam_max) - sqrt(lam_min)) = 2 sqrt(beta), so
    alpha = 4 / (sqrt(lam_max) + sqrt(lam_min))^2, sqrt(beta) = rho =
    (sqrt(kappa) - 1) / (sqrt(kappa) + 1).
    """
    if not (0.0 < lam_min <= lam_max):
        raise OracleError("need 0 < lam_min <= lam_max")
    a, c = np.sqrt(lam_max), np.sqrt(lam_min)
    alpha = 4.0 / (a + c) ** 2
    rho = (a - c) / (a + c)
    return float(alpha), float(rho * rho), float(rho)


def normal_spectrum(Cb: list[np.ndarray]):
    """(lam_min, lam_max) of sum_i C_i^T C_i, the Hessian of the D-HBM
    objective (1/2) sum_i ||C_i x - d_i||^2 (Sec. 4.3)."""
    n = Cb[0].shape[1]
    H = np.zeros((n, n))
    for Ci in Cb:
        H = H + Ci.T @ Ci
    lam = np.linalg.eigvalsh(H)
    if lam[0] <= n * EPS * lam[-1]:
        raise OracleError("singular normal matrix: no unique solution")
    return float(lam[0]), float(lam[-1])


def precondition(A: np.ndarray, B: np.ndarray, off: np.ndarray):
    """Sec. 6: every machine premultiplies its equations by (A_i A_i^T)^{-1/2};
    returns the blocks C_i = (A_i A_i^T)^{-1/2} A_i and
    d_i = (A_i A_i^T)^{-1/2} b_i.  The inverse square root is taken from the
    symmetric eigendecomposition of A_i A_i^T."""
    A = np.asarray(A, dtype=np.float64)
    B = _as_cols(B)
    Cb, db = [], []
    for Ai, bi in zip(blocks(A, off), blocks(B, off)):
        lam, U = np.linalg.eigh(Ai @ Ai.T)
        if lam[0] <= Ai.shape[1] * EPS * lam[-1]:
            raise OracleError("rank-deficient block")
        S = U @ np.diag(1.0 / np.sqrt(lam)) @ U.T
        Cb.append(S @ Ai)
        db.append(S @ bi)
    return Cb, db


def dhbm_step(Cb, db, x: np.ndarray, z: np.ndarray, alpha: float, beta: float):
    """One D-HBM update (Sec. 4.3): every machine forms its gradient
    C_i^T (C_i x - d_i); the master sums them in block order, then
    z <- beta z + sum, x <- x - alpha z."""
    g = np.zeros_like(x)
    for Ci, di in zip(Cb, db):
        g = g + Ci.T @ (Ci @ x - di)
    zn = beta * z + g
    return x - alpha * zn, zn


def dhbm_run(A, B, off, T: int, preconditioned: bool = False, alpha: float | None = None,
             beta: float | None = None, x0=None, xstar=None, keep_traj: bool = False):
    """T updates of D-HBM (Sec. 4.3) on the blocks [A_i, b_i], or on the
    preconditioned blocks of Sec. 6.  alpha/beta default to the optimum for the
    spectrum of sum_i C_i^T C_i.  The start is x(0) = APC's initial average
    (Alg. 1 with reading R2), z(0) = 0 (reading R13), unless x0 is given."""
    A = np.asarray(A, dtype=np.float64)
    B = _as_cols(B)
    if preconditioned:
        Cb, db = precondition(A, B, off)
    else:
        Cb, db = blocks(A, off), blocks(B, off)
    lam_min, lam_max = normal_spectrum(Cb)
    a_opt, b_opt, rho = hbm_optimal_params(lam_min, lam_max)
    alpha = a_opt if alpha is None else alpha
    beta = b_opt if beta is None else beta
    if x0 is None:
        Qt, R = factor(A, off)
        x = initial_average(init_local(Qt, R, B, off))
    else:
        x = _as_cols(np.array(x0, dtype=np.float64))
    z = np.zeros_like(x)
    out = {"alpha": alpha, "beta": beta, "rho": rho, "lam_min": lam_min, "lam_max": lam_max}
    errs, traj = [], []
    for t in range(T + 1):
        if xstar is not None:
            errs.append(rel_error(x, xstar))
        if keep_traj:
            traj.append(x.copy())
        if t < T:
            x, z = dhbm_step(Cb, db, x, z, alpha, beta)
    out["x"] = x
    if xstar is not None:
        out["err"] = np.array(errs)
    if keep_traj:
        out["traj"] = np.stack(traj)
    return out
