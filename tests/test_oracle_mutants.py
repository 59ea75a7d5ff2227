"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins in
test_oracle.py catch each one.  This guards the pins themselves: a pin that
passes on a wrong oracle is no pin."""

import numpy as np
import pytest

from oracle import apc_oracle as O
from tests import test_oracle as P


def _step_wrong_sign(Qt, x, xbar, gamma, eta):
    m = x.shape[0]
    xn = np.empty_like(x)
    for i in range(m):
        d = xbar - x[i]
        xn[i] = x[i] + gamma * (d + Qt[i].T @ (Qt[i] @ d))      # sign of Q Q^T d flipped
    return xn, (eta / m) * xn.sum(0) + (1 - eta) * xbar


def _step_dropped_memory(Qt, x, xbar, gamma, eta):
    m = x.shape[0]
    xn = np.empty_like(x)
    for i in range(m):
        d = xbar - x[i]
        xn[i] = x[i] + gamma * (d - Qt[i].T @ (Qt[i] @ d))
    return xn, (eta / m) * xn.sum(0)                             # (1 - eta) x_bar dropped


def _step_stale_average(Qt, x, xbar, gamma, eta):
    m = x.shape[0]
    xn = np.empty_like(x)
    for i in range(m):
        d = xbar - x[i]
        xn[i] = x[i] + gamma * (d - Qt[i].T @ (Qt[i] @ d))
    return xn, (eta / m) * x.sum(0) + (1 - eta) * xbar           # averages x_i(t), not x_i(t+1)


def _step_wrong_direction(Qt, x, xbar, gamma, eta):
    m = x.shape[0]
    xn = np.empty_like(x)
    for i in range(m):
        d = x[i] - xbar                                          # d sign flipped
        xn[i] = x[i] + gamma * (d - Qt[i].T @ (Qt[i] @ d))
    return xn, (eta / m) * xn.sum(0) + (1 - eta) * xbar


def _params_swapped(mu_min, mu_max):
    g, e, r = _orig_params(mu_min, mu_max)
    return e, g, r                                               # gamma/eta roots swapped


def _params_plain_kappa(mu_min, mu_max):
    g, e, r = _orig_params(mu_min, mu_max)
    k = mu_max / mu_min
    return g, e, (k - 1) / (k + 1)                               # Cimmino rate instead of APC's


def _init_transposed(Qt, R, B, off):
    from scipy.linalg import solve_triangular
    B = B[:, None] if B.ndim == 1 else B
    xs = []
    for Qti, Ri, bi in zip(Qt, R, O.blocks(B, off)):
        ci = solve_triangular(Ri, bi, trans="N", lower=False)    # R^{-1} instead of R^{-T}
        xs.append(Qti.T @ ci)
    return np.stack(xs)


def _X_missing_inverse(A, off):
    A = np.asarray(A, dtype=np.float64)
    m = len(off) - 1
    return sum(Ai.T @ Ai for Ai in O.blocks(A, off)) / m        # (A_i A_i^T)^{-1} dropped


def _rel_error_mean(xbar, xstar):
    xb, xs = O._as_cols(xbar), O._as_cols(xstar)
    return float(np.mean(np.linalg.norm(xb - xs, axis=0) / np.linalg.norm(xs, axis=0)))  # mean, not max


def _rel_error_as_fro(xbar, xstar):
    xb, xs = O._as_cols(xbar), O._as_cols(xstar)
    return float(np.linalg.norm(xb - xs) / np.linalg.norm(xs))  # Frobenius in place of the gate


def _rel_error_fro_unnormalised(xbar, xstar):
    xb, xs = O._as_cols(xbar), O._as_cols(xstar)
    return float(np.linalg.norm(xb - xs))                        # ||X*|| dropped


def _residual_max_column(A, B, X):
    B = O._as_cols(B)
    R = B - np.asarray(A) @ O._as_cols(X)
    return float(np.max(np.linalg.norm(R, axis=0)) / np.linalg.norm(B))  # max column, not F-norm


def _residual_sign(A, B, X):
    B = O._as_cols(B)
    return float(np.linalg.norm(B + np.asarray(A) @ O._as_cols(X)) / np.linalg.norm(B))  # B + AX


_orig_params = O.optimal_params
_orig_adjoint = O.apc_adjoint


def _adjoint_variant(direct_average_path=True, start_transposed=False):
    """The oracle's adjoint with one planted mistake (same steps otherwise)."""
    from scipy.linalg import solve_triangular

    def adj(A, B, off, T, gamma, eta, dxbar):
        B = B[:, None] if B.ndim == 1 else B
        dxbar = dxbar[:, None] if dxbar.ndim == 1 else dxbar
        Qt, R = O.factor(A, off)
        x = O.init_local(Qt, R, B, off)
        xbar = O.initial_average(x)
        m = x.shape[0]
        xs, xbars = [x], [xbar]
        for _ in range(T):
            x, xbar = O.apc_step(Qt, x, xbar, gamma, eta)
            xs.append(x)
            xbars.append(xbar)
        lam, mu, dg, de = np.zeros_like(xs[0]), dxbar.copy(), 0.0, 0.0
        for t in range(T - 1, -1, -1):
            de += float(np.sum(mu * (xs[t + 1].mean(0) - xbars[t])))
            lam_new, push = np.empty_like(lam), np.zeros_like(mu)
            for i in range(m):
                li = lam[i] + ((eta / m) * mu if direct_average_path else 0.0)
                pli = O.project(Qt[i], li)
                dg += float(np.sum(pli * (xbars[t] - xs[t][i])))
                lam_new[i] = li - gamma * pli
                push = push + pli
            mu, lam = (1.0 - eta) * mu + gamma * push, lam_new
        dB = np.zeros_like(B)
        for i, (Qti, Ri) in enumerate(zip(Qt, R)):
            gi = Qti @ (lam[i] + mu / m)
            dB[off[i]:off[i + 1]] = solve_triangular(Ri, gi, trans="T" if start_transposed else "N",
                                                     lower=False)
        return dB, dg, de
    return adj


def _hbm_params_unsquared(lam_min, lam_max):
    alpha, beta, rho = _orig_hbm_params(lam_min, lam_max)
    return alpha, rho, rho                                       # momentum rho instead of rho^2


def _precondition_full_inverse(A, B, off):
    B = B[:, None] if B.ndim == 1 else B
    Cb, db = [], []
    for Ai, bi in zip(O.blocks(A, off), O.blocks(B, off)):
        S = np.linalg.inv(Ai @ Ai.T)                             # (A_i A_i^T)^{-1}, not ^{-1/2}
        Cb.append(S @ Ai)
        db.append(S @ bi)
    return Cb, db


def _dhbm_step_gradient_first(Cb, db, x, z, alpha, beta):
    g = sum(Ci.T @ (Ci @ x - di) for Ci, di in zip(Cb, db))
    return x - alpha * g, beta * z + g                           # x moves along g, not along new z


def _dhbm_step_wrong_sign(Cb, db, x, z, alpha, beta):
    g = sum(Ci.T @ (di - Ci @ x) for Ci, di in zip(Cb, db))      # gradient sign flipped
    zn = beta * z + g
    return x - alpha * zn, zn


_orig_hbm_params = O.hbm_optimal_params

_adjoint_no_average_path = _adjoint_variant(direct_average_path=False)
_adjoint_no_average_path.__name__ = "_adjoint_no_average_path"
_adjoint_start_transposed = _adjoint_variant(start_transposed=True)
_adjoint_start_transposed.__name__ = "_adjoint_start_transposed"

MUTANTS = [
    ("apc_step", _step_wrong_sign, ["test_single_update_solves_the_constrained_problem",
                                    "test_one_step_matches_stacked_error_recursion"]),
    ("apc_step", _step_dropped_memory, ["test_one_step_matches_stacked_error_recursion",
                                        "test_gamma_one_is_block_cimmino"]),
    ("apc_step", _step_stale_average, ["test_one_step_matches_stacked_error_recursion"]),
    ("apc_step", _step_wrong_direction, ["test_single_update_solves_the_constrained_problem",
                                         "test_converges_to_direct_solve"]),
    ("optimal_params", _params_swapped, ["test_optimal_params_satisfy_theorem1",
                                         "test_stacked_radius_at_optimum_is_rho_star"]),
    ("optimal_params", _params_plain_kappa, ["test_optimal_params_satisfy_theorem1"]),
    ("init_local", _init_transposed, ["test_init_is_min_norm_solution"]),
    ("X_matrix", _X_missing_inverse, ["test_X_matrix_properties"]),
    ("apc_adjoint", _adjoint_no_average_path, ["test_adjoint_matches_central_differences",
                                               "test_adjoint_converged_gradient"]),
    ("apc_adjoint", _adjoint_start_transposed, ["test_adjoint_matches_central_differences",
                                                "test_adjoint_of_the_start",
                                                "test_adjoint_converged_gradient"]),
    ("hbm_optimal_params", _hbm_params_unsquared, ["test_hbm_params_minimise_radius",
                                                   "test_dhbm_radius_at_optimum_is_the_paper_rate",
                                                   "test_apc_average_is_preconditioned_heavy_ball"]),
    ("precondition", _precondition_full_inverse, ["test_preconditioner_identities",
                                                  "test_preconditioned_dhbm_rate_equals_apc_rate"]),
    ("dhbm_step", _dhbm_step_gradient_first, ["test_dhbm_step_is_the_heavy_ball_recursion",
                                              "test_apc_average_is_preconditioned_heavy_ball"]),
    ("dhbm_step", _dhbm_step_wrong_sign, ["test_dhbm_step_is_the_heavy_ball_recursion",
                                          "test_dhbm_converges_to_direct_solve"]),
    ("rel_error", _rel_error_mean, ["test_error_metrics_on_a_hand_worked_case",
                                    "test_error_metrics_invariances"]),
    ("rel_error", _rel_error_as_fro, ["test_error_metrics_on_a_hand_worked_case",
                                      "test_error_metrics_invariances"]),
    ("rel_error_fro", _rel_error_fro_unnormalised, ["test_error_metrics_on_a_hand_worked_case",
                                                    "test_residual_with_orthonormal_columns_is_the_error"]),
    ("residual", _residual_max_column, ["test_residual_of_a_perturbed_direct_solve"]),
    ("residual", _residual_sign, ["test_residual_of_a_perturbed_direct_solve",
                                  "test_residual_with_orthonormal_columns_is_the_error"]),
]


def _run_pin(name):
    fn = getattr(P, name)
    if name == "test_optimal_params_satisfy_theorem1":
        for seed in range(5):
            fn(seed)
    elif name == "test_adjoint_matches_central_differences":
        fn(24, 12, 3, 2, 15, 5)
    elif name == "test_apc_average_is_preconditioned_heavy_ball":
        fn(None, None)
    else:
        fn()


@pytest.mark.parametrize("attr,mutant,pins", MUTANTS,
                         ids=[f"{a}-{m.__name__}" for a, m, _ in MUTANTS])
def test_pins_catch_planted_mistake(monkeypatch, attr, mutant, pins):
    monkeypatch.setattr(O, attr, mutant)
    caught = 0
    for name in pins:
        try:
            _run_pin(name)
        except (AssertionError, O.OracleError, np.linalg.LinAlgError):
            caught += 1
    assert caught == len(pins), f"{mutant.__name__}: only {caught}/{len(pins)} pins failed"
