"""CPU oracle for the transform coefficients of the imaginary time/frequency
grid (Sec. II.A.3, Eqs. (4)-(9)).

TEST INFRASTRUCTURE ONLY.  Only the test-suite may import this module.  The
package's grid generator never calls it and shares no code with it.

What is computed, for a given tau/omega grid and transition energies x in
[x_min, x_max] (eV), per frequency omega_k:

* the error functions of Eqs. (5) and (8),
      eta^c(x) = 2x/(x^2 + omega_k^2)     - sum_j c_kj exp(-x tau_j),
      eta^s(x) = 2omega_k/(x^2 + omega_k^2) - sum_j s_kj exp(-x tau_j),
  whose exact terms are the cosine and sine transforms of exp(-x tau);
* coefficients minimising the maximum of |eta| / (exact term) over x, with the
  amplification sum_j |c_kj| exp(-x tau_j) / (exact term) bounded by twice
  that of the least-squares fit with a 1e-6 ridge on column-scaled
  coefficients (the reading the generator documents), written as a linear
  program over a log-spaced sample of x and solved by an interior-point
  method (scipy.optimize.linprog, one step);
* the inverse transforms of Eqs. (6) and (9) as matrix inverses.

Pins (tests/test_oracle_grid_pins.py): the Chebyshev alternation of the
unconstrained optimum (N + 1 points of equal error and alternating sign, with
de la Vallee-Poussin's lower bound), exact recovery of a target that is
itself a sum of the exponentials, the Laplace pairs of Eqs. (5) and (8) on a
dense Gauss-Legendre grid (the optimum is no worse than that exact
discretisation), and a planted cosine/sine mix-up.  Parity unpinned: none.
"""
from __future__ import annotations

import numpy as np

__all__ = ["exact_term", "relative_error", "amplification", "ridge_reference", "lp_minimax",
           "coefficients"]


def exact_term(kind, x, w):
    """The exact transform of exp(-x tau) under the brace of Eq. (5) (kind
    "cos") or Eq. (8) ("sin")."""
    return 2.0 * x / (x * x + w * w) if kind == "cos" else 2.0 * w / (x * x + w * w)


def relative_error(c, tau, target, x):
    """max_x |target(x) - sum_j c_j exp(-x tau_j)| / |target(x)|, target given
    as values on x."""
    e = np.exp(-np.outer(x, tau))
    return float((np.abs(target - e @ c) / np.abs(target)).max())


def amplification(c, tau, target, x):
    """max_x sum_j |c_j| exp(-x tau_j) / |target(x)|."""
    e = np.exp(-np.outer(x, tau))
    return float(((e @ np.abs(c)) / np.abs(target)).max())


def ridge_reference(tau, target, x, ridge=1e-6):
    """Least squares of the relative residual 1 - sum_j c_j exp(-x tau_j)/target
    with a ridge on the coefficients scaled by their column norms."""
    a = np.exp(-np.outer(x, tau)) / target[:, None]
    norms = np.linalg.norm(a, axis=0)
    lhs = np.vstack([a / norms, ridge * np.eye(tau.shape[0])])
    rhs = np.concatenate([np.ones(x.shape[0]), np.zeros(tau.shape[0])])
    return np.linalg.lstsq(lhs, rhs, rcond=None)[0] / norms


def lp_minimax(tau, target, x, amp_bound=None):
    """min t subject to |1 - sum_j c_j exp(-x_i tau_j)/target_i| <= t for every
    sample x_i and, when amp_bound is given,
    sum_j |c_j| exp(-x_i tau_j)/|target_i| <= amp_bound; variables c = p - q
    with p, q >= 0.  Returns (c, t)."""
    from scipy.optimize import linprog
    n = tau.shape[0]
    m = x.shape[0]
    b = np.exp(-np.outer(x, tau)) / target[:, None]
    scale = np.abs(b).max(axis=0)
    b = b / scale                                  # unknowns c_j * scale_j
    rows = [np.hstack([-b, b, -np.ones((m, 1))]), np.hstack([b, -b, -np.ones((m, 1))])]
    rhs = [-np.ones(m), np.ones(m)]
    if amp_bound is not None:
        rows.append(np.hstack([np.abs(b), np.abs(b), np.zeros((m, 1))]))
        rhs.append(np.full(m, float(amp_bound)))
    cost = np.zeros(2 * n + 1)
    cost[-1] = 1.0
    r = linprog(cost, A_ub=np.vstack(rows), b_ub=np.concatenate(rhs),
                bounds=[(0, None)] * (2 * n + 1), method="highs-ipm")
    if r.status != 0:
        raise RuntimeError(r.message)
    return (r.x[:n] - r.x[n:2 * n]) / scale, float(r.x[-1])


def coefficients(tau, omega, kind, x_min, x_max, n_sample=1600):
    """Per omega_k the bounded minimax coefficients of Eq. (5) or (8); returns
    (matrix [n_omega][n_tau], optimum per k, bound per k)."""
    tau = np.asarray(tau, dtype=np.float64)
    x = np.geomspace(x_min, x_max, n_sample)
    out = np.empty((len(omega), tau.shape[0]))
    opt = np.empty(len(omega))
    bound = np.empty(len(omega))
    for k, w in enumerate(omega):
        target = exact_term(kind, x, w)
        c0 = ridge_reference(tau, target, x)
        bound[k] = 2.0 * amplification(c0, tau, target, x)
        out[k], opt[k] = lp_minimax(tau, target, x, bound[k])
    return out, opt, bound
