"""Imaginary time/frequency grids and the transform coefficients of the
space-time method (Sec. II.A.2-3, Eqs. (4)-(9)).

This module prepares inputs only: it holds none of the polarizability,
screened-interaction or self-energy arithmetic.  Host FP64.

For transition energies x in [x_min, x_max] (eV):

* Cosine coefficients (Eq. (5)): for each omega_k the coefficients
  c_kj = gamma_kj cos(omega_k tau_j) that minimise the maximum over x of the
  error function relative to its exact term,
      |eta^c(x)| / f_k(x),   eta^c(x) = f_k(x) - sum_j c_kj exp(-x tau_j),
      f_k(x) = 2x/(x^2 + omega_k^2),
  subject to a bound on the transform's amplification,
      sum_j |c_kj| exp(-x tau_j) / f_k(x) <= A_k   for every x,
  A_k being twice that of the ridge least-squares fit on the same grid.  A
  linear program over a log-spaced sample of x (scipy's HiGHS), one per omega_k.
* Sine coefficients (Eq. (8)): the same with f_k(x) = 2 omega_k/(x^2 + omega_k^2),
  s_kj = lambda_kj sin(omega_k tau_j).
* Inverse transforms (Eqs. (6) and (9)): xi cos(tau omega) and
  zeta sin(tau omega) are the matrix inverses of the forward matrices.
* Grid: omega_k log-spaced in [x_min/2, x_max]; tau_j from a three-parameter
  log-spaced family, chosen to minimise log(fit error) + log(amplification)/2
  of the ridge least-squares fit (a fast stand-in for the minimax error during
  the search).
* ``time_grid``: the minimax quadrature of the energy denominator of the
  direct MP2 energy in imaginary time (Sec. II.A.2), 1/y = int exp(-y t) dt by
  N exponentials with the smallest maximum error over y in [1, R],
  R = x_max/x_min, tau_j = t_j/x_min -- a nonlinear Remez exchange with Newton
  steps on the 2N + 1 alternation equations, continued in N from one term, in
  extended precision (numpy.longdouble).  Offered as ``minimax_grid(...,
  tau_kind="mp2")``; the default family grid transforms with smaller
  amplification on these workloads (measured).

Readings (the paper names the error functions but not their norm, weight or
any conditioning constraint): the relative maximum error, because the build's
tolerance is relative per frequency; and the amplification bound, because the
unconstrained minimax drives the coefficients to cancel as the range narrows
(amplification of chi(tau) norms measured up to 1e5 at 20 points over
[10, 75] eV), which FP32 and split-BF16 inputs cannot absorb.
"""
from __future__ import annotations

import dataclasses
import functools
import json
import math
import os
from typing import Callable, Optional, Tuple

import numpy as np

__all__ = ["time_grid", "ridge_fit", "minimax_fit", "fit_transform", "cosine_target",
           "sine_target", "MinimaxGrid", "minimax_grid", "amplification", "relative_error"]

LD = np.longdouble
_TWO_PI = LD(2) * LD(math.pi)


def _gsolve(a, b):
    """Gaussian elimination with partial pivoting (works in longdouble)."""
    a = a.copy()
    b = b.copy()
    n = b.shape[0]
    for k in range(n):
        piv = k + int(np.argmax(np.abs(a[k:, k])))
        if a[piv, k] == 0:
            raise np.linalg.LinAlgError("singular alternation system")
        if piv != k:
            a[[k, piv]] = a[[piv, k]]
            b[[k, piv]] = b[[piv, k]]
        f = a[k + 1:, k] / a[k, k]
        a[k + 1:, k:] -= np.outer(f, a[k, k:])
        b[k + 1:] -= f * b[k]
    x = np.zeros(n, dtype=a.dtype)
    for k in range(n - 1, -1, -1):
        x[k] = (b[k] - a[k, k + 1:] @ x[k + 1:]) / a[k, k]
    return x


def _alternation(e, x, nref):
    """The nref largest alternating extrema of the sampled error e(x)."""
    idx = [0] + [i for i in range(1, x.shape[0] - 1)
                 if (e[i] - e[i - 1]) * (e[i + 1] - e[i]) <= 0] + [x.shape[0] - 1]
    pts = []
    for i in idx:
        if pts and np.sign(e[i]) == np.sign(e[pts[-1]]):
            if abs(e[i]) > abs(e[pts[-1]]):
                pts[-1] = i
        else:
            pts.append(i)
    while len(pts) > nref:
        if abs(e[pts[0]]) < abs(e[pts[-1]]):
            pts.pop(0)
        else:
            pts.pop()
    return np.asarray(pts, dtype=np.int64)


# ---------------------------------------------------------------------------
# Nonlinear minimax of 1/y by N terms b_j phi(y, exp(q_j)), parameters
# p = (log b, log q).
# ---------------------------------------------------------------------------

def _time_terms(p, y):
    n = p.shape[0] // 2
    a, t = np.exp(p[:n]), np.exp(p[n:])
    e = np.exp(-np.outer(y, t))
    # value, d/dlog a, d/dlog t
    return e @ a, e * a[None, :], -e * (a * t)[None, :] * y[:, None]


def _newton(terms, p, e_lev, yr):
    n = p.shape[0] // 2
    s = LD(-1) ** np.arange(yr.shape[0])
    for _ in range(80):
        v, da, dq = terms(p, yr)
        f = 1 / yr - v - s * e_lev
        jac = np.empty((yr.shape[0], 2 * n + 1), dtype=LD)
        jac[:, :n] = -da
        jac[:, n:2 * n] = -dq
        jac[:, 2 * n] = -s
        d = _gsolve(jac, -f)
        step, f0 = LD(1), np.abs(f).max()
        while True:
            pn, en = p + step * d[:2 * n], e_lev + step * d[2 * n]
            fn = 1 / yr - terms(pn, yr)[0] - s * en
            if np.all(np.isfinite(fn)) and np.abs(fn).max() <= f0 * (1 - LD(1e-4) * step):
                break
            step /= 2
            if step < LD(1e-6):
                return p, e_lev, f0 < LD(1e-17)
        p, e_lev = pn, en
        if np.abs(fn).max() < LD(1e-18):
            break
    return p, e_lev, True


def _remez_nonlinear(terms, p, yr, r, n_sample=40000, iters=40):
    """Exchange loop: Newton on the alternation system, then the new extrema.
    Returns (p, E, max error, references) or None when it does not resolve."""
    y = np.geomspace(1.0, r, n_sample).astype(LD)
    nref = p.shape[0] + 1
    e_lev = LD(0)
    emax = None
    for _ in range(iters):
        try:
            p, e_lev, ok = _newton(terms, p, e_lev, yr)
        except np.linalg.LinAlgError:
            return None
        if not ok:
            return None
        err = 1 / y - terms(p, y)[0]
        pts = _alternation(err, y, nref)
        emax = np.abs(err).max()
        if pts.shape[0] == nref:
            yr = y[pts]
        if abs(emax - abs(e_lev)) < LD(1e-6) * abs(e_lev):
            break
    return p, abs(e_lev), emax, yr


def _extend(p, yr, n_new):
    """Start for n_new terms from an n-term solution: log parameters
    interpolated over the sorted terms, weights scaled by the spacing ratio,
    references interpolated in log y."""
    n = p.shape[0] // 2
    lb, lq = p[:n], p[n:]
    o = np.argsort(lq)
    lb, lq = lb[o].astype(float), lq[o].astype(float)
    if n == 1:
        lq2 = np.array([lq[0] - 1.5, lq[0] + 1.0])
        lb2 = np.array([lb[0] - 1.0, lb[0]])
    else:
        s_old = np.arange(n) / (n - 1.0)
        s_new = np.arange(n_new) / (n_new - 1.0)
        lq2 = np.interp(s_new, s_old, lq)
        lb2 = np.interp(s_new, s_old, lb) + math.log((n - 1.0) / (n_new - 1.0))
    ly = np.log(yr.astype(float))
    yr2 = np.exp(np.interp(np.linspace(0, 1, 2 * n_new + 1), np.linspace(0, 1, yr.shape[0]), ly))
    return np.concatenate([lb2, lq2]).astype(LD), yr2.astype(LD)


def _one_term_start(terms, r):
    """Coarse search for the one-term problem, then its exchange loop."""
    y = np.geomspace(1.0, r, 300).astype(LD)
    best = None
    for lb in np.linspace(-3.0, 3.0, 61):
        for lq in np.linspace(-6.0, 3.0, 91):
            p = np.array([lb, lq], dtype=LD)
            e = np.abs(1 / y - terms(p, y)[0]).max()
            if best is None or e < best[0]:
                best = (e, p)
    p = best[1]
    err = 1 / y - terms(p, y)[0]
    pts = _alternation(err, y, 3)
    yr = y[pts] if pts.shape[0] == 3 else np.array([1.0, math.sqrt(r), r], dtype=LD)
    return _remez_nonlinear(terms, p, yr, r)


def _solve_nonlinear(terms, n, r):
    """n-term minimax on [1, r], continued in the number of terms; None if
    some step does not resolve."""
    res = _one_term_start(terms, r)
    if res is None:
        return None
    for m in range(2, n + 1):
        p0, yr0 = _extend(res[0], res[3], m)
        res = _remez_nonlinear(terms, p0, yr0, r)
        if res is None:
            return None
    return res


@functools.lru_cache(maxsize=256)
def _nonlinear_grid(kind, n, r):
    terms = _time_terms
    rr = float(r)
    for _ in range(40):
        res = _solve_nonlinear(terms, n, rr)
        if res is not None:
            p, e_lev, emax, _ = res
            w, q = np.exp(p[:n]).astype(float), np.exp(p[n:]).astype(float)
            o = np.argsort(q)
            return q[o], w[o], float(emax), rr
        rr *= 1.5          # not resolvable at this range: the next wider one
    raise RuntimeError(f"minimax {kind} grid with {n} points did not converge")


def time_grid(n: int, x_min: float, x_max: float):
    """(tau [n], alpha [n], max error of the scaled problem, range used R')."""
    t, a, err, r_used = _nonlinear_grid("time", int(n), float(x_max / x_min))
    return t / x_min, a / x_min, err, r_used




# ---------------------------------------------------------------------------
# Transform coefficients on a given grid.
# ---------------------------------------------------------------------------

def cosine_target(x, w):
    """2x/(x^2 + w^2): the exact cosine transform of exp(-x tau) (Eq. (5))."""
    return 2.0 * x / (x * x + w * w)


def sine_target(x, w):
    """2w/(x^2 + w^2): the exact sine transform of exp(-x tau) (Eq. (8))."""
    return 2.0 * w / (x * x + w * w)


def relative_error(c, tau, w, target, x):
    """max_x |target(x) - sum_j c_j exp(-x tau_j)| / target(x)."""
    f = target(x, w)
    return float((np.abs(f - np.exp(-np.outer(x, tau)) @ c) / f).max())


def amplification(c, tau, w, target, x):
    """max_x sum_j |c_j| exp(-x tau_j) / target(x)."""
    return float(((np.exp(-np.outer(x, tau)) @ np.abs(c)) / target(x, w)).max())


def ridge_fit(tau, w, target, x, ridge=1e-6):
    """Least squares of the relative residual with a small ridge on
    column-scaled coefficients (the conditioning reference)."""
    a = np.exp(-np.outer(x, tau)) / target(x, w)[:, None]
    s = np.sqrt((a * a).sum(0))
    m = np.vstack([a / s, ridge * np.eye(len(tau))])
    rhs = np.concatenate([np.ones(len(x)), np.zeros(len(tau))])
    return np.linalg.lstsq(m, rhs, rcond=None)[0] / s


def minimax_fit(tau, w, target, x, amp_bound):
    """Coefficients minimising max_x |1 - sum_j c_j exp(-x tau_j)/target(x)|
    subject to sum_j |c_j| exp(-x tau_j)/target(x) <= amp_bound, over the
    sample x: a linear program in (c+, c-, t) with c = c+ - c-, each column
    scaled to a maximum of one.  Returns None if neither HiGHS method solves it."""
    from scipy.optimize import linprog
    n = len(tau)
    b = np.exp(-np.outer(x, tau)) / target(x, w)[:, None]
    sc = b.max(axis=0)
    b = b / sc
    ones = np.ones((len(x), 1))
    zero = np.zeros((len(x), 1))
    a_ub = np.vstack([np.hstack([-b, b, -ones]),       # 1 - b c <= t
                      np.hstack([b, -b, -ones]),       # b c - 1 <= t
                      np.hstack([b, b, zero])])        # amplification
    b_ub = np.concatenate([-np.ones(len(x)), np.ones(len(x)), np.full(len(x), amp_bound)])
    cost = np.zeros(2 * n + 1)
    cost[-1] = 1.0
    for method in ("highs-ds", "highs-ipm"):
        r = linprog(cost, A_ub=a_ub, b_ub=b_ub, bounds=[(0, None)] * (2 * n + 1), method=method)
        if r.status == 0:
            return (r.x[:n] - r.x[n:2 * n]) / sc
    return None


def _sample(x_min, x_max, n=800):
    return np.geomspace(x_min, x_max, n)


def _fit_all(tau, omega, target, x_min, x_max):
    x = _sample(x_min, x_max)
    out = np.empty((len(omega), len(tau)))
    err = 0.0
    for k, w in enumerate(omega):
        c0 = ridge_fit(tau, w, target, x)
        c = minimax_fit(tau, w, target, x, 2.0 * amplification(c0, tau, w, target, x))
        # the ridge fit where the program cannot be solved, or where it does not
        # improve the maximum error (the sample and solver tolerances bound it)
        if c is None or relative_error(c, tau, w, target, x) > relative_error(c0, tau, w, target, x):
            c = c0
        out[k] = c
        err = max(err, relative_error(out[k], tau, w, target, x))
    return out, err


def fit_transform(tau, omega, kind, x_min, x_max):
    """Coefficients of the cosine (kind "cos", Eq. (5)) or sine ("sin",
    Eq. (8)) transform on a given grid; returns (matrix [n_omega][n_tau],
    max relative error)."""
    return _fit_all(tau, omega, cosine_target if kind == "cos" else sine_target, x_min, x_max)


def _family(n_tau, x_min, x_max, a, b, p):
    t = np.linspace(0.0, 1.0, n_tau) ** p
    lo, hi = math.log(a / x_max), math.log(b / x_min)
    return np.exp(lo + t * (hi - lo))


def _family_search(n, x_min, x_max):
    """tau from the three-parameter family with the best
    log(ridge-fit error) + log(amplification)/2 over the cosine targets."""
    x = np.geomspace(x_min, x_max, 600)
    omega = np.geomspace(x_min / 2.0, x_max, n)
    best = None
    for a in (0.05, 0.1, 0.2, 0.3, 0.5):
        for b in (1.0, 2.0, 3.0, 5.0, 8.0):
            for p in (0.7, 0.85, 1.0, 1.2):
                tau = _family(n, x_min, x_max, a, b, p)
                err = amp = 0.0
                for w in omega:
                    c = ridge_fit(tau, w, cosine_target, x, ridge=0.0)
                    err = max(err, relative_error(c, tau, w, cosine_target, x))
                    amp = max(amp, amplification(c, tau, w, cosine_target, x))
                score = math.log(err) + 0.5 * math.log(amp)
                if best is None or score < best[0]:
                    best = (score, tau)
    return best[1], omega


@dataclasses.dataclass
class MinimaxGrid:
    tau: np.ndarray          # [n]
    omega: np.ndarray        # [n]
    ct: np.ndarray           # [n][n] gamma_kj cos(omega_k tau_j)   (Eq. (4))
    st: np.ndarray           # [n][n] lambda_kj sin(omega_k tau_j)  (Eq. (7))
    ict: Optional[np.ndarray]   # [n][n] xi_jk cos(tau_j omega_k)   (Eq. (6)); None if singular
    ist: Optional[np.ndarray]   # [n][n] zeta_jk sin(tau_j omega_k) (Eq. (9)); None if singular
    err_cos: float           # max over k and x of |eta^c| / f_k
    err_sin: float           # max over k and x of |eta^s| / f_k


_TABLES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grid_tables.json")


def _key(n, x_min, x_max, tau_kind):
    return f"{tau_kind}:{n}:{x_min!r}:{x_max!r}"


@functools.lru_cache(maxsize=1)
def _tables():
    try:
        with open(_TABLES) as f:
            return json.load(f)
    except OSError:
        return {}


def _compute(n, x_min, x_max, tau_kind):
    if tau_kind == "mp2":
        tau = time_grid(n, x_min, x_max)[0]
        omega = np.geomspace(x_min / 2.0, x_max, n)
    else:
        tau, omega = _family_search(n, x_min, x_max)
    ct, ec = _fit_all(tau, omega, cosine_target, x_min, x_max)
    st, es = _fit_all(tau, omega, sine_target, x_min, x_max)
    return {"tau": tau.tolist(), "omega": omega.tolist(), "ct": ct.tolist(), "st": st.tolist(),
            "err_cos": ec, "err_sin": es}


def _inverse(m):
    """The matrix inverse, or None for a numerically singular matrix (many
    points over a narrow range make the forward matrices nearly dependent)."""
    try:
        inv = np.linalg.inv(m)
    except np.linalg.LinAlgError:
        return None
    return inv if np.all(np.isfinite(inv)) and np.linalg.cond(m) < 1e13 else None


@functools.lru_cache(maxsize=64)
def _grid_cached(n, x_min, x_max, tau_kind):
    d = _tables().get(_key(n, x_min, x_max, tau_kind))
    if d is None:
        d = _compute(n, x_min, x_max, tau_kind)
    ct, st = np.array(d["ct"]), np.array(d["st"])
    return MinimaxGrid(tau=np.array(d["tau"]), omega=np.array(d["omega"]), ct=ct, st=st,
                       ict=_inverse(ct), ist=_inverse(st), err_cos=float(d["err_cos"]),
                       err_sin=float(d["err_sin"]))


def minimax_grid(n: int, x_min: float, x_max: float, tau_kind: str = "family") -> MinimaxGrid:
    """The n-point grid with its four transform matrices for transition
    energies in [x_min, x_max] (eV).  Grids listed in grid_tables.json (the
    workload configurations, written by ``python -m
    paper_1607_02859_amd.minimax``) are read from it; others are computed and
    cached for the process."""
    g = _grid_cached(int(n), float(x_min), float(x_max), tau_kind)
    return dataclasses.replace(g, **{f.name: np.copy(getattr(g, f.name))
                                     for f in dataclasses.fields(g)
                                     if isinstance(getattr(g, f.name), np.ndarray)})


# grids kept in grid_tables.json: (points, x_min, x_max) of the workload
# configurations (the 32-system batch has gaps 0.1 * 100^(s/7) eV) and of the
# smaller synthetic items and screened-interaction inputs
TABLE_GRIDS = sorted(set(
    [(n, lo, 75.0) for n in range(1, 21) for lo in (0.5, 1.0)]
    + [(n, 0.5, 50.0) for n in range(1, 21)]
    + [(20, 0.1 * 100.0 ** (s / 7.0), 75.0) for s in range(8)]))


if __name__ == "__main__":
    out = {}
    for n, lo, hi in TABLE_GRIDS:
        out[_key(n, float(lo), float(hi), "family")] = _compute(n, float(lo), float(hi), "family")
        print(n, lo, hi, out[_key(n, float(lo), float(hi), "family")]["err_cos"], flush=True)
    with open(_TABLES, "w") as f:
        json.dump(out, f, separators=(",", ":"))
