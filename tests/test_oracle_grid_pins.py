"""Pins of the grid-coefficient oracle (oracle/grid.py) and parity of the
package's generator (minimax.py) against it.

Pins: the Chebyshev alternation theorem for the unconstrained optimum (the
exponentials exp(-x tau_j) with distinct tau_j form a Haar system, so the
best relative approximation equioscillates at N + 1 points), de la
Vallee-Poussin's lower bound, exact recovery of a target in the span, the
Laplace pairs of Eqs. (5) and (8) on a dense Gauss-Legendre grid, the inverse
transforms of Eqs. (6) and (9), and a planted cosine/sine mix-up.
"""
import numpy as np
import pytest

from oracle import grid as og
from paper_1607_02859_amd import minimax, synth


def _extrema(err):
    """signed values at the alternating extrema of a sampled error curve"""
    idx = [0] + [i for i in range(1, len(err) - 1)
                 if (err[i] - err[i - 1]) * (err[i + 1] - err[i]) <= 0] + [len(err) - 1]
    out = []
    for i in idx:
        if out and np.sign(err[i]) == np.sign(out[-1]):
            if abs(err[i]) > abs(out[-1]):
                out[-1] = err[i]
        else:
            out.append(err[i])
    return np.array(out)


@pytest.mark.parametrize("kind", ["cos", "sin"])
def test_unconstrained_optimum_equioscillates(kind):
    tau = np.array([0.02, 0.1, 0.4, 1.5])
    x = np.geomspace(1.0, 20.0, 4000)
    target = og.exact_term(kind, x, 3.0)
    c, t = og.lp_minimax(tau, target, x)
    err = 1.0 - (np.exp(-np.outer(x, tau)) @ c) / target
    ext = _extrema(err)
    big = ext[np.abs(ext) >= 0.999 * t]
    # N + 1 = 5 extrema of the optimum level with alternating signs
    assert big.shape[0] >= tau.shape[0] + 1
    assert np.all(np.sign(big[1:]) != np.sign(big[:-1]))
    # de la Vallee-Poussin: any N + 1 alternating errors bound the optimum below,
    # so the level t is optimal up to the sampling
    assert np.abs(big).min() <= t * (1 + 1e-6)


def test_target_in_the_span_is_recovered():
    tau = np.array([0.05, 0.3, 1.1, 4.0])
    d = np.array([0.7, -0.2, 1.3, 0.4])
    x = np.geomspace(0.5, 40.0, 1500)
    target = np.exp(-np.outer(x, tau)) @ d
    c, t = og.lp_minimax(tau, target, x)
    assert t <= 1e-7
    assert np.allclose(c, d, rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("kind", ["cos", "sin"])
def test_laplace_pair_on_dense_quadrature(kind):
    """On Gauss-Legendre nodes the discretised integral 2 sum_j w_j cos/sin(omega tau_j)
    exp(-x tau_j) is the exact term of Eq. (5) / (8) to ~1e-9; the bounded
    optimum with those nodes is at least as good (it is a minimum)."""
    omega = np.array([1.3])
    tau, ct = synth.gauss_legendre_ct(omega, 40.0, panel=1.0, nodes=24)
    _, st = synth.gauss_legendre_st(omega, 40.0, panel=1.0, nodes=24)
    tau = tau[::8]                      # a subset keeps the program small
    x = np.geomspace(1.0, 20.0, 400)
    target = og.exact_term(kind, x, omega[0])
    full = ct[0] if kind == "cos" else st[0]
    tau_all, _ = synth.gauss_legendre_ct(omega, 40.0, panel=1.0, nodes=24)
    assert og.relative_error(full, tau_all, target, x) < 1e-8
    c, t = og.lp_minimax(tau, target, x)
    assert t <= og.relative_error(ridge := og.ridge_reference(tau, target, x), tau, target, x)


def test_planted_cos_sin_mixup_is_caught():
    omega = np.array([2.0])
    tau, ct = synth.gauss_legendre_ct(omega, 40.0, panel=1.0, nodes=24)
    x = np.geomspace(1.0, 20.0, 400)
    # the cosine discretisation measured against the sine term fails
    assert og.relative_error(ct[0], tau, og.exact_term("sin", x, 2.0), x) > 0.1


@pytest.mark.parametrize("n,x_min,x_max", [(6, 0.5, 75.0), (12, 0.5, 75.0), (20, 0.1, 75.0),
                                           (20, 1.3894954943731375, 75.0)])
def test_generator_parity(n, x_min, x_max):
    """The generator's coefficients against the oracle's program on a denser
    sample: within the oracle's amplification bound and no worse than its
    optimum beyond the sampling difference (5 %) and the solvers' primal
    feasibility tolerance (1e-7 on the scaled constraint rows of each of the
    two programs, hence 2e-7 on the relative error); inverses of Eqs. (6) and
    (9)."""
    g = minimax.minimax_grid(n, x_min, x_max)
    x = np.geomspace(x_min, x_max, 1600)
    for kind, mat in (("cos", g.ct), ("sin", g.st)):
        ref, opt, bound = og.coefficients(g.tau, g.omega, kind, x_min, x_max)
        for k, w in enumerate(g.omega):
            target = og.exact_term(kind, x, w)
            err = og.relative_error(mat[k], g.tau, target, x)
            amp = og.amplification(mat[k], g.tau, target, x)
            assert amp <= bound[k] * 1.02
            assert err <= opt[k] * 1.05 + 2e-7
    # a backward-stable inverse leaves a residual of order n eps cond
    for fwd, inv in ((g.ct, g.ict), (g.st, g.ist)):
        if inv is not None:
            bound = 10 * n * np.finfo(float).eps * np.linalg.cond(fwd)
            assert np.abs(inv @ fwd - np.eye(n)).max() < bound


def test_mp2_time_grid_equioscillates():
    """The direct-MP2 time quadrature (Sec. II.A.2): 1/y by N exponentials on
    [1, R]; the optimum equioscillates at 2N + 1 points."""
    n, r = 5, 50.0
    tau, alpha, err, r_used = minimax.time_grid(n, 1.0, r)
    assert r_used == r
    y = np.geomspace(1.0, r, 20000)
    e = 1.0 / y - np.exp(-np.outer(y, tau)) @ alpha
    ext = _extrema(e)
    big = ext[np.abs(ext) >= 0.999 * np.abs(e).max()]
    assert big.shape[0] >= 2 * n + 1
    assert np.all(np.sign(big[1:]) != np.sign(big[:-1]))
