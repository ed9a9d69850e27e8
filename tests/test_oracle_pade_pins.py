"""Pins of the CPU oracle for the analytic continuation (Thiele's reciprocal
differences, Sec. II.E.1, Eqs. (72)-(74)).

Checked against what the mathematics fixes, not against the oracle's own
formulas: the interpolation property the paper states, rational functions an
N-point Thiele fraction represents exactly, and a rational interpolant of the
same degrees obtained independently by a linear solve.  Planted index
mistakes fail the same checks.
"""
import numpy as np
import pytest

from oracle import pade as op


def _grid(n, wmax=30.0):
    # imaginary frequencies, log-spaced as on the paper's grids
    return 1j * np.exp(np.linspace(np.log(0.05), np.log(wmax), n))


def _poles(m, seed, span=20.0):
    rng = np.random.default_rng(seed)
    e = rng.uniform(-span, span, m) + 1j * rng.uniform(-0.5, 0.5, m)   # pole positions
    r = rng.uniform(0.2, 2.0, m) * np.exp(1j * rng.uniform(-0.3, 0.3, m))
    return e, r


def _f_poles(e, r, z):
    return (r[None, :] / (z[:, None] - e[None, :])).sum(axis=1)


@pytest.mark.parametrize("n", [1, 2, 5, 12, 20])
def test_interpolates_the_nodes(n):
    z = _grid(n)
    e, r = _poles(6, n)
    f = _f_poles(e, r, z) + 0.3
    p = op.continue_to(z, f, z)
    assert np.abs(p - f).max() <= 1e-9 * np.abs(f).max()


def test_constant_is_exact():
    """A constant has a_2 = 0 exactly; the fraction ends there (the reading
    for an exactly zero reciprocal-difference denominator)."""
    z = _grid(8)
    f = np.full(8, 2.5 - 0.5j)
    a = op.coefficients(z, f)
    assert a[0] == 2.5 - 0.5j and np.all(a[1:] == 0)
    w = np.linspace(-10, 10, 7) + 0.01j
    assert np.abs(op.continue_to(z, f, w) - (2.5 - 0.5j)).max() < 1e-13


def test_one_pole_with_more_points_terminates():
    """One pole needs 2 points; with 6 the later reciprocal differences vanish
    (up to rounding or exactly) and the continuation stays exact."""
    z = _grid(6)
    e, r = np.array([0.7 - 0.3j]), np.array([1.1 + 0.0j])
    f = _f_poles(e, r, z)
    w = np.linspace(-5, 5, 21) + 0.05j
    out = op.continue_to(z, f, w)
    assert np.all(np.isfinite(out))
    assert np.abs(out - _f_poles(e, r, w)).max() < 1e-8


def test_single_pole_is_exact_on_the_real_axis():
    z = _grid(6)
    e, r = np.array([1.7 - 0.2j]), np.array([0.8 + 0.1j])
    f = _f_poles(e, r, z)
    w = np.linspace(-5, 5, 41) + 0.05j
    assert np.abs(op.continue_to(z, f, w) - _f_poles(e, r, w)).max() < 1e-10


@pytest.mark.parametrize("m", [2, 3, 4])
def test_sum_of_poles_with_enough_points_is_exact(m):
    """M poles form a rational function of degrees (M-1, M); 2M + 1 points
    determine it, so the continuation reproduces it off the imaginary axis
    (poles within the span of the nodes, where the continuation is well
    conditioned: errors 1e-14 .. 1e-10)."""
    n = 2 * m + 1
    z = _grid(n, 30.0)
    e, r = _poles(m, 40 + m, span=5.0)
    f = _f_poles(e, r, z)
    w = np.linspace(-8, 8, 101) + 0.2j
    ref = _f_poles(e, r, w)
    err = np.abs(op.continue_to(z, f, w) - ref).max() / np.abs(ref).max()
    assert err < 1e-8


def _rational_by_solve(z, f, w):
    """Interpolant p(z)/q(z) with deg p = floor((N-1)/2), deg q = ceil((N-1)/2),
    q monic in its top power, from the linear conditions p(z_j) - f_j q(z_j) = 0."""
    n = z.shape[0]
    dp, dq = (n - 1) // 2, n - 1 - (n - 1) // 2
    a = np.zeros((n, n), dtype=np.complex128)
    rhs = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        for k in range(dp + 1):
            a[j, k] = z[j] ** k
        for k in range(dq):
            a[j, dp + 1 + k] = -f[j] * z[j] ** k
        rhs[j] = f[j] * z[j] ** dq
    c = np.linalg.solve(a, rhs)
    p = sum(c[k] * w ** k for k in range(dp + 1))
    q = sum(c[dp + 1 + k] * w ** k for k in range(dq)) + w ** dq
    return p / q


@pytest.mark.parametrize("n", [3, 4, 5, 6, 7])
def test_matches_rational_interpolant_by_linear_solve(n):
    """The N-point Thiele fraction is the rational interpolant of degrees
    (floor((N-1)/2), ceil((N-1)/2)); solving for it directly must agree."""
    z = _grid(n, 5.0)
    rng = np.random.default_rng(n)
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    w = np.linspace(-3, 3, 13) + 0.3j
    a = op.continue_to(z, f, w)
    b = _rational_by_solve(z, f, w)
    assert np.abs(a - b).max() <= 1e-8 * max(1.0, np.abs(b).max())


def test_planted_index_mistakes_are_caught():
    n = 7
    z = _grid(n, 30.0)
    e, r = _poles(3, 7, span=5.0)
    f = _f_poles(e, r, z)
    w = np.linspace(-8, 8, 51) + 0.2j
    ref = _f_poles(e, r, w)
    a = op.coefficients(z, f)
    good = op.evaluate(z, a, w)
    assert np.abs(good - ref).max() / np.abs(ref).max() < 1e-7
    # evaluation shifted by one node: (w - z_n) in place of (w - z_{n-1})
    t = np.ones_like(w)
    for k in range(n - 1, 0, -1):
        t = 1.0 + a[k] * (w - z[k]) / t
    assert np.abs(a[0] / t - ref).max() / np.abs(ref).max() > 1e-3
    # coefficients from the unreduced values (g_n(z_n) replaced by f_n)
    assert np.abs(op.evaluate(z, f, w) - ref).max() / np.abs(ref).max() > 1e-3


def test_batched_shapes():
    z = _grid(5)
    f = np.random.default_rng(1).standard_normal((3, 4, 5)) + 0j
    w = np.linspace(-1, 1, 6) + 0.1j
    out = op.continue_to(z, f, w)
    assert out.shape == (3, 4, 6)
    assert np.allclose(out[2, 1], op.continue_to(z, f[2, 1], w))


# ---------------------------------------------------------------------------
# The recursion against exact rational arithmetic.  The inputs are FP64
# numbers, hence exact rationals; the recursion of Eqs. (73)-(74) run in
# fractions.Fraction gives the exact coefficients, which the FP64 oracle must
# reproduce to its rounding error.  Generic (non-rational) data keep every
# level well conditioned, so this holds for every point count up to 32.
# ---------------------------------------------------------------------------

def _exact_coefficients(z, f):
    from fractions import Fraction as Fr

    def cx(c):
        return (Fr(float(c.real)), Fr(float(c.imag)))

    def sub(a, b):
        return (a[0] - b[0], a[1] - b[1])

    def mul(a, b):
        return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])

    def div(a, b):
        d = b[0] * b[0] + b[1] * b[1]
        return ((a[0] * b[0] + a[1] * b[1]) / d, (a[1] * b[0] - a[0] * b[1]) / d)

    zz = [cx(c) for c in z]
    g = [cx(c) for c in f]
    n = len(zz)
    a = [g[0]]
    for k in range(1, n):
        prev = g[k - 1]
        for j in range(k, n):
            den = mul(sub(zz[j], zz[k - 1]), g[j])
            g[j] = (Fr(0), Fr(0)) if den == (0, 0) else div(sub(prev, g[j]), den)
        a.append(g[k])
    return np.array([complex(float(c[0]), float(c[1])) for c in a])


@pytest.mark.parametrize("n", [13, 16, 20, 24, 32])
def test_coefficients_match_exact_rational_arithmetic(n):
    rng = np.random.default_rng(700 + n)
    z = 1j * np.exp(np.linspace(np.log(0.05), np.log(30.0), n))
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    exact = _exact_coefficients(z, f)
    got = op.coefficients(z, f)
    err = np.abs(got - exact) / np.abs(exact)
    assert err.max() <= 1e-12
