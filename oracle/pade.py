"""CPU FP64 oracle for the analytic continuation by Thiele's reciprocal
differences.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The library's compute
path never calls it and shares no code with it.

What is computed (space-time GW, Liu, Kaltak, Klimes, Kresse,
arXiv:1607.02859, Sec. II.E.1, Eqs. (72)-(74)), for a
function known at N complex points (z_j, f_j), j = 1..N (the diagonal
self-energy at the imaginary frequencies i omega_k):

1. The coefficients by the reciprocal-difference recursion (Eqs. (73)-(74)):
       g_1(z_j) = f_j,
       g_n(z)   = (g_{n-1}(z_{n-1}) - g_{n-1}(z)) / ((z - z_{n-1}) g_{n-1}(z)),  n >= 2,
       a_n      = g_n(z_n).
2. The N-point continued fraction of Eq. (72),
       P_N(z) = a_1 / (1 + a_2 (z - z_1) / (1 + ... a_N (z - z_{N-1}) / 1)).
   Reading: the tail (z - z_N) g_{N+1}(z) of the last denominator, which
   would make the fraction exact for the function itself, is dropped; the
   approximant ends with 1.  It is evaluated from the innermost level out.
   Reading: a reciprocal difference whose denominator is exactly zero (the
   function is already represented by fewer levels, e.g. a constant) is
   taken as 0, which ends the fraction there (the paper does not treat
   this breakdown).

Everything is plain Python/NumPy complex128.  Pins
(tests/test_oracle_pade_pins.py): the interpolation property P_N(z_j) = f_j
the paper states, exactness for rational functions that an N-point Thiele
fraction represents (a constant, one pole, a sum of poles with N >= 2M + 1
points), agreement with a brute-force rational interpolant obtained by a
linear solve, and planted index mistakes that fail them.  Parity unpinned:
none.
"""
from __future__ import annotations

import numpy as np

__all__ = ["coefficients", "evaluate", "continue_to"]


def coefficients(z, f) -> np.ndarray:
    """a_1..a_N of Eqs. (73)-(74) for points z[N] and values f[..., N]."""
    z = np.asarray(z, dtype=np.complex128)
    f = np.asarray(f, dtype=np.complex128)
    n = z.shape[0]
    g = f.copy()                                   # g[..., j] = g_n(z_j), updated in n
    a = np.empty_like(f)
    a[..., 0] = g[..., 0]
    for k in range(1, n):                          # level n = k + 1
        prev = g[..., k - 1].copy()                # g_{n-1}(z_{n-1}) = a_{n-1}
        for j in range(k, n):
            den = (z[j] - z[k - 1]) * g[..., j]
            # an exactly zero denominator ends the fraction: the difference
            # (and every deeper one) is taken as 0
            safe = np.where(den == 0, 1.0, den)
            g[..., j] = np.where(den == 0, 0.0, (prev - g[..., j]) / safe)
        a[..., k] = g[..., k]
    return a


def evaluate(z, a, w) -> np.ndarray:
    """P_N(w) of Eq. (72) (last denominator 1) for coefficients a[..., N] at
    points w[M]; returns [..., M]."""
    z = np.asarray(z, dtype=np.complex128)
    a = np.asarray(a, dtype=np.complex128)
    w = np.asarray(w, dtype=np.complex128)
    n = z.shape[0]
    t = np.ones(a.shape[:-1] + w.shape, dtype=np.complex128)
    for k in range(n - 1, 0, -1):                  # levels N .. 2, innermost first
        t = 1.0 + a[..., k, None] * (w - z[k - 1]) / t
    return a[..., 0, None] / t


def continue_to(z, f, w) -> np.ndarray:
    """Coefficients from (z, f), then P_N at w."""
    return evaluate(z, coefficients(z, f), w)
