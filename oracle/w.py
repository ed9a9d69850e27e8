"""CPU FP64 oracle for the screened interaction built from the polarizability.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The library's compute
path never calls it and shares no code with it.

What is computed (space-time GW, Liu, Kaltak, Klimes, Kresse,
arXiv:1607.02859, Sec. II.C steps (iii)-(iv)), for one k-point and every
imaginary frequency omega_k, from chi(G, G', i omega_k):

1. The symmetric bare Coulomb kernel of Eq. (47),
       v(G, G') = s(G) s(G'),   s(G) = sqrt(4 pi e^2) / |k + G|,
   with s supplied by the caller (s = 0 drops a plane wave, e.g. G = 0 at
   k = 0).
2. The symmetric RPA dielectric matrix of Eq. (48), products element by
   element:
       eps(G, G') = delta_GG' - v(G, G') chi(G, G').
3. The screened interaction of Eq. (46), W(G, G') = v(G, G') eps^-1(G, G'),
   and its correlated part of Eq. (49).  Reading: the bare term removed in
   Eq. (49) is the part of W that the delta of Eq. (48) produces, so
       W~(G, G') = v(G, G') (eps^-1(G, G') - delta_GG'),
   which is W - v for the bare Coulomb operator v(G) delta_GG' and satisfies
   the RPA Dyson equation W = v + v chi W (pinned in the tests).
4. The inverse cosine transform of Eq. (50),
       W~(i tau_j) = sum_k xi_jk cos(tau_j omega_k) W~(i omega_k),
   where the matrix xi cos(tau omega) is the inverse of the forward matrix
   gamma cos(omega tau) of Eq. (4) (stated with Eq. (6)); the grids are
   square (N tau points, N frequencies).

The inverse is a library routine (numpy.linalg.inv) used as one step;
``w_tilde_rows`` gives selected rows of the same result through linear solves
(numpy.linalg.solve) for sizes where full inverses on the CPU are slow.
Pins (tests/test_oracle_w_pins.py): the Dyson equation by matrix products
only, the closed form for a diagonal chi, Hermiticity and negative
semidefiniteness of W~(i omega) for a Hermitian negative semidefinite chi,
and the inverse transform against the exact Laplace pair exp(-x tau) <->
2x / (x^2 + omega^2) of Eq. (5).  Parity unpinned: none.
"""
from __future__ import annotations

import numpy as np

__all__ = ["inverse_ct", "coulomb_kernel", "w_tilde_omega", "w_tilde_tau", "w_tilde_rows",
           "w_tilde_omega_rows"]


def inverse_ct(ct: np.ndarray) -> np.ndarray:
    """xi_jk cos(tau_j omega_k) as the inverse of ct[k][j] = gamma_kj cos(omega_k tau_j)
    (Eq. (6), used in Eq. (50)); shape [n_tau][n_omega]."""
    ct = np.asarray(ct, dtype=np.float64)
    if ct.ndim != 2 or ct.shape[0] != ct.shape[1]:
        raise ValueError("the inverse cosine transform needs a square grid")
    return np.linalg.inv(ct)


def coulomb_kernel(s: np.ndarray) -> np.ndarray:
    """v(G, G') = s(G) s(G') of Eq. (47)."""
    s = np.asarray(s, dtype=np.float64)
    return np.outer(s, s)


def w_tilde_omega(chi_w: np.ndarray, s: np.ndarray) -> np.ndarray:
    """W~(G, G', i omega_k) for every k (Eqs. (46)-(49)); chi_w [n_omega][n_g][n_g]."""
    chi_w = np.asarray(chi_w, dtype=np.complex128)
    v = coulomb_kernel(s)
    n_g = v.shape[0]
    eye = np.eye(n_g)
    out = np.empty_like(chi_w)
    for k in range(chi_w.shape[0]):
        eps = eye - v * chi_w[k]                     # Eq. (48)
        w = v * np.linalg.inv(eps)                   # Eq. (46)
        out[k] = w - v * eye                         # Eq. (49), bare part v delta
    return out


def w_tilde_tau(chi_w: np.ndarray, s: np.ndarray, ct: np.ndarray, return_omega=False):
    """W~(G, G', i tau_j) for every j (Eq. (50)) from chi(i omega_k)."""
    w_w = w_tilde_omega(chi_w, s)
    ict = inverse_ct(ct)
    n_tau, n_omega = ict.shape
    if n_omega != w_w.shape[0]:
        raise ValueError("chi has a different number of frequencies than the grid")
    out = np.zeros((n_tau,) + w_w.shape[1:], dtype=np.complex128)
    for j in range(n_tau):
        for k in range(n_omega):                     # summed in increasing k
            out[j] += ict[j, k] * w_w[k]
    return (out, w_w) if return_omega else out


def w_tilde_rows(chi_w: np.ndarray, s: np.ndarray, ct: np.ndarray, rows) -> np.ndarray:
    """Rows ``rows`` of W~(G, G', i tau_j) for every j, shape [n_tau][len(rows)][n_g].

    Row g of eps^-1 is e_g^T eps^-1 = (eps^-T e_g)^T, one linear solve per
    frequency for all selected rows; then Eqs. (46), (49) and (50) as above."""
    chi_w = np.asarray(chi_w, dtype=np.complex128)
    w_w = np.stack([w_tilde_omega_rows(chi_w[k], s, rows) for k in range(chi_w.shape[0])])
    ict = inverse_ct(ct)
    out = np.zeros((ict.shape[0],) + w_w.shape[1:], dtype=np.complex128)
    for j in range(ict.shape[0]):
        for k in range(ict.shape[1]):                               # Eq. (50)
            out[j] += ict[j, k] * w_w[k]
    return out


def w_tilde_omega_rows(chi: np.ndarray, s: np.ndarray, rows) -> np.ndarray:
    """Rows ``rows`` of W~(G, G', i omega) for one frequency (Eqs. (46)-(49));
    row g of eps^-1 is e_g^T eps^-1 = (eps^-T e_g)^T, one linear solve."""
    chi = np.asarray(chi, dtype=np.complex128)
    s = np.asarray(s, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    n_g = s.shape[0]
    v = coulomb_kernel(s)
    e = np.zeros((n_g, rows.shape[0]))
    e[rows, np.arange(rows.shape[0])] = 1.0
    eps = np.eye(n_g) - v * chi                                     # Eq. (48)
    inv_rows = np.linalg.solve(eps.T, e).T                          # rows of eps^-1
    return v[rows] * inv_rows - v[rows] * e.T                       # Eqs. (46), (49)
