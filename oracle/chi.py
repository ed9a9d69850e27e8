"""CPU FP64 oracle for the imaginary-time polarizability build.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The library's compute
path never calls it and shares no code with it.

What is computed (space-time GW, Liu, Kaltak, Klimes, Kresse,
arXiv:1607.02859), for one item and every imaginary time tau_j:

1. Weights of the Green's functions (Sec. II.A.1, Eqs. (1)-(2) with the
   Fermi level mu; the product of the two weights is the time dependence
   xi_ia(tau) = exp(-(eps_a - eps_i) tau) stated under Eq. (16)):
       w_i = exp((eps_i - mu) tau_j),   w_a = exp(-(eps_a - mu) tau_j).
2. Green's functions on the real-space grid, as dense band sums:
       G_occ(r, r')   = sum_i w_i phi_i(r) conj(phi_i(r'))
       G_unocc(r, r') = sum_a w_a phi_a(r) conj(phi_a(r')).
3. Pointwise product in real space and imaginary time (Eqs. (14)-(15)):
       chi(r, r') = -G_occ(r, r') * conj(G_unocc(r, r')).
   This is the tau < 0 branch of Eq. (15) (obtained there by exchanging the
   occupied and unoccupied functions); for real orbitals both branches
   coincide.
4. Spatial transform of both indices (Sec. II.C step (i), Eqs. (43)-(44)):
       chi(G, r')  = sum_r  exp(-i G.r)  chi(r, r')     (first index)
       chi(G, G')  = sum_r' chi(G, r') exp(+i G'.r')    (second index)
   with r on the integer grid (i0/n0, i1/n1, i2/n2) and G restricted to the
   caller's plane-wave list (flat FFT indices in output order).  No 1/N_r,
   volume or spin factor.
5. Cosine transform to imaginary frequency (Eq. (4) applied as in Eq. (45)):
       chi(G, G', i omega_k) = sum_j ct[k][j] chi(G, G', i tau_j),
   ct[k][j] = gamma_kj cos(omega_k tau_j), summed in FP64 in increasing j.

Also here, for pinning the above:

* ``chi_pairsum`` -- the reciprocal-space pair sum of Eq. (16) (Adler-Wiser
  form) with the time dependence integrated by the same cosine transform:
  chi(G,G',i w_k) = -sum_ia c_k(eps_a - eps_i) rho_ia(G) conj(rho_ia(G')),
  rho_ia(G) = sum_r exp(-i G.r) phi_i(r) conj(phi_a(r)),
  c_k(x) = sum_j ct[k][j] exp(-x tau_j).
* ``chi_rows`` -- selected rows of the same pair sum, evaluated through one
  FFT over r' per row, so that large grids can be checked on samples.
* ``chi_laplace`` -- the closed form reached when the cosine coefficients
  integrate exactly: c_k(x) -> 2x/(x^2 + omega_k^2), the integral under the
  brace of Eq. (5).

Every routine is plain NumPy/SciPy in FP64.  Parity unpinned: none.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft

__all__ = [
    "validate",
    "weights",
    "chi_tau",
    "chi_omega",
    "chi_pairsum",
    "chi_rows",
    "chi_laplace",
    "pair_densities",
    "kappa_F",
    "rel_frobenius",
]

# FFT threads: the process's thread budget when one is set, else every core
_WORKERS = max(1, int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1)


def _phi(item, which):
    return item.phi_occ if which == "o" else item.phi_unocc


def validate(item) -> None:
    """Reject inputs the method is not defined for (raises ValueError).

    The Fermi level must lie strictly between the occupied and unoccupied
    eigenvalues (Sec. II.A.1); imaginary times are positive; the plane-wave
    list holds distinct in-range flat indices.
    """
    n_r = int(np.prod(item.n))
    if any(int(v) <= 0 for v in item.n):
        raise ValueError("grid size must be positive")
    if item.phi_occ.shape[0] < 1 or item.phi_unocc.shape[0] < 1:
        raise ValueError("need at least one occupied and one unoccupied band")
    if item.phi_occ.shape[1] != n_r or item.phi_unocc.shape[1] != n_r:
        raise ValueError("orbital length != grid size")
    for a in (item.phi_occ, item.phi_unocc, item.eps_occ, item.eps_unocc, item.tau, item.ct):
        if not np.all(np.isfinite(a)):
            raise ValueError("non-finite input")
    if not math.isfinite(item.mu):
        raise ValueError("non-finite mu")
    if not (item.eps_occ.max() < item.mu < item.eps_unocc.min()):
        raise ValueError("mu must lie strictly inside the gap")
    if np.any(item.tau <= 0):
        raise ValueError("tau must be positive")
    g = np.asarray(item.g_index)
    if g.size < 1 or g.min() < 0 or g.max() >= n_r or np.unique(g).size != g.size:
        raise ValueError("g_index out of range or duplicated")
    if item.ct.shape[1] != item.tau.shape[0]:
        raise ValueError("ct must be n_omega x n_tau")


def weights(item, tau):
    """Step 1: w_i = exp((eps_i - mu) tau), w_a = exp(-(eps_a - mu) tau)."""
    w_o = np.exp((item.eps_occ - item.mu) * tau)
    w_u = np.exp(-(item.eps_unocc - item.mu) * tau)
    return w_o, w_u


def chi_tau(item, j, slab=2048):
    """Steps 1-4 for one imaginary time tau_j: chi(G, G', i tau_j), complex128
    of shape (n_g, n_g).  The r' index is processed in slabs of ``slab``
    columns so that the N_r x N_r matrices never exist whole."""
    n0, n1, n2 = (int(v) for v in item.n)
    n_r = n0 * n1 * n2
    g = np.asarray(item.g_index, dtype=np.int64)
    w_o, w_u = weights(item, float(item.tau[j]))
    phi_o = item.phi_occ.astype(np.complex128)
    phi_u = item.phi_unocc.astype(np.complex128)
    # step 2 operands: rows r, columns bands
    a_o = phi_o.T * w_o[None, :]
    a_u = phi_u.T * w_u[None, :]
    chi_gr = np.empty((g.size, n_r), dtype=np.complex128)
    for s in range(0, n_r, slab):
        e = min(n_r, s + slab)
        g_o = a_o @ phi_o[:, s:e].conj()          # G_occ(r, r' in slab)
        g_u = a_u @ phi_u[:, s:e].conj()          # G_unocc(r, r' in slab)
        chi = -g_o * g_u.conj()                   # step 3
        cube = chi.reshape(n0, n1, n2, e - s)
        f = sfft.fftn(cube, axes=(0, 1, 2), workers=_WORKERS)   # exp(-i G.r)
        chi_gr[:, s:e] = f.reshape(n_r, e - s)[g, :]
    cube = chi_gr.reshape(g.size, n0, n1, n2)
    # sum_r' exp(+i G'.r') = N_r * inverse DFT
    f = sfft.ifftn(cube, axes=(1, 2, 3), workers=_WORKERS) * n_r
    return f.reshape(g.size, n_r)[:, g]


def chi_omega(item, slab=2048, return_tau=False):
    """Steps 1-5: chi(G, G', i omega_k), complex128 (n_omega, n_g, n_g)."""
    validate(item)
    xs = [chi_tau(item, j, slab) for j in range(item.n_tau)]
    out = np.zeros((item.n_omega, item.n_g, item.n_g), dtype=np.complex128)
    for k in range(item.n_omega):
        for j in range(item.n_tau):          # increasing j
            out[k] += item.ct[k, j] * xs[j]
    if return_tau:
        return out, np.stack(xs)
    return out


def pair_densities(item):
    """rho_ia(G) = sum_r exp(-i G.r) phi_i(r) conj(phi_a(r)) for all pairs,
    complex128 of shape (n_occ, n_unocc, n_g) (the matrix elements of
    Eq. (16))."""
    n0, n1, n2 = (int(v) for v in item.n)
    g = np.asarray(item.g_index, dtype=np.int64)
    out = np.empty((item.n_occ, item.n_unocc, g.size), dtype=np.complex128)
    for i in range(item.n_occ):
        prod = item.phi_occ[i][None, :] * item.phi_unocc.conj()
        f = sfft.fftn(prod.reshape(item.n_unocc, n0, n1, n2), axes=(1, 2, 3), workers=_WORKERS)
        out[i] = f.reshape(item.n_unocc, -1)[:, g]
    return out


def _ck(item, x):
    """c_k(x) = sum_j ct[k][j] exp(-x tau_j): the cosine transform of the pair
    time dependence exp(-x tau), shape (n_omega,) + x.shape."""
    e = np.exp(-np.multiply.outer(x, item.tau))          # x.shape + (n_tau,)
    return np.moveaxis(e @ item.ct.T, -1, 0)


def chi_pairsum(item):
    """Brute-force pair sum of Eq. (16), transformed by the same cosine
    coefficients: chi(i w_k) = -sum_ia c_k(eps_a - eps_i) rho_ia rho_ia^H."""
    validate(item)
    rho = pair_densities(item).reshape(-1, item.n_g)
    x = (item.eps_unocc[None, :] - item.eps_occ[:, None]).ravel()
    ck = _ck(item, x)                                      # (n_omega, P)
    out = np.empty((item.n_omega, item.n_g, item.n_g), dtype=np.complex128)
    for k in range(item.n_omega):
        out[k] = -(rho.T * ck[k][None, :]) @ rho.conj()
    return out


def chi_rows(item, rows):
    """Rows ``rows`` (positions in g_index) of chi(G, G', i omega_k) from the
    pair sum of Eq. (16), shape (n_omega, len(rows), n_g).

    For a fixed row G_s the pair sum is rearranged exactly as
      chi(G_s, G') = sum_r' exp(+i G'.r') [ -sum_ia c_k(eps_a - eps_i)
                       rho_ia(G_s) conj(phi_i(r')) phi_a(r') ],
    one dense contraction and one FFT over r' per (row, omega)."""
    validate(item)
    n0, n1, n2 = (int(v) for v in item.n)
    n_r = n0 * n1 * n2
    g = np.asarray(item.g_index, dtype=np.int64)
    i0, rem = np.divmod(np.arange(n_r), n1 * n2)
    i1, i2 = np.divmod(rem, n2)
    phi_o = item.phi_occ.astype(np.complex128)
    phi_u = item.phi_unocc.astype(np.complex128)
    x = item.eps_unocc[None, :] - item.eps_occ[:, None]
    ck = _ck(item, x)                                       # (n_omega, n_o, n_u)
    out = np.empty((item.n_omega, len(rows), g.size), dtype=np.complex128)
    for s, row in enumerate(rows):
        f = int(g[row])
        k0, rem = divmod(f, n1 * n2)
        k1, k2 = divmod(rem, n2)
        ph = np.exp(-2j * np.pi * (k0 * i0 / n0 + k1 * i1 / n1 + k2 * i2 / n2))
        rho_s = (phi_o * ph[None, :]) @ phi_u.conj().T      # (n_o, n_u)
        for k in range(item.n_omega):
            m = ck[k] * rho_s
            t = m @ phi_u                                   # (n_o, n_r)
            col = -(phi_o.conj() * t).sum(0)                # over i
            fr = sfft.ifftn(col.reshape(n0, n1, n2), workers=_WORKERS).ravel() * n_r
            out[k, s] = fr[g]
    return out


def chi_laplace(item, omega):
    """Closed form of the exact cosine transform:
    chi(i w) = -sum_ia 2x/(x^2 + w^2) rho_ia rho_ia^H, x = eps_a - eps_i."""
    rho = pair_densities(item).reshape(-1, item.n_g)
    x = (item.eps_unocc[None, :] - item.eps_occ[:, None]).ravel()
    out = np.empty((len(omega), item.n_g, item.n_g), dtype=np.complex128)
    for k, w in enumerate(omega):
        c = 2.0 * x / (x * x + w * w)
        out[k] = -(rho.T * c[None, :]) @ rho.conj()
    return out


def kappa_F(item, chi_tau_stack, chi_w):
    """Cosine-transform amplification per omega:
    kappa_F(k) = sum_j |ct[k][j]| ||chi(tau_j)||_F / ||chi(i omega_k)||_F."""
    nt = np.sqrt((np.abs(chi_tau_stack) ** 2).sum(axis=(1, 2)))
    nw = np.sqrt((np.abs(chi_w) ** 2).sum(axis=(1, 2)))
    return (np.abs(item.ct) @ nt) / nw


def rel_frobenius(a, b):
    """max over omega of ||a_k - b_k||_F / ||b_k||_F (b is the reference)."""
    a = np.asarray(a)
    b = np.asarray(b)
    num = np.sqrt((np.abs(a - b) ** 2).reshape(b.shape[0], -1).sum(1))
    den = np.sqrt((np.abs(b) ** 2).reshape(b.shape[0], -1).sum(1))
    return float((num / den).max())
