"""Seeded synthetic inputs for the imaginary-time polarizability build.

This module only *prepares inputs*: orbitals, eigenvalues, the plane-wave
sphere, the imaginary time/frequency grids and the cosine-transform
coefficients.  It holds none of the polarizability arithmetic (no Green's
functions, no products, no FFT of chi, no transform of chi), so both the
GPU path and the CPU oracle can draw their inputs from it.

Workload shapes follow the space-time GW method of Liu, Kaltak, Klimes and
Kresse (arXiv:1607.02859):

* orbitals on a real-space grid, occupied below and unoccupied above the
  Fermi level, which sits at zero (Sec. II.A.1, the text after Eqs. (1)-(2));
* a response cutoff sphere of plane waves (Sec. II.C step (i), the cutoff
  sphere after Eqs. (43)-(44));
* a small nonuniform time/frequency grid (Sec. II.A.2) with cosine and sine
  coefficients obtained by minimising the maximum of the error functions of
  Eqs. (5) and (8) over a range of transition energies (Sec. II.A.3), from
  the ``minimax`` module of this package.

The physical orbitals of the paper are not available; the stand-ins here are
seeded Gaussian columns orthonormalised by QR.  They fix only shapes, value
ranges and conditioning.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import List, Optional, Sequence

import numpy as np

from . import minimax

__all__ = [
    "Item",
    "g_sphere",
    "ct_grid",
    "make_item",
    "make_config",
    "CONFIGS",
    "algorithmic_flops",
    "WItem",
    "coulomb_sqrt",
    "make_w_item",
    "make_pade_input",
    "st_fit",
    "gauss_legendre_st",
    "SigmaItem",
    "make_sigma_item",
]


@dataclasses.dataclass
class Item:
    """One independent polarizability problem (one k-point or one system).

    Arrays use the C-ABI layout: orbitals band-major ``[band][r]`` (complex
    arrays are interleaved re/im in memory), ``ct`` row-major ``[k][j]``.
    """

    n: tuple                 # FFT grid (n0, n1, n2); r = (i0*n1 + i1)*n2 + i2
    phi_occ: np.ndarray      # (n_occ, N_r) float64 or complex128
    phi_unocc: np.ndarray    # (n_unocc, N_r)
    eps_occ: np.ndarray      # (n_occ,) eV
    eps_unocc: np.ndarray    # (n_unocc,) eV
    mu: float                # eV, strictly inside the gap
    tau: np.ndarray          # (n_tau,) eV^-1, > 0
    omega: np.ndarray        # (n_omega,) eV (kept for reporting; the build uses ct)
    ct: np.ndarray           # (n_omega, n_tau): gamma_kj * cos(omega_k tau_j)
    g_index: np.ndarray      # (n_g,) int32 flat FFT indices, output order

    @property
    def n_r(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def is_complex(self) -> bool:
        return np.iscomplexobj(self.phi_occ)

    @property
    def n_occ(self) -> int:
        return self.phi_occ.shape[0]

    @property
    def n_unocc(self) -> int:
        return self.phi_unocc.shape[0]

    @property
    def n_tau(self) -> int:
        return self.tau.shape[0]

    @property
    def n_omega(self) -> int:
        return self.ct.shape[0]

    @property
    def n_g(self) -> int:
        return self.g_index.shape[0]


# ----------------------------------------------------------------------------
# Plane-wave sphere
# ----------------------------------------------------------------------------

def g_sphere(n: Sequence[int], frac2: float = 5.0 / 36.0) -> np.ndarray:
    """Flat FFT indices of the plane waves m with |m|^2 <= floor(frac2 * n^2).

    Integer vectors m lie in the open box (-n/2, n/2) per axis, so no vector
    sits on a Nyquist plane.  Ordering is by (|m|^2, m0, m1, m2).  For a cubic
    grid this gives 389 / 895 / 1309 / 1743 / 2969 / 4729 / 7123 plane waves
    at n = 12 / 16 / 18 / 20 / 24 / 28 / 32, about 22 % of the grid.
    """
    n0, n1, n2 = (int(v) for v in n)
    nmin = min(n0, n1, n2)
    cut = math.floor(frac2 * nmin * nmin)

    def rng(nd):
        h = (nd - 1) // 2
        return np.arange(-h, h + 1)

    m0, m1, m2 = np.meshgrid(rng(n0), rng(n1), rng(n2), indexing="ij")
    m0, m1, m2 = m0.ravel(), m1.ravel(), m2.ravel()
    q = m0 * m0 + m1 * m1 + m2 * m2
    keep = q <= cut
    m0, m1, m2, q = m0[keep], m1[keep], m2[keep], q[keep]
    order = np.lexsort((m2, m1, m0, q))
    m0, m1, m2 = m0[order], m1[order], m2[order]
    flat = ((m0 % n0) * n1 + (m1 % n1)) * n2 + (m2 % n2)
    return flat.astype(np.int32)


# ----------------------------------------------------------------------------
# Time / frequency grid and cosine-transform coefficients
# ----------------------------------------------------------------------------

def ct_grid(n_tau: int, x_min: float, x_max: float):
    """Nonuniform tau/omega grids and cosine coefficients for transition
    energies x in [x_min, x_max] (eV): the grid of ``minimax.minimax_grid``
    (omega_k log-spaced in [x_min/2, x_max], tau_j from a three-parameter
    log-spaced family) with the minimax coefficients of Eq. (5) under an
    amplification bound.  Returns (tau, omega, ct, max relative fit error)
    with ct of shape (n_omega, n_tau)."""
    g = minimax.minimax_grid(int(n_tau), float(x_min), float(x_max))
    return g.tau, g.omega, g.ct, g.err_cos


def st_fit(tau: np.ndarray, omega: np.ndarray, x_min: float, x_max: float):
    """Sine-transform coefficients st[k][j] = lambda_kj sin(omega_k tau_j) on a
    given tau/omega grid: the minimax coefficients of Eq. (8) under the same
    amplification bound as the cosine ones.  Returns (st, max relative fit
    error).  On the grids of ``ct_grid`` this equals ``minimax_grid(...).st``."""
    g = minimax.minimax_grid(len(tau), float(x_min), float(x_max))
    if np.array_equal(g.tau, np.asarray(tau)) and np.array_equal(g.omega, np.asarray(omega)):
        return g.st, g.err_sin
    return minimax.fit_transform(np.asarray(tau, float), np.asarray(omega, float), "sin",
                                 float(x_min), float(x_max))


def gauss_legendre_st(omega: np.ndarray, t_max: float, panel: float = 0.1, nodes: int = 8):
    """Dense-quadrature sine coefficients on the nodes of ``gauss_legendre_ct``:
    st[k][j] = 2 w_j sin(omega_k tau_j), so that sum_j st[k][j] exp(-x tau_j) ->
    2 int_0^inf sin(omega tau) exp(-x tau) dtau = 2 omega/(x^2 + omega^2), the
    closed form under the brace of Eq. (8)."""
    n_pan = int(math.ceil(t_max / panel))
    h = t_max / n_pan
    xg, wg = np.polynomial.legendre.leggauss(nodes)
    left = np.arange(n_pan) * h
    tau = (left[:, None] + (xg[None, :] + 1.0) * 0.5 * h).ravel()
    w = np.tile(wg * 0.5 * h, n_pan)
    st = 2.0 * w[None, :] * np.sin(np.outer(omega, tau))
    return tau, st


def gauss_legendre_ct(omega: np.ndarray, t_max: float, panel: float = 0.1, nodes: int = 8):
    """Dense-quadrature cosine coefficients for the Laplace-identity check.

    Composite Gauss-Legendre rule on [0, t_max] with panels of width <= panel
    and ``nodes`` nodes each: ct[k][j] = 2 w_j cos(omega_k tau_j), so that
    sum_j ct[k][j] exp(-x tau_j) -> 2 int_0^inf cos(omega tau) exp(-x tau) dtau
    = 2x/(x^2+omega^2), the closed form under the brace of Eq. (5).
    """
    n_pan = int(math.ceil(t_max / panel))
    h = t_max / n_pan
    xg, wg = np.polynomial.legendre.leggauss(nodes)
    left = np.arange(n_pan) * h
    tau = (left[:, None] + (xg[None, :] + 1.0) * 0.5 * h).ravel()
    w = np.tile(wg * 0.5 * h, n_pan)
    ct = 2.0 * w[None, :] * np.cos(np.outer(omega, tau))
    return tau, ct


# ----------------------------------------------------------------------------
# Items and configurations
# ----------------------------------------------------------------------------

def _orbitals(rng, n_r, k, cplx):
    a = rng.standard_normal((n_r, k))
    if cplx:
        a = a + 1j * rng.standard_normal((n_r, k))
    q, _ = np.linalg.qr(a, mode="reduced")
    return np.ascontiguousarray(q.T)


def make_item(seed, n, n_occ, n_unocc, cplx, n_tau, *, gap=1.0, x_min=None,
              eps_lo=-15.0, eps_hi=60.0, x_max=75.0, mu=0.0, n_g=None, ct=None) -> Item:
    """One seeded item.

    Eigenvalues: occupied uniform in [eps_lo, -gap/2], unoccupied uniform in
    [gap/2, eps_hi], sorted, then shifted by mu.  The tau/omega grid covers
    transition energies [x_min, x_max] (x_min defaults to the gap).
    """
    rng = np.random.default_rng(seed)
    n = tuple(int(v) for v in n)
    n_r = n[0] * n[1] * n[2]
    phi = _orbitals(rng, n_r, n_occ + n_unocc, cplx)
    eps_o = np.sort(rng.uniform(eps_lo, -gap / 2.0, n_occ))
    eps_u = np.sort(rng.uniform(gap / 2.0, eps_hi, n_unocc))
    if ct is None:
        tau, omega, ctm, _ = ct_grid(n_tau, gap if x_min is None else x_min, x_max)
    else:
        tau, omega, ctm = ct
    g = g_sphere(n)
    if n_g is not None:
        g = g[:n_g]
    return Item(n=n, phi_occ=np.ascontiguousarray(phi[:n_occ]),
                phi_unocc=np.ascontiguousarray(phi[n_occ:]),
                eps_occ=eps_o + mu, eps_unocc=eps_u + mu, mu=float(mu),
                tau=np.asarray(tau, float), omega=np.asarray(omega, float),
                ct=np.ascontiguousarray(ctm, dtype=float), g_index=g)


def _cfg5_system(s):
    n = [16, 18, 20, 24, 28][(5 * s) // 32]
    n_o = 16 + int(round(80 * s / 31))
    return n, n_o, 16 * n_o, 0.1 * 100.0 ** ((s % 8) / 7.0)


CONFIGS = {
    # id: description used in reports
    1: "gamma-only real, 12^3, 16+112 bands, 6 tau",
    2: "gamma-only complex, 24^3, 64+960 bands, 12 tau, 2048-column slabs",
    3: "8 k-points, 24^3 complex, occ 48-64 / unocc 700-1000, 16 tau",
    4: "32^3 complex, 128+2048 bands, 16 tau",
    5: "32 real systems, 16^3-28^3, 16/256-96/1536 bands, gaps 0.1-10 eV, 20 tau",
}


def make_config(cfg: int, *, scale: Optional[float] = None) -> List[Item]:
    """The items of a workload configuration, seeded by (cfg, item).

    ``scale`` is not used to shrink anything silently: callers that want a
    small variant build it with :func:`make_item` directly.
    """
    if cfg == 1:
        return [make_item([1, 0], (12, 12, 12), 16, 112, False, 6, x_min=0.5)]
    if cfg == 2:
        return [make_item([2, 0], (24, 24, 24), 64, 960, True, 12, x_min=0.5)]
    if cfg == 3:
        out = []
        rng = np.random.default_rng([3, 99])
        occ = rng.integers(48, 65, 8)
        unocc = rng.integers(700, 1001, 8)
        for k in range(8):
            out.append(make_item([3, k], (24, 24, 24), int(occ[k]), int(unocc[k]), True, 16,
                                 x_min=0.5))
        return out
    if cfg == 4:
        return [make_item([4, 0], (32, 32, 32), 128, 2048, True, 16, x_min=0.5)]
    if cfg == 5:
        out = []
        for s in range(32):
            n, n_o, n_u, gap = _cfg5_system(s)
            out.append(make_item([5, s], (n, n, n), n_o, n_u, False, 20, gap=gap))
        return out
    raise ValueError(f"unknown configuration {cfg}")


def algorithmic_flops(item: Item) -> float:
    """Flops per build the method must spend on the band contractions,
    counting the full N_r x N_r square: 8 N_r^2 K per tau (complex) or
    2 N_r^2 K (real), K = n_occ + n_unocc."""
    per = 8.0 if item.is_complex else 2.0
    return per * item.n_r ** 2 * (item.n_occ + item.n_unocc) * item.n_tau


# ----------------------------------------------------------------------------
# Inputs of the screened-interaction step (W~ from chi)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class WItem:
    """One screened-interaction problem: chi(G, G', i omega_k) of one k-point,
    the square root of the Coulomb kernel per plane wave and the forward
    cosine matrix of the same grid (``ct[k][j]``, square)."""

    chi: np.ndarray          # (n_omega, n_g, n_g) complex128, Hermitian negative semidefinite
    sqrt_v: np.ndarray       # (n_g,) float64, >= 0
    ct: np.ndarray           # (n_omega, n_tau) float64, n_tau == n_omega
    omega: np.ndarray        # (n_omega,)

    @property
    def n_g(self) -> int:
        return self.chi.shape[1]

    @property
    def n_omega(self) -> int:
        return self.chi.shape[0]

    @property
    def n_tau(self) -> int:
        return self.ct.shape[1]


def coulomb_sqrt(n: Sequence[int], g_index: np.ndarray, alpha: float = 1.0,
                 k: Sequence[float] = (0.0, 0.0, 0.0)) -> np.ndarray:
    """alpha / |k + m| per plane wave, m the integer vector of the flat FFT index
    (cubic cell in units where the reciprocal lattice vectors are unit
    vectors), and 0 where k + m = 0 (the G = 0 term at k = 0 is dropped)."""
    n0, n1, n2 = (int(v) for v in n)
    g = np.asarray(g_index, dtype=np.int64)
    k0, rem = np.divmod(g, n1 * n2)
    k1, k2 = np.divmod(rem, n2)

    def signed(kd, nd):
        return np.where(kd > nd // 2, kd - nd, kd).astype(np.float64)

    q = np.stack([signed(k0, n0) + k[0], signed(k1, n1) + k[1], signed(k2, n2) + k[2]], axis=1)
    norm = np.sqrt((q * q).sum(axis=1))
    out = np.zeros(g.shape[0])
    nz = norm > 0
    out[nz] = alpha / norm[nz]
    return out


def make_w_item(seed, n, n_tau, *, rank=None, strength=1.0, alpha=1.0,
                x_min=0.5, x_max=50.0, n_g=None, k=(0.0, 0.0, 0.0)) -> WItem:
    """Seeded chi(i omega_k) of the shape the polarizability build returns:
    Hermitian, negative semidefinite, decaying with omega.  It is a sum of
    ``rank`` (default n_g / 4) rank-one terms -b_m b_m^H with Lorentzian weights
    x_m^2 / (x_m^2 + omega_k^2), x_m log-spaced in [x_min, x_max]; the plane
    waves are the sphere of grid ``n`` (its first ``n_g`` when given) and
    ``sqrt_v`` is ``coulomb_sqrt`` at ``k``.  ``strength`` scales chi; the
    dielectric matrix stays positive definite for any strength >= 0."""
    g_index = g_sphere(n)
    if n_g is not None:
        g_index = g_index[:int(n_g)]
    n_g = g_index.shape[0]
    rank = max(1, n_g // 4) if rank is None else int(rank)
    rng = np.random.default_rng(seed)
    tau, omega, ct, _ = ct_grid(n_tau, x_min, x_max)
    b = (rng.standard_normal((n_g, rank)) + 1j * rng.standard_normal((n_g, rank))) / math.sqrt(2.0 * n_g)
    x = np.exp(np.linspace(math.log(x_min), math.log(x_max), rank))
    chi = np.empty((omega.shape[0], n_g, n_g), dtype=np.complex128)
    for kk, w in enumerate(omega):
        lw = strength * x * x / (x * x + w * w)
        chi[kk] = -(b * lw[None, :]) @ b.conj().T
        chi[kk] = 0.5 * (chi[kk] + chi[kk].conj().T)
    return WItem(chi=chi, sqrt_v=coulomb_sqrt(n, g_index, alpha, k), ct=ct, omega=omega)


# ----------------------------------------------------------------------------
# Inputs of the analytic continuation
# ----------------------------------------------------------------------------

def make_pade_input(seed, n_fun, n_points, n_eval, *, n_poles=4, span=5.0, eta=0.05,
                    w_max=30.0):
    """Seeded functions of the shape of diagonal self-energies on the
    imaginary axis: f(z) = c + sum_p r_p / (z - e_p) with n_poles poles per
    function, e_p with real parts in [-span, span] eV and imaginary parts of
    the sign that keeps f analytic in the upper half plane (a retarded
    function), residues of order one, c real.  z_j = i omega_j with omega_j
    log-spaced in [0.05, w_max] eV; the evaluation points are a real
    frequency grid in [-2 span, 2 span] shifted by i eta.
    Returns (z [N], f [n_fun][N], w [M], e [n_fun][P], r [n_fun][P], c [n_fun])."""
    rng = np.random.default_rng(seed)
    z = 1j * np.exp(np.linspace(math.log(0.05), math.log(w_max), n_points))
    e = rng.uniform(-span, span, (n_fun, n_poles)) - 1j * rng.uniform(0.05, 0.5, (n_fun, n_poles))
    r = rng.uniform(0.1, 1.5, (n_fun, n_poles)) * np.exp(1j * rng.uniform(-0.2, 0.2, (n_fun, n_poles)))
    c = rng.uniform(-2.0, 2.0, n_fun)
    f = c[:, None] + (r[:, None, :] / (z[None, :, None] - e[:, None, :])).sum(axis=2)
    w = np.linspace(-2 * span, 2 * span, n_eval) + 1j * eta
    return z, f.astype(np.complex128), w, e, r, c


# ----------------------------------------------------------------------------
# Inputs of the self-energy step
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class SigmaItem:
    """One self-energy problem at the Gamma point: orbitals and eigenvalues as
    for the polarizability, the tau/omega grid with its cosine (ct) and sine
    (st) coefficients, the correlated screened interaction W~(G, G', i tau_j)
    on the plane-wave list, and the states whose diagonal elements are wanted
    (index b < n_occ: occupied band b; otherwise unoccupied band b - n_occ)."""

    n: tuple
    phi_occ: np.ndarray      # (n_occ, N_r) complex128
    phi_unocc: np.ndarray    # (n_unocc, N_r)
    eps_occ: np.ndarray
    eps_unocc: np.ndarray
    mu: float
    tau: np.ndarray          # (n_tau,)
    omega: np.ndarray        # (n_omega,)
    ct: np.ndarray           # (n_omega, n_tau)
    st: np.ndarray           # (n_omega, n_tau)
    g_index: np.ndarray      # (n_g,) int32
    w_tau: np.ndarray        # (n_tau, n_g, n_g) complex128, Hermitian per tau
    states: np.ndarray       # (n_states,) int32

    @property
    def n_r(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def n_occ(self) -> int:
        return self.phi_occ.shape[0]

    @property
    def n_unocc(self) -> int:
        return self.phi_unocc.shape[0]

    @property
    def n_tau(self) -> int:
        return self.tau.shape[0]

    @property
    def n_omega(self) -> int:
        return self.ct.shape[0]

    @property
    def n_g(self) -> int:
        return self.g_index.shape[0]

    @property
    def n_states(self) -> int:
        return self.states.shape[0]


def make_sigma_item(seed, n, n_occ, n_unocc, n_tau, n_states, *, gap=1.0, x_min=0.5,
                    x_max=75.0, n_g=None, rank=None, strength=1.0) -> SigmaItem:
    """One seeded self-energy item with complex orbitals.

    Orbitals, eigenvalues, grid and cosine coefficients are those of
    ``make_item``; the sine coefficients are the grid's minimax ones (Eq. (8)).
    The screened interaction is a Hermitian, negative semidefinite stand-in
    that decays in tau like the correlated interaction:
        W~(i tau_j) = -strength sum_m exp(-x_m tau_j) b_m b_m^H,
    ``rank`` terms (default n_g / 4), b_m complex Gaussian over the plane waves
    (variance 1/n_g), x_m log-spaced in [x_min, x_max].  The states are the
    n_states bands nearest the gap, half below and half above it."""
    it = make_item(seed, n, n_occ, n_unocc, True, n_tau, gap=gap, x_min=x_min, x_max=x_max,
                   n_g=n_g)
    st = minimax.minimax_grid(n_tau, x_min, x_max).st
    rng = np.random.default_rng([seed, 77])
    g = it.g_index.shape[0]
    rank = max(1, g // 4) if rank is None else int(rank)
    b = (rng.standard_normal((g, rank)) + 1j * rng.standard_normal((g, rank))) / math.sqrt(2.0 * g)
    x = np.exp(np.linspace(math.log(x_min), math.log(x_max), rank))
    w = np.empty((it.tau.shape[0], g, g), dtype=np.complex128)
    for j, t in enumerate(it.tau):
        w[j] = -(b * (strength * np.exp(-x * t))[None, :]) @ b.conj().T
        w[j] = 0.5 * (w[j] + w[j].conj().T)
    n_below = min(n_occ, (n_states + 1) // 2)
    n_above = min(n_unocc, n_states - n_below)
    states = np.concatenate([np.arange(n_occ - n_below, n_occ),
                             np.arange(n_occ, n_occ + n_above)]).astype(np.int32)
    return SigmaItem(n=it.n, phi_occ=it.phi_occ, phi_unocc=it.phi_unocc, eps_occ=it.eps_occ,
                     eps_unocc=it.eps_unocc, mu=it.mu, tau=it.tau, omega=it.omega, ct=it.ct,
                     st=np.ascontiguousarray(st), g_index=it.g_index, w_tau=w, states=states)
