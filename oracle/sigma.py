"""CPU FP64 oracle for the correlation self-energy in space and imaginary time.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The library's compute
path never calls it and shares no code with it.

What is computed (space-time GW, Liu, Kaltak, Klimes, Kresse,
arXiv:1607.02859, Sec. II.D), for one Gamma-point item (orbitals on the grid
of one cell, k = 0), every imaginary time tau_j > 0 and every requested state n:

1. The correlated screened interaction in real space from its plane-wave
   matrix, by the two spatial transforms of Eqs. (51)-(52) at k = 0:
       W~(r, G')  = sum_G  exp(+i G.r) W~(G, G', i tau_j),
       W~(r, r')  = sum_G' W~(r, G') exp(-i G'.r').
   No 1/N_r or volume factor (bare sums, as for the polarizability).
2. The Green's functions of Eqs. (1)-(2) at +tau_j (unoccupied) and at
   -tau_j (occupied), with the Fermi level mu:
       Gbar(r, r', i tau)  = -sum_a phi_a(r) conj(phi_a(r')) exp(-(eps_a - mu) tau),
       Gund(r, r', -i tau) = +sum_i phi_i(r) conj(phi_i(r')) exp(+(eps_i - mu) tau).
3. The products in real space and imaginary time (Eq. (53), the plane-wave
   term Sigma^(1) of Eq. (55)), W~ being even in tau (it is obtained by the
   inverse cosine transform of Eq. (50)):
       Sigma_bar(r, r', i tau)  = -Gbar(r, r', i tau)  W~(r, r', i tau),
       Sigma_und(r, r', -i tau) = -Gund(r, r', -i tau) W~(r, r', i tau).
4. Diagonal matrix elements, the first line of Eq. (62):
       Sigma_nn = sum_{r, r'} conj(psi_n(r)) Sigma(r, r') psi_n(r').
5. The even and odd parts of Eqs. (67)-(68):
       Sigma^c(i tau) = (Sigma_bar(i tau) + Sigma_und(-i tau)) / 2,
       Sigma^s(i tau) = (Sigma_bar(i tau) - Sigma_und(-i tau)) / 2.
6. The cosine and sine transforms of Eqs. (69)-(71):
       Sigma(i omega_k) = sum_j ct[k][j] Sigma^c(i tau_j) + i sum_j st[k][j] Sigma^s(i tau_j),
   ct[k][j] = gamma_kj cos(omega_k tau_j), st[k][j] = lambda_kj sin(omega_k tau_j),
   each summed in FP64 in increasing j.

Readings (the paper is silent on them): the items are Gamma-point systems
(the k-sum of Eq. (62) and cross-k terms are left to the caller); W~(-i tau)
= W~(i tau); only the plane-wave term Sigma^(1) is formed (the one-centre PAW
terms need PAW data).

``sigma_pairsum_tau`` evaluates the same matrix elements without any
real-space W~, as sums over bands of plane-wave pair densities
(rho_b(G) = sum_r exp(-i G.r) psi_n(r) conj(phi_b(r))):
    sum_{r,r'} conj(psi_n(r)) phi_b(r) W~(r, r') conj(phi_b(r')) psi_n(r')
      = rho_b^H W~ rho_b,
which pins steps 1-4.  ``sigma_laplace`` is the exact frequency result for a
screened interaction that is a constant in space, c exp(-y tau), reached when
the cosine and sine coefficients integrate exactly; it pins steps 5-6 and
their signs.  Every routine is plain NumPy/SciPy in FP64.  Parity unpinned:
none.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

__all__ = ["validate", "weights", "w_first_index", "w_real_space_rows", "sigma_tau", "sigma_omega",
           "sigma_from_tau", "sigma_pairsum_tau", "sigma_laplace", "state_orbitals",
           "rel_l2"]

_WORKERS = max(1, int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1)


def validate(item) -> None:
    """Reject inputs the method is not defined for (raises ValueError)."""
    n_r = int(np.prod(item.n))
    if item.phi_occ.shape[1] != n_r or item.phi_unocc.shape[1] != n_r:
        raise ValueError("orbital length != grid size")
    if not (item.eps_occ.max() < item.mu < item.eps_unocc.min()):
        raise ValueError("mu must lie strictly inside the gap")
    if np.any(item.tau <= 0):
        raise ValueError("tau must be positive")
    g = np.asarray(item.g_index)
    if g.min() < 0 or g.max() >= n_r or np.unique(g).size != g.size:
        raise ValueError("g_index out of range or duplicated")
    k = item.n_occ + item.n_unocc
    s = np.asarray(item.states)
    if s.size < 1 or s.min() < 0 or s.max() >= k:
        raise ValueError("state index out of range")
    if item.w_tau.shape != (item.tau.shape[0], g.size, g.size):
        raise ValueError("w_tau must be n_tau x n_g x n_g")
    if item.ct.shape[1] != item.tau.shape[0] or item.st.shape != item.ct.shape:
        raise ValueError("ct and st must be n_omega x n_tau")


def weights(item, tau):
    """exp(+(eps_i - mu) tau) for the occupied, exp(-(eps_a - mu) tau) for the
    unoccupied bands (Eqs. (1)-(2) at -tau and +tau)."""
    return np.exp((item.eps_occ - item.mu) * tau), np.exp(-(item.eps_unocc - item.mu) * tau)


def state_orbitals(item):
    """psi_n for the requested states: index b < n_occ is occupied band b,
    otherwise unoccupied band b - n_occ; shape (n_states, N_r) complex."""
    phi = np.concatenate([item.phi_occ, item.phi_unocc]).astype(np.complex128)
    return phi[np.asarray(item.states, dtype=np.int64)]


def w_first_index(item, j):
    """Step 1, first transform: W~(r, G', i tau_j) = sum_G exp(+i G.r) W~(G, G'),
    shape (N_r, n_g)."""
    n0, n1, n2 = (int(v) for v in item.n)
    n_r = n0 * n1 * n2
    g = np.asarray(item.g_index, dtype=np.int64)
    cube = np.zeros((n_r, g.size), dtype=np.complex128)
    cube[g, :] = np.asarray(item.w_tau[j], dtype=np.complex128)
    # scatter each column onto the grid, N_r * inverse DFT
    return sfft.ifftn(cube.reshape(n0, n1, n2, g.size), axes=(0, 1, 2),
                      workers=_WORKERS).reshape(n_r, g.size) * n_r


def w_real_space_rows(item, j, rows, w_rg=None):
    """Step 1: W~(r, r', i tau_j) for the grid points r in ``rows`` and every
    r', shape (len(rows), N_r); ``w_rg`` is the first transform when already
    computed."""
    n0, n1, n2 = (int(v) for v in item.n)
    n_r = n0 * n1 * n2
    g = np.asarray(item.g_index, dtype=np.int64)
    if w_rg is None:
        w_rg = w_first_index(item, j)
    # W~(r, r') = sum_G' W~(r, G') exp(-i G'.r'): scatter each row, forward DFT
    sel = w_rg[np.asarray(rows, dtype=np.int64)]
    cube = np.zeros((sel.shape[0], n_r), dtype=np.complex128)
    cube[:, g] = sel
    return sfft.fftn(cube.reshape(-1, n0, n1, n2), axes=(1, 2, 3),
                     workers=_WORKERS).reshape(-1, n_r)


def sigma_tau(item, j, block=1024):
    """Steps 1-4 at tau_j: (Sigma_und_nn(-i tau_j), Sigma_bar_nn(i tau_j)) for
    the requested states, each complex of shape (n_states,).  The rows r are
    processed in blocks of ``block`` so that no N_r x N_r matrix exists whole."""
    n_r = int(np.prod(item.n))
    tau = float(item.tau[j])
    w_o, w_u = weights(item, tau)
    phi_o = item.phi_occ.astype(np.complex128)
    phi_u = item.phi_unocc.astype(np.complex128)
    psi = state_orbitals(item)                       # (n_s, N_r)
    s_und = np.zeros(psi.shape[0], dtype=np.complex128)
    s_bar = np.zeros(psi.shape[0], dtype=np.complex128)
    w_rg = w_first_index(item, j)
    for r0 in range(0, n_r, block):
        rows = np.arange(r0, min(n_r, r0 + block))
        wt = w_real_space_rows(item, j, rows, w_rg)                 # W~(r in block, r')
        g_und = (phi_o[:, rows].T * w_o[None, :]) @ phi_o.conj()    # Gund(r, r', -i tau)
        g_bar = -(phi_u[:, rows].T * w_u[None, :]) @ phi_u.conj()   # Gbar(r, r', i tau)
        sig_und = -g_und * wt                                       # step 3
        sig_bar = -g_bar * wt
        # step 4: sum_r conj(psi_n(r)) sum_r' Sigma(r, r') psi_n(r')
        s_und += (psi[:, rows].conj() * (sig_und @ psi.T).T).sum(axis=1)
        s_bar += (psi[:, rows].conj() * (sig_bar @ psi.T).T).sum(axis=1)
    return s_und, s_bar


def sigma_from_tau(item, s_und, s_bar):
    """Steps 5-6 from the matrix elements at every tau, arrays (n_tau, n_states):
    Sigma_nn(i omega_k), complex (n_states, n_omega)."""
    s_und = np.asarray(s_und, dtype=np.complex128)
    s_bar = np.asarray(s_bar, dtype=np.complex128)
    s_c = 0.5 * (s_bar + s_und)                      # Eq. (67)
    s_s = 0.5 * (s_bar - s_und)                      # Eq. (68)
    n_omega, n_tau = item.ct.shape
    out = np.zeros((s_und.shape[1], n_omega), dtype=np.complex128)
    for k in range(n_omega):
        c = np.zeros(s_und.shape[1], dtype=np.complex128)
        s = np.zeros(s_und.shape[1], dtype=np.complex128)
        for j in range(n_tau):                       # increasing j
            c += item.ct[k, j] * s_c[j]
            s += item.st[k, j] * s_s[j]
        out[:, k] = c + 1j * s                       # Eqs. (69)-(71)
    return out


def sigma_omega(item, return_tau=False):
    """Steps 1-6: Sigma_nn(i omega_k), complex (n_states, n_omega); with
    ``return_tau`` also the (n_tau, n_states) arrays of Sigma_und(-i tau_j)
    and Sigma_bar(i tau_j)."""
    validate(item)
    und, bar = zip(*[sigma_tau(item, j) for j in range(item.tau.shape[0])])
    und, bar = np.stack(und), np.stack(bar)
    out = sigma_from_tau(item, und, bar)
    return (out, und, bar) if return_tau else out


def sigma_pairsum_tau(item, j):
    """Steps 1-4 at tau_j by the plane-wave pair form, without real-space W~:
    (Sigma_und(-i tau_j), Sigma_bar(i tau_j)) per state, from
    sum_{r,r'} conj(psi_n(r)) G(r, r') W~(r, r') psi_n(r') = sum_b w_b rho_b^H W~ rho_b,
    rho_b(G) = sum_r exp(-i G.r) psi_n(r) conj(phi_b(r))."""
    n0, n1, n2 = (int(v) for v in item.n)
    g = np.asarray(item.g_index, dtype=np.int64)
    w = np.asarray(item.w_tau[j], dtype=np.complex128)
    w_o, w_u = weights(item, float(item.tau[j]))
    psi = state_orbitals(item)
    out_und = np.empty(psi.shape[0], dtype=np.complex128)
    out_bar = np.empty(psi.shape[0], dtype=np.complex128)
    for s in range(psi.shape[0]):
        terms = []
        for phi, wts in ((item.phi_occ, w_o), (item.phi_unocc, w_u)):
            prod = psi[s][None, :] * np.conj(phi.astype(np.complex128))
            rho = sfft.fftn(prod.reshape(-1, n0, n1, n2), axes=(1, 2, 3),
                            workers=_WORKERS).reshape(phi.shape[0], -1)[:, g]
            q = np.einsum("bg,gh,bh->b", rho.conj(), w, rho)
            terms.append((wts * q).sum())
        out_und[s] = -terms[0]          # -sum_i w_i <...>  (Gund carries +)
        out_bar[s] = +terms[1]          # Gbar carries -, Sigma_bar = -Gbar W~
    return out_und, out_bar


def sigma_laplace(item, c, y, omega):
    """Exact Sigma_nn(i omega) for W~(r, r', i tau) = c exp(-y |tau|) (constant
    in space) and orthonormal orbitals: only the state's own band contributes,
    unoccupied:  c / (x - i omega),  x = eps_n - mu + y;
    occupied:   -c / (x + i omega),  x = mu - eps_n + y;
    the Fourier integral -int G(i tau) W~(i tau) exp(i omega tau) d tau of Eq. (64)
    done in closed form.  Shape (n_states, len(omega))."""
    eps = np.concatenate([item.eps_occ, item.eps_unocc])[np.asarray(item.states)]
    occ = np.asarray(item.states) < item.n_occ
    om = np.asarray(omega, dtype=np.float64)[None, :]
    out = np.empty((eps.shape[0], om.shape[1]), dtype=np.complex128)
    x_u = (eps - item.mu + y)[:, None]
    x_o = (item.mu - eps + y)[:, None]
    out[:] = np.where(occ[:, None], -c / (x_o + 1j * om), c / (x_u - 1j * om))
    return out


def rel_l2(a, b):
    """max over omega of ||a[:, k] - b[:, k]||_2 / ||b[:, k]||_2 over the states
    (b is the reference)."""
    a = np.asarray(a)
    b = np.asarray(b)
    num = np.sqrt((np.abs(a - b) ** 2).sum(axis=0))
    den = np.sqrt((np.abs(b) ** 2).sum(axis=0))
    return float((num / den).max())
