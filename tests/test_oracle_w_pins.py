"""Pins of the CPU oracle for the screened interaction (W~ from chi).

Each test checks the oracle against something other than its own formulas:
the RPA Dyson equation by matrix products, a closed form, invariants, and the
exact Laplace transform pair for the inverse cosine transform.  A planted
mistake (the other reading of the bare-Coulomb subtraction, a transposed
inverse transform) must fail the same checks.
"""
import numpy as np
import pytest

from oracle import w as ow
from paper_1607_02859_amd import synth


@pytest.fixture(scope="module")
def witem():
    return synth.make_w_item(11, (12, 12, 12), 6, strength=4.0)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_dyson_equation(witem):
    """W = v + v chi W with the bare Coulomb operator v = diag(s^2) (Sec. II.C
    step (iii)); for the correlated part: W~ = v chi v + v chi W~.  Checked
    with matrix products only, no inversion."""
    wt = ow.w_tilde_omega(witem.chi, witem.sqrt_v)
    vd = np.diag(witem.sqrt_v ** 2)
    for k in range(witem.n_omega):
        rhs = vd @ witem.chi[k] @ vd + vd @ witem.chi[k] @ wt[k]
        assert _rel(rhs, wt[k]) < 1e-12


def test_planted_full_v_subtraction_is_caught(witem):
    """Subtracting the whole v(G, G') matrix in Eq. (49) instead of its
    diagonal part breaks the Dyson equation."""
    v = ow.coulomb_kernel(witem.sqrt_v)
    wrong = ow.w_tilde_omega(witem.chi, witem.sqrt_v) + v * np.eye(witem.n_g) - v
    vd = np.diag(witem.sqrt_v ** 2)
    rhs = vd @ witem.chi[0] @ vd + vd @ witem.chi[0] @ wrong[0]
    assert _rel(rhs, wrong[0]) > 1e-2


def test_diagonal_chi_closed_form():
    """chi = diag(c): W~ = diag(s^4 c / (1 - s^2 c))."""
    rng = np.random.default_rng(3)
    n = 40
    s = rng.uniform(0.1, 2.0, n)
    c = -rng.uniform(0.0, 3.0, (2, n))
    chi = np.stack([np.diag(ci).astype(np.complex128) for ci in c])
    wt = ow.w_tilde_omega(chi, s)
    for k in range(2):
        expect = np.diag(s ** 4 * c[k] / (1.0 - s ** 2 * c[k]))
        assert np.abs(wt[k] - expect).max() < 1e-13 * np.abs(expect).max()


def test_one_plane_wave():
    """1 x 1: W~ = s^2 (1 / (1 - s^2 chi) - 1)."""
    s = np.array([1.7])
    chi = np.array([[[-0.8 + 0j]]])
    wt = ow.w_tilde_omega(chi, s)
    expect = 1.7 ** 2 * (1.0 / (1.0 + 1.7 ** 2 * 0.8) - 1.0)
    assert abs(wt[0, 0, 0] - expect) < 1e-15


def test_hermitian_negative_semidefinite(witem):
    """For a Hermitian negative semidefinite chi, eps >= 1 and W~(i omega) is
    Hermitian negative semidefinite."""
    wt = ow.w_tilde_omega(witem.chi, witem.sqrt_v)
    for k in range(witem.n_omega):
        assert np.abs(wt[k] - wt[k].conj().T).max() < 1e-13 * np.abs(wt[k]).max()
        ev = np.linalg.eigvalsh(0.5 * (wt[k] + wt[k].conj().T))
        assert ev.max() <= 1e-12 * np.abs(ev).max()
        assert ev.min() < 0


def test_dropped_plane_wave_gives_zero_row_and_column(witem):
    """s(G) = 0 (G = 0 at k = 0): that row and column of W~ vanish."""
    z = np.flatnonzero(witem.sqrt_v == 0)
    assert z.size == 1
    wt = ow.w_tilde_tau(witem.chi, witem.sqrt_v, witem.ct)
    assert np.abs(wt[:, z, :]).max() == 0 and np.abs(wt[:, :, z]).max() == 0


@pytest.mark.parametrize("n_tau", [12, 16, 20])
def test_inverse_ct_recovers_laplace_pair(n_tau):
    """The inverse transform of 2x / (x^2 + omega_k^2) returns exp(-x tau_j)
    (the pair under the brace of Eq. (5)) within the grid's error: with the
    forward fit error eta(x) = f_w(x) - ct f_t(x) (Eq. (5)), the inverse gives
    ict f_w - f_t = ict eta, bounded by ||ict||_inf max_k |eta_k(x)|, for
    transition energies across the fitted range."""
    tau, om, ct, _ = synth.ct_grid(n_tau, 0.5, 50.0)
    ict = ow.inverse_ct(ct)
    norm_inf = np.abs(ict).sum(axis=1).max()
    worst = worst_t = 0.0
    for x in np.exp(np.linspace(np.log(0.5), np.log(50.0), 41)):
        f_w = 2 * x / (x * x + om * om)
        f_t = np.exp(-x * tau)
        eta = np.abs(f_w - ct @ f_t).max()
        err = np.abs(ict @ f_w - f_t).max()
        assert err <= 1.000001 * norm_inf * eta + 1e-14
        worst = max(worst, err)
        worst_t = max(worst_t, np.abs(ict.T @ f_w - f_t).max())
    assert worst < 1e-2
    assert worst_t > 0.05        # a transposed inverse is caught


def test_tau_transform_is_linear_in_frequencies(witem):
    """W~(i tau_j) is the inverse transform of W~(i omega_k) element by element:
    applying the forward matrix returns W~(i omega)."""
    wt, ww = ow.w_tilde_tau(witem.chi, witem.sqrt_v, witem.ct, return_omega=True)
    back = np.einsum("kj,jab->kab", witem.ct, wt)
    assert _rel(back, ww) < 1e-11


def test_inverse_ct_rejects_non_square():
    with pytest.raises(ValueError):
        ow.inverse_ct(np.ones((3, 4)))


def test_rows_by_solves_match_full_inverse(witem):
    """The sampled-row form (linear solves) agrees with the full inverse."""
    full = ow.w_tilde_tau(witem.chi, witem.sqrt_v, witem.ct)
    rows = [0, 1, 57, witem.n_g - 1]
    part = ow.w_tilde_rows(witem.chi, witem.sqrt_v, witem.ct, rows)
    assert _rel(part, full[:, rows, :]) < 1e-12
