"""Pins of the self-energy oracle (oracle/sigma.py) against what the paper and
the mathematics fix, independently of the oracle's own real-space route:

* the plane-wave pair form (no real-space W~) for every tau, complex orbitals
  on cubic and non-cubic grids;
* the exact frequency result for a screened interaction constant in space,
  reached with dense Gauss-Legendre cosine and sine coefficients (pins the
  even/odd split, the transforms and the sign of the sine part);
* a two-point example derived by hand (tests/golden/sigma_two_point.json);
* invariants: real tau-domain elements (Hermitian G and W~), a common shift of
  the eigenvalues and the Fermi level, per-band phases, additivity over band
  sets;
* planted mistakes (a transposed W~, the sine part with the wrong sign, the
  even/odd parts swapped) fail them.
"""
import json
import os

import numpy as np
import pytest

from oracle import sigma as osg
from paper_1607_02859_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def small():
    return synth.make_sigma_item(11, (6, 6, 5), 4, 20, 6, 6)


@pytest.mark.parametrize("n,bands", [((6, 6, 5), (4, 20)), ((4, 6, 5), (3, 9)), ((8, 8, 8), (6, 30))])
def test_matches_pair_form(n, bands):
    it = synth.make_sigma_item(12 + n[0], n, bands[0], bands[1], 4, 5)
    for j in range(it.n_tau):
        und, bar = osg.sigma_tau(it, j)
        und2, bar2 = osg.sigma_pairsum_tau(it, j)
        assert np.abs(und - und2).max() <= 1e-13 * np.abs(und2).max()
        assert np.abs(bar - bar2).max() <= 1e-13 * np.abs(bar2).max()


def _constant_w_item(c, y, n_tau_panels_t_max=40.0):
    it = synth.make_sigma_item(21, (4, 4, 3), 3, 9, 2, 12, gap=2.0)
    omega = np.array([0.5, 2.0, 5.0, 10.0])
    x_min = 1.0 + y                     # smallest |eps - mu| + y
    tau, ct = synth.gauss_legendre_ct(omega, n_tau_panels_t_max / x_min)
    _, st = synth.gauss_legendre_st(omega, n_tau_panels_t_max / x_min)
    w = np.zeros((tau.shape[0], it.n_g, it.n_g), dtype=np.complex128)
    g0 = int(np.flatnonzero(it.g_index == 0)[0])
    w[:, g0, g0] = c * np.exp(-y * tau)
    it.tau, it.omega, it.ct, it.st, it.w_tau = tau, omega, ct, st, w
    return it


def test_laplace_closed_form():
    """W~(r, r', i tau) = c exp(-y tau) (the G = G' = 0 element only): the dense
    quadrature of Eqs. (69)-(71) must give c/(x - i omega) for unoccupied and
    -c/(x + i omega) for occupied states (the integral of Eq. (64))."""
    c, y = 0.8, 0.3
    it = _constant_w_item(c, y)
    got = osg.sigma_omega(it)
    ref = osg.sigma_laplace(it, c, y, it.omega)
    assert osg.rel_l2(got, ref) <= 1e-11


def test_two_point_golden():
    d = json.load(open(os.path.join(HERE, "golden", "sigma_two_point.json")))
    wt = d["w_tau"]
    b = complex(*wt["b_01"])
    w = np.array([[[wt["a_00"], b], [np.conj(b), wt["d_11"]]]], dtype=np.complex128)
    it = synth.SigmaItem(n=tuple(d["grid"]), phi_occ=np.array(d["phi_occ"], complex),
                         phi_unocc=np.array(d["phi_unocc"], complex),
                         eps_occ=np.array(d["eps_occ"]), eps_unocc=np.array(d["eps_unocc"]),
                         mu=d["mu"], tau=np.array(d["tau"]), omega=np.array([1.0]),
                         ct=np.array(d["ct"]), st=np.array(d["st"]),
                         g_index=np.array(d["g_index"], np.int32), w_tau=w,
                         states=np.array(d["states"], np.int32))
    out, und, bar = osg.sigma_omega(it, return_tau=True)
    for s, key in enumerate(("state_occupied", "state_unoccupied")):
        e = d["expected"][key]
        assert und[0, s] == pytest.approx(e["sigma_und_minus_tau"], abs=1e-15)
        assert bar[0, s] == pytest.approx(e["sigma_bar_tau"], abs=1e-15)
        assert out[s, 0] == pytest.approx(complex(*e["sigma_omega"]), abs=1e-15)


def test_tau_elements_are_real(small):
    for j in range(small.n_tau):
        und, bar = osg.sigma_tau(small, j)
        assert np.abs(und.imag).max() <= 1e-14 * np.abs(und).max()
        assert np.abs(bar.imag).max() <= 1e-14 * np.abs(bar).max()


def test_common_energy_shift(small):
    ref = osg.sigma_omega(small)
    sh = synth.SigmaItem(**{**small.__dict__, "eps_occ": small.eps_occ + 0.37,
                            "eps_unocc": small.eps_unocc + 0.37, "mu": small.mu + 0.37})
    assert osg.rel_l2(osg.sigma_omega(sh), ref) <= 1e-13


def test_band_phase_invariance(small):
    ref = osg.sigma_omega(small)
    rng = np.random.default_rng(3)
    po = small.phi_occ * np.exp(1j * rng.uniform(0, 6.3, small.n_occ))[:, None]
    pu = small.phi_unocc * np.exp(1j * rng.uniform(0, 6.3, small.n_unocc))[:, None]
    ph = synth.SigmaItem(**{**small.__dict__, "phi_occ": po, "phi_unocc": pu})
    assert osg.rel_l2(osg.sigma_omega(ph), ref) <= 1e-13


def test_additive_over_unoccupied_bands(small):
    """Sigma_bar is a sum over the unoccupied bands: splitting the unoccupied
    set into two parts splits it into two terms (occupied set fixed, states
    taken from the occupied bands so they stay in both parts)."""
    it = synth.SigmaItem(**{**small.__dict__, "states": np.array([0, 2, 3], np.int32)})
    _, _, bar = osg.sigma_omega(it, return_tau=True)
    parts = []
    for sl in (slice(0, 8), slice(8, None)):
        p = synth.SigmaItem(**{**it.__dict__, "phi_unocc": it.phi_unocc[sl],
                               "eps_unocc": it.eps_unocc[sl]})
        parts.append(osg.sigma_omega(p, return_tau=True)[2])
    assert np.abs(parts[0] + parts[1] - bar).max() <= 1e-14 * np.abs(bar).max()


def test_planted_transposed_w_is_caught(small, monkeypatch):
    it = small
    orig = osg.w_real_space_rows

    def planted(item, j, rows, w_rg=None):
        t = synth.SigmaItem(**{**item.__dict__, "w_tau": np.transpose(item.w_tau, (0, 2, 1)).copy()})
        return orig(t, j, rows)

    monkeypatch.setattr(osg, "w_real_space_rows", planted)
    und, bar = osg.sigma_tau(it, 1)
    und2, bar2 = osg.sigma_pairsum_tau(it, 1)
    assert np.abs(bar - bar2).max() > 1e-6 * np.abs(bar2).max()


def test_planted_transform_mistakes_are_caught(monkeypatch):
    c, y = 0.8, 0.3
    it = _constant_w_item(c, y)
    ref = osg.sigma_laplace(it, c, y, it.omega)
    _, und, bar = osg.sigma_omega(it, return_tau=True)
    # the sine part with the wrong sign
    bad = synth.SigmaItem(**{**it.__dict__, "st": -it.st})
    assert osg.rel_l2(osg.sigma_from_tau(bad, und, bar), ref) > 1e-2
    # the even and odd parts exchanged
    assert osg.rel_l2(osg.sigma_from_tau(it, -und, bar), ref) > 1e-2
