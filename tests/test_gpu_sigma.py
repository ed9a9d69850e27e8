"""GPU parity of the self-energy step (Sec. II.D: W~ to real space, the
products with the Green's functions, diagonal matrix elements, even/odd split,
cosine and sine transforms) against the CPU FP64 oracle, through the C ABI.

Bounds, per precision, on the maximum over frequencies of the relative
2-norm error over the states: 1e-10 (FP64), 1e-5 (FP32), 1e-4 (split-BF16)
-- the tiers of the polarizability build.  The tau-domain elements are
compared with the same bounds relative to their largest magnitude.  Cases
span several GEMM tiles with ragged edges, non-cubic grids, the specialised
cubic sizes, several r' slabs, several items in one call, the device entry,
and the 24^3 workload (64 + 960 bands, 12 taus, 2969 plane waves) on
sampled taus.
"""
import sys

import numpy as np
import pytest

from oracle import sigma as osg
from paper_1607_02859_amd import gwchi, synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-4}
PRECS = ["fp64", "fp32", "bf16x3"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = gwchi.Context(0)
    yield c
    c.close()


CASES = {
    "noncubic": lambda: synth.make_sigma_item(201, (6, 6, 5), 4, 20, 6, 6),
    "cplx8": lambda: synth.make_sigma_item(202, (8, 8, 8), 8, 40, 6, 10),
    "ragged": lambda: synth.make_sigma_item(203, (10, 12, 9), 20, 100, 4, 9),
    "cubic16": lambda: synth.make_sigma_item(204, (16, 16, 16), 8, 56, 3, 12),
}
_REF = {}


def case(name):
    if name not in _REF:
        it = CASES[name]()
        _REF[name] = (it,) + tuple(osg.sigma_omega(it, return_tau=True))
    return _REF[name]


def tau_err(got, und, bar):
    """max over tau of max |error| / max |reference| over the states, both parts"""
    g_und, g_bar = got[:, :, 0].T, got[:, :, 1].T          # (n_tau, n_states)
    e1 = np.abs(g_und - und.real).max(axis=1) / np.abs(und).max(axis=1)
    e2 = np.abs(g_bar - bar.real).max(axis=1) / np.abs(bar).max(axis=1)
    return float(max(e1.max(), e2.max()))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", list(CASES))
def test_parity(ctx, name, prec):
    it, ref, und, bar = case(name)
    say(f"[sigma] case={name} prec={prec} n={it.n} K={it.n_occ}+{it.n_unocc} states={it.n_states}")
    (outs, taus), rep = ctx.sigma_build([it], prec, tau_out=True, report=True)
    err = osg.rel_l2(outs[0], ref)
    et = tau_err(taus[0], und, bar)
    say(f"   err(omega)={err:.3e} err(tau)={et:.3e} ms={rep['ms_total']:.3f}")
    assert np.all(np.isfinite(outs[0])) and err <= TOL[prec] and et <= TOL[prec]


def test_several_slabs_and_items(ctx):
    """Two items of different grids in one call, with 256-column slabs (the
    16^3 grid runs 16 slabs) and the FP32 path."""
    a, ra, *_ = case("cubic16")
    b, rb, *_ = case("ragged")
    ctx.set_options(slab_width=256)
    outs = ctx.sigma_build([a, b], "fp32")
    ctx.set_options(slab_width=0)
    for o, r in zip(outs, (ra, rb)):
        err = osg.rel_l2(o, r)
        say(f"[sigma] two items, 256-column slabs: err={err:.3e}")
        assert err <= TOL["fp32"]


def test_device_entry_matches_host_entry(ctx):
    import torch
    dev = torch.device("cuda:0")
    it, ref, *_ = case("cplx8")
    host = ctx.sigma_build([it], "fp64")[0]
    po = torch.from_numpy(it.phi_occ).to(dev)
    pu = torch.from_numpy(it.phi_unocc).to(dev)
    w = torch.from_numpy(it.w_tau).to(dev)
    out = torch.empty((it.n_states, it.n_omega), dtype=torch.complex128, device=dev)
    rep = ctx.sigma_build_device([it], [(po, pu)], [w], [out], prec="fp64", report=True)
    torch.cuda.synchronize()
    say(f"[sigma] device entry ms={rep['ms_total']:.3f}")
    assert np.array_equal(out.cpu().numpy(), host)
    assert osg.rel_l2(host, ref) <= TOL["fp64"]


def test_constant_interaction_closed_form(ctx):
    """W~ constant in space (only G = G' = 0), c exp(-y tau) on a dense
    Gauss-Legendre grid: the GPU result approaches the closed form of the
    Fourier integral to the quadrature's accuracy, as the oracle does."""
    it = synth.make_sigma_item(205, (4, 4, 3), 3, 9, 2, 12, gap=2.0)
    c, y = 0.8, 0.3
    omega = np.array([0.5, 2.0, 5.0, 10.0])
    tau, ct = synth.gauss_legendre_ct(omega, 40.0 / (1.0 + y), panel=1.0, nodes=24)
    _, st = synth.gauss_legendre_st(omega, 40.0 / (1.0 + y), panel=1.0, nodes=24)
    w = np.zeros((tau.shape[0], it.n_g, it.n_g), dtype=np.complex128)
    g0 = int(np.flatnonzero(it.g_index == 0)[0])
    w[:, g0, g0] = c * np.exp(-y * tau)
    it.tau, it.omega, it.ct, it.st, it.w_tau = tau, omega, ct, st, w
    got = ctx.sigma_build([it], "fp64")[0]
    exact = osg.sigma_laplace(it, c, y, omega)
    err = osg.rel_l2(got, exact)
    say(f"[sigma] closed form ({tau.shape[0]} taus): err={err:.3e}")
    assert err <= 1e-8


def test_workload_24cubed_sampled_taus(ctx):
    """The 24^3 workload (64 + 960 complex bands, 12 taus, 2969 plane waves,
    8 states at the gap) in FP32 and FP64: every state's tau-domain elements
    against the oracle at three of the twelve taus."""
    it = synth.make_sigma_item([2, 0], (24, 24, 24), 64, 960, 12, 8)
    js = [0, 5, 11]
    refs = [osg.sigma_tau(it, j) for j in js]
    for prec in ("fp32", "fp64"):
        (outs, taus), rep = ctx.sigma_build([it], prec, tau_out=True, report=True)
        t = taus[0]
        worst = 0.0
        for j, (und, bar) in zip(js, refs):
            e1 = np.abs(t[:, j, 0] - und.real).max() / np.abs(und).max()
            e2 = np.abs(t[:, j, 1] - bar.real).max() / np.abs(bar).max()
            worst = max(worst, e1, e2)
        say(f"[sigma24] prec={prec} ms={rep['ms_total']:.1f} (gemm {rep['ms_gemm']:.1f}, "
            f"fft {rep['ms_fft']:.1f}) err(sampled taus)={worst:.3e}")
        assert np.all(np.isfinite(outs[0])) and worst <= TOL[prec]


def test_chain_chi_w_sigma_pade(ctx):
    """The whole chain on the GPU, each step fed by the previous one's device
    output -- chi(i omega) (polarizability build), W~(i tau) (screened
    interaction), Sigma_nn(i omega) (self-energy), then the continuation to
    real frequencies -- against the oracle chain run on the same seeded
    inputs (each oracle step fed by the previous oracle step), FP64."""
    import torch
    from oracle import chi as oc, pade as op, w as ow
    dev = torch.device("cuda:0")
    n_tau = 8
    it = synth.make_item(211, (8, 8, 8), 8, 40, True, n_tau, x_min=1.0)
    s_v = synth.coulomb_sqrt(it.n, it.g_index)
    st, _ = synth.st_fit(it.tau, it.omega, 1.0, 75.0)
    states = np.array([6, 7, 8, 9], np.int32)
    # oracle chain
    chi_ref = oc.chi_omega(it)
    w_ref = ow.w_tilde_tau(chi_ref, s_v, it.ct)
    sitem = synth.SigmaItem(n=it.n, phi_occ=it.phi_occ, phi_unocc=it.phi_unocc,
                            eps_occ=it.eps_occ, eps_unocc=it.eps_unocc, mu=it.mu, tau=it.tau,
                            omega=it.omega, ct=it.ct, st=st, g_index=it.g_index, w_tau=w_ref,
                            states=states)
    sig_ref = osg.sigma_omega(sitem)
    z = 1j * it.omega
    wr = np.linspace(-5.0, 5.0, 41) + 0.1j
    pade_ref = op.continue_to(z, sig_ref, wr)
    # GPU chain, device buffers passed along
    po = torch.from_numpy(it.phi_occ).to(dev)
    pu = torch.from_numpy(it.phi_unocc).to(dev)
    chi = torch.empty((it.n_omega, it.n_g, it.n_g), dtype=torch.complex128, device=dev)
    ctx.build_device([it], [(po, pu)], [chi], "fp64")
    witem = synth.WItem(chi=None, sqrt_v=s_v, ct=it.ct, omega=it.omega)
    w_tau = torch.empty((n_tau, it.n_g, it.n_g), dtype=torch.complex128, device=dev)
    ctx.w_build_device([witem], [chi], [w_tau])
    sig = torch.empty((len(states), it.n_omega), dtype=torch.complex128, device=dev)
    ctx.sigma_build_device([sitem], [(po, pu)], [w_tau], [sig], prec="fp64")
    out = torch.empty((len(states), len(wr)), dtype=torch.complex128, device=dev)
    ctx.pade_device(z, sig, wr, out)
    torch.cuda.synchronize()
    e_sig = osg.rel_l2(sig.cpu().numpy(), sig_ref)
    got = out.cpu().numpy()
    e_pade = float(np.abs(got - pade_ref).max() / np.abs(pade_ref).max())
    say(f"[chain] sigma err={e_sig:.3e} continuation err={e_pade:.3e}")
    assert e_sig <= 1e-10 and e_pade <= 1e-8
