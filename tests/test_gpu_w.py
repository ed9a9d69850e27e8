"""GPU parity of the screened-interaction step (W~ from chi, Sec. II.C steps
(iii)-(iv)) against the CPU FP64 oracle, through the C ABI.

The path is FP64 throughout; every comparison uses the FP64 bound of
1e-10 on the maximum, over the tau (or omega) matrices, of the relative
Frobenius error of each matrix.  Cases span several 64 x 64 update tiles
and 64-pivot blocks with ragged tails, sizes below one block, several items
of different sizes in one call, the device entry, the full 24^3 sphere
(2969 plane waves, 12 frequencies) and the 32^3 sphere (7123 plane waves) on
sampled rows, and the error paths.
"""
import sys

import numpy as np
import pytest

from oracle import w as ow
from paper_1607_02859_amd import gwchi, synth

pytestmark = pytest.mark.gpu

TOL = 1e-10
K_SHIFT = (0.11, 0.23, 0.07)     # k off the Gamma point: no plane wave is dropped


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    """max over the leading (tau or omega) index of ||a_j - b_j||_F / ||b_j||_F"""
    a = np.asarray(a).reshape(np.shape(b)[0], -1)
    b = np.asarray(b).reshape(np.shape(b)[0], -1)
    return float((np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)).max())


def tau_bound(ref_t, ref_w, ct, err_w):
    """The bound the inverse cosine transform (Eq. (50)) puts on the error of
    W~(i tau_j) given the error err_w of every W~(i omega_k):
    ||dW_j|| <= sum_k |xi_jk| ||dW_k|| <= (err_w + n eps) sum_k |xi_jk| ||W_k||,
    relative to ||W_j||; the maximum over j."""
    ict = ow.inverse_ct(ct)
    nw = np.linalg.norm(ref_w.reshape(ref_w.shape[0], -1), axis=1)
    nt = np.linalg.norm(ref_t.reshape(ref_t.shape[0], -1), axis=1)
    kappa = (np.abs(ict) @ nw) / nt
    return float(((err_w + ict.shape[0] * np.finfo(float).eps) * kappa).max())


@pytest.fixture(scope="module")
def ctx():
    c = gwchi.Context(0)
    yield c
    c.close()


def test_sphere12_host_entry(ctx):
    w = synth.make_w_item(21, (12, 12, 12), 6, strength=4.0)
    say(f"[w] sphere12 n_g={w.n_g} n_omega={w.n_omega}")
    (taus, oms), rep = ctx.w_build([w], omega=True, report=True)
    ref_t, ref_w = ow.w_tilde_tau(w.chi, w.sqrt_v, w.ct, return_omega=True)
    et, ew = rel(taus[0], ref_t), rel(oms[0], ref_w)
    say(f"   err tau={et:.3e} omega={ew:.3e} ms={rep['ms_total']:.3f} launches={rep['n_launches']}")
    assert et <= TOL and ew <= TOL
    z = np.flatnonzero(w.sqrt_v == 0)           # G = 0 at k = 0 is dropped
    assert np.all(taus[0][:, z, :] == 0) and np.all(taus[0][:, :, z] == 0)


@pytest.mark.parametrize("n_g", [1, 2, 31, 32, 33, 64, 65, 97, 130])
def test_edge_sizes(ctx, n_g):
    w = synth.make_w_item(30 + n_g, (12, 12, 12), 4, strength=3.0, n_g=n_g, k=K_SHIFT)
    say(f"[w] edge n_g={n_g}")
    out = ctx.w_build([w])[0]
    ref = ow.w_tilde_tau(w.chi, w.sqrt_v, w.ct)
    err = rel(out, ref)
    say(f"   err={err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("n_tau", [1, 20])
def test_grid_sizes(ctx, n_tau):
    """One frequency (a 1 x 1 cosine matrix), and 20 (the widest register set
    of the final pass: up to 32 taus).  W~(i omega) meets the FP64 bound; each
    W~(i tau_j) is the inverse transform of them, whose amplification on the
    20-point grid (|xi| up to 1e3 against matrices of smaller norm) the bound
    for the tau matrices takes from the conditioning (tau_bound)."""
    w = synth.make_w_item(90 + n_tau, (8, 8, 8), n_tau, strength=3.0, n_g=70, k=K_SHIFT)
    (taus, oms) = ctx.w_build([w], omega=True)
    ref_t, ref_w = ow.w_tilde_tau(w.chi, w.sqrt_v, w.ct, return_omega=True)
    et, ew = rel(taus[0], ref_t), rel(oms[0], ref_w)
    bound = max(TOL, tau_bound(ref_t, ref_w, w.ct, ew))
    say(f"[w] n_tau={n_tau} err tau={et:.3e} (bound {bound:.1e}) omega={ew:.3e}")
    assert ew <= TOL and et <= bound


def test_several_items_one_call(ctx):
    ws = [synth.make_w_item(41, (12, 12, 12), 5, strength=2.0, n_g=200, k=K_SHIFT),
          synth.make_w_item(42, (12, 12, 12), 5, strength=5.0),
          synth.make_w_item(43, (12, 12, 12), 5, strength=1.0, n_g=77, k=K_SHIFT)]
    outs = ctx.w_build(ws)
    for w, o in zip(ws, outs):
        err = rel(o, ow.w_tilde_tau(w.chi, w.sqrt_v, w.ct))
        say(f"[w] multi n_g={w.n_g} err={err:.3e}")
        assert err <= TOL


def test_device_entry_matches_host_entry(ctx):
    import torch
    dev = torch.device("cuda:0")
    ws = [synth.make_w_item(51, (12, 12, 12), 6, strength=4.0),
          synth.make_w_item(52, (12, 12, 12), 6, strength=2.0, n_g=150, k=K_SHIFT)]
    chis = [torch.from_numpy(w.chi).to(dev) for w in ws]
    taus = [torch.empty((w.n_tau, w.n_g, w.n_g), dtype=torch.complex128, device=dev) for w in ws]
    oms = [torch.empty((w.n_omega, w.n_g, w.n_g), dtype=torch.complex128, device=dev) for w in ws]
    rep = ctx.w_build_device(ws, chis, taus, oms, report=True)
    torch.cuda.synchronize()
    say(f"[w] device entry ms={rep['ms_total']:.3f}")
    host = ctx.w_build(ws, omega=True)
    for t, w in enumerate(ws):
        got_t, got_w = taus[t].cpu().numpy(), oms[t].cpu().numpy()
        assert np.array_equal(got_t, host[0][t]) and np.array_equal(got_w, host[1][t])
        ref_t, ref_w = ow.w_tilde_tau(w.chi, w.sqrt_v, w.ct, return_omega=True)
        assert rel(got_t, ref_t) <= TOL and rel(got_w, ref_w) <= TOL
    # a second call into the same outputs, without a report (enqueue only)
    ctx.w_build_device(ws[1:], chis[1:], taus[1:])
    torch.cuda.synchronize()
    assert np.array_equal(taus[1].cpu().numpy(), host[0][1])


def test_sphere18_full(ctx):
    """The 18^3 sphere (1309 plane waves, 21 tiles per side: every XCD
    partition owns several column tiles, including the second, reversed group
    of the snake), compared in full."""
    w = synth.make_w_item(65, (18, 18, 18), 6, strength=4.0)
    say(f"[w] sphere18 n_g={w.n_g}")
    (taus, oms) = ctx.w_build([w], omega=True)
    ref_t, ref_w = ow.w_tilde_tau(w.chi, w.sqrt_v, w.ct, return_omega=True)
    et, ew = rel(taus[0], ref_t), rel(oms[0], ref_w)
    say(f"   err tau={et:.3e} omega={ew:.3e}")
    assert et <= TOL and ew <= TOL


def test_full_sphere24_sampled_rows(ctx):
    """The 24^3 sphere (2969 plane waves) and 12 frequencies, the size of the
    headline polarizability workload: sampled rows against linear solves."""
    w = synth.make_w_item(61, (24, 24, 24), 12, strength=4.0)
    say(f"[w] sphere24 n_g={w.n_g}")
    (taus, oms), rep = ctx.w_build([w], omega=True, report=True)
    say(f"   ms total={rep['ms_total']:.2f} invert={rep['ms_invert']:.2f} "
        f"TFLOP/s={rep['alg_flops'] / rep['ms_total'] * 1e-9:.1f}")
    rows = [0, 1, 777, 1500, w.n_g - 1]
    ref = ow.w_tilde_rows(w.chi, w.sqrt_v, w.ct, rows)
    err = rel(taus[0][:, rows, :], ref)
    say(f"   err(sampled rows)={err:.3e}")
    assert err <= TOL
    # W~(i omega) is Hermitian and negative semidefinite (checked on one matrix)
    m = oms[0][0]
    assert np.abs(m - m.conj().T).max() <= 1e-10 * np.abs(m).max()
    ev = np.linalg.eigvalsh(0.5 * (m + m.conj().T))
    assert ev.max() <= 1e-10 * np.abs(ev).max()


def test_sphere32_sampled_rows(ctx):
    """The 32^3 sphere (7123 plane waves, 112 pivot blocks, a ragged last
    block of 19), the plane-wave count of the largest polarizability
    workload, with 4 frequencies: sampled rows against linear solves."""
    w = synth.make_w_item(67, (32, 32, 32), 4, strength=4.0)
    say(f"[w] sphere32 n_g={w.n_g} n_omega={w.n_omega}")
    (taus, oms), rep = ctx.w_build([w], omega=True, report=True)
    say(f"   ms total={rep['ms_total']:.2f} invert={rep['ms_invert']:.2f}")
    rows = [0, 1, 64, 3000, 7040, w.n_g - 1]
    ref_w = np.stack([ow.w_tilde_omega_rows(w.chi[k], w.sqrt_v, rows) for k in range(w.n_omega)])
    ict = ow.inverse_ct(w.ct)
    ref = np.zeros_like(ref_w)
    for j in range(ict.shape[0]):
        for k in range(ict.shape[1]):                   # Eq. (50), increasing k
            ref[j] += ict[j, k] * ref_w[k]
    err = rel(taus[0][:, rows, :], ref)
    err_w = rel(oms[0][:, rows, :], ref_w)
    say(f"   err(sampled rows) tau={err:.3e} omega={err_w:.3e}")
    assert err <= TOL and err_w <= TOL


def test_not_positive_definite_is_reported(ctx):
    n = 40
    w = synth.WItem(chi=np.tile((2.0 * np.eye(n)).astype(np.complex128), (4, 1, 1)),
                    sqrt_v=np.ones(n), ct=synth.ct_grid(4, 0.5, 50.0)[2],
                    omega=np.zeros(4))
    with pytest.raises(gwchi.GwchiError) as e:
        ctx.w_build([w])
    assert e.value.status == 5
    # the context stays usable
    w2 = synth.make_w_item(71, (12, 12, 12), 4, n_g=50, k=K_SHIFT)
    assert rel(ctx.w_build([w2])[0], ow.w_tilde_tau(w2.chi, w2.sqrt_v, w2.ct)) <= TOL


def test_invalid_grid_is_rejected(ctx):
    w = synth.make_w_item(81, (12, 12, 12), 4, n_g=20, k=K_SHIFT)
    w.ct = w.ct[:, :3].copy()
    with pytest.raises(gwchi.GwchiError) as e:
        ctx.w_build([w])
    assert e.value.status == 1
