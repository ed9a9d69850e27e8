"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Tolerances are max-over-omega relative Frobenius errors: 1e-10 (FP64),
1e-5 (FP32), 1e-4 (split-BF16).  Cases span several GEMM tiles, ragged
grid and band counts, non-cubic grids, real and complex orbitals.
"""
import sys

import numpy as np
import pytest

from oracle import chi as oc
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
    "real6": lambda: synth.make_item(101, (6, 6, 6), 4, 20, False, 5, x_min=1.0),
    "cplx_noncubic": lambda: synth.make_item(102, (4, 6, 5), 3, 9, True, 4, x_min=1.0),
    "cplx8": lambda: synth.make_item(103, (8, 8, 8), 8, 40, True, 6, x_min=1.0),
    "ragged": lambda: synth.make_item(104, (10, 12, 9), 20, 100, True, 4, x_min=1.0),
    "ragged_real": lambda: synth.make_item(105, (9, 10, 14), 13, 77, False, 3, x_min=1.0),
    # cubic grids with specialised FFT kernels (column-grouped and contiguous
    # plane kernels, radices 4, 2, 3, 5)
    "cplx16": lambda: synth.make_item(107, (16, 16, 16), 8, 40, True, 4, x_min=1.0),
    "real18": lambda: synth.make_item(108, (18, 18, 18), 6, 30, False, 3, x_min=1.0),
    "cplx20": lambda: synth.make_item(109, (20, 20, 20), 6, 30, True, 3, x_min=1.0),
    "cfg1": lambda: synth.make_config(1)[0],
    # complex cubic grids of the single-launch first-index FFT (one batch of
    # planes at 12^3, two batches with a partial one at 18^3), and a slab
    # narrower than the grid so that several slabs and the lower-triangle
    # batches at their diagonals are exercised
    "cplx12": lambda: synth.make_item(115, (12, 12, 12), 5, 27, True, 3, x_min=1.0),
    "cplx18": lambda: synth.make_item(116, (18, 18, 18), 6, 30, True, 3, x_min=1.0),
}

_ORACLE = {}


def case(name):
    if name not in _ORACLE:
        it = CASES[name]()
        _ORACLE[name] = (it, oc.chi_omega(it))
    return _ORACLE[name]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", list(CASES))
def test_parity(ctx, name, prec):
    it, ref = case(name)
    say(f"[parity] case={name} prec={prec} n={it.n} K={it.n_occ}+{it.n_unocc}")
    ctx.set_options(use_graph=1, hermitian=0, skip_zero_bands=0, slab_width=0, tile_id=0)
    out, rep = ctx.build([it], prec, report=True)
    err = oc.rel_frobenius(out[0], ref)
    say(f"   err={err:.3e} kappa_F={rep['kappa_F_max']:.2f} ms={rep['ms_total']:.3f}")
    assert np.all(np.isfinite(out[0]))
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_every_tile_config(ctx, prec):
    it, ref = case("ragged")
    for t in range(1, 7):
        ctx.set_options(tile_id=t, use_graph=0)
        out = ctx.build([it], prec)
        err = oc.rel_frobenius(out[0], ref)
        say(f"[tile] prec={prec} tile={t} err={err:.3e}")
        assert err <= TOL[prec]
    ctx.set_options(tile_id=0, use_graph=1)
    for t in range(1, 7):
        ctx.set_options(tile_id=t, use_graph=0)
        it2, ref2 = case("ragged_real")
        out = ctx.build([it2], prec)
        assert oc.rel_frobenius(out[0], ref2) <= TOL[prec]
    ctx.set_options(tile_id=0, use_graph=1)


@pytest.mark.parametrize("prec", PRECS)
def test_hermitian_mode(ctx, prec):
    for name in ("ragged", "ragged_real", "cfg1"):
        it, ref = case(name)
        ctx.set_options(hermitian=1)
        out = ctx.build([it], prec)
        ctx.set_options(hermitian=0)
        err = oc.rel_frobenius(out[0], ref)
        say(f"[hermitian] case={name} prec={prec} err={err:.3e}")
        assert err <= TOL[prec]


def test_slab_width_bitwise(ctx):
    it, _ = case("ragged")        # N_r = 1080: five 256-column slabs, ragged last
    ctx.set_options(slab_width=0)
    a = ctx.build([it], "fp32")[0]
    ctx.set_options(slab_width=256)
    b = ctx.build([it], "fp32")[0]
    ctx.set_options(slab_width=0)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_skip_zero_bands_bitwise(ctx, prec):
    # large tau makes far bands underflow to exact zeros in FP32
    it = synth.make_item(106, (8, 8, 6), 6, 60, True, 5, x_min=0.5)
    it.tau = it.tau * 4.0
    ctx.set_options(skip_zero_bands=0)
    a = ctx.build([it], prec)[0]
    ctx.set_options(skip_zero_bands=1)
    b = ctx.build([it], prec)[0]
    ctx.set_options(skip_zero_bands=0)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", PRECS)
def test_batch_equals_single(ctx, prec):
    items = [case("cplx8")[0], case("ragged")[0], case("cplx_noncubic")[0]]
    single = [ctx.build([it], prec)[0] for it in items]
    batch = ctx.build(items, prec)
    for s, b in zip(single, batch):
        assert np.array_equal(s, b)


def test_mixed_real_and_complex_rejected(ctx):
    with pytest.raises(gwchi.GwchiError) as e:
        ctx.build([case("real6")[0], case("cplx8")[0]], "fp32")
    assert e.value.status == 1
    # the context stays usable
    it, ref = case("cplx8")
    assert oc.rel_frobenius(ctx.build([it], "fp32")[0], ref) <= TOL["fp32"]


def test_graph_replay_identical(ctx):
    it, ref = case("cplx8")
    ctx.set_options(use_graph=1)
    outs = [ctx.build([it], "fp32", report=True) for _ in range(3)]
    assert outs[1][1]["graph_replayed"] == 1
    assert np.array_equal(outs[0][0][0], outs[1][0][0])
    assert np.array_equal(outs[0][0][0], outs[2][0][0])
    ctx.set_options(use_graph=0)
    eager = ctx.build([it], "fp32")[0]
    ctx.set_options(use_graph=1)
    assert np.array_equal(eager, outs[0][0][0])


def test_device_entry_matches_host(ctx):
    import torch
    it, _ = case("ragged")
    host = ctx.build([it], "fp32")[0]
    dev = torch.device("cuda:0")
    po = torch.from_numpy(it.phi_occ).to(dev)
    pu = torch.from_numpy(it.phi_unocc).to(dev)
    out = torch.empty((it.n_omega, it.n_g, it.n_g), dtype=torch.complex128, device=dev)
    ctx.build_device([it], [(po, pu)], [out], "fp32")
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), host)


def test_timing_report(ctx):
    it, _ = case("cfg1")
    ctx.set_options(timing=1)
    _, rep = ctx.build([it], "fp32", report=True)
    ctx.set_options(timing=0)
    say(f"[timing] {rep}")
    assert rep["ms_gemm"] > 0 and rep["n_gemm_launches"] >= 1
    assert rep["alg_flops"] == synth.algorithmic_flops(it)


def test_config2_full_size_sampled_rows(ctx):
    """Config 2 at full size in the benchmark's launch configuration (FP32),
    checked on sampled rows of chi(i omega) from the pair-sum oracle."""
    it = synth.make_config(2)[0]
    say(f"[cfg2] n={it.n} K={it.n_occ}+{it.n_unocc} n_g={it.n_g}")
    ctx.set_options(use_graph=1, hermitian=0, skip_zero_bands=0, slab_width=0, tile_id=0)
    out = ctx.build([it], "fp32")[0]
    rows = [0, 1, 57, 1500, it.n_g - 1]
    ref = oc.chi_rows(it, rows)
    err = oc.rel_frobenius(out[:, rows, :], ref)
    say(f"   sampled-row err={err:.3e}")
    assert err <= TOL["fp32"]
    herm = np.abs(out - np.conj(np.transpose(out, (0, 2, 1)))).max() / np.abs(out).max()
    assert herm < 1e-5


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["cplx12", "cplx16", "real18", "cplx18", "cplx20"])
@pytest.mark.parametrize("slab", [0, 1024])
def test_cubic_hermitian_default(ctx, name, prec, slab):
    """The default options (Hermitian completion, persistent launch, graph) on
    the cubic grids with specialised FFT kernels, with the planner's slab
    width and with 1024-column slabs."""
    it, ref = case(name)
    ctx.set_options(use_graph=1, hermitian=1, skip_zero_bands=0, slab_width=slab, tile_id=0)
    out = ctx.build([it], prec)[0]
    err = oc.rel_frobenius(out, ref)
    say(f"[cubic-herm] case={name} prec={prec} slab={slab} err={err:.3e}")
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_cplx28_sampled_rows(ctx, prec):
    """28^3 complex (radix-7 line transforms, the largest-register plane
    kernels), default options, checked on sampled rows from the pair-sum
    oracle."""
    it = synth.make_item(110, (28, 28, 28), 4, 20, True, 2, x_min=1.0)
    say(f"[cplx28] prec={prec} n_g={it.n_g}")
    ctx.set_options(use_graph=1, hermitian=1, skip_zero_bands=0, slab_width=0, tile_id=0)
    out = ctx.build([it], prec)[0]
    rows = [0, 1, 333, it.n_g - 1]
    err = oc.rel_frobenius(out[:, rows, :], oc.chi_rows(it, rows))
    say(f"   sampled-row err={err:.3e}")
    assert err <= TOL[prec]


_BIG = {}


def big_case(n):
    """A 28^3 or 32^3 complex item with few bands (4 + 20, 2 taus) and its
    pair-sum result over the whole plane-wave sphere (4729 or 7123 waves)."""
    if n not in _BIG:
        it = synth.make_item(120 + n, (n, n, n), 4, 20, True, 2, x_min=1.0)
        _BIG[n] = (it, oc.chi_pairsum(it))
    return _BIG[n]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("herm", [1, 0])
@pytest.mark.parametrize("n", [28, 32])
def test_full_matrix_28_32(ctx, n, herm, prec):
    """The two largest specialised grids (radix 7 at 28^3; at 32^3 the plane
    column that exceeds the LDS) compared in full against the pair sum of
    Eq. (16), with and without Hermitian completion.  Without it the output is
    not Hermitian by construction, so Hermiticity is a real check there."""
    it, ref = big_case(n)
    say(f"[full{n}] herm={herm} prec={prec} n_g={it.n_g}")
    ctx.set_options(use_graph=1, hermitian=herm, skip_zero_bands=0, slab_width=0, tile_id=0)
    out = ctx.build([it], prec)[0]
    err = oc.rel_frobenius(out, ref)
    say(f"   err={err:.3e}")
    assert np.all(np.isfinite(out)) and err <= TOL[prec]
    if herm == 0:
        dev = np.abs(out - np.conj(np.transpose(out, (0, 2, 1)))).max() / np.abs(out).max()
        say(f"   hermiticity deviation={dev:.1e}")
        assert dev <= (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("herm", [1, 0])
@pytest.mark.parametrize("prec", PRECS)
def test_kappa_F_matches_oracle(ctx, prec, herm):
    """The reported kappa_F (norms of chi(tau_j) and chi(i omega_k) summed from
    per-block partial sums in a fixed order) against the oracle's kappa_F of
    the same item, and identical on a second build."""
    it = synth.make_item(131, (10, 12, 9), 20, 100, True, 6, x_min=1.0)
    if "k131" not in _ORACLE:
        w, xs = oc.chi_omega(it, return_tau=True)
        _ORACLE["k131"] = (w, float(oc.kappa_F(it, xs, w).max()))
    _, ref = _ORACLE["k131"]
    ctx.set_options(use_graph=1, hermitian=herm, skip_zero_bands=0, slab_width=0, tile_id=0,
                    kappa=1)
    _, rep = ctx.build([it], prec, report=True)
    _, rep2 = ctx.build([it], prec, report=True)
    got = rep["kappa_F_max"]
    say(f"[kappa] prec={prec} herm={herm} gpu={got:.12f} oracle={ref:.12f}")
    assert got == rep2["kappa_F_max"]
    assert abs(got - ref) <= (1e-12 if prec == "fp64" else 1e-5) * ref


# Degenerate shapes: one occupied and one unoccupied band, one tau point, two
# plane waves, and grids far smaller than one GEMM tile.
DEGENERATE = {
    "one_pair_two_pw": lambda: synth.make_item(111, (3, 4, 5), 1, 1, True, 1, x_min=1.0, n_g=2),
    "real_tiny": lambda: synth.make_item(112, (3, 3, 3), 1, 2, False, 2, x_min=1.0, n_g=5),
    "one_occ": lambda: synth.make_item(113, (6, 6, 6), 1, 3, True, 2, x_min=1.0),
}
_DEG = {}


# Real orbitals: the first-index transform packs two real columns into one
# complex line, and when the plane-wave list is closed under G -> -G only one
# half of the rows is transformed over the second index, the other half
# following by conjugation.  A shuffled closed list makes the -G map
# non-trivial; a list with one point of a +-G pair dropped takes the path that
# transforms every row.
def _real_sphere(kind):
    it = synth.make_item(114, (12, 12, 12), 6, 40, False, 3, x_min=1.0)
    g = np.asarray(it.g_index)
    if kind == "shuffled":
        g = np.random.default_rng(5).permutation(g)
    else:
        g = np.concatenate([g[:7], g[8:]])     # drops m = (-1, -1, 0), keeps (1, 1, 0)
    it.g_index = np.ascontiguousarray(g, dtype=np.int32)
    return it


_REAL = {}


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("herm", [0, 1])
@pytest.mark.parametrize("kind", ["shuffled", "open"])
def test_real_sphere_symmetry(ctx, kind, herm, prec):
    if kind not in _REAL:
        it = _real_sphere(kind)
        _REAL[kind] = (it, oc.chi_omega(it))
    it, ref = _REAL[kind]
    say(f"[real sphere] kind={kind} herm={herm} prec={prec} n_g={len(it.g_index)}")
    ctx.set_options(use_graph=1, hermitian=herm, skip_zero_bands=0, slab_width=0, tile_id=0)
    out = ctx.build([it], prec)[0]
    err = oc.rel_frobenius(out, ref)
    say(f"   err={err:.3e}")
    assert np.all(np.isfinite(out)) and err <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("herm", [0, 1])
@pytest.mark.parametrize("name", list(DEGENERATE))
def test_degenerate_shapes(ctx, name, herm, prec):
    if name not in _DEG:
        it = DEGENERATE[name]()
        _DEG[name] = (it, oc.chi_omega(it))
    it, ref = _DEG[name]
    ctx.set_options(use_graph=1, hermitian=herm, skip_zero_bands=0, slab_width=0, tile_id=0)
    out = ctx.build([it], prec)[0]
    err = oc.rel_frobenius(out, ref)
    say(f"[degenerate] case={name} herm={herm} prec={prec} err={err:.3e}")
    assert err <= TOL[prec]
    # the G = 0 row and column vanish (orthonormal orbitals), up to the
    # rounding level of the path
    scale = np.abs(ref).max()
    assert np.abs(out[:, 0, :]).max() <= 10 * TOL[prec] * scale
    assert np.abs(out[:, :, 0]).max() <= 10 * TOL[prec] * scale


@pytest.mark.parametrize("prec", PRECS)
def test_multi_pass_bitwise(ctx, prec):
    """Jobs split over several passes (an item's taus straddling passes, the
    cosine transform continuing its sums) give the single-pass result bit for
    bit, and stay within tolerance of the oracle."""
    items = [case("cplx8")[0], case("ragged")[0]]
    ctx.set_options(tau_batch=0, use_graph=1)
    one = ctx.build(items, prec)
    ctx.set_options(tau_batch=3)
    many, rep = ctx.build(items, prec, report=True)
    ctx.set_options(tau_batch=0)
    assert rep["tau_batch"] == 3
    for a, b in zip(one, many):
        assert np.array_equal(a, b)
    assert oc.rel_frobenius(many[1], case("ragged")[1]) <= TOL[prec]


def test_small_memory_budget(ctx):
    """A device-memory cap forces narrower slabs and more passes; the result is
    unchanged.  A cap below one job is reported as ENOMEM."""
    it, ref = case("ragged")
    ctx.set_options(max_device_bytes=0)
    a = ctx.build([it], "fp32")[0]
    ctx.set_options(max_device_bytes=80 << 20)
    outs, rep = ctx.build([it], "fp32", report=True)
    b = outs[0]
    assert rep["tau_batch"] < it.n_tau
    assert np.array_equal(a, b)
    ctx.set_options(max_device_bytes=1 << 20)
    with pytest.raises(gwchi.GwchiError) as e:
        ctx.build([it], "fp32")
    assert e.value.status == 2
    ctx.set_options(max_device_bytes=0)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_persistent_matches_one_block_per_tile(ctx, prec):
    """The persistent ticketed launch computes every tile exactly as a launch
    with one workgroup per tile."""
    items = [case("cplx8")[0], case("ragged")[0]]
    ctx.set_options(persistent=1)
    a = ctx.build(items, prec)
    ctx.set_options(persistent=0)
    b = ctx.build(items, prec)
    ctx.set_options(persistent=1)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_autotune_picks_the_fastest_measured_tile(tmp_path):
    """The autotuner measures every tile's GEMM time whatever the context's
    timing option (off here, the default), keeps the fastest, writes it under
    the architecture-keyed name, and later builds use it."""
    import json
    path = str(tmp_path / "tune.json")
    it, ref = case("cfg1")
    big = synth.make_item(141, (16, 16, 16), 32, 480, False, 3, x_min=1.0)
    c = gwchi.Context(0, tune_cache=path)
    assert c.options()["timing"] == 0
    c.autotune([big], "fp32")
    ms, chosen = c.autotune_times("fp32", is_complex=False)
    c.close()
    say(f"[autotune] ms={ms} chosen={chosen}")
    assert all(m > 0 for m in ms)
    assert chosen == int(np.argmin(ms))
    data = json.load(open(path))
    assert data["gfx950/fp32/r"] == chosen
    c2 = gwchi.Context(0, tune_cache=path)
    out, rep = c2.build([it], "fp32", report=True)
    c2.close()
    assert rep["tile_id"] == chosen + 1
    assert oc.rel_frobenius(out[0], ref) <= TOL["fp32"]
