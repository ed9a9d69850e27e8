"""Full-size workload configurations on the GPU, in the launch configuration
the benchmark times (Hermitian completion, persistent launch, graph),
checked against the oracle on sampled rows of chi(i omega) (pair sum + one FFT
over r' per row).  Hermiticity is checked where it is not built in (the
full-matrix tests of the parity suite run without completion).

* 8 k-points on 24^3 with uneven band counts, all in one call;
* 32^3 with 128 + 2048 complex bands;
* 32 real systems of mixed grid size (16^3 .. 28^3), gaps 0.1 .. 10 eV, one call.
"""
import sys

import numpy as np
import pytest

from oracle import chi as oc
from paper_1607_02859_amd import gwchi, synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-4}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = gwchi.Context(0)
    yield c
    c.close()


_ITEMS = {}


def items_of(cfg):
    if cfg not in _ITEMS:
        _ITEMS[cfg] = synth.make_config(cfg)
    return _ITEMS[cfg]


_REF = {}


def ref_rows(cfg, t, rows):
    key = (cfg, t, tuple(rows))
    if key not in _REF:
        _REF[key] = oc.chi_rows(items_of(cfg)[t], list(rows))
    return _REF[key]


def check(cfg, outs, sample, prec):
    worst = 0.0
    for t, rows in sample:
        it = items_of(cfg)[t]
        out = outs[t]
        assert out.shape == (it.n_omega, it.n_g, it.n_g)
        assert np.all(np.isfinite(out))
        err = oc.rel_frobenius(out[:, list(rows), :], ref_rows(cfg, t, rows))
        say(f"   item {t} (n={it.n[0]}, K={it.n_occ}+{it.n_unocc}) rows {rows}: err={err:.3e}")
        worst = max(worst, err)
    assert worst <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp64"])
def test_kpoint_batch_uneven_bands(ctx, prec):
    items = items_of(3)
    say(f"[cfg3] prec={prec} bands={[(i.n_occ, i.n_unocc) for i in items]}")
    ctx.set_options(use_graph=1, hermitian=1, slab_width=0, tile_id=0)
    outs, rep = ctx.build(items, prec, report=True)
    say(f"   ms={rep['ms_total']:.1f} kappa_F={rep['kappa_F_max']:.2f} tau_batch={rep['tau_batch']}")
    check(3, outs, [(0, (0, 700)), (2, (11, 2000)), (5, (3, 2968)), (7, (1, 1234))], prec)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp64"])
def test_32cubed(ctx, prec):
    items = items_of(4)
    say(f"[cfg4] prec={prec}")
    ctx.set_options(use_graph=1, hermitian=1, slab_width=0, tile_id=0)
    outs, rep = ctx.build(items, prec, report=True)
    say(f"   ms={rep['ms_total']:.1f} kappa_F={rep['kappa_F_max']:.2f} slab={rep['slab_width']}")
    check(4, outs, [(0, (1, 100, 2500, 5000, 7122))], prec)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp64"])
def test_multi_system_batch(ctx, prec):
    items = items_of(5)
    say(f"[cfg5] prec={prec} grids={sorted(set(i.n[0] for i in items))}")
    ctx.set_options(use_graph=1, hermitian=1, slab_width=0, tile_id=0)
    outs, rep = ctx.build(items, prec, report=True)
    say(f"   ms={rep['ms_total']:.1f} kappa_F={rep['kappa_F_max']:.2f}")
    # one system of every grid size (16, 18, 20, 24, 28), the smallest and
    # largest gaps among them
    check(5, outs, [(0, (0, 5)), (9, (2, 100)), (16, (3, 1700)), (20, (1, 1000)),
                    (31, (7, 4000))], prec)
