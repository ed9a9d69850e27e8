"""The allocation-free build (gwchi_chi_build_device_noalloc) against the
device build it mirrors (gwchi_chi_build_device), through the C ABI, on two
calls in a row -- the second with a smaller input, so it runs over the first
call's leftovers in the fixed scratch -- in every precision, to the parity
bounds (max relative Frobenius error 1e-10 / 1e-5 / 1e-4), and the error
for a job that cannot fit the fixed scratch."""
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


def _run(ctx, it, prec, noalloc):
    import torch
    dev = torch.device("cuda:0")
    po = torch.from_numpy(it.phi_occ).to(dev)
    pu = torch.from_numpy(it.phi_unocc).to(dev)
    out = torch.full((it.n_omega, it.n_g, it.n_g), float("nan"), dtype=torch.complex128,
                     device=dev)
    if noalloc:
        ctx.build_device_noalloc([it], [(po, pu)], [out], prec)
    else:
        ctx.build_device([it], [(po, pu)], [out], prec)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_noalloc_matches_device_entry_twice(ctx, prec):
    big = synth.make_config(1)[0]                                     # 12^3 real, 6 taus
    small = synth.make_item(151, (8, 8, 8), 8, 40, True, 4, x_min=1.0)   # 8^3 complex
    ctx.set_options(use_graph=1, hermitian=1, skip_zero_bands=0, slab_width=0, tile_id=0)
    for name, it in (("12^3 real", big), ("8^3 complex", small)):
        say(f"[noalloc] prec={prec} case={name}")
        ref = _run(ctx, it, prec, noalloc=False)
        got = _run(ctx, it, prec, noalloc=True)
        assert np.all(np.isfinite(got))
        err = oc.rel_frobenius(got, ref)
        say(f"   vs device entry: rel err={err:.3e} identical={np.array_equal(got, ref)}")
        assert err <= TOL[prec]


def test_noalloc_rejects_a_job_beyond_the_scratch(ctx):
    import torch
    it = synth.make_item(152, (32, 32, 32), 4, 20, True, 2, x_min=1.0)
    dev = torch.device("cuda:0")
    po = torch.from_numpy(it.phi_occ).to(dev)
    pu = torch.from_numpy(it.phi_unocc).to(dev)
    out = torch.empty((it.n_omega, it.n_g, it.n_g), dtype=torch.complex128, device=dev)
    with pytest.raises(gwchi.GwchiError) as e:
        ctx.build_device_noalloc([it], [(po, pu)], [out], "fp32")
    say(f"[noalloc] 32^3: {e.value}")
    assert e.value.status == 2 and "fixed scratch" in str(e.value)
    # the entry still works afterwards
    small = synth.make_item(153, (6, 6, 6), 4, 20, False, 3, x_min=1.0)
    got = _run(ctx, small, "fp64", noalloc=True)
    assert oc.rel_frobenius(got, oc.chi_omega(small)) <= TOL["fp64"]
