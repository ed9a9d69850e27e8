"""The C-ABI library loads, exports every symbol gwchi.h declares, and its
host-only validation rejects what the header says it rejects (no device is
touched by gwchi_validate)."""
import os
import re

import numpy as np
import pytest

from paper_1607_02859_amd import gwchi, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "gwchi.h")).read()
    # declarations: a return type, the name, then the parameter list
    return sorted(set(re.findall(r"^(?:gwchi_status|const char \*)\s*(gwchi_[a-z_]+)\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gwchi.LIB_PATH):
        from paper_1607_02859_amd import build
        build.build()
    return gwchi.load()


def test_exports_match_header(lib):
    syms = header_symbols()
    assert set(syms) == set(gwchi.EXPORTS)
    for s in syms:
        assert hasattr(lib, s), s


def test_version(lib):
    assert b"gfx950" in lib.gwchi_version()


@pytest.fixture(scope="module")
def item():
    return synth.make_item(7, (6, 5, 4), 3, 9, True, 4, x_min=1.0)


def clone(it, **kw):
    d = dict(it.__dict__)
    d.update(kw)
    return synth.Item(**d)


def test_valid_item_passes(lib, item):
    assert gwchi.validate([item]) == 0


@pytest.mark.parametrize("mut", [
    lambda it: clone(it, mu=float(it.eps_unocc.min()) + 0.1),          # mu above the gap
    lambda it: clone(it, mu=float(it.eps_occ.max())),                   # mu on an edge
    lambda it: clone(it, tau=np.concatenate([it.tau[:-1], [0.0]])),     # tau <= 0
    lambda it: clone(it, tau=np.concatenate([it.tau[:-1], [np.nan]])),  # non-finite tau
    lambda it: clone(it, ct=it.ct * np.inf),                            # non-finite ct
    lambda it: clone(it, g_index=np.array([0, 1, 1], np.int32)),        # duplicate G
    lambda it: clone(it, g_index=np.array([0, 120], np.int32)),         # G out of range
    lambda it: clone(it, g_index=np.array([-1], np.int32)),
    lambda it: clone(it, eps_occ=np.array([np.nan, -1.0, -2.0])),
])
def test_validate_rejects(lib, item, mut):
    assert gwchi.validate([mut(item)]) == 1


def test_validate_nonfinite_orbital(lib, item):
    bad = clone(item, phi_occ=item.phi_occ.copy())
    bad.phi_occ[1, 3] = np.nan
    assert gwchi.validate([bad], check_orbitals=True) == 1
    assert gwchi.validate([bad], check_orbitals=False) == 0


def test_validate_unsupported_grid(lib):
    it = synth.make_item(8, (11, 4, 4), 2, 5, True, 3, x_min=1.0)   # 11 is not 7-smooth
    assert gwchi.validate([it]) == 4
    it = synth.make_item(8, (33, 1, 1), 2, 5, True, 3, x_min=1.0)   # > 32
    assert gwchi.validate([it]) == 4


def test_validate_empty_batch(lib):
    arr = (gwchi.GwchiItem * 1)()
    assert lib.gwchi_validate(arr, 0, 1) == 1
    assert b"n_items" in lib.gwchi_last_error(None)


def test_validate_null_pointer(lib, item):
    keep = gwchi._Keep()
    it = gwchi.make_item(keep, item, chi_out=np.zeros(1, complex))
    it.g_index = 0
    arr = (gwchi.GwchiItem * 1)(it)
    assert lib.gwchi_validate(arr, 1, 1) == 1
    assert b"NULL" in lib.gwchi_last_error(None)


def test_struct_layout_matches_header(lib, tmp_path):
    """Every field offset of the ctypes mirrors equals the C compiler's."""
    import ctypes as C
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gwchi.h"', 'int main(void){']
    mirrors = [("gwchi_item", gwchi.GwchiItem), ("gwchi_report", gwchi.GwchiReport),
               ("gwchi_options", gwchi.GwchiOptions), ("gwchi_w_item", gwchi.GwchiWItem),
               ("gwchi_w_report", gwchi.GwchiWReport), ("gwchi_pade_item", gwchi.GwchiPadeItem),
               ("gwchi_sigma_item", gwchi.GwchiSigmaItem),
               ("gwchi_sigma_report", gwchi.GwchiSigmaReport)]
    for cname, py in mirrors:
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = []
    for _, py in mirrors:
        want.append(C.sizeof(py))
        want += [getattr(py, f).offset for f, _ in py._fields_]
    assert got == want


# ---- screened-interaction entry: host-only validation ----------------------

@pytest.fixture(scope="module")
def witem():
    return synth.make_w_item(5, (12, 12, 12), 6)


def test_w_valid_item_passes(lib, witem):
    assert gwchi.w_validate([witem]) == 0


def _w_mut(witem, **kw):
    import copy
    w = copy.copy(witem)
    for k, v in kw.items():
        setattr(w, k, v)
    return w


@pytest.mark.parametrize("mut", [
    "neg_s", "nan_s", "nan_ct", "singular_ct", "non_square", "too_many_tau"])
def test_w_validate_rejects(lib, witem, mut):
    if mut == "neg_s":
        s = witem.sqrt_v.copy()
        s[3] = -1.0
        w = _w_mut(witem, sqrt_v=s)
    elif mut == "nan_s":
        s = witem.sqrt_v.copy()
        s[0] = np.nan
        w = _w_mut(witem, sqrt_v=s)
    elif mut == "nan_ct":
        c = witem.ct.copy()
        c[1, 2] = np.inf
        w = _w_mut(witem, ct=c)
    elif mut == "singular_ct":
        c = witem.ct.copy()
        c[1] = c[0]
        w = _w_mut(witem, ct=c)
    elif mut == "non_square":
        w = _w_mut(witem, ct=witem.ct[:, :-1].copy())
    else:
        n = 33
        w = _w_mut(witem, ct=np.eye(n), chi=np.zeros((n, 4, 4), np.complex128),
                   sqrt_v=np.ones(4))
    assert gwchi.w_validate([w]) == 1


def test_w_validate_empty_and_null(lib, witem):
    import ctypes as C
    assert lib.gwchi_w_validate(None, 0) == 1
    keep = gwchi._Keep()
    it = gwchi.make_w_item(keep, witem, w_tau=None)
    arr = (gwchi.GwchiWItem * 1)(it)
    assert lib.gwchi_w_validate(arr, 1) == 1
    assert b"NULL" in lib.gwchi_last_error(None)


# ---- analytic continuation: host-only validation ---------------------------

@pytest.fixture(scope="module")
def pade_in():
    z, f, w, *_ = synth.make_pade_input(3, 5, 12, 40)
    return z, f, w


def test_pade_valid_passes(lib, pade_in):
    assert gwchi.pade_validate(*pade_in) == 0


@pytest.mark.parametrize("mut", ["repeated_z", "nan_z", "inf_w", "too_many_points", "no_points"])
def test_pade_validate_rejects(lib, pade_in, mut):
    z, f, w = (x.copy() for x in pade_in)
    if mut == "repeated_z":
        z[5] = z[2]
    elif mut == "nan_z":
        z[0] = np.nan
    elif mut == "inf_w":
        w[3] = np.inf
    elif mut == "too_many_points":
        z = 1j * np.arange(1, 34, dtype=float)
        f = np.ones((5, 33), np.complex128)
    else:
        z = np.zeros(0, np.complex128)
        f = np.ones((5, 0), np.complex128)
    assert gwchi.pade_validate(z, f, w) == 1


def test_pade_validate_null(lib):
    assert lib.gwchi_pade_validate(None) == 1


def test_validate_rejects_mixed_real_and_complex(lib):
    real = synth.make_item(7, (4, 4, 4), 2, 6, False, 3, x_min=1.0)
    cplx = synth.make_item(8, (4, 4, 4), 2, 6, True, 3, x_min=1.0)
    assert gwchi.validate([real, real]) == 0
    assert gwchi.validate([cplx, cplx]) == 0
    assert gwchi.validate([real, cplx]) == 1
    assert b"all real or all complex" in lib.gwchi_last_error(None)


# ---- self-energy entry: host-only validation --------------------------------

@pytest.fixture(scope="module")
def sitem():
    return synth.make_sigma_item(9, (6, 5, 4), 3, 9, 4, 4)


def _s_mut(sitem, **kw):
    d = dict(sitem.__dict__)
    d.update(kw)
    return synth.SigmaItem(**d)


def test_sigma_valid_item_passes(lib, sitem):
    assert gwchi.sigma_validate([sitem]) == 0


@pytest.mark.parametrize("mut", ["state_high", "state_neg", "nan_st", "mu_in_band", "tau_zero",
                                 "no_states", "too_many_states"])
def test_sigma_validate_rejects(lib, sitem, mut):
    if mut == "state_high":
        w = _s_mut(sitem, states=np.array([0, 12], np.int32))
    elif mut == "state_neg":
        w = _s_mut(sitem, states=np.array([-1], np.int32))
    elif mut == "nan_st":
        st = sitem.st.copy()
        st[0, 1] = np.nan
        w = _s_mut(sitem, st=st)
    elif mut == "mu_in_band":
        w = _s_mut(sitem, mu=float(sitem.eps_unocc.min()) + 0.1)
    elif mut == "tau_zero":
        w = _s_mut(sitem, tau=np.concatenate([sitem.tau[:-1], [0.0]]))
    elif mut == "no_states":
        w = _s_mut(sitem, states=np.zeros(0, np.int32))
    else:
        w = _s_mut(sitem, states=np.zeros(1025, np.int32))
    assert gwchi.sigma_validate([w]) == 1


def test_sigma_validate_real_orbitals_unsupported(lib, sitem):
    w = _s_mut(sitem, phi_occ=sitem.phi_occ.real.copy(), phi_unocc=sitem.phi_unocc.real.copy())
    assert gwchi.sigma_validate([w]) == 4
    assert b"real orbitals" in lib.gwchi_last_error(None)


def test_sigma_validate_null(lib, sitem):
    keep = gwchi._Keep()
    it = gwchi.make_sigma_item(keep, sitem, sigma_out=None)
    arr = (gwchi.GwchiSigmaItem * 1)(it)
    assert lib.gwchi_sigma_validate(arr, 1, 1) == 1
    assert b"NULL" in lib.gwchi_last_error(None)
    assert lib.gwchi_sigma_validate(None, 0, 1) == 1
