"""ctypes binding of libgwchi.so (gwchi.h): argument marshalling only.

Every step of the polarizability build runs in the library's HIP kernels.
There is no CPU fallback: if the shared library is missing, importing the
compute entry points raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgwchi.so")

FP64, FP32, BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOTSUP", 5: "ENUMERIC"}

EXPORTS = ["gwchi_create", "gwchi_destroy", "gwchi_set_options", "gwchi_get_options",
           "gwchi_validate", "gwchi_chi_build", "gwchi_chi_build_device", "gwchi_autotune",
           "gwchi_autotune_times", "gwchi_last_error", "gwchi_version", "gwchi_w_build",
           "gwchi_w_build_device", "gwchi_w_validate", "gwchi_pade", "gwchi_pade_device",
           "gwchi_pade_validate", "gwchi_chi_build_device_noalloc", "gwchi_sigma_validate",
           "gwchi_sigma_build", "gwchi_sigma_build_device"]


class GwchiItem(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3),
        ("is_complex", C.c_int32),
        ("n_occ", C.c_int32),
        ("n_unocc", C.c_int32),
        ("phi_occ", C.c_void_p),
        ("phi_unocc", C.c_void_p),
        ("eps_occ", C.c_void_p),
        ("eps_unocc", C.c_void_p),
        ("mu", C.c_double),
        ("n_tau", C.c_int32),
        ("n_omega", C.c_int32),
        ("tau", C.c_void_p),
        ("ct", C.c_void_p),
        ("n_g", C.c_int32),
        ("g_index", C.c_void_p),
        ("chi_out", C.c_void_p),
    ]


class GwchiReport(C.Structure):
    _fields_ = [
        ("ms_total", C.c_double),
        ("ms_stage", C.c_double),
        ("ms_gemm", C.c_double),
        ("ms_fft_r", C.c_double),
        ("ms_fft_rp", C.c_double),
        ("ms_ct", C.c_double),
        ("n_gemm_launches", C.c_int32),
        ("n_fft_launches", C.c_int32),
        ("alg_flops", C.c_double),
        ("mfma_flops", C.c_double),
        ("slab_width", C.c_int32),
        ("tau_batch", C.c_int32),
        ("tile_id", C.c_int32),
        ("graph_replayed", C.c_int32),
        ("kappa_F_max", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GwchiOptions(C.Structure):
    _fields_ = [
        ("slab_width", C.c_int32),
        ("tau_batch", C.c_int32),
        ("tile_id", C.c_int32),
        ("use_graph", C.c_int32),
        ("check_output", C.c_int32),
        ("timing", C.c_int32),
        ("skip_zero_bands", C.c_int32),
        ("hermitian", C.c_int32),
        ("persistent", C.c_int32),
        ("kappa", C.c_int32),
        ("max_device_bytes", C.c_int64),
    ]


class GwchiWItem(C.Structure):
    _fields_ = [
        ("n_g", C.c_int32),
        ("n_omega", C.c_int32),
        ("n_tau", C.c_int32),
        ("chi", C.c_void_p),
        ("sqrt_v", C.c_void_p),
        ("ct", C.c_void_p),
        ("w_tau_out", C.c_void_p),
        ("w_omega_out", C.c_void_p),
    ]


class GwchiWReport(C.Structure):
    _fields_ = [
        ("ms_total", C.c_double),
        ("ms_eps", C.c_double),
        ("ms_invert", C.c_double),
        ("ms_final", C.c_double),
        ("alg_flops", C.c_double),
        ("n_launches", C.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GwchiSigmaItem(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3),
        ("is_complex", C.c_int32),
        ("n_occ", C.c_int32),
        ("n_unocc", C.c_int32),
        ("phi_occ", C.c_void_p),
        ("phi_unocc", C.c_void_p),
        ("eps_occ", C.c_void_p),
        ("eps_unocc", C.c_void_p),
        ("mu", C.c_double),
        ("n_tau", C.c_int32),
        ("n_omega", C.c_int32),
        ("tau", C.c_void_p),
        ("ct", C.c_void_p),
        ("st", C.c_void_p),
        ("n_g", C.c_int32),
        ("g_index", C.c_void_p),
        ("w_tau", C.c_void_p),
        ("n_states", C.c_int32),
        ("states", C.c_void_p),
        ("sigma_out", C.c_void_p),
        ("sigma_tau_out", C.c_void_p),
    ]


class GwchiSigmaReport(C.Structure):
    _fields_ = [
        ("ms_total", C.c_double),
        ("ms_stage", C.c_double),
        ("ms_fft", C.c_double),
        ("ms_gemm", C.c_double),
        ("ms_final", C.c_double),
        ("n_gemm_launches", C.c_int32),
        ("slab_width", C.c_int32),
        ("tau_batch", C.c_int32),
        ("alg_flops", C.c_double),
        ("mfma_flops", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GwchiPadeItem(C.Structure):
    _fields_ = [
        ("n_points", C.c_int32),
        ("z", C.c_void_p),
        ("n_fun", C.c_int32),
        ("f", C.c_void_p),
        ("n_eval", C.c_int32),
        ("w", C.c_void_p),
        ("out", C.c_void_p),
        ("coef", C.c_void_p),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} not built; run paper_1607_02859_amd/build.py")
    # PyTorch-ROCm ships its own HIP runtime with the same soname.  Loading
    # torch first makes this library bind to that runtime, so that torch
    # tensors, streams and this library share one HIP runtime in the process.
    try:
        import torch  # noqa: F401
    except Exception:
        pass
    lib = C.CDLL(path)
    P = C.POINTER
    lib.gwchi_create.argtypes = [P(C.c_void_p), C.c_int32, C.c_char_p]
    lib.gwchi_destroy.argtypes = [C.c_void_p]
    lib.gwchi_set_options.argtypes = [C.c_void_p, P(GwchiOptions)]
    lib.gwchi_get_options.argtypes = [C.c_void_p, P(GwchiOptions)]
    lib.gwchi_validate.argtypes = [P(GwchiItem), C.c_int32, C.c_int32]
    lib.gwchi_chi_build.argtypes = [C.c_void_p, P(GwchiItem), C.c_int32, C.c_int, P(GwchiReport)]
    lib.gwchi_chi_build_device.argtypes = [C.c_void_p, P(GwchiItem), C.c_int32, C.c_int,
                                           C.c_void_p, P(GwchiReport)]
    lib.gwchi_autotune.argtypes = [C.c_void_p, P(GwchiItem), C.c_int32, C.c_int]
    lib.gwchi_chi_build_device_noalloc.argtypes = [C.c_void_p, P(GwchiItem), C.c_int32, C.c_int,
                                                   C.c_void_p]
    lib.gwchi_autotune_times.argtypes = [C.c_void_p, C.c_int, C.c_int32, P(C.c_double), C.c_int32,
                                         P(C.c_int32)]
    lib.gwchi_w_build.argtypes = [C.c_void_p, P(GwchiWItem), C.c_int32, P(GwchiWReport)]
    lib.gwchi_sigma_validate.argtypes = [P(GwchiSigmaItem), C.c_int32, C.c_int32]
    lib.gwchi_sigma_build.argtypes = [C.c_void_p, P(GwchiSigmaItem), C.c_int32, C.c_int,
                                      P(GwchiSigmaReport)]
    lib.gwchi_sigma_build_device.argtypes = [C.c_void_p, P(GwchiSigmaItem), C.c_int32, C.c_int,
                                             C.c_void_p, P(GwchiSigmaReport)]
    lib.gwchi_w_validate.argtypes = [P(GwchiWItem), C.c_int32]
    lib.gwchi_pade_validate.argtypes = [P(GwchiPadeItem)]
    lib.gwchi_pade.argtypes = [C.c_void_p, P(GwchiPadeItem), P(C.c_double)]
    lib.gwchi_pade_device.argtypes = [C.c_void_p, P(GwchiPadeItem), C.c_void_p, P(C.c_double)]
    lib.gwchi_w_build_device.argtypes = [C.c_void_p, P(GwchiWItem), C.c_int32, C.c_void_p,
                                         P(GwchiWReport)]
    lib.gwchi_last_error.argtypes = [C.c_void_p]
    lib.gwchi_last_error.restype = C.c_char_p
    lib.gwchi_version.restype = C.c_char_p
    for f in ("gwchi_create", "gwchi_destroy", "gwchi_set_options", "gwchi_get_options",
              "gwchi_validate", "gwchi_chi_build", "gwchi_chi_build_device", "gwchi_autotune",
              "gwchi_autotune_times", "gwchi_w_build", "gwchi_w_build_device", "gwchi_w_validate",
              "gwchi_pade", "gwchi_pade_device", "gwchi_pade_validate",
              "gwchi_chi_build_device_noalloc", "gwchi_sigma_validate", "gwchi_sigma_build",
              "gwchi_sigma_build_device"):
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


class GwchiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _ptr(a) -> int:
    if a is None:
        return 0
    if hasattr(a, "data_ptr"):      # torch tensor
        return int(a.data_ptr())
    return int(a.ctypes.data)


class _Keep:
    """Holds host arrays alive while the library reads them."""

    def __init__(self):
        self.refs = []

    def f64(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        self.refs.append(a)
        return a

    def i32(self, a):
        a = np.ascontiguousarray(a, dtype=np.int32)
        self.refs.append(a)
        return a


def make_item(keep: _Keep, item, phi_occ=None, phi_unocc=None, chi_out=None) -> GwchiItem:
    """Fill a GwchiItem from a synth.Item.  phi_* and chi_out default to host
    arrays taken from ``item``; pass device tensors for the device entry."""
    it = GwchiItem()
    it.n[0], it.n[1], it.n[2] = (int(v) for v in item.n)
    cplx = bool(np.iscomplexobj(item.phi_occ))
    it.is_complex = 1 if cplx else 0
    it.n_occ = item.phi_occ.shape[0]
    it.n_unocc = item.phi_unocc.shape[0]
    if phi_occ is None:
        dt = np.complex128 if cplx else np.float64
        phi_occ = np.ascontiguousarray(item.phi_occ, dtype=dt)
        phi_unocc = np.ascontiguousarray(item.phi_unocc, dtype=dt)
        keep.refs += [phi_occ, phi_unocc]
    it.phi_occ = _ptr(phi_occ)
    it.phi_unocc = _ptr(phi_unocc)
    it.eps_occ = _ptr(keep.f64(item.eps_occ))
    it.eps_unocc = _ptr(keep.f64(item.eps_unocc))
    it.mu = float(item.mu)
    it.n_tau = int(np.asarray(item.tau).shape[0])
    it.n_omega = int(np.asarray(item.ct).shape[0])
    it.tau = _ptr(keep.f64(item.tau))
    it.ct = _ptr(keep.f64(item.ct))
    g = keep.i32(item.g_index)
    it.n_g = int(g.shape[0])
    it.g_index = _ptr(g)
    it.chi_out = _ptr(chi_out)
    return it


def make_w_item(keep: _Keep, witem, chi=None, w_tau=None, w_omega=None) -> GwchiWItem:
    """Fill a GwchiWItem from a synth.WItem (or any object with ``chi``,
    ``sqrt_v`` and ``ct``).  ``chi`` defaults to the host array of the item;
    pass device tensors (and device outputs) for the device entry."""
    it = GwchiWItem()
    ct = keep.f64(witem.ct)
    it.n_omega, it.n_tau = int(ct.shape[0]), int(ct.shape[1])
    if chi is None:
        chi = np.ascontiguousarray(witem.chi, dtype=np.complex128)
        keep.refs.append(chi)
    it.n_g = int(chi.shape[1])
    it.chi = _ptr(chi)
    it.sqrt_v = _ptr(keep.f64(witem.sqrt_v))
    it.ct = _ptr(ct)
    it.w_tau_out = _ptr(w_tau)
    it.w_omega_out = _ptr(w_omega)
    return it


def make_sigma_item(keep: _Keep, item, phi_occ=None, phi_unocc=None, w_tau=None, sigma_out=None,
                    sigma_tau_out=None) -> GwchiSigmaItem:
    """Fill a GwchiSigmaItem from a synth.SigmaItem.  Orbitals and W~ default to
    host arrays of ``item``; pass device tensors (and device outputs) for the
    device entry."""
    it = GwchiSigmaItem()
    it.n[0], it.n[1], it.n[2] = (int(v) for v in item.n)
    it.is_complex = 1 if np.iscomplexobj(item.phi_occ) else 0
    it.n_occ = item.phi_occ.shape[0]
    it.n_unocc = item.phi_unocc.shape[0]
    if phi_occ is None:
        dt = np.complex128 if it.is_complex else np.float64
        phi_occ = np.ascontiguousarray(item.phi_occ, dtype=dt)
        phi_unocc = np.ascontiguousarray(item.phi_unocc, dtype=dt)
        keep.refs += [phi_occ, phi_unocc]
    if w_tau is None:
        w_tau = np.ascontiguousarray(item.w_tau, dtype=np.complex128)
        keep.refs.append(w_tau)
    it.phi_occ = _ptr(phi_occ)
    it.phi_unocc = _ptr(phi_unocc)
    it.eps_occ = _ptr(keep.f64(item.eps_occ))
    it.eps_unocc = _ptr(keep.f64(item.eps_unocc))
    it.mu = float(item.mu)
    it.n_tau = int(np.asarray(item.tau).shape[0])
    it.n_omega = int(np.asarray(item.ct).shape[0])
    it.tau = _ptr(keep.f64(item.tau))
    it.ct = _ptr(keep.f64(item.ct))
    it.st = _ptr(keep.f64(item.st))
    g = keep.i32(item.g_index)
    it.n_g = int(g.shape[0])
    it.g_index = _ptr(g)
    it.w_tau = _ptr(w_tau)
    s = keep.i32(item.states)
    it.n_states = int(s.shape[0])
    it.states = _ptr(s)
    it.sigma_out = _ptr(sigma_out)
    it.sigma_tau_out = _ptr(sigma_tau_out)
    return it


def sigma_validate(items, check_orbitals=True) -> int:
    """gwchi_sigma_validate on host arrays; returns the status code."""
    lib = load()
    keep = _Keep()
    its = []
    for it in items:
        o = np.zeros(1, np.complex128)
        keep.refs.append(o)
        its.append(make_sigma_item(keep, it, sigma_out=o))
    arr = (GwchiSigmaItem * len(its))(*its)
    return int(lib.gwchi_sigma_validate(arr, len(its), 1 if check_orbitals else 0))


def validate(items, check_orbitals=True) -> int:
    """gwchi_validate on host arrays; returns the status code."""
    lib = load()
    keep = _Keep()
    outs = [np.zeros(1, np.complex128) for _ in items]
    arr = (GwchiItem * len(items))(*[make_item(keep, it, chi_out=o) for it, o in zip(items, outs)])
    return int(lib.gwchi_validate(arr, len(items), 1 if check_orbitals else 0))


def w_validate(witems) -> int:
    """gwchi_w_validate on host arrays; returns the status code."""
    lib = load()
    keep = _Keep()
    its = []
    for w in witems:
        t = np.zeros(1, np.complex128)
        keep.refs.append(t)
        its.append(make_w_item(keep, w, w_tau=t))
    arr = (GwchiWItem * len(its))(*its)
    return int(lib.gwchi_w_validate(arr, len(its)))


def make_pade_item(keep: _Keep, z, f, w, out, coef=None) -> GwchiPadeItem:
    """Fill a GwchiPadeItem: z [N] and w [M] host complex arrays; f [n_fun][N],
    out [n_fun][M] and coef [n_fun][N] host arrays or device tensors (complex128)."""
    it = GwchiPadeItem()
    z = np.ascontiguousarray(z, dtype=np.complex128)
    w = np.ascontiguousarray(w, dtype=np.complex128)
    keep.refs += [z, w]
    it.n_points = int(z.shape[0])
    it.z = _ptr(z)
    it.n_fun = int(f.shape[0])
    it.f = _ptr(f)
    it.n_eval = int(w.shape[0])
    it.w = _ptr(w) if w.shape[0] > 0 else 0
    it.out = _ptr(out)
    it.coef = _ptr(coef)
    return it


def pade_validate(z, f, w) -> int:
    """gwchi_pade_validate on host arrays; returns the status code."""
    lib = load()
    keep = _Keep()
    f = np.ascontiguousarray(f, dtype=np.complex128)
    out = np.zeros((f.shape[0], max(1, len(w))), np.complex128)
    keep.refs += [f, out]
    it = make_pade_item(keep, z, f, w, out)
    return int(lib.gwchi_pade_validate(C.byref(it)))


class Context:
    """One gwchi context on a HIP device."""

    def __init__(self, device: int = 0, tune_cache: Optional[str] = None, **options):
        self.lib = load()
        h = C.c_void_p()
        st = self.lib.gwchi_create(C.byref(h), int(device),
                                   tune_cache.encode() if tune_cache else None)
        if st != 0:
            raise GwchiError(st, self.lib.gwchi_last_error(None).decode())
        self.h = h
        if options:
            self.set_options(**options)

    def close(self):
        if getattr(self, "h", None):
            self.lib.gwchi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, st):
        return GwchiError(st, self.lib.gwchi_last_error(self.h).decode())

    def options(self) -> dict:
        o = GwchiOptions()
        self.lib.gwchi_get_options(self.h, C.byref(o))
        return {k: getattr(o, k) for k, _ in o._fields_}

    def set_options(self, **kw):
        cur = self.options()
        cur.update(kw)
        o = GwchiOptions(**cur)
        st = self.lib.gwchi_set_options(self.h, C.byref(o))
        if st != 0:
            raise self._err(st)

    def build(self, items: Sequence, prec="fp32", report=False):
        """Host-memory build: returns a list of complex128 arrays
        (n_omega, n_g, n_g) and optionally the report dict."""
        keep = _Keep()
        outs = [np.empty((np.asarray(it.ct).shape[0], len(it.g_index), len(it.g_index)),
                         np.complex128) for it in items]
        arr = (GwchiItem * len(items))(*[make_item(keep, it, chi_out=o) for it, o in zip(items, outs)])
        rep = GwchiReport()
        st = self.lib.gwchi_chi_build(self.h, arr, len(items), PRECISIONS[prec],
                                      C.byref(rep) if report else None)
        if st != 0:
            raise self._err(st)
        return (outs, rep.as_dict()) if report else outs

    def build_device(self, items: Sequence, phis, outs, prec="fp32", stream=None, report=False):
        """Device-memory build.  ``phis`` is a list of (phi_occ, phi_unocc)
        device tensors (float64 real or complex128 complex, band-major) and
        ``outs`` a list of complex128 device tensors (n_omega, n_g, n_g).
        ``stream`` is a torch.cuda.Stream or None (the current stream)."""
        keep = _Keep()
        arr = (GwchiItem * len(items))(*[
            make_item(keep, it, phi_occ=p[0], phi_unocc=p[1], chi_out=o)
            for it, p, o in zip(items, phis, outs)])
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        sh = int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream or 0)
        rep = GwchiReport()
        st = self.lib.gwchi_chi_build_device(self.h, arr, len(items), PRECISIONS[prec],
                                             C.c_void_p(sh), C.byref(rep) if report else None)
        if st != 0:
            raise self._err(st)
        return rep.as_dict() if report else None

    def build_device_noalloc(self, items: Sequence, phis, outs, prec="fp32", stream=None):
        """gwchi_chi_build_device_noalloc: as build_device, every scratch buffer
        in the library's fixed device array (no allocation, no report)."""
        keep = _Keep()
        arr = (GwchiItem * len(items))(*[
            make_item(keep, it, phi_occ=p[0], phi_unocc=p[1], chi_out=o)
            for it, p, o in zip(items, phis, outs)])
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        sh = int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream or 0)
        st = self.lib.gwchi_chi_build_device_noalloc(self.h, arr, len(items), PRECISIONS[prec],
                                                     C.c_void_p(sh))
        if st != 0:
            raise self._err(st)

    def autotune(self, items: Sequence, prec="fp32"):
        keep = _Keep()
        outs = [np.empty((np.asarray(it.ct).shape[0], len(it.g_index), len(it.g_index)),
                         np.complex128) for it in items]
        arr = (GwchiItem * len(items))(*[make_item(keep, it, chi_out=o) for it, o in zip(items, outs)])
        st = self.lib.gwchi_autotune(self.h, arr, len(items), PRECISIONS[prec])
        if st != 0:
            raise self._err(st)

    def autotune_times(self, prec="fp32", is_complex=True, n=6):
        """(GEMM ms per tile measured by the last autotune of this family,
        index of the tile kept)."""
        ms = (C.c_double * n)()
        chosen = C.c_int32(-1)
        st = self.lib.gwchi_autotune_times(self.h, PRECISIONS[prec], 1 if is_complex else 0, ms, n,
                                           C.byref(chosen))
        if st != 0:
            raise self._err(st)
        return list(ms), int(chosen.value)

    def w_build(self, witems: Sequence, omega=False, report=False):
        """Host-memory W~ (gwchi_w_build): returns a list of complex128 arrays
        W~(i tau) (n_tau, n_g, n_g), with W~(i omega) when ``omega``, and the
        report dict when ``report``."""
        keep = _Keep()
        taus, oms, its = [], [], []
        for w in witems:
            n_g, K = w.chi.shape[1], w.chi.shape[0]
            t = np.empty((np.asarray(w.ct).shape[1], n_g, n_g), np.complex128)
            o = np.empty((K, n_g, n_g), np.complex128) if omega else None
            taus.append(t)
            oms.append(o)
            its.append(make_w_item(keep, w, w_tau=t, w_omega=o))
        arr = (GwchiWItem * len(its))(*its)
        rep = GwchiWReport()
        st = self.lib.gwchi_w_build(self.h, arr, len(its), C.byref(rep) if report else None)
        if st != 0:
            raise self._err(st)
        out = (taus, oms) if omega else taus
        return (out, rep.as_dict()) if report else out

    def w_build_device(self, witems: Sequence, chis, w_taus, w_omegas=None, stream=None,
                       report=False):
        """Device-memory W~ (gwchi_w_build_device).  ``chis``: complex128 device
        tensors (n_omega, n_g, n_g); ``w_taus`` (and optionally ``w_omegas``):
        complex128 device outputs."""
        keep = _Keep()
        if w_omegas is None:
            w_omegas = [None] * len(witems)
        arr = (GwchiWItem * len(witems))(*[
            make_w_item(keep, w, chi=c, w_tau=t, w_omega=o)
            for w, c, t, o in zip(witems, chis, w_taus, w_omegas)])
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        sh = int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream or 0)
        rep = GwchiWReport()
        st = self.lib.gwchi_w_build_device(self.h, arr, len(witems), C.c_void_p(sh),
                                           C.byref(rep) if report else None)
        if st != 0:
            raise self._err(st)
        return rep.as_dict() if report else None

    def sigma_build(self, items: Sequence, prec="fp32", tau_out=False, report=False):
        """Host-memory self-energy (gwchi_sigma_build): returns a list of
        complex128 arrays Sigma_nn(i omega) (n_states, n_omega), with the
        (n_states, n_tau, 2) tau-domain elements when ``tau_out`` and the
        report dict when ``report``."""
        keep = _Keep()
        outs, taus, its = [], [], []
        for it in items:
            o = np.empty((len(it.states), np.asarray(it.ct).shape[0]), np.complex128)
            t = np.empty((len(it.states), len(it.tau), 2), np.float64) if tau_out else None
            outs.append(o)
            taus.append(t)
            its.append(make_sigma_item(keep, it, sigma_out=o, sigma_tau_out=t))
        arr = (GwchiSigmaItem * len(its))(*its)
        rep = GwchiSigmaReport()
        st = self.lib.gwchi_sigma_build(self.h, arr, len(its), PRECISIONS[prec],
                                        C.byref(rep) if report else None)
        if st != 0:
            raise self._err(st)
        res = (outs, taus) if tau_out else outs
        return (res, rep.as_dict()) if report else res

    def sigma_build_device(self, items: Sequence, phis, w_taus, outs, tau_outs=None, prec="fp32",
                           stream=None, report=False):
        """Device-memory self-energy (gwchi_sigma_build_device): ``phis`` a list
        of (phi_occ, phi_unocc) complex128 device tensors, ``w_taus`` complex128
        device tensors (n_tau, n_g, n_g), ``outs`` complex128 device outputs
        (n_states, n_omega), ``tau_outs`` optional float64 (n_states, n_tau, 2)."""
        keep = _Keep()
        if tau_outs is None:
            tau_outs = [None] * len(items)
        arr = (GwchiSigmaItem * len(items))(*[
            make_sigma_item(keep, it, phi_occ=p[0], phi_unocc=p[1], w_tau=w, sigma_out=o,
                            sigma_tau_out=t)
            for it, p, w, o, t in zip(items, phis, w_taus, outs, tau_outs)])
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        sh = int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream or 0)
        rep = GwchiSigmaReport()
        st = self.lib.gwchi_sigma_build_device(self.h, arr, len(items), PRECISIONS[prec],
                                               C.c_void_p(sh), C.byref(rep) if report else None)
        if st != 0:
            raise self._err(st)
        return rep.as_dict() if report else None

    def pade(self, z, f, w, coef=False, report=False):
        """Host-memory continuation (gwchi_pade): f [n_fun][N] complex at the
        points z [N]; returns P_N at w [M] as [n_fun][M] (and the coefficients
        [n_fun][N] when ``coef``; the kernel time in ms when ``report``)."""
        keep = _Keep()
        f = np.ascontiguousarray(f, dtype=np.complex128)
        out = np.empty((f.shape[0], len(w)), np.complex128)
        cf = np.empty_like(f) if coef else None
        keep.refs += [f, out]
        it = make_pade_item(keep, z, f, w, out, cf)
        ms = C.c_double(0.0)
        st = self.lib.gwchi_pade(self.h, C.byref(it), C.byref(ms))
        if st != 0:
            raise self._err(st)
        res = (out, cf) if coef else out
        return (res, ms.value) if report else res

    def pade_device(self, z, f, w, out, coef=None, stream=None, report=False):
        """Device-memory continuation (gwchi_pade_device): f, out (and coef)
        complex128 device tensors; z and w host arrays."""
        keep = _Keep()
        it = make_pade_item(keep, z, f, w, out, coef)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        sh = int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream or 0)
        ms = C.c_double(0.0)
        st = self.lib.gwchi_pade_device(self.h, C.byref(it), C.c_void_p(sh),
                                        C.byref(ms) if report else None)
        if st != 0:
            raise self._err(st)
        return ms.value if report else None
