"""Benchmark of the chi(G, G', i omega) build on one MI355X.

`value` is the effective throughput: the method's algorithmic flops for the
full r x r' square, 8 N_r^2 (N_occ + N_unocc) per tau, divided by the wall
time of a build ("value_kind" says so; "executed_tflops" beside it counts the
flops the band-GEMM tiles actually execute).  With Hermitian completion (the
default) the GEMM computes only the lower block triangle, so the roofline of
the dominant kernel is taken on the flops it actually executes.

Workload: the Gamma-only complex configuration -- 24^3 grid, 64 occupied +
960 unoccupied orbitals, 12 tau/omega points, r' streamed in 2048-column
slabs -- with inputs resident in HBM.  A step is one complete build (all
tau points: weights, fused band contractions + Hadamard product, both sphere
FFTs, cosine transform).  The FP32 path is the headline; the FP64 path it
is compared against and the split-BF16 path are timed the same way.

Prints one JSON line (see the "paths", "roofline" and "cpu_baseline" keys).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "chi(G,G',iw) build: TFLOP/s + ms per tau point vs FP64 GPU path at stated error"
TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-4}
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}   # MI355X dense MFMA
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3->f32"}
SAMPLE_ROWS = (0, 1, 57, 1500, 2968)
WORKLOADS = {
    1: "gamma-only real 12^3 grid, 16+112 bands, 6 tau/omega, 389 plane waves",
    2: "gamma-only complex 24^3 grid, 64+960 bands, 12 tau/omega, 2048-column r' slabs, "
       "2969 plane waves",
    3: "8 k-points, complex 24^3 grid, occ 48-64 / unocc 700-1000 per k, 16 tau/omega, "
       "2969 plane waves, one batched build",
    4: "complex 32^3 grid, 128+2048 bands, 16 tau/omega, 2048-column r' slabs, 7123 plane waves",
    5: "32 real systems, 16^3-28^3 grids, 16/256-96/1536 bands, gaps 0.1-10 eV, 20 tau/omega, "
       "one batched build",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "chi_build_gamma_complex_24cubed_hbm_traffic.md")
W_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_w_update_sphere24_hbm_traffic.md")


def gemm_traffic(kernel_prefix: str, profile: str = TRAFFIC_PROFILE, source: str = "k_gemm.hip"):
    """HBM bytes per launch of a kernel from a committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by its reading for a plain
    copy of known size), or None when that summary was taken on a different
    version of the kernel's source file than the one built here."""
    import hashlib
    import re
    try:
        txt = open(profile).read()
    except OSError:
        return None
    m = re.search(re.escape(source) + r" sha256 when measured: `([0-9a-f]+)`", txt)
    src = os.path.join(ROOT, "paper_1607_02859_amd", "csrc", source)
    if not m or hashlib.sha256(open(src, "rb").read()).hexdigest() != m.group(1):
        return None
    ird = iwr = None
    for line in txt.splitlines():
        cols = [c.strip() for c in line.strip().strip("|").split("|")]
        if line.startswith("| kernel"):
            ird = next(i for i, c in enumerate(cols) if "read GB" in c)
            iwr = next(i for i, c in enumerate(cols) if "write GB" in c)
        elif ird is not None and line.startswith("| `" + kernel_prefix):
            return (float(cols[ird]) + float(cols[iwr])) * 1e9
    return None


def gemm_kernel_name(prec: str, cplx: bool, tile_id: int) -> str:
    """Kernel name prefix of GEMM tile tile_id (1-based menu entry, as in the
    report) of a precision's tile menu in k_gemm.hip."""
    import re
    fam = {"fp64": "FP64", "fp32": "FP32", "bf16x3": "BF16"}[prec] + ("_C" if cplx else "_R")
    src = open(os.path.join(ROOT, "paper_1607_02859_amd", "csrc", "k_gemm.hip")).read()
    body = re.search(r"#define GW_TILES_" + fam + r"\(X\)(.*?)\n\n", src, re.S).group(1)
    tiles = re.findall(r"X\(P_\w+, (true|false), (\d+), (\d+), (\d+), (\d+), (\d+)\)", body)
    c, a, b, k, o, w = tiles[tile_id - 1]
    p = {"fp64": 0, "fp32": 1, "bf16x3": 2}[prec]
    return f"void k_gemm<{p}, {c}, {a}, {b}, {k}, {o}, {w}>"


def cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo), or "unknown"."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(item, n_tau_sample: int = 1):
    """The oracle (unchanged) on a bounded sample: n_tau_sample tau points of
    the same item through the full space-time path, FP64 on the host."""
    from oracle import chi as oc
    import threadpoolctl
    a = np.ones((64, 64))
    _ = a @ a
    info = threadpoolctl.threadpool_info()
    blas_threads = max([i.get("num_threads", 1) for i in info] or [1])
    cores = max(blas_threads, oc._WORKERS)
    t0 = time.perf_counter()
    for j in range(n_tau_sample):
        oc.chi_tau(item, j)
    dt = time.perf_counter() - t0
    flops = 8.0 * item.n_r ** 2 * (item.n_occ + item.n_unocc) * n_tau_sample
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{n_tau_sample} of {item.n_tau} tau points of the same workload "
                      f"(space-time steps 1-4, FP64 NumPy/SciPy), {dt:.1f} s"}


def bench_w(ctx, item, args):
    """The screened-interaction step after the build (Sec. II.C steps (iii)-(iv)):
    W~(G, G', i tau) from chi(G, G', i omega) on the workload's plane-wave
    sphere and frequency grid, FP64.  chi is a seeded Hermitian negative
    semidefinite stand-in of the same shape, resident in HBM; one step is one
    call (dielectric matrices, their inversion, W~ and the inverse cosine
    transform).  Algorithmic flops: 8 n_g^3 per frequency (complex inversion)."""
    import torch
    from paper_1607_02859_amd import synth
    dev = torch.device("cuda:0")
    w = synth.make_w_item(61, item.n, item.n_tau, strength=4.0)
    chi = torch.from_numpy(w.chi).to(dev)
    w_tau = torch.empty((w.n_tau, w.n_g, w.n_g), dtype=torch.complex128, device=dev)
    w_om = torch.empty((w.n_omega, w.n_g, w.n_g), dtype=torch.complex128, device=dev)
    for _ in range(max(1, args.warmup)):
        ctx.w_build_device([w], [chi], [w_tau], [w_om], report=True)
    reps = [ctx.w_build_device([w], [chi], [w_tau], [w_om], report=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    ms = sum(r["ms_total"] for r in reps) / len(reps)
    ms_inv = sum(r["ms_invert"] for r in reps) / len(reps)
    flops = reps[0]["alg_flops"]
    t_side = (w.n_g + 63) // 64
    lower_frac = t_side * (t_side + 1) / 2 / t_side ** 2
    out = {
        "metric": "W~(G,G',i tau) from chi(G,G',i omega): TFLOP/s (8 n_g^3 per frequency)",
        "value": flops / ms * 1e-9, "unit": "TFLOP/s", "ms_per_step": ms, "dtype": "f64",
        "config": {"n_g": w.n_g, "n_omega": w.n_omega, "n_tau": w.n_tau,
                   "data": "seeded Hermitian negative semidefinite chi(i omega) of the "
                           "workload's sphere and frequency grid"},
        "ms_phases": {"eps": sum(r["ms_eps"] for r in reps) / len(reps), "invert": ms_inv,
                      "final": sum(r["ms_final"] for r in reps) / len(reps)},
        # the inversion executes only the block-lower tiles of the sweep (eps is
        # Hermitian): T (T + 1) / 2 of T^2 64 x 64 tiles, T = ceil(n_g / 64)
        "roofline": {"bound": "mfma", "kernel": "inversion (k_w_diag + k_w_panel + k_w_update)",
                     "executed_flops": flops * lower_frac,
                     "achieved": flops * lower_frac / ms_inv * 1e-9, "peak": PEAK_TFLOPS["fp64"],
                     "unit": "TFLOP/s",
                     "frac": flops * lower_frac / ms_inv * 1e-9 / PEAK_TFLOPS["fp64"],
                     # HBM bytes of one k_w_update launch (the inversion's dominant
                     # kernel) on this workload, against 2 x 16 n_g^2 K algorithmic
                     "traffic_k_w_update": gemm_traffic("k_w_update", W_TRAFFIC_PROFILE, "k_w.hip")
                     if (w.n_g == 2969 and w.n_omega == 12) else None,
                     "traffic_k_w_update_algorithmic": 32.0 * w.n_g ** 2 * w.n_omega,
                     "traffic_source": os.path.relpath(W_TRAFFIC_PROFILE, ROOT)},
    }
    if not args.no_check:
        rows = [0, w.n_g // 2, w.n_g - 1]
        got = w_om.cpu().numpy()
        from oracle import w as ow
        errs = [float(np.linalg.norm(got[k][rows] - ow.w_tilde_omega_rows(w.chi[k], w.sqrt_v, rows))
                      / np.linalg.norm(ow.w_tilde_omega_rows(w.chi[k], w.sqrt_v, rows)))
                for k in (0, w.n_omega - 1)]
        out["err_vs_oracle_sampled"] = max(errs)
    if not args.no_cpu:
        from oracle import w as ow
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] or [1])
        t0 = time.perf_counter()
        ow.w_tilde_omega(w.chi[:1], w.sqrt_v)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 8.0 * w.n_g ** 3 / dt * 1e-12, "unit": "TFLOP/s",
                               "cores": int(cores), "kind": "oracle",
                               "sample": f"1 of {w.n_omega} frequencies (dense inverse, FP64 "
                                         f"NumPy), {dt:.1f} s"}
    log(f"[bench] w_tilde: {ms:.2f} ms/step (invert {ms_inv:.2f}), "
        f"{out['value']:.1f} TFLOP/s, err {out.get('err_vs_oracle_sampled', float('nan')):.2e}")
    return out


def bench_sigma(ctx, item, args):
    """The self-energy step (Sec. II.D) on the workload's grid, bands and tau
    grid: diagonal Sigma_nn(i omega) of the 8 states nearest the gap from a
    seeded Hermitian W~(G, G', i tau) stand-in; inputs and outputs in HBM.  One
    step is one call (staging, W~ to real space, the fused band GEMM with the
    products and matrix elements, the sums and the cosine and sine transforms).
    The dominant kernel is the band GEMM: its executed flops (lower-triangle
    tiles, 8 BM BN K each) over its event-timed duration."""
    import torch
    from paper_1607_02859_amd import synth
    dev = torch.device("cuda:0")
    s = synth.make_sigma_item([2, 0], item.n, item.n_occ, item.n_unocc, item.n_tau, 8)
    po = torch.from_numpy(s.phi_occ).to(dev)
    pu = torch.from_numpy(s.phi_unocc).to(dev)
    w = torch.from_numpy(s.w_tau).to(dev)
    out = torch.empty((s.n_states, s.n_omega), dtype=torch.complex128, device=dev)
    tau_out = torch.empty((s.n_states, s.n_tau, 2), dtype=torch.float64, device=dev)
    paths = {}
    for prec in args.precisions.split(","):
        for _ in range(max(1, args.warmup)):
            ctx.sigma_build_device([s], [(po, pu)], [w], [out], [tau_out], prec=prec, report=True)
        reps = [ctx.sigma_build_device([s], [(po, pu)], [w], [out], [tau_out], prec=prec,
                                       report=True) for _ in range(args.steps)]
        torch.cuda.synchronize()
        ms = sum(r["ms_total"] for r in reps) / len(reps)
        gemm = sum(r["ms_gemm"] for r in reps) / len(reps)
        issued = reps[0]["mfma_flops"] / (gemm * 1e-3) / 1e12
        p = {"ms_per_step": ms, "ms_phases": {k: sum(r[k] for r in reps) / len(reps)
                                               for k in ("ms_stage", "ms_fft", "ms_gemm", "ms_final")},
             "tflops": reps[0]["alg_flops"] / (ms * 1e-3) / 1e12,
             "gemm_tflops_issued": issued, "gemm_frac_of_peak": issued / PEAK_TFLOPS[prec],
             "gemm_launches": reps[0]["n_gemm_launches"]}
        if not args.no_check:
            from oracle import sigma as osg
            und, bar = osg.sigma_tau(s, 0)
            got = tau_out.cpu().numpy()[:, 0, :]
            p["err_vs_oracle_tau0"] = float(max(np.abs(got[:, 0] - und.real).max() / np.abs(und).max(),
                                                np.abs(got[:, 1] - bar.real).max() / np.abs(bar).max()))
        paths[prec] = p
        log(f"[bench] sigma {prec}: {ms:.1f} ms/step (gemm {gemm:.1f}, fft {p['ms_phases']['ms_fft']:.1f}), "
            f"gemm {issued:.1f} TFLOP/s issued ({100 * p['gemm_frac_of_peak']:.0f}% of peak), "
            f"err {p.get('err_vs_oracle_tau0', float('nan')):.2e}")
    head = "fp32" if "fp32" in paths else list(paths)[0]
    H = paths[head]
    out_d = {
        "metric": "Sigma_nn(i omega) (self-energy, 8 states): TFLOP/s (8 N_r^2 K per tau, the two "
                  "Green's functions)",
        "value": H["tflops"], "unit": "TFLOP/s", "ms_per_step": H["ms_per_step"], "dtype": DTYPE[head],
        "config": {"workload": WORKLOADS[args.config], "n_states": s.n_states,
                   "data": "seeded Hermitian W~(G, G', i tau) stand-in of the workload's sphere"},
        "paths": paths,
        "roofline": {"bound": "mfma", "kernel": "k_gemm_sigma (band contractions, products with W~, "
                                                "matrix elements)",
                     "achieved": H["gemm_tflops_issued"], "peak": PEAK_TFLOPS[head], "unit": "TFLOP/s",
                     "frac": H["gemm_frac_of_peak"], "traffic": None},
    }
    if not args.no_cpu:
        from oracle import sigma as osg
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] or [1])
        t0 = time.perf_counter()
        osg.sigma_tau(s, 1)
        dt = time.perf_counter() - t0
        out_d["cpu_baseline"] = {"value": 8.0 * s.n_r ** 2 * (s.n_occ + s.n_unocc) / dt * 1e-12,
                                 "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
                                 "cpu_model": cpu_model(),
                                 "sample": f"1 of {s.n_tau} tau points (FP64 NumPy/SciPy), {dt:.1f} s"}
    return out_d


PADE_FUNCS, PADE_EVAL = 8192, 4096


def pade_flops(n_fun, n, m):
    """Nominal FP64 work of the continuation: 20 flops per complex level (one
    complex product, one complex division, two additions), N - 1 levels per
    evaluated point and N (N - 1) / 2 for the recursion of each function."""
    return 20.0 * n_fun * ((n - 1) * m + n * (n - 1) / 2)


def bench_pade(ctx, item, args):
    """The analytic continuation (Sec. II.E.1): PADE_FUNCS seeded functions of
    the shape of diagonal self-energies, known at the workload's N imaginary
    frequencies, continued to PADE_EVAL real frequencies; inputs and outputs
    in HBM.  One step is one call (coefficients and evaluation)."""
    import torch
    from paper_1607_02859_amd import synth
    dev = torch.device("cuda:0")
    n = item.n_tau
    z, f, w, *_ = synth.make_pade_input(71, PADE_FUNCS, n, PADE_EVAL, n_poles=24)
    fd = torch.from_numpy(f).to(dev)
    od = torch.empty((PADE_FUNCS, PADE_EVAL), dtype=torch.complex128, device=dev)
    for _ in range(max(1, args.warmup)):
        ctx.pade_device(z, fd, w, od, report=True)
    ms = sum(ctx.pade_device(z, fd, w, od, report=True) for _ in range(args.steps)) / args.steps
    torch.cuda.synchronize()
    fl = pade_flops(PADE_FUNCS, n, PADE_EVAL)
    out = {
        "metric": "analytic continuation (Thiele reciprocal differences): TFLOP/s "
                  "(20 flops per complex level)",
        "value": fl / ms * 1e-9, "unit": "TFLOP/s", "ms_per_step": ms, "dtype": "f64",
        "config": {"n_functions": PADE_FUNCS, "n_points": n, "n_eval": PADE_EVAL,
                   "data": "seeded 24-pole functions on the workload's imaginary frequencies"},
        "roofline": {"bound": "alu", "kernel": "k_pade", "achieved": fl / ms * 1e-9,
                     "peak": 78.6, "unit": "TFLOP/s", "frac": fl / ms * 1e-9 / 78.6,
                     "traffic": None,
                     "bytes_algorithmic": 16.0 * PADE_FUNCS * (n + PADE_EVAL)},
    }
    if not args.no_check:
        from oracle import pade as op
        rows = [0, PADE_FUNCS // 2, PADE_FUNCS - 1]
        got = od[rows].cpu().numpy()
        ref = op.continue_to(z, f[rows], w)
        out["err_vs_oracle_sampled"] = float(np.abs(got - ref).max() / np.abs(ref).max())
    if not args.no_cpu:
        from oracle import pade as op
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] or [1])
        sample = 256
        t0 = time.perf_counter()
        op.continue_to(z, f[:sample], w)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": pade_flops(sample, n, PADE_EVAL) / dt * 1e-12,
                               "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
                               "sample": f"{sample} of {PADE_FUNCS} functions (NumPy), {dt:.1f} s"}
    log(f"[bench] pade: {ms:.3f} ms/step, {out['value']:.1f} TFLOP/s, "
        f"err {out.get('err_vs_oracle_sampled', float('nan')):.2e}")
    return out


def bench_config(args, cfg, sample, tune=None, timed=2, kappa=True):
    """One more workload configuration on every path, in one persistent launch
    per slab over all its (item, tau) jobs: GEMM tiles autotuned on the items
    tune(items) selects (else the menu's default), one warm-up, then `timed`
    builds timed with per-launch events (GEMM time) and by the wall clock;
    error against the oracle on the sampled rows [(item, rows)]."""
    import torch
    from paper_1607_02859_amd import gwchi, synth
    dev = torch.device("cuda:0")
    items = synth.make_config(cfg)
    phis = [(torch.from_numpy(it.phi_occ).to(dev), torch.from_numpy(it.phi_unocc).to(dev))
            for it in items]
    outs = [torch.empty((it.n_omega, it.n_g, it.n_g), dtype=torch.complex128, device=dev)
            for it in items]
    alg = sum(synth.algorithmic_flops(it) for it in items)
    refs = None
    if not args.no_check:
        from oracle import chi as oc
        refs = {t: oc.chi_rows(items[t], rows) for t, rows in sample}
    ctx = gwchi.Context(0)
    ctx.set_options(use_graph=1, timing=1, hermitian=1, kappa=0)
    stream = torch.cuda.current_stream()
    out = {"config": {"workload": WORKLOADS[cfg], "items": len(items)}, "paths": {}}
    for prec in args.precisions.split(","):
        if tune is not None:
            ctx.autotune(tune(items), prec)
        ctx.build_device(items, phis, outs, prec, stream=stream, report=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = [ctx.build_device(items, phis, outs, prec, stream=stream, report=True)
                for _ in range(timed)]
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / timed
        gemm_ms = sum(r["ms_gemm"] for r in reps) / timed
        issued = reps[-1]["mfma_flops"] / (gemm_ms * 1e-3) / 1e12
        p = {"ms_per_step": 1e3 * wall, "ms_per_tau": 1e3 * wall / max(it.n_tau for it in items),
             "tflops": alg / wall / 1e12, "gemm_ms": gemm_ms,
             "mfma_tflops_issued": issued, "mfma_frac_of_peak": issued / PEAK_TFLOPS[prec],
             "phase_ms": {k: sum(r[k] for r in reps) / timed
                          for k in ("ms_stage", "ms_gemm", "ms_fft_r", "ms_fft_rp", "ms_ct")},
             "tile_id": reps[-1]["tile_id"]}
        if kappa:
            ctx.set_options(kappa=1)
            p["kappa_F"] = ctx.build_device(items, phis, outs, prec, stream=stream,
                                            report=True)["kappa_F_max"]
            ctx.set_options(kappa=0)
        if refs is not None:
            from oracle import chi as oc
            errs = [oc.rel_frobenius(outs[t].cpu().numpy()[:, rows, :], refs[t])
                    for t, rows in sample]
            p["err_vs_oracle_sampled_rows"] = max(errs)
            p["within_tol"] = bool(max(errs) <= TOL[prec])
        out["paths"][prec] = p
        log(f"[bench] config {cfg} {prec}: {p['ms_per_step']:.0f} ms/step, {p['tflops']:.1f} TFLOP/s, "
            f"gemm {issued:.1f} TFLOP/s issued ({100 * p['mfma_frac_of_peak']:.0f}% of peak), "
            + (f"kappa_F {p['kappa_F']:.2f}, " if "kappa_F" in p else "")
            + f"err {p.get('err_vs_oracle_sampled_rows', float('nan')):.2e}")
    ctx.close()
    del phis, outs
    torch.cuda.empty_cache()
    if "fp64" in out["paths"]:
        for prec, p in out["paths"].items():
            p["speedup_vs_fp64"] = out["paths"]["fp64"]["ms_per_step"] / p["ms_per_step"]
    return out


def bench_batched(args):
    """The 32-system batch (configuration 5: real orbitals, 16^3-28^3 grids,
    16/256 .. 96/1536 bands, gaps 0.1-10 eV, 20 taus) on every path: tiles
    autotuned on the six 24^3 systems, two timed builds; sampled rows of one
    system of every grid size."""
    return bench_config(args, 5, [(0, [0, 5]), (9, [2, 100]), (16, [3, 1700]), (20, [1, 1000]),
                                  (31, [7, 4000])],
                        tune=lambda items: [it for it in items if it.n[0] == 24])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precisions", default="fp64,fp32,bf16x3")
    ap.add_argument("--headline", default="fp32")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled oracle check")
    ap.add_argument("--hermitian", type=int, default=1)
    ap.add_argument("--skip-zero-bands", type=int, default=0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before timing, copy MIB mebibytes device-to-device once (a plain copy "
                         "of known size against which HBM byte counters are scaled)")
    ap.add_argument("--config", type=int, default=2,
                    help="workload configuration (2 is the headline; 1, 3, 4, 5 for the record)")
    ap.add_argument("--w", type=int, default=None,
                    help="also time the screened-interaction step W~ from chi(i omega) on the "
                         "plane-wave sphere of the workload (default: on for configuration 2)")
    ap.add_argument("--pade", type=int, default=None,
                    help="also time the analytic continuation of many functions known at the "
                         "workload's imaginary frequencies (default: on for configuration 2)")
    ap.add_argument("--sigma", type=int, default=None,
                    help="also time the self-energy step on the workload (default: on for "
                         "configuration 2)")
    ap.add_argument("--sigma-only", action="store_true",
                    help="time only the self-energy step (prints one JSON line with the sigma object)")
    ap.add_argument("--pade-only", action="store_true",
                    help="time only the continuation (prints one JSON line with the pade object)")
    ap.add_argument("--w-only", action="store_true",
                    help="time only the W~ step (prints one JSON line with the w_tilde object)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="time every GEMM tile on the workload before the warm-up and use the "
                         "fastest (default on)")
    ap.add_argument("--batched", type=int, default=None,
                    help="also time the 32-system batch (configuration 5) on every path, one "
                         "warm-up and two timed builds (default: on for configuration 2)")
    ap.add_argument("--more-configs", type=int, default=None,
                    help="also time the 8-k-point batch (configuration 3) and the 32^3 grid "
                         "(configuration 4) on every path, tiles autotuned on the first item, "
                         "one warm-up and one timed build (default: on for configuration 2)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1607_02859_amd import gwchi, synth

    dev = torch.device("cuda:0")
    items = synth.make_config(args.config)
    item = items[0]
    log(f"[bench] config {args.config}: {len(items)} item(s), first n={item.n} "
        f"K={item.n_occ}+{item.n_unocc} n_tau={item.n_tau} n_g={item.n_g}")
    if args.calibrate_copy > 0:
        n = args.calibrate_copy << 20
        a = torch.empty(n, dtype=torch.uint8, device=dev).fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.w_only or args.pade_only or args.sigma_only:
        ctx = gwchi.Context(0)
        if args.w_only:
            out = {"w_tilde": bench_w(ctx, item, args)}
        elif args.sigma_only:
            out = {"sigma": bench_sigma(ctx, item, args)}
        else:
            out = {"pade": bench_pade(ctx, item, args)}
        ctx.close()
        print(json.dumps(out), flush=True)
        return
    phis = [(torch.from_numpy(it.phi_occ).to(dev), torch.from_numpy(it.phi_unocc).to(dev))
            for it in items]
    outs = [torch.empty((it.n_omega, it.n_g, it.n_g), dtype=torch.complex128, device=dev)
            for it in items]
    ctx = gwchi.Context(0)
    ctx.set_options(use_graph=1, timing=1, slab_width=2048, hermitian=args.hermitian,
                    skip_zero_bands=args.skip_zero_bands, kappa=0)
    stream = torch.cuda.current_stream()
    alg = sum(synth.algorithmic_flops(it) for it in items)

    ref_rows = None
    if not args.no_check:
        from oracle import chi as oc
        t0 = time.perf_counter()
        rows = [r for r in SAMPLE_ROWS if r < item.n_g]
        ref_rows = oc.chi_rows(item, rows)
        log(f"[bench] oracle sampled rows in {time.perf_counter() - t0:.1f} s")

    paths = {}
    for prec in args.precisions.split(","):
        if args.autotune:
            t0 = time.perf_counter()
            ctx.autotune(items, prec)
            log(f"[bench] {prec}: autotuned GEMM tiles in {time.perf_counter() - t0:.1f} s")
        for _ in range(args.warmup):
            ctx.build_device(items, phis, outs, prec, stream=stream, report=True)
        torch.cuda.synchronize()
        reps = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            reps.append(ctx.build_device(items, phis, outs, prec, stream=stream, report=True))
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        ms_step = 1e3 * wall
        gemm_ms = sum(r["ms_gemm"] for r in reps) / len(reps)
        n_launch = reps[-1]["n_gemm_launches"]
        p = {
            "ms_per_step": ms_step,
            "ms_per_tau": ms_step / max(it.n_tau for it in items),
            "tflops": alg / wall / 1e12,
            "gemm_ms_per_step": gemm_ms,
            "gemm_launches_per_step": n_launch,
            "gemm_ms_per_launch": gemm_ms / max(1, n_launch),
            "gemm_effective_tflops": alg / (gemm_ms * 1e-3) / 1e12,
            "mfma_flops_per_step": reps[-1]["mfma_flops"],
            "mfma_tflops_issued": reps[-1]["mfma_flops"] / (gemm_ms * 1e-3) / 1e12,
            "mfma_frac_of_peak": reps[-1]["mfma_flops"] / (gemm_ms * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
            "phase_ms": {k: sum(r[k] for r in reps) / len(reps)
                         for k in ("ms_stage", "ms_gemm", "ms_fft_r", "ms_fft_rp", "ms_ct")},
            "kappa_F": None,
            "graph_replayed": reps[-1]["graph_replayed"],
            "tile_id": reps[-1]["tile_id"],
        }
        if ref_rows is not None:
            got = outs[0].cpu().numpy()[:, rows, :]
            num = np.sqrt((np.abs(got - ref_rows) ** 2).reshape(item.n_omega, -1).sum(1))
            den = np.sqrt((np.abs(ref_rows) ** 2).reshape(item.n_omega, -1).sum(1))
            p["err_vs_oracle_sampled_rows"] = float((num / den).max())
            p["within_tol"] = bool(p["err_vs_oracle_sampled_rows"] <= TOL[prec])
        # kappa_F of this result (norm pass outside the timed steps)
        ctx.set_options(kappa=1)
        p["kappa_F"] = ctx.build_device(items, phis, outs, prec, stream=stream,
                                        report=True)["kappa_F_max"]
        ctx.set_options(kappa=0)
        # the same build replayed from the captured hipGraph (no per-launch events)
        ctx.set_options(timing=0)
        for _ in range(max(1, args.warmup)):
            ctx.build_device(items, phis, outs, prec, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.build_device(items, phis, outs, prec, stream=stream)
        torch.cuda.synchronize()
        p["ms_per_step_graph"] = 1e3 * (time.perf_counter() - t0) / args.steps
        ctx.set_options(timing=1)
        paths[prec] = p
        log(f"[bench] {prec}: {ms_step:.2f} ms/step, {p['ms_per_tau']:.3f} ms/tau, "
            f"{p['tflops']:.1f} TFLOP/s, gemm {p['mfma_tflops_issued']:.1f} TFLOP/s issued "
            f"({100 * p['mfma_frac_of_peak']:.0f}% of peak), "
            f"err {p.get('err_vs_oracle_sampled_rows', float('nan')):.2e}")

    head = args.headline if args.headline in paths else list(paths)[0]
    H = paths[head]
    res = {
        "metric": METRIC,
        "value": H["tflops"],
        "unit": "TFLOP/s",
        "value_kind": "effective: full-square algorithmic flops 8 N_r^2 K per tau / build time",
        "executed_tflops": H["mfma_flops_per_step"] / (H["ms_per_step"] * 1e-3) / 1e12
        / (3.0 if head == "bf16x3" else 1.0),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": H["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[head],
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config],
                   "precision": head, "hermitian": args.hermitian,
                   "skip_zero_bands": args.skip_zero_bands,
                   "autotune": args.autotune},
        "ms_per_tau": H["ms_per_tau"],
        "speedup_vs_fp64": (paths["fp64"]["ms_per_step"] / H["ms_per_step"]) if "fp64" in paths else None,
        "err_vs_oracle": H.get("err_vs_oracle_sampled_rows"),
        "kappa_F": H["kappa_F"],
        "paths": paths,
    }
    # dominant kernel: flops it executes per launch (the tiles it computes, each
    # 8*BM*BN*K for complex orbitals; split-BF16 issues three products per flop)
    per_launch = H["mfma_flops_per_step"] / H["gemm_launches_per_step"]
    achieved = per_launch / (H["gemm_ms_per_launch"] * 1e-3) / 1e12
    res["roofline"] = {
        "bound": "mfma",
        "kernel": "k_gemm (fused band contractions + Hadamard product)",
        "achieved": achieved,
        "peak": PEAK_TFLOPS[head],
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_TFLOPS[head],
        "traffic": gemm_traffic(gemm_kernel_name(head, True, H["tile_id"]))
        if (head == "fp32" and args.config == 2) else None,
        "tile": gemm_kernel_name(head, item.is_complex, H["tile_id"]),
        "traffic_source": os.path.relpath(TRAFFIC_PROFILE, ROOT),
        "per_launch_flops": per_launch,
        "avg_launch_ms": H["gemm_ms_per_launch"],
        "launches_per_step": H["gemm_launches_per_step"],
    }
    if not args.no_cpu and args.config == 2:
        res["cpu_baseline"] = cpu_baseline(item, 6)
    if args.w is None:
        args.w = 1 if args.config == 2 else 0
    if args.w:
        res["w_tilde"] = bench_w(ctx, item, args)
    if args.pade is None:
        args.pade = 1 if args.config == 2 else 0
    if args.pade:
        res["pade"] = bench_pade(ctx, item, args)
    if args.sigma is None:
        args.sigma = 1 if args.config == 2 else 0
    if args.sigma:
        res["sigma"] = bench_sigma(ctx, item, args)
    ctx.close()
    del phis, outs
    torch.cuda.empty_cache()
    if args.batched is None:
        args.batched = 1 if args.config == 2 else 0
    if args.batched:
        res["batched"] = bench_batched(args)
    if args.more_configs is None:
        args.more_configs = 1 if args.config == 2 else 0
    if args.more_configs:
        first = lambda items: items[:1]
        res["config3"] = bench_config(args, 3, [(0, [0, 700]), (5, [3, 2968])], tune=first,
                                      timed=1, kappa=False)
        res["config4"] = bench_config(args, 4, [(0, [1, 7122])], tune=first, timed=1,
                                      kappa=False)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
