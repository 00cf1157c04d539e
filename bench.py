#!/usr/bin/env python3
"""Benchmark of the LDDMM hot path on one MI355X.

Workload (pair128): one template/target pair on a 128^3 periodic grid, nt = 10
Heun steps, L = (Id - 0.0025 Laplacian)^2, sigma^2 = 1, FP32 fields with FP64
reductions.  Template = seeded phantom (24 blobs, sigmas 4-12 voxels, tissue
classes 0.2/0.5/0.8, ellipsoidal shell); target = template shot by a seeded
band-limited v0 (max |v0| = 6 voxels) on the GPU in FP64, plus N(0, 0.01^2)
noise.  Synthetic data stand in for the paper's brain volumes.

One timed step = one full inexact Gauss-Newton-Krylov solve from v0 = 0 (10
outer iterations, <= 20 CG iterations each, Armijo line search), i.e. every
stage of the hot path: shooting with trajectory store, final conditions, the
adjoint sweep, Hessian-vector products inside CG in V, line-search shoots.
``value`` = solves per minute.  The same run also reports Hessian-vector
products/s and gradients/s (HIP events on the library stream), the plain FP64
path, the roofline of the dominant kernel and the CPU oracle on the host.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s

# Algorithmic bytes per launch (each distinct operand read once, each result
# written once) as a function of the grid; V = vector field, S = scalar field,
# C = one component's half spectrum (N0 N1 (N2/2+1) complex).  The spectral
# kernels always process the three components of a vector field here.
def kernel_bytes(n, esize):
    n0, n1, n2 = n
    N = n0 * n1 * n2
    S = N * esize
    V = 3 * S
    C = n0 * n1 * (n2 // 2 + 1) * 2 * esize
    return {
        "fft_plane_fwd": 3 * (S + C),
        "fft_pencil_symbol": 3 * 2 * C,
        "fft_plane_inv": 3 * (C + S),
        "fft_plane_inv_add": 3 * (C + 2 * S),
        "fft_rows_fwd": 3 * (S + C),
        "fft_pencil_x1_fwd": 3 * 2 * C,
        "fft_pencil_x1_inv": 3 * 2 * C,
        "fft_rows_inv": 3 * (C + S),
        "tangent_stage_pred": 7 * V,
        "tangent_stage_corr": 9 * V,
        "adjoint_stage_pred": 7 * V,
        "adjoint_stage_corr": 9 * V,
        # the sweeps' first stages, which do not read their zero start field
        "tangent_stage_pred_first": 6 * V,
        "tangent_stage_corr_first": 8 * V,
        "adjoint_stage_corr_first": 8 * V,
        "epdiff_stage_pred": 3 * V,
        "epdiff_stage_corr": 4 * V,
        "sl_step": 4 * V,
        "compose": 2 * S + V,
        "residual_grad": 3 * S + V,
        "gn_final_condition": 3 * V,
        "final_condition": S + 2 * V,
    }


# Compulsory HBM floor of the Hessian-vector product (16 V per time step and
# sweep): per step and sweep the stage kernels read the 4 coefficient fields and
# read and write the 2-field state once (8 V over the step's 2 stage launches,
# 4 V each), and each of the 2 K applications makes 2 round trips of a vector
# field (4 V, shared by its 3 transform passes).  Per Hv: 32 V nt.
def floor_bytes_per_launch(group, n, esize):
    V = 3 * n[0] * n[1] * n[2] * esize
    if group.startswith("fft_"):
        return 4 * V / 3
    if group.endswith("_stage"):
        return 4 * V
    return None


def hv_floor_bytes(n, nt, esize):
    return 32 * 3 * n[0] * n[1] * n[2] * esize * nt


# Profiler launch names -> kernel template (the rocprof kernel name without its
# template arguments): predictor, corrector and first-stage launches of one
# template form one group.
def kernel_group(name):
    if name.startswith("tangent_stage"):
        return "tangent_stage"
    if name.startswith("adjoint_stage"):
        return "adjoint_stage"
    if name.startswith("epdiff_stage"):
        return "epdiff_stage"
    if name.startswith("fft_plane_inv"):
        return "fft_plane_inv"
    return name


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Transform launch shape that the autotuner chose; HBM traffic is recorded per shape.
TUNED_KEYS = (
    "fft.plane_threads",
    "fft.plane_grid",
    "fft.plane_halves_used",
    "fft.pencil_threads",
    "fft.pencil_tb",
    "fft.rows_rb",
    "fft.fused",
    "fft.static_kernels",
    "stencil.rowvec",
    "stencil.pair_rows",
)
KERNEL_SOURCES = {
    "fft": ("paper_1807_04638_amd/csrc/fft.hip", "paper_1807_04638_amd/csrc/fft_core.h",
            "paper_1807_04638_amd/csrc/index_math.h"),
    "stencil": ("paper_1807_04638_amd/csrc/stencil.hip", "paper_1807_04638_amd/csrc/index_math.h"),
}
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "hbm_traffic_pair128_fp32.md")


def source_digest(group):
    import hashlib

    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[group]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel, tuned):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE
    record, or None when the record is missing, was taken with another launch
    shape, or the kernel's sources changed since."""
    try:
        with open(TRAFFIC_RECORD) as f:
            text = f.read()
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    if rec.get("sources", {}).get(k["sources"]) != source_digest(k["sources"]):
        return None
    if any(rec.get("tuned", {}).get(key) != tuned.get(key) for key in shape_keys(kernel)):
        return None
    return int(k["fetch_bytes"] + k["write_bytes"])


def shape_keys(kernel):
    """Launch-shape options that change a kernel's memory traffic."""
    if kernel.startswith("fft_pencil"):
        return ("fft.pencil_tb", "fft.pencil_threads", "fft.fused", "fft.static_kernels", "fft.plane_halves_used")
    if kernel.startswith("fft_"):
        return ("fft.plane_threads", "fft.rows_rb", "fft.fused", "fft.static_kernels", "fft.plane_halves_used")
    return ("stencil.rowvec",)


def make_pair(spec, dtype, dev, torch, Registration, synth):
    I0 = synth.phantom(spec.n, spec.n_blobs, spec.sigma_range, spec.classes, 1000, shells=spec.shells)
    v0t = synth.random_velocity(spec.n, 2000, spec.disp_vox)
    nz = synth.noise(spec.n, 3000, spec.noise_sd)
    # target: FP64 GPU shoot of the seeded v0, plus noise
    R = Registration(spec.n, spec.nt, spec.alpha, spec.s, spec.sigma2, dtype=torch.float64, device=dev)
    t0 = torch.tensor(I0, dtype=torch.float64, device=dev)
    R.set_images(t0, t0)
    J1 = R.shoot(torch.tensor(v0t, dtype=torch.float64, device=dev), want=("J1",))["J1"]
    I1 = (J1 + torch.tensor(nz, dtype=torch.float64, device=dev)).cpu().numpy()
    R.close()
    return I0, I1, v0t


def time_events(torch, fn, reps):
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(reps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / reps  # ms


def median_events(torch, fn, reps, warmup=3):
    """Median over `reps` calls of fn, each bracketed by its own pair of events on
    the current stream, after `warmup` untimed calls (ms)."""
    for _ in range(warmup):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) for a, b in ev)
    return t[len(t) // 2] if len(t) % 2 else 0.5 * (t[len(t) // 2 - 1] + t[len(t) // 2])


def cpu_baseline(spec, I0, I1, v0t, rep):
    """Time the FP64 oracle on the host on a bounded sample of the workload: one
    linearization (shoot with trajectory store, SL transport, final conditions),
    one adjoint sweep (the gradient at that linearization) and one Gauss-Newton
    Hessian-vector product, all at the full grid and nt, each timed once.  A
    solve is extrapolated from these per-operation times and the GPU solve's
    operation counts (linearizations, adjoint sweeps, Hessian-vector products)."""
    import numpy as np

    import oracle as O
    from synth import random_field

    p = O.Params(spec.n, spec.alpha, spec.s, spec.nt, spec.sigma2)
    v = 0.5 * np.asarray(v0t)
    dv = random_field(spec.n, 7)
    t = time.perf_counter()
    lin = O.linearize(v, I0, I1, p)
    t_lin = time.perf_counter() - t
    log(f"[bench] oracle linearization {t_lin:.1f} s")
    t = time.perf_counter()
    O.gradient(v, I0, I1, p, lin)
    t_bw = time.perf_counter() - t
    log(f"[bench] oracle adjoint sweep {t_bw:.1f} s")
    t = time.perf_counter()
    O.hessvec(dv, lin, p)
    t_hv = time.perf_counter() - t
    log(f"[bench] oracle Hessian-vector product {t_hv:.1f} s")
    n_lin = 1 + rep["shoots"]
    n_bw = rep["gradients"]
    n_hv = rep["hessvecs"]
    per_solve = n_lin * t_lin + n_bw * t_bw + n_hv * t_hv
    cores = O.lddmm_oracle._WORKERS
    return {
        "value": round(60.0 / per_solve, 5),
        "unit": "GN solves/min",
        "cores": cores,
        "kind": "oracle",
        "extrapolated": True,
        "sample": (
            f"FP64 oracle at {spec.n[0]}x{spec.n[1]}x{spec.n[2]}, nt={spec.nt}, timed once each: linearization "
            f"{t_lin:.1f} s, adjoint sweep {t_bw:.1f} s, Hessian-vector product {t_hv:.1f} s (scipy.fft on {cores} "
            f"threads, numpy elementwise on one); a GN solve extrapolated as {n_lin} linearizations + {n_bw} adjoint "
            f"sweeps + {n_hv} Hessian-vector products (the GPU solve's counts) = {per_solve:.0f} s"
        ),
        "hv_per_s": round(1.0 / t_hv, 5),
        "gradients_per_s": round(1.0 / (t_lin + t_bw), 5),
        "shoot_s": round(t_lin, 2),
    }


def batch_bench(args, torch, synth, Batch, Registration):
    """16 pairs of uneven sizes N in {64, 80, 96, 112, 128} (drawn with seed
    4000), phantom recipe scaled by N/128, FP32, nt = 10: aggregate Hv/s and
    solves/min in lockstep (one host thread, each phase enqueued for all pairs,
    graphs spanning the pairs) and on one host thread per pair, against the same
    batch run one pair after the other."""
    import numpy as np

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(4000)
    sizes = [int(x) for x in rng.choice([64, 80, 96, 112, 128], size=16)]
    specs, data = [], []
    for i, N in enumerate(sizes):
        f = N / 128.0
        n = (N, N, N)
        I0 = synth.phantom(n, 24, (4.0 * f, 12.0 * f), True, 1000 + i)
        v0 = synth.random_velocity(n, 2000 + i, 6.0 * f)
        R = Registration(n, 10, 0.0025, 2, 1.0, dtype=torch.float64, device=dev)
        t0 = torch.tensor(I0, dtype=torch.float64, device=dev)
        R.set_images(t0, t0)
        J1 = R.shoot(torch.tensor(v0, dtype=torch.float64, device=dev), want=("J1",))["J1"]
        I1 = (J1 + torch.tensor(synth.noise(n, 3000 + i, 0.01), device=dev)).float()
        R.close()
        specs.append(dict(n=n, nt=10, alpha=0.0025, s=2, sigma2=1.0))
        data.append((torch.tensor(I0, dtype=torch.float32, device=dev), I1))
        log(f"[bench] pair {i}: {N}^3")
    B = Batch(specs, dtype=torch.float32, device=dev)
    for i, (I0, I1) in enumerate(data):
        B.contexts[i].set_images(I0, I1)
    B.autotune(reps=3)
    out = {}
    # per-voxel rate of the largest grid alone: one Hv of the first 128^3 pair
    big = max(range(len(specs)), key=lambda i: specs[i]["n"][0])
    nb = specs[big]["n"]
    dvb = torch.randn((3,) + nb, device=dev)
    hvb = torch.empty_like(dvb)
    Rb = B.contexts[big]
    Rb.linearize(torch.zeros((3,) + nb, device=dev))
    Rb.hessvec(dvb, out=hvb)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.hv_reps):
        Rb.hessvec(dvb, out=hvb)
    torch.cuda.synchronize()
    t_big = (time.perf_counter() - t) / args.hv_reps
    vox = sum(sp["n"][0] * sp["n"][1] * sp["n"][2] for sp in specs) / float(nb[0] * nb[1] * nb[2])
    hv_bound = len(specs) / (t_big * vox)
    log(f"[bench] largest grid alone {1e3 * t_big:.3f} ms per Hv; {vox:.2f} of its volumes in the batch -> "
        f"bandwidth-proportional bound {hv_bound:.1f} Hv/s")
    for mode in ("sequential", "threads", "lockstep"):
        vs = [torch.zeros((3,) + sp["n"], device=dev) for sp in specs]
        B.gn_solve(vs, gn_iters=2, cg_iters=5, mode=mode)  # warm-up (graph capture, caches)
        vs = [torch.zeros((3,) + sp["n"], device=dev) for sp in specs]
        torch.cuda.synchronize()
        t = time.perf_counter()
        reps = B.gn_solve(vs, mode=mode)
        T = time.perf_counter() - t
        hv = sum(r["hessvecs"] for r in reps)
        dvs = [torch.randn((3,) + sp["n"], device=dev) for sp in specs]
        hvs = [torch.empty_like(d) for d in dvs]
        B.hessvec(dvs, hvs, reps=1, mode=mode)
        t = time.perf_counter()
        B.hessvec(dvs, hvs, reps=args.hv_reps, mode=mode)
        Th = time.perf_counter() - t
        out[mode] = {
            "gn_solves_per_min": round(60.0 * len(specs) / T, 3),
            "s_per_batch": round(T, 3),
            "hessvecs_in_solves": hv,
            "hv_per_s": round(len(specs) * args.hv_reps / Th, 2),
            "mse_rel_final_mean": round(float(np.mean([r["mse_rel_final"] for r in reps])), 4),
        }
        log(f"[bench] {mode}: {out[mode]}")
    line = {
        "metric": "aggregate Hessian-vector products/s & GN solves/min, 16 uneven pairs",
        "value": max(out["lockstep"]["hv_per_s"], out["threads"]["hv_per_s"]),
        "unit": "Hv/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch16: 16 pairs, N drawn from {64,80,96,112,128} with seed 4000, nt=10, "
                               "alpha=0.0025, s=2, sigma2=1, GN<=10, CG<=20", "sizes": sizes},
        "lockstep": out["lockstep"],
        "threads": out["threads"],
        "sequential": out["sequential"],
        "speedup_hv": {m: round(out[m]["hv_per_s"] / out["sequential"]["hv_per_s"], 3) for m in ("lockstep", "threads")},
        "speedup_solves": {m: round(out[m]["gn_solves_per_min"] / out["sequential"]["gn_solves_per_min"], 3)
                           for m in ("lockstep", "threads")},
        # bandwidth-proportional bound: every pair at the per-voxel rate of the
        # largest grid alone (its sequential Hv time scaled by voxel count)
        "hv_per_s_bound": round(hv_bound, 2),
    }
    B.close()
    return line


def precision_bench(args, torch, synth, Registration, spec):
    """Precision policy on a brain-shaped grid: FP32 fields with FP64 reductions
    against the plain FP64 path (the FP64 GPU path is the reference here; it
    matches the FP64 oracle to ~1e-15 at the sizes the oracle finishes).
    Reports relative-L2 differences of v0 after the GN solve, the warped image,
    and the <mu, v> drift of the final geodesic, with solve/Hv timings."""
    import numpy as np

    dev = torch.device("cuda:0")
    n = spec.n
    I0 = synth.phantom(n, spec.n_blobs, spec.sigma_range, spec.classes, 1000, shells=spec.shells)
    v0t = synth.random_velocity(n, 2000, spec.disp_vox)
    res = {}
    I1 = None
    for dt in (torch.float64, torch.float32):
        R = Registration(n, spec.nt, spec.alpha, spec.s, spec.sigma2, dtype=dt, device=dev)
        t0 = torch.tensor(I0, dtype=dt, device=dev)
        if I1 is None:
            R.set_images(t0, t0)
            J = R.shoot(torch.tensor(v0t, dtype=dt, device=dev), want=("J1",))["J1"]
            I1 = (J + torch.tensor(synth.noise(n, 3000, spec.noise_sd), dtype=dt, device=dev)).cpu().numpy()
        R.set_images(t0, torch.tensor(I1, dtype=dt, device=dev))
        tried, ms = R.autotune(reps=3)
        R.set_option("exec.graph", 1)
        log(f"[bench] {dt}: autotune {tried} variants, K {1e3 * ms:.1f} us; {R.get_option('fft.static_kernels')} compile-time passes")
        v = torch.zeros((3,) + n, dtype=dt, device=dev)
        R.gn_solve(v, gn_iters=1, cg_iters=2)  # warm-up
        v = torch.zeros((3,) + n, dtype=dt, device=dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        tr = R.gn_solve(v, gn_iters=spec.gn_iters, cg_iters=spec.cg_iters)
        torch.cuda.synchronize()
        Ts = time.perf_counter() - t
        sh = R.shoot(v, want=("J1", "v1"))
        mu0, mu1 = R.apply_L(v), R.apply_L(sh["v1"])
        drift = R.dot(mu1, sh["v1"]) / R.dot(mu0, v) - 1.0
        dv = torch.randn((3,) + n, dtype=dt, device=dev, generator=torch.Generator(device=dev).manual_seed(5))
        R.hessvec(dv)
        hv_ms = time_events(torch, lambda: R.hessvec(dv), 5)
        res[dt] = dict(v=v.double().cpu().numpy(), J1=sh["J1"].double().cpu().numpy(), drift=drift, s=Ts,
                       hv_ms=hv_ms, rep=tr.report)
        log(f"[bench] {dt}: solve {Ts:.2f} s, Hv {hv_ms:.2f} ms, drift {drift:.3e}, report {tr.report}")
        del R
        torch.cuda.empty_cache()
    a, b = res[torch.float32], res[torch.float64]

    def rel(x, y):
        return float(np.linalg.norm(x - y) / np.linalg.norm(y))

    line = {
        "metric": "FP32 vs FP64 relative-L2 error (v0 after GN, warped image, drift) and solve speed",
        "value": round(60.0 / a["s"], 3),
        "unit": "GN solves/min",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{spec.name}: {n[0]}x{n[1]}x{n[2]} head phantom (3 shells, {spec.n_blobs} blobs), "
                               f"nt={spec.nt}, alpha={spec.alpha}, s={spec.s}, sigma2={spec.sigma2}, disp {spec.disp_vox} vox, "
                               "noise 0.01, GN<=10, CG<=20"},
        "rel_l2_v0": rel(a["v"], b["v"]),
        "rel_l2_J1": rel(a["J1"], b["J1"]),
        "drift_fp32": a["drift"],
        "drift_fp64": b["drift"],
        "mse_rel_final": {"fp32": a["rep"]["mse_rel_final"], "fp64": b["rep"]["mse_rel_final"]},
        "E_final": {"fp32": a["rep"]["E_final"], "fp64": b["rep"]["E_final"]},
        "solve_s": {"fp32": round(a["s"], 3), "fp64": round(b["s"], 3)},
        "hv_ms": {"fp32": round(a["hv_ms"], 3), "fp64": round(b["hv_ms"], 3)},
        "fp32_speedup_vs_fp64": round(b["s"] / a["s"], 3),
        "reference": "FP64 GPU path (checked against the FP64 oracle on this grid at nt = 2 and on small grids)",
    }
    return line


def pde_bench(args, torch, Registration, spec, I0, I1):
    """PDE-LDDMM (the comparison method of Section 2.3) on the same pair: a
    Gauss-Newton-Krylov solve from v = 0 with stationary and with non-stationary
    velocities (nt + 1 fields), FP32, and Gauss-Newton Hessian products/s."""
    dev = torch.device("cuda:0")
    R = Registration(spec.n, spec.nt, spec.alpha, spec.s, spec.sigma2, dtype=torch.float32, device=dev)
    R.set_images(torch.tensor(I0, dtype=torch.float32, device=dev), torch.tensor(I1, dtype=torch.float32, device=dev))
    R.autotune(reps=3)
    out = {}
    for stationary in (True, False):
        key = "stationary" if stationary else "non_stationary"
        v = R.empty_velocity(stationary).zero_()
        R.pde_gn_solve(v, stationary, gn_iters=1, cg_iters=2)  # warm-up
        v.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        tr = R.pde_gn_solve(v, stationary, gn_iters=spec.gn_iters, cg_iters=spec.cg_iters)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t
        dv = torch.randn(v.shape, device=dev, generator=torch.Generator(device=dev).manual_seed(11))
        hv = torch.empty_like(dv)
        R.pde_hessvec(dv, stationary, v=v, out=hv)
        ms = time_events(torch, lambda: R.pde_hessvec(dv, stationary, out=hv), 5)
        rep = tr.report
        out[key] = {"solves_per_min": round(60.0 / ts, 3), "ms_per_solve": round(1e3 * ts, 1),
                    "hv_per_s": round(1e3 / ms, 2), "iters": rep["iters"], "cg_total": rep["cg_total"],
                    "line_search_shoots": rep["shoots"], "mse_rel_final": rep["mse_rel_final"],
                    "E_final": rep["E_final"], "stop_reason": rep["stop_reason"]}
        log(f"[bench] PDE-LDDMM {key}: {out[key]}")
    R.close()
    return {"workload": f"{spec.name}: the same pair, PDE-LDDMM (velocity over time), FP32, nt={spec.nt}, "
                        f"GN<={spec.gn_iters}, PCG<={spec.cg_iters} in L2 with preconditioner K", **out}


def table1_bench(args, torch, synth, Registration, spec, pairs=15):
    """Table-1-shaped report on seeded synthetic pairs of the pair128 recipe (the
    paper registers 15 NIREP pairs; these stand in for them): for every method
    the paper compares (gradient descent in V, stationary and non-stationary
    PDE-LDDMM, Gauss-Newton in V and in L2) and the Newton-Krylov variant, mean
    and standard deviation over the pairs of the final MSE_rel (percent), the
    final infinity-norm gradient relative to the one at v = 0 (each solver's own
    norm: V for the V methods, L2 for the L2 and PDE ones), the extrema of
    det(I + D u1) of the inverse map, the Krylov iterations and the outer
    iterations, with the time per solve.  FP32 fields, the bench's launch shape."""
    import numpy as np

    dev = torch.device("cuda:0")
    n = spec.n
    R64 = Registration(n, spec.nt, spec.alpha, spec.s, spec.sigma2, dtype=torch.float64, device=dev)
    R = Registration(n, spec.nt, spec.alpha, spec.s, spec.sigma2, dtype=torch.float32, device=dev)
    methods = ("gd", "pde_stationary", "pde_non_stationary", "gn_v", "gn_l2", "newton")
    rows = {m: [] for m in methods}
    tuned = False
    for i in range(pairs):
        I0 = synth.phantom(n, spec.n_blobs, spec.sigma_range, spec.classes, 1000 + i, shells=spec.shells)
        t0 = torch.tensor(I0, dtype=torch.float64, device=dev)
        R64.set_images(t0, t0)
        J1 = R64.shoot(torch.tensor(synth.random_velocity(n, 2000 + i, spec.disp_vox), dtype=torch.float64,
                                    device=dev), want=("J1",))["J1"]
        I1 = J1 + torch.tensor(synth.noise(n, 3000 + i, spec.noise_sd), dtype=torch.float64, device=dev)
        R.set_images(t0.float(), I1.float())
        if not tuned:
            R.autotune(reps=3)
            R.set_option("exec.graph", 1)
            tuned = True
        zero = torch.zeros((3,) + n, dtype=torch.float32, device=dev)
        g0v, _ = R.gradient(zero)
        g0 = {"v": g0v.abs().max().item(), "l2": R.apply_L(g0v).abs().max().item()}
        for m in methods:
            pde = m.startswith("pde")
            st = m == "pde_stationary"
            v = R.empty_velocity(st).zero_() if pde else zero.clone()
            if pde:
                g0p = R.pde_gradient(v, st)[0].abs().max().item()
            torch.cuda.synchronize()
            t = time.perf_counter()
            tr = R.pde_gn_solve(v, st) if pde else R.gn_solve(v, method=m)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t)
            if pde:
                ginf = R.pde_gradient(v, st)[0].abs().max().item() / g0p
                u1 = R.pde_displacement(v, st)
            else:
                g, _ = R.gradient(v)
                ginf = (R.apply_L(g).abs().max().item() / g0["l2"]) if m == "gn_l2" else g.abs().max().item() / g0["v"]
                u1 = R.shoot(v, want=("u1",))["u1"]
            _, dmin, dmax = R.jacobian_det(u1)
            rep = tr.report
            rows[m].append([rep["mse_rel_final"], ginf, dmin, dmax, rep["cg_total"], rep["iters"], ms])
        log(f"[bench] table1 pair {i + 1}/{pairs}: " + ", ".join(f"{m} {rows[m][-1][0]:.2f}%" for m in methods))
    R.close()
    R64.close()
    cols = ("mse_rel", "g_inf_rel", "det_min", "det_max", "krylov_iters", "outer_iters", "ms_per_solve")
    out = {}
    for m in methods:
        a = np.asarray(rows[m], dtype=np.float64)
        out[m] = {c: {"mean": round(float(a[:, k].mean()), 5), "sd": round(float(a[:, k].std(ddof=1)), 5)}
                  for k, c in enumerate(cols)}
    return {"workload": f"{spec.name} recipe, {pairs} seeded pairs (template 1000+i, v0 2000+i, noise 3000+i), FP32, "
                        f"nt={spec.nt}; GD <= 50 iterations, GN/Newton <= 10, Krylov <= 20",
            "columns": list(cols), "methods": out}


def memory_bench(args, torch, synth, Registration, spec):
    """Trajectory memory policies at 256^3, nt = 32 (FP32): store every step,
    checkpoint every 4 steps, full recompute.  For each: device bytes the
    context holds (trajectory and the whole context), the drop in free device
    memory while it runs, and Hessian-vector products/s at one linearization.
    The three give bitwise the same Hv (checked here on the first component)."""
    dev = torch.device("cuda:0")
    n = spec.n
    log(f"[bench] memory policies {spec.name}: building inputs")
    I0 = synth.phantom(n, spec.n_blobs, spec.sigma_range, spec.classes, 1000, shells=spec.shells)
    v0t = synth.random_velocity(n, 2000, spec.disp_vox)
    R = Registration(n, spec.nt, spec.alpha, spec.s, spec.sigma2, dtype=torch.float32, device=dev,
                     checkpoint_every=-1)
    t0 = torch.tensor(I0, dtype=torch.float32, device=dev)
    R.set_images(t0, t0)
    vt = torch.tensor(v0t, dtype=torch.float32, device=dev)
    I1 = R.shoot(vt, want=("J1",))["J1"] + torch.tensor(synth.noise(n, 3000, spec.noise_sd), dtype=torch.float32,
                                                         device=dev)
    R.close()
    del R
    vlin = 0.5 * vt
    dv = torch.randn((3,) + n, device=dev, generator=torch.Generator(device=dev).manual_seed(9))
    out = {}
    first = None
    for name, every in (("store_all", 0), ("checkpoint_4", 4), ("recompute", -1)):
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        free0 = torch.cuda.mem_get_info(dev)[0]
        R = Registration(n, spec.nt, spec.alpha, spec.s, spec.sigma2, dtype=torch.float32, device=dev,
                         checkpoint_every=every)
        R.set_images(t0, I1)
        if every == 0 and not args.no_graph:
            R.set_option("exec.graph", 1)
        R.linearize(vlin)
        hv = torch.empty_like(dv)
        R.hessvec(dv, out=hv)
        reps = 3 if every >= 0 else 2
        ms = time_events(torch, lambda: R.hessvec(dv, out=hv), reps)
        free1 = torch.cuda.mem_get_info(dev)[0]
        if first is None:
            first = hv.clone()
            same = True
        else:
            same = bool(torch.equal(hv, first))
        out[name] = {
            "checkpoint_every": every,
            "traj_policy": R.get_option("traj.policy"),
            "trajectory_bytes": R.get_option("traj.bytes"),
            "context_bytes": R.memory_bytes(),
            "device_bytes_in_use": int(free0 - free1),
            "hv_per_s": round(1e3 / ms, 3),
            "ms_per_hv": round(ms, 2),
            "hv_bitwise_equal_to_store_all": same,
        }
        log(f"[bench] {name}: {out[name]}")
        R.close()
        del R, hv
    torch.cuda.empty_cache()
    return {
        "workload": f"{spec.name}: {n[0]}x{n[1]}x{n[2]} pair, nt={spec.nt}, FP32, alpha={spec.alpha}, s={spec.s}",
        "policies": out,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="pair128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the GN-L2 and gradient-descent solves")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the head-grid, batch16, 256^3 memory-policy and PDE-LDDMM workloads")
    ap.add_argument("--hv-reps", type=int, default=20)
    ap.add_argument("--no-tune", action="store_true", help="keep the default transform launch shapes")
    ap.add_argument("--no-graph", action="store_true", help="launch Hessian-vector products kernel by kernel")
    ap.add_argument(
        "--shape",
        default=None,
        metavar="JSON",
        help='launch shape to use instead of autotuning, e.g. the "launch_shape" of an earlier bench line '
        "(read-only keys in it are checked, not set)",
    )
    ap.add_argument(
        "--profile-hv",
        type=int,
        default=0,
        metavar="K",
        help="profiling mode: K Hessian-vector products at the workload's linearization (pair128 or "
        "head180x216x180), then 4 plain copies of 256 MiB (counter calibration), and exit",
    )
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(
            "bench.py measures one GPU only: the hot path runs on one MI355X per registration "
            "problem; run it with --gpus 1",
            file=sys.stderr,
        )
        sys.exit(2)

    import torch

    import synth
    from paper_1807_04638_amd import Batch, Registration

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "batch16":
        print(json.dumps(batch_bench(args, torch, synth, Batch, Registration)), flush=True)
        return
    # everything runs on a dedicated stream so the contexts can replay graphs
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    if args.workload == "table1":
        print(json.dumps(table1_bench(args, torch, synth, Registration, synth.WORKLOADS["pair128"])), flush=True)
        return
    spec = synth.WORKLOADS[args.workload]
    if args.workload == "head180x216x180" and not args.profile_hv:
        print(json.dumps(precision_bench(args, torch, synth, Registration, spec)), flush=True)
        return
    if args.workload == "pair256":
        print(json.dumps(memory_bench(args, torch, synth, Registration, spec)), flush=True)
        return
    log(f"[bench] workload {spec.name} n={spec.n} nt={spec.nt}: building inputs")
    I0, I1, v0t = make_pair(spec, torch.float64, dev, torch, Registration, synth)

    def context(dtype):
        R = Registration(spec.n, spec.nt, spec.alpha, spec.s, spec.sigma2, dtype=dtype, device=dev)
        R.set_images(torch.tensor(I0, dtype=dtype, device=dev), torch.tensor(I1, dtype=dtype, device=dev))
        if args.shape and dtype == torch.float32:
            shape = json.loads(args.shape)
            for key, val in shape.items():
                if key == "fft.plane_halves_used":
                    R.set_option("fft.plane_halves", val)
                elif key not in ("fft.fused", "fft.static_kernels"):
                    R.set_option(key, val)
            for key in ("fft.fused", "fft.static_kernels", "fft.plane_halves_used"):
                if key in shape and R.get_option(key) != shape[key]:
                    raise SystemExit(f"bench.py: launch shape {key}={shape[key]} is not what this grid gives")
            log(f"[bench] launch shape set: {shape}")
        elif not args.no_tune:
            tried, ms = R.autotune(reps=5)
            log(f"[bench] autotune {dtype}: {tried} variants, K application {1e3 * ms:.1f} us")
        if not args.no_graph:
            R.set_option("exec.graph", 1)
        return R

    def solve(R, dtype):
        v = torch.zeros((3,) + spec.n, dtype=dtype, device=dev)
        return R.gn_solve(v, gn_iters=spec.gn_iters, cg_iters=spec.cg_iters)

    R = context(torch.float32)
    if args.profile_hv:
        vlin = torch.tensor(0.5 * v0t, dtype=torch.float32, device=dev)
        dv = torch.randn((3,) + spec.n, device=dev, generator=torch.Generator(device=dev).manual_seed(7))
        hv = torch.empty_like(dv)
        R.linearize(vlin)
        for i in range(args.profile_hv):
            R.hessvec(dv, out=hv)
            torch.cuda.synchronize()
            log(f"[bench] profile hessvec {i + 1}/{args.profile_hv}")
        src = torch.ones(64 * 2**20, dtype=torch.float32, device=dev)  # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        tuned = {k: R.get_option(k) for k in TUNED_KEYS}
        digests = {g: source_digest(g) for g in KERNEL_SOURCES}
        print(
            json.dumps(
                {"profile_hv": args.profile_hv, "copy_bytes_each_way": src.numel() * 4, "tuned": tuned, "sources": digests}
            ),
            flush=True,
        )
        return
    log(f"[bench] warmup {args.warmup} solve(s)")
    for _ in range(args.warmup):
        solve(R, torch.float32)
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} solve(s)")
    t0 = time.perf_counter()
    traces = []
    for _ in range(args.steps):
        traces.append(solve(R, torch.float32))
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    rep = traces[-1].report
    ms_per_step = 1e3 * T / args.steps
    log(f"[bench] {ms_per_step:.1f} ms per solve, report {rep}")

    # Hessian-vector products and gradients (HIP events on the library stream)
    vlin = torch.tensor(0.5 * v0t, dtype=torch.float32, device=dev)
    dv = torch.randn((3,) + spec.n, device=dev, generator=torch.Generator(device=dev).manual_seed(7))
    hv = torch.empty_like(dv)
    g = torch.empty_like(dv)
    R.linearize(vlin)
    R.hessvec(dv, out=hv)
    # medians of single calls after 3 untimed ones: >= 20 Hessian-vector products, 5 gradients, 5 shoots
    hv_ms = median_events(torch, lambda: R.hessvec(dv, out=hv), max(20, args.hv_reps))
    grad_ms = median_events(torch, lambda: R.gradient(vlin, out=g), 5)
    shoot_ms = median_events(torch, lambda: R.shoot(vlin, want=("J1",)), 5)
    log(f"[bench] hessvec {hv_ms:.3f} ms, gradient {grad_ms:.3f} ms, shoot {shoot_ms:.3f} ms")

    # per-kernel HIP-event timing over Hessian-vector products -> roofline
    R.linearize(vlin)
    R.profile_enable(True)
    for _ in range(5):
        R.hessvec(dv, out=hv)
    prof = R.profile_read()
    R.profile_enable(False)
    nbytes = kernel_bytes(spec.n, 4)
    tuned = {k: R.get_option(k) for k in TUNED_KEYS}
    total_ms = sum(v[1] for v in prof.values())
    kernels = {}
    for name, (cnt, ms) in prof.items():
        avg_us = 1e3 * ms / max(cnt, 1)
        kb = nbytes.get(name)
        kernels[name] = {
            "group": kernel_group(name),
            "launches_per_hv": cnt / 5,
            "avg_us": round(avg_us, 2),
            "share": round(ms / total_ms, 4),
            "ledger_bytes": kb,
            "ledger_GBps": round(kb / (avg_us * 1e-6) / 1e9, 1) if kb else None,
            "traffic": recorded_traffic(name, tuned),
        }
    # kernel templates (predictor, corrector and first stages together), each
    # priced at its share of the Hessian-vector product's compulsory floor
    groups = {}
    for name, k in kernels.items():
        g = groups.setdefault(k["group"], {"launches_per_hv": 0.0, "ms_per_hv": 0.0, "members": [], "traffic_sum": 0.0,
                                           "traffic_known": True})
        g["launches_per_hv"] += k["launches_per_hv"]
        g["ms_per_hv"] += prof[name][1] / 5
        g["members"].append(name)
        if k["traffic"] is None:
            g["traffic_known"] = False
        else:
            g["traffic_sum"] += k["traffic"] * k["launches_per_hv"]
    for gname, g in groups.items():
        fb = floor_bytes_per_launch(gname, spec.n, 4)
        avg_us = 1e3 * g["ms_per_hv"] / g["launches_per_hv"]
        g["avg_us"] = round(avg_us, 2)
        g["floor_bytes_per_launch"] = int(fb) if fb else None
        g["floor_GBps"] = round(fb / (avg_us * 1e-6) / 1e9, 1) if fb else None
        g["traffic"] = int(g["traffic_sum"] / g["launches_per_hv"]) if g["traffic_known"] else None
        g["ms_per_hv"] = round(g["ms_per_hv"], 4)
        del g["traffic_sum"], g["traffic_known"]
    dom = max((g for g in groups if groups[g]["floor_bytes_per_launch"]), key=lambda g: groups[g]["ms_per_hv"])
    dom_bytes = groups[dom]["floor_bytes_per_launch"]
    dom_avg_s = groups[dom]["avg_us"] * 1e-6
    achieved = dom_bytes / dom_avg_s / 1e9
    hv_ledger = sum(nbytes[k] * kernels[k]["launches_per_hv"] for k in kernels if k in nbytes)
    hv_floor = hv_floor_bytes(spec.n, spec.nt, 4)
    counted = [k for k in kernels if kernels[k]["traffic"] is not None]
    hv_counter = (sum(kernels[k]["traffic"] * kernels[k]["launches_per_hv"] for k in kernels)
                  if len(counted) == len(kernels) else None)
    log(f"[bench] dominant kernel template {dom}: {groups[dom]}")

    # practical HBM ceiling for reference: a plain 1 GiB device copy (read + write)
    src = torch.ones(256 * 2**20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    copy_ms = time_events(torch, lambda: dst.copy_(src), 10)
    copy_GBps = 2 * src.numel() * 4 / (copy_ms * 1e-3) / 1e9
    del src, dst
    log(f"[bench] device copy 1 GiB: {copy_ms:.3f} ms, {copy_GBps:.0f} GB/s (read + write)")

    # the other optimisers on the same pair: Gauss-Newton with PCG in L2
    # (preconditioner K), gradient descent in V (50 iterations) and Newton-Krylov
    # on the full Hessian
    variants = {}
    vlin_newton = torch.tensor(0.5 * v0t, dtype=torch.float32, device=dev)
    dvn = torch.randn((3,) + spec.n, device=dev, generator=torch.Generator(device=dev).manual_seed(8))
    hvn = torch.empty_like(dvn)
    if not args.no_variants:
        for method in ("gn_l2", "gd", "newton"):
            v = torch.zeros((3,) + spec.n, dtype=torch.float32, device=dev)
            R.gn_solve(v, gn_iters=1, cg_iters=2, method=method)  # warm-up (graph capture)
            v.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            trv = R.gn_solve(v, cg_iters=spec.cg_iters, method=method)
            torch.cuda.synchronize()
            sv = time.perf_counter() - t1
            r = trv.report
            if method == "newton":
                R.linearize(vlin_newton)
                R.hessvec(dvn, out=hvn, newton=True)
                nms = time_events(torch, lambda: R.hessvec(dvn, out=hvn, newton=True), 5)
            variants[method] = {
                "solves_per_min": round(60.0 / sv, 3),
                "ms_per_solve": round(1e3 * sv, 1),
                "iters": r["iters"],
                "cg_total": r["cg_total"],
                "gradients": r["gradients"],
                "line_search_shoots": r["shoots"],
                "mse_rel_final": r["mse_rel_final"],
                "E_final": r["E_final"],
                "g_rel_final": r["g_rel_final"],
            }
            if method == "newton":
                variants[method]["hv_per_s"] = round(1e3 / nms, 2)
            log(f"[bench] {method}: {variants[method]}")

    # plain FP64 path
    fp64 = None
    if not args.no_fp64:
        R.close()
        R = None
        torch.cuda.empty_cache()
        R64 = context(torch.float64)
        v64 = torch.tensor(0.5 * v0t, dtype=torch.float64, device=dev)
        d64 = dv.double()
        R64.hessvec(d64, v0=v64)
        hv64_ms = time_events(torch, lambda: R64.hessvec(d64), max(5, args.hv_reps // 4))
        t1 = time.perf_counter()
        tr64 = solve(R64, torch.float64)
        torch.cuda.synchronize()
        s64 = time.perf_counter() - t1
        fp64 = {
            "gn_solves_per_min": round(60.0 / s64, 3),
            "ms_per_solve": round(1e3 * s64, 1),
            "hv_per_s": round(1e3 / hv64_ms, 2),
            "mse_rel_final": tr64.report["mse_rel_final"],
            "E_final": tr64.report["E_final"],
            "hessvecs": tr64.report["hessvecs"],
        }
        log(f"[bench] fp64 {fp64}")
        del R64
        torch.cuda.empty_cache()

    # the other workloads, bounded in time: precision policy on the head grid,
    # the batch of 16 uneven pairs, trajectory memory policies at 256^3
    extra = {}
    if not args.no_extra:
        if R is not None:
            R.close()
            R = None
        torch.cuda.empty_cache()
        for key, fn in (
            ("head180x216x180", lambda: precision_bench(args, torch, synth, Registration,
                                                        synth.WORKLOADS["head180x216x180"])),
            ("batch16", lambda: batch_bench(args, torch, synth, Batch, Registration)),
            ("pair256_memory", lambda: memory_bench(args, torch, synth, Registration, synth.WORKLOADS["pair256"])),
            ("pair128_pde_lddmm", lambda: pde_bench(args, torch, Registration, spec, I0, I1)),
            ("table1_pair128x15", lambda: table1_bench(args, torch, synth, Registration, spec)),
        ):
            log(f"[bench] extra workload {key}")
            try:
                extra[key] = fn()
                torch.cuda.synchronize()
            except Exception as e:  # an extra workload never costs the headline line
                log(f"[bench] extra workload {key} failed: {type(e).__name__}: {e}")
                extra[key] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(spec, I0, I1, v0t, rep)

    value = 60.0 * args.steps / T
    out = {
        "metric": "Hessian-vector products/s & GN solves/min at 128^3 vs FP64 path; % HBM peak",
        "value": round(value, 3),
        "unit": "GN solves/min",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{spec.name}: {spec.n[0]}x{spec.n[1]}x{spec.n[2]} pair, nt={spec.nt}, alpha={spec.alpha}, "
            f"s={spec.s}, sigma2={spec.sigma2}, GN<= {spec.gn_iters}, CG<= {spec.cg_iters}, FP32 fields + FP64 reductions",
            "global_batch": 1,
            "grid": list(spec.n),
            "parallelism": "single GPU",
        },
        "hv_per_s": round(1e3 / hv_ms, 2),
        "ms_per_hv": round(hv_ms, 3),
        "gradients_per_s": round(1e3 / grad_ms, 2),
        "shoots_per_s": round(1e3 / shoot_ms, 2),
        "solve": {
            "iters": rep["iters"],
            "hessvecs": rep["hessvecs"],
            "gradients": rep["gradients"],
            "line_search_shoots": rep["shoots"],
            "mse_rel_final": rep["mse_rel_final"],
            "E_first": rep["E_first"],
            "E_final": rep["E_final"],
        },
        "fp64": fp64,
        "fp32_speedup_vs_fp64": round(fp64["ms_per_solve"] / ms_per_step, 3) if fp64 else None,
        "variants": variants,
        "hv_floor_bytes": int(hv_floor),
        "floor_frac": round(hv_floor / (hv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "hv_ledger_bytes": int(hv_ledger),
        "hv_ledger_GBps": round(hv_ledger / (hv_ms * 1e-3) / 1e9, 1),
        "hv_counter_bytes": int(hv_counter) if hv_counter else None,
        "counter_over_floor": round(hv_counter / hv_floor, 3) if hv_counter else None,
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": groups[dom]["traffic"],
            "bytes_per_launch": int(dom_bytes),
            "avg_launch_us": groups[dom]["avg_us"],
            "launches_per_hv": groups[dom]["launches_per_hv"],
        },
        "launch_shape": tuned,
        "kernel_groups": groups,
        "kernels": kernels,
        "hbm_copy_GBps": round(copy_GBps, 1),
        "cpu_baseline": cpu,
        "workloads": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
