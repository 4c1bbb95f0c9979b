#!/usr/bin/env python
"""Benchmark of the fast direct solver on one MI355X.

Metric (one JSON line on stdout): preconditioned-CFIE right-hand-side solves per second at
N = 16384 with rel.err <= 1e-6, plus setup seconds.  Workload: the seed-0 convex
Fourier-perturbed circle (10 nodes per wavelength, k = 1638.38), 1024 TE plane waves.

A step is one pass of the whole hot path on device-resident data: assembly of the BEM
matrices and the circulant spectrum (cfie_assemble), randomized skeleton and capacitance LU
(cfie_factor), plane-wave right-hand sides (cfie_plane_wave_rhs) and the Woodbury solve of
all right-hand sides (cfie_solve).  `value` is the solve throughput (nrhs / solve seconds,
the solve being the per-right-hand-side cost once the factorisation exists); `setup_s` is
assemble + factor.  Accuracy of the timed output is checked against the FP64 residual of
the assembled operator and, where stored oracle solutions exist, against the oracle.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "preconditioned-CFIE RHS solves/s at N=16384, rel.err ≤1e-6; setup seconds"
PEAKS = {"zgemm_f64": ("mfma", 78.6, "TFLOP/s"), "zgemm_f32": ("mfma", 157.3, "TFLOP/s"),
         "circ_fft": ("hbm", 8000.0, "GB/s")}
FP64_PEAK = 78.6e12
HBM_PEAK = 8.0e12
# FP64 flops per Gauss point pair of the far-pair assembly kernels, counted on the metric
# workload with rocprofv3 (64 x (ADD_F64 + MUL_F64 + 2 FMA_F64) wave instructions of the four
# far kernels on the contour, 2.129e12, over its N^2 q^2 = 6.711e9 point pairs;
# profiles/valu_hbm_kernels_perturbed16384.md)
FAR_FLOPS_PER_PAIR = 317.2


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--solve-reps", type=int, default=5,
                    help="solves per step on the same right-hand sides; the step's solve time "
                         "is their median (RHS/s is taken over the median of at least 5 solves)")
    ap.add_argument("--workload", default="perturbed16384",
                    help="perturbed16384 (the metric), ellipse4096, ellipse256, batch64, "
                         "shapegrad8192 or serve16384")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--sketch", choices=("srft", "gaussian"), default="srft",
                    help="test matrix of the range finder's blocks after the first")
    ap.add_argument("--refine", choices=("factored", "dense"), default="dense",
                    help="mixed precision: residuals factor by factor or with C formed densely "
                         "in FP64 at factor time")
    ap.add_argument("--eps", type=float, default=None,
                    help="compression tolerance (default 1e-5 fp64, 1e-3 mixed)")
    ap.add_argument("--compare", action=argparse.BooleanOptionalAction, default=True,
                    help="also run one step of the other precision and report it")
    ap.add_argument("--cpu-baseline", action=argparse.BooleanOptionalAction, default=True)
    ap.add_argument("--tight", action=argparse.BooleanOptionalAction, default=True,
                    help="also run one FP64 step at epsilon = 1e-10 (the FP64 parity level)")
    ap.add_argument("--profile", action=argparse.BooleanOptionalAction, default=True,
                    help="HIP-event timing of every hot launch inside the library")
    ap.add_argument("--serve-m", type=int, default=8,
                    help="right-hand sides per call of the serve16384 workload")
    ap.add_argument("--serve-workload", default="perturbed16384",
                    help="problem of the serve16384 workload (default: the metric's)")
    ap.add_argument("--remainder", choices=("auto", "factored", "dense"), default=None,
                    help="how the factorisation applies C - C_c (default: auto; dense for "
                         "shapegrad8192, whose remainder has full rank at 1e-10)")
    ap.add_argument("--autotune", action=argparse.BooleanOptionalAction, default=True,
                    help="GEMM tile autotuner (bitwise-neutral; on by default)")
    ap.add_argument("--grouped", action=argparse.BooleanOptionalAction, default=False,
                    help="batch64: every problem's solve in one recorded launch "
                         "(cfie_solve_batch_grouped) after all are factored")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the steps, copy a MIB-mebibyte device buffer once (a kernel of "
                         "known HBM traffic, the reference for hardware byte counters)")
    return ap.parse_args()


def step(P, w, prec, eps, profile, form=0, refine=0, solve_reps=1, sketch=None):
    """One pass of the hot path: assemble, factor, right-hand sides, solve.  The solve runs
    solve_reps times on the same right-hand sides (each a full solve); its time is their
    median."""
    import torch
    s = P.Solver(precision=prec, compress_tol=eps, block=256, refine_tol=1e-8,
                 profile=profile, remainder_form=form, refine_form=refine,
                 test_matrix=P.SKETCH_SRFT if sketch is None else sketch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.assemble(w.zhat, w.n_nodes, w.k)
    s.factor()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    B = s.plane_wave_rhs(w.angles)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    solves = []
    for _ in range(max(1, solve_reps)):
        ts = time.perf_counter()
        X = s.solve(B)
        torch.cuda.synchronize()
        solves.append(time.perf_counter() - ts)
    t3 = time.perf_counter()
    solve_s = sorted(solves)[len(solves) // 2]
    return s, B, X, dict(setup_s=t1 - t0, rhs_s=t2 - t1, solve_s=solve_s, step_s=t3 - t0)


def accuracy(P, s, w, B, X):
    """max over sampled columns of ||b - C x|| / ||b|| (FP64, assembled operator) and, where
    oracle solutions are stored for this workload, max rel.err against them."""
    import numpy as np
    import torch
    m = B.shape[0]
    cols = torch.arange(0, m, max(1, m // 32), device=B.device)
    Xs, Bs = X[cols].contiguous(), B[cols].contiguous()
    R = s.apply(P.OP_C, Xs) - Bs
    res = float((R.abs().pow(2).sum(1).sqrt() / Bs.abs().pow(2).sum(1).sqrt()).max())
    err = None
    gpath = os.path.join(ROOT, "tests", "golden", w.name + ".npz")
    if os.path.exists(gpath):
        g = np.load(gpath)
        if int(g["N"]) == w.n_nodes and abs(float(g["k"]) - w.k) < 1e-12 * w.k:
            idx = g["cols_rhs"]
            x = X[torch.as_tensor(idx, device=X.device)].cpu().numpy().T
            xr = g["x"]
            err = float(np.max(np.linalg.norm(x - xr, axis=0) / np.linalg.norm(xr, axis=0)))
    return res, err


def _oracle_sample(w, Ns, cores, ms=64):
    """Phase times of the oracle at Ns nodes of w's contour at w's nodes per wavelength:
    dense assembly, form C + LU, LU solve of ms right-hand sides."""
    import numpy as np
    import scipy.linalg as sla
    from oracle import assembly as A
    from oracle import system as S
    ks = w.k * Ns / w.n_nodes
    L = S.Contour(w.zhat).L
    kts = S.ktilde(ks, L)
    t0 = time.perf_counter()
    M = A.assemble(w.zhat, Ns, ks, kts, workers=cores)
    t1 = time.perf_counter()
    C = S.form_C(M)
    lu = sla.lu_factor(C)
    t2 = time.perf_counter()
    angles = 2 * math.pi * np.arange(ms) / ms
    e, hh = S.excitation(w.zhat, Ns, ks, angles)
    b = S.rhs(M, e, hh, ks)
    t3 = time.perf_counter()
    sla.lu_solve(lu, b)
    t4 = time.perf_counter()
    return dict(asm=t1 - t0, lu=t2 - t1, solve=(t4 - t3) / ms, total=t4 - t0)


def cpu_baseline(w):
    """The CPU oracle on a bounded sample of this workload, scaled to it.

    Sample: the oracle's dense assembly, its dense C and LU, and the triangular solves of 64
    right-hand sides at N_s = 1024 and 2048 nodes of the same contour and the same nodes per
    wavelength (about 15 s of CPU work on 16 cores).  Scaling to N from the 2048 sample:
    assembly ~ N^2 (pairs of elements), form C + LU ~ N^3, solve ~ N^2 per right-hand side;
    the exponents measured between the two samples are reported beside them.  The oracle's
    one full-size run (tests/golden/perturbed16384.npz, on the 8 cores where the references
    were written) is reported for comparison."""
    import numpy as np
    # at most 16 host threads: the host share that comes with one GPU
    cores = max(1, min(16, os.cpu_count() or 1))
    a = _oracle_sample(w, 1024, cores)
    b = _oracle_sample(w, 2048, cores)
    Ns = 2048
    r = w.n_nodes / Ns
    t_asm = b["asm"] * r * r
    t_lu = b["lu"] * r ** 3
    t_solve_per_rhs = b["solve"] * r * r
    expo = {k: round(math.log2(b[k] / a[k]), 2) for k in ("asm", "lu", "solve")}
    out = {"value": 1.0 / t_solve_per_rhs, "unit": "RHS/s", "cores": cores, "kind": "oracle",
           "setup_s": t_asm + t_lu,
           "sample": f"oracle at N=1024 and N={Ns} (same contour, same nodes/wavelength): "
                     f"dense assembly {b['asm']:.1f} s x (N/{Ns})^2, form C + LU "
                     f"{b['lu']:.1f} s x (N/{Ns})^3, LU solve {b['solve'] * 1e3:.2f} ms per "
                     f"RHS x (N/{Ns})^2",
           "measured_exponents_1024_2048": {"assembly": expo["asm"], "form_C_LU": expo["lu"],
                                            "solve_per_rhs": expo["solve"]},
           "sample_cpu_s": round(a["total"] + b["total"], 1)}
    gpath = os.path.join(ROOT, "tests", "golden", w.name + ".npz")
    if os.path.exists(gpath):
        g = np.load(gpath)
        if int(g["N"]) == w.n_nodes:
            out["full_size_reference"] = {
                "cores": 8, "assembly_s": round(float(g["t_assemble_s"]), 1),
                "form_C_LU_solve_s": round(float(g["t_lu_s"]), 1),
                "note": "the oracle's full run at this N when its stored solutions were "
                        "written (8-core build host, 4 right-hand sides)"}
    return out


def phase_roofline(w, info, prof_tot, steps, solve_s, nrhs):
    """Achieved fraction of each phase's bound (the last timed step's device times).

    assembly: FP64 VALU -- Gauss point pairs of the far kernels x their counted FP64 flops per
    pair over the assembly's device time (the near band, the circle row and the DFTs inside
    that time are not credited).  capacitance LU: FP64 matrix cores -- the executed flops of
    K = I + V^T U~ (6 r^2 N, 3M form) and of the LU's trailing updates (2 r^3 of the
    (8/3) r^3 classical count, 3M form) over the phase's device time.  solve: the sum of the
    phase floors over the measured solve time -- the two Woodbury products at the FP64
    matrix-core peak (6 N r m executed flops each) plus the HBM floor of the right-hand
    sides read and the solutions written and the circulant product's one read and one
    write of the batch (64 N m bytes)."""
    N, r, m = w.n_nodes, info["rank"], nrhs
    out = {}
    far = prof_tot.get("assemble_far")
    t_asm = info["t_assemble_ms"] / 1e3
    if far and far[0] and t_asm > 0:
        flops = far[1] / steps * FAR_FLOPS_PER_PAIR
        out["assembly"] = {"bound": "fp64_valu", "achieved_tflops": flops / t_asm / 1e12,
                           "peak_tflops": FP64_PEAK / 1e12, "frac": flops / t_asm / FP64_PEAK}
    t_lu = info["t_factor_phase_ms"][2] / 1e3
    if r > 0 and t_lu > 0:
        flops = 6.0 * r * r * N + 2.0 * r ** 3
        out["capacitance_lu"] = {"bound": "mfma_fp64", "achieved_tflops": flops / t_lu / 1e12,
                                 "peak_tflops": FP64_PEAK / 1e12,
                                 "frac": flops / t_lu / FP64_PEAK}
    if solve_s > 0:
        t_gemm = 2 * 6.0 * N * r * m / FP64_PEAK
        t_hbm = 64.0 * N * m / HBM_PEAK
        out["solve"] = {"floor_ms": 1e3 * (t_gemm + t_hbm), "gemm_floor_ms": 1e3 * t_gemm,
                        "hbm_floor_ms": 1e3 * t_hbm, "measured_ms": 1e3 * solve_s,
                        "frac": (t_gemm + t_hbm) / solve_s}
    return out


def measured_traffic(kernel, launches_per_step):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC summary, or None when
    the summary is missing, was taken on a different version of the kernel's source, or on a
    step with a different number of launches of it (a different mix of shapes)."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", f"{kernel}_perturbed16384.md")
    src = os.path.join(ROOT, "paper_2203_13283_amd", "csrc",
                       {"zgemm_f64": "k_gemm.hip", "zgemm_f32": "k_gemm.hip"}.get(kernel, ""))
    if not (os.path.exists(prof) and os.path.isfile(src)):
        return None
    vals = {}
    for line in open(prof):
        k, _, v = line.strip().partition(": ")
        if k in ("traffic_bytes_per_launch", "source_sha256", "launches_per_step"):
            vals[k] = v.strip()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if vals.get("source_sha256") != sha or "traffic_bytes_per_launch" not in vals:
        return None
    if vals.get("launches_per_step") != str(launches_per_step):
        return None
    return float(vals["traffic_bytes_per_launch"])


def batch_main(a):
    """--workload batch64: 64 seeded perturbed ellipses, N log-uniform in [512, 8192], 32-512
    plane waves each, every problem's whole path (assembly, factor, right-hand sides, solve)
    through cfie_solve_batch over four streams.  value = aggregate right-hand sides solved per
    second of wall time for the whole batch (setup included)."""
    import torch
    import workloads as W
    import paper_2203_13283_amd as P
    probs = W.batch_problems()
    prec = P.CFIE_FP64 if a.precision == "fp64" else P.CFIE_MIXED
    eps = a.eps if a.eps is not None else (1e-6 if prec == P.CFIE_FP64 else 1e-3)
    nrhs = sum(p["angles"].size for p in probs)
    sk = P.SKETCH_SRFT if a.sketch == "srft" else P.SKETCH_GAUSSIAN
    for _ in range(a.warmup):
        P.solve_batch(probs[:4], precision=prec, compress_tol=eps, block=128, test_matrix=sk)
    torch.cuda.synchronize()
    times = []
    for _ in range(a.steps):
        t0 = time.perf_counter()
        sols, res = P.solve_batch(probs, precision=prec, compress_tol=eps, block=128,
                                  refine_tol=1e-8, n_streams=4, grouped=a.grouped,
                                  sweeps=2, test_matrix=sk)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    med = sorted(times)[len(times) // 2]
    # accuracy of the last batch: FP64 residual of a few columns of three problems
    worst = 0.0
    for i in (0, len(probs) // 2, len(probs) - 1):
        pr = probs[i]
        s = P.Solver(compress_tol=eps, block=128)
        s.assemble(pr["zhat"], pr["n_nodes"], pr["k"])
        X = sols[i][:4].contiguous()
        B = s.plane_wave_rhs(pr["angles"][:4])
        R = s.apply(P.OP_C, X) - B
        worst = max(worst, float((R.abs().pow(2).sum(1).sqrt() /
                                  B.abs().pow(2).sum(1).sqrt()).max()))
        del s
    Ns = [p["n_nodes"] for p in probs]
    out = {
        "metric": "batched preconditioned-CFIE RHS solves/s (64 contours, uneven N, setup "
                  "included)",
        "value": nrhs / med, "unit": "RHS/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * med, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == P.CFIE_FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": "batch64: seeded perturbed ellipses a~U(0.8,1.2), "
                               "b~U(0.4,0.8), N log-uniform in [512, 8192], 32-512 plane "
                               "waves, 10 nodes/wavelength",
                   "problems": len(probs), "N_min": min(Ns), "N_max": max(Ns),
                   "nrhs_total": nrhs, "compress_tol": eps, "streams": 4,
                   "precision": a.precision, "gemm_autotune": bool(a.autotune),
                   "grouped_solve": bool(a.grouped), "sketch": a.sketch},
        "problems_per_s": len(probs) / med,
        "rel_residual_sampled": worst,
        "max_rank": max(r["rank"] for r in res),
    }
    print(json.dumps(out), flush=True)


def serve_main(a):
    """--workload serve16384: the metric's problem (perturbed16384) factored once, then many
    small solves (--serve-m right-hand sides per call, 200 calls), as a serving loop would
    issue them: direct cfie_solve against recorded solves (options.solve_graphs).
    value = right-hand sides per second of the recorded solves."""
    import torch
    import workloads as W
    import paper_2203_13283_amd as P
    w = W.get(a.serve_workload)
    m, calls = a.serve_m, 200
    eps = a.eps if a.eps is not None else 1e-5
    out_modes = {}
    for graphs in (False, True):
        s = P.Solver(compress_tol=eps, block=256, solve_graphs=graphs)
        s.assemble(w.zhat, w.n_nodes, w.k)
        s.factor()
        B = s.plane_wave_rhs(w.angles[:m])
        X = torch.empty_like(B)
        for _ in range(5):
            s.solve(B, out=X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(calls):
            s.solve(B, out=X)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / calls
        out_modes["graph" if graphs else "direct"] = dict(ms_per_call=1e3 * dt,
                                                          rhs_per_s=m / dt)
        rank = s.info()["rank"]
        del s, B, X
        torch.cuda.empty_cache()
    g = out_modes["graph"]
    out = {
        "metric": "preconditioned-CFIE RHS solves/s in small batches (serving loop)",
        "value": g["rhs_per_s"], "unit": "RHS/s", "n_gpus": 1, "steps": calls, "warmup": 5,
        "ms_per_step": g["ms_per_call"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"serve16384: {w.name}: {w.description}, factored once, {m} "
                               "plane waves per call", "N": w.n_nodes, "nrhs_per_call": m, "calls": calls,
                   "compress_tol": eps},
        "rank": rank, "modes": out_modes,
        "graph_speedup": out_modes["direct"]["ms_per_call"] / g["ms_per_call"],
    }
    print(json.dumps(out), flush=True)


def shapegrad_main(a):
    """--workload shapegrad8192: the shape-differentiation workload (r = 1 + sum_{m<=64}
    s_m cos + t_m sin, s_m, t_m ~ N(0, (0.01/m)^2), seed 0, N = 8192, 10 nodes/wavelength,
    16 plane waves, 181 backscatter observation angles each).  A step is the forward pass
    (assemble, factor, right-hand sides, solve, far field) and the gradient of the loss
    sum |F|^2 with respect to the 128 shape coefficients (cfie_shape_gradient).
    value = gradient evaluations per second (forward + backward)."""
    import numpy as np
    import torch
    import workloads as W
    import paper_2203_13283_amd as P
    pr = W.shape_problem()
    N, k, inc, obs = pr["n_nodes"], pr["k"], pr["angles"], pr["obs"]
    m, n_obs = obs.shape
    mmax = pr["s"].size
    eps = a.eps if a.eps is not None else 1e-10
    sel = np.zeros((m, m * n_obs))
    for j in range(m):
        sel[j, j * n_obs:(j + 1) * n_obs] = 1.0
    sel = torch.as_tensor(sel, device="cuda")
    J = W.shape_jacobian(mmax)
    form = {"auto": 0, "factored": 1, "dense": 2}[a.remainder or "dense"]

    def one():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = P.Solver(compress_tol=eps, block=256, remainder_form=form)
        s.assemble(pr["zhat"], N, k)
        s.factor()
        X = s.solve(s.plane_wave_rhs(inc))
        F = s.far_field(X, obs.ravel())
        L = float(((F.abs() ** 2) * sel).sum())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gz = s.shape_gradient(inc, X, obs.ravel(), (2 * F * sel).contiguous())
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        info = s.info()
        return dict(fwd=t1 - t0, bwd=t2 - t1, L=L, g=J.T @ gz.reshape(-1), rank=info["rank"],
                    asm=info["t_assemble_ms"] / 1e3, fac=info["t_factor_ms"] / 1e3)

    for _ in range(a.warmup):
        one()
    runs = [one() for _ in range(a.steps)]
    tot = sorted(r["fwd"] + r["bwd"] for r in runs)[len(runs) // 2]
    r = runs[-1]
    out = {
        "metric": "shape-gradient evaluations/s (far-field backscatter loss, 128 shape "
                  "coefficients)",
        "value": 1.0 / tot, "unit": "gradients/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * tot, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "shapegrad8192: r = 1 + sum_{m=1..64} s_m cos(m t) + t_m sin(m t),"
                               " s_m, t_m ~ N(0, (0.01/m)^2) seed 0, 10 nodes/wavelength, "
                               "16 plane waves x 181 backscatter angles",
                   "N": N, "k": k, "nrhs": m, "n_obs": n_obs, "compress_tol": eps,
                   "remainder_form": a.remainder or "dense"},
        "phase_s": {"forward": sorted(x["fwd"] for x in runs)[len(runs) // 2],
                    "gradient": sorted(x["bwd"] for x in runs)[len(runs) // 2],
                    "assemble_dev": r["asm"], "factor_dev": r["fac"]},
        "rank": r["rank"], "loss": r["L"], "grad_norm": float(np.linalg.norm(r["g"])),
    }
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported (the solver "
              "has no multi-GPU path).", file=sys.stderr)
        sys.exit(2)
    if not a.autotune:
        import paper_2203_13283_amd as P
        P.set_gemm_autotune(False)
    if a.workload == "batch64":
        batch_main(a)
        return
    if a.workload == "shapegrad8192":
        shapegrad_main(a)
        return
    if a.workload == "serve16384":
        serve_main(a)
        return
    import workloads as W
    w = W.get(a.workload)
    # the CPU leg runs first, before this process touches the GPU (its oracle workers fork)
    cpu = cpu_baseline(w) if a.cpu_baseline else None
    import torch
    import paper_2203_13283_amd as P
    prec = P.CFIE_FP64 if a.precision == "fp64" else P.CFIE_MIXED
    eps = a.eps if a.eps is not None else (1e-5 if prec == P.CFIE_FP64 else 1e-3)
    form = {"auto": 0, "factored": 1, "dense": 2}[a.remainder or "auto"]
    if a.calibrate_copy > 0:
        src = torch.ones(a.calibrate_copy << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cold = None
    refine = P.REFINE_DENSE if a.refine == "dense" else P.REFINE_FACTORED
    sk = P.SKETCH_SRFT if a.sketch == "srft" else P.SKETCH_GAUSSIAN
    for _ in range(a.warmup):
        s, B, X, _t = step(P, w, prec, eps, False, form, refine, sketch=sk)
        cold = _t["setup_s"] if cold is None else cold
        del s, B, X
    torch.cuda.synchronize()
    times = []
    prof_tot = {}
    t_start = time.perf_counter()
    last = None
    for _ in range(a.steps):
        if last is not None:
            del last
        s, B, X, t = step(P, w, prec, eps, a.profile, form, refine, a.solve_reps, sketch=sk)
        cold = t["setup_s"] if cold is None else cold
        times.append(t)
        for name, (n, work, ms) in s.profile().items():
            c = prof_tot.setdefault(name, [0, 0.0, 0.0])
            c[0] += n
            c[1] += work
            c[2] += ms
        last = (s, B, X)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    s, B, X = last
    info = s.info()
    res, err = accuracy(P, s, w, B, X)
    med = sorted(times, key=lambda d: d["solve_s"])[len(times) // 2]
    solve_s = sorted(d["solve_s"] for d in times)[len(times) // 2]
    setup_s = sorted(d["setup_s"] for d in times)[len(times) // 2]
    nrhs = w.nrhs
    out = {
        "metric": METRIC,
        "value": nrhs / solve_s,
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * t_total / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == P.CFIE_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.description}", "N": w.n_nodes, "nrhs": nrhs,
                   "k": w.k, "compress_tol": eps, "solve_reps": a.solve_reps,
                   "precision": "fp64" if prec == P.CFIE_FP64 else "mixed",
                   "sketch": a.sketch},
        "setup_s": setup_s,
        "setup_cold_s": cold,
        "phase_s": {"assemble+factor": setup_s, "rhs": med["rhs_s"], "solve": solve_s,
                    "assemble_dev": info["t_assemble_ms"] / 1e3,
                    "factor_dev": info["t_factor_ms"] / 1e3,
                    "factor_range_finder_dev": info["t_factor_phase_ms"][0] / 1e3,
                    "factor_projection_dev": info["t_factor_phase_ms"][1] / 1e3,
                    "factor_capacitance_lu_dev": info["t_factor_phase_ms"][2] / 1e3,
                    "factor_kinv_vt_dev": info["t_factor_phase_ms"][3] / 1e3},
        "rank": info["rank"],
        "rel_residual": res,
        "rel_err_bound": 4.0 * res,
        "rel_err_vs_oracle": err,
        "refine_sweeps": info["refine_sweeps"],
    }
    kern = {}
    for name, (n, work, ms) in prof_tot.items():
        if n == 0:
            continue
        kern[name] = {"launches": n, "ms_total": ms / a.steps, "avg_launch_ms": ms / n,
                      "work_per_launch": work / n}
        if name in PEAKS:
            bound, peak, unit = PEAKS[name]
            scale = 1e-12 if unit == "TFLOP/s" else 1e-9
            ach = (work / n) * scale / (ms / n / 1e3)
            kern[name].update({"bound": bound, "achieved": ach, "unit": unit, "frac": ach / peak})
            if name == "circ_fft":
                # the four-step split makes three passes over the data for N > 4096
                passes = 3 if w.n_nodes > 4096 else 1
                kern[name].update({"passes": passes, "frac_per_pass": passes * ach / peak})
    out["kernels"] = kern
    out["phase_roofline"] = phase_roofline(w, info, prof_tot, a.steps, solve_s, nrhs)
    dom = max((k for k in kern if k in PEAKS), key=lambda k: kern[k]["ms_total"], default=None)
    if dom is not None:
        bound, peak, unit = PEAKS[dom]
        d = kern[dom]
        scale = 1e-12 if unit == "TFLOP/s" else 1e-9
        achieved = d["work_per_launch"] * scale / (d["avg_launch_ms"] / 1e3)
        out["roofline"] = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak,
                           "unit": unit, "frac": achieved / peak,
                           "traffic": measured_traffic(dom, d["launches"] // a.steps)}
    del last, s, B, X
    torch.cuda.empty_cache()
    if a.compare:
        other = P.CFIE_MIXED if prec == P.CFIE_FP64 else P.CFIE_FP64
        eps_o = 1e-3 if other == P.CFIE_MIXED else 1e-5
        # mixed precision: the refinement's residual factor by factor and with C formed
        # densely in FP64 at factor time
        forms = (P.REFINE_FACTORED, P.REFINE_DENSE) if other == P.CFIE_MIXED else (0,)
        legs = []
        for rf in forms:
            torch.cuda.empty_cache()
            so, Bo, Xo, to = step(P, w, other, eps_o, False, form, rf, sketch=sk)
            io = so.info()
            res_o, err_o = accuracy(P, so, w, Bo, Xo)
            legs.append({"precision": "mixed" if other == P.CFIE_MIXED else "fp64",
                         "compress_tol": eps_o, "value": nrhs / to["solve_s"],
                         "setup_s": to["setup_s"], "rank": io["rank"],
                         "refine_form": "dense" if rf == P.REFINE_DENSE else "factored",
                         "refine_sweeps": io["refine_sweeps"], "rel_residual": res_o,
                         "rel_err_vs_oracle": err_o})
            del so, Bo, Xo
        out["compare"] = legs[-1]
        if len(legs) > 1:
            out["compare_refine_factored"] = legs[0]
    if a.tight and prec == P.CFIE_FP64 and a.eps is None:
        # the FP64 path at the parity level of 1e-10 (nearly full rank at this size)
        torch.cuda.empty_cache()
        st, Bt, Xt, tt = step(P, w, P.CFIE_FP64, 1e-10, False, form, sketch=sk)
        it = st.info()
        res_t, err_t = accuracy(P, st, w, Bt, Xt)
        out["fp64_tight"] = {"compress_tol": 1e-10, "value": nrhs / tt["solve_s"],
                             "setup_s": tt["setup_s"], "rank": it["rank"],
                             "rel_residual": res_t, "rel_err_vs_oracle": err_t}
        del st, Bt, Xt
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
