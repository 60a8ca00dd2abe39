#!/usr/bin/env python
"""Benchmark of the lagged-diffusivity TV deblurring hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms all|none] [--cpu-steps S]

Headline (one step = one complete tvdeblur_solve, input already in HBM): the
512 x 512 anti-reflective workload (64-shape phantom, 21 x 21 Gaussian PSF
sigma 3, 1% noise, alpha 5e-4, beta 0.05, X_D preconditioner, 15 fixed-point
steps, PCG tol 1e-6, at most 100 iterations) in FP32-mixed precision.
`value` = the median restore time (s) of the K timed solves; PCG iterations
per second of whole solves, the same rate counting only the iterations the
FP64 oracle needs, and the inner-loop-only rate sit beside it.  Rooflines are
HBM rooflines: the algorithmic bytes of a launch (the words per pixel each
stage of the method must move, ALGO_WORDS) over its duration, taken from a
burst of back-to-back launches between HIP events right after the timed
solves (tvdeblur_time_kernel); `roofline` is the class with the largest share
of the loop, `iteration_roofline` the whole PCG iteration (13 words per
pixel).  Which class dominates comes from one more, untimed solve in which one
launch in PROFILE_EVERY of each class carries a start/stop event pair on its
own dispatch.

Forms (default --forms all): the plain FP64 path on the same workload, the
batching form on the 64-image ragged workload against 64 single-image solves,
the differentiation form (forward + adjoint against forward), each with its
speedup over the plain GPU FP64 path and its error against the FP64 oracle,
the alpha sweep of the headline image under both boundary conditions (one
batched solve per BC: restoration error per alpha, the best alpha), the
reblurring system, and the other single-image workloads (64^2, 256^2 under
both BCs and precisions, 1024^2 with both PSFs) with their rooflines and
errors against the oracle's stored results.  The oracle itself is timed on
this host's cores on a bounded sample (cpu_baseline).
"""

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor peak
MFMA_PEAK_TFLOPS = {"f32_mixed": 157.3, "f64": 78.6}   # dense matrix-core peaks
# FP32 products of the 64 x 64 tiles run as six bf16 products of split
# operands: their ceiling in FP32 flops is the dense bf16 peak over six
SPLIT_BF16_PEAK_TFLOPS = round(2500.0 / 6, 1)

# Algorithmic HBM words per pixel of each HBM-bound PCG-loop kernel (what that
# stage of the method must read + write; w bytes per word):
#   band_normal  p_old, z, kappa read; p_new, q written            -> 5
#   row_forward  x, r, p, q, s read; x, r, T1 written              -> 8
#   column       T1, 1/mu read; T2 written                         -> 3
#   row_inverse  T2, s, r read; z written                          -> 4
#   update       x, r, p, q, s read; x, r, t written               -> 8
#   x_pass       z read; w written                                 -> 2
#   transform_gemm  one product of the product form: operand and basis
#                   matrix read, result written                    -> 3
ALGO_WORDS = {"band_normal": 5, "row_forward": 8, "column": 3, "row_inverse": 4, "update": 8, "x_pass": 2,
              "transform_gemm": 3}
# The products also run as dense n x n x n products on the matrix cores
# (2 n^3 flop per launch); that rate is reported beside the HBM roofline.
MFMA_CLASSES = ("transform_gemm",)
BURST_CLASSES = ("band_normal", "column", "update", "transform_gemm", "x_pass")   # tvdeblur_time_kernel classes
BURST_REPS = 100
# Per PCG iteration the method moves x, r, p (R/W), q, z (W/R), kappa, s,
# 1/mu (R): 13 words per pixel, plus 4 for the two transform intermediates.
ITER_WORDS = 13
ITER_WORDS_WITH_TRANSPOSES = 17

# HBM traffic per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE
# counters on the 512x512 FP32-mixed workload, scaled by the same counters on
# a plain copy kernel of known size (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0), for
# the kernel source whose SHA-256 prefix is recorded; ignored (null) once the
# kernel source has changed since.  Source: profiles/m512_f32_traffic.md.
TRAFFIC = {"source_sha256": "bc786f8fdecec389",
           "bytes_per_launch": {"transform_gemm": 8281342, "band_normal": 8908638, "update": 8136657}}

# The per-class breakdown samples 1 launch in PROFILE_EVERY of each class
# (a timed launch delays the next by ~9 us), in a solve outside the timing.
PROFILE_EVERY = 32

WORKLOAD = ("512x512 piecewise-constant phantom (64 rectangles/disks, seed 512), 21x21 Gaussian PSF "
            "sigma 3, 1% noise, anti-reflective BCs, X_D (M_D) DST-I preconditioner, alpha 5e-4, "
            "beta 0.05, 15 fixed-point steps, PCG tol 1e-6, max 100")


def kernel_source_sha():
    with open(os.path.join(ROOT, "paper_1011_5964_amd", "csrc", "tvd_kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def rel2(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def time_calls(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    times, out = [], None
    for _ in range(steps):
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return times, out


def hbm_roofline(kind, avg_s, N, w):
    """One kernel class against the HBM roofline: the algorithmic bytes of
    one launch (ALGO_WORDS words per pixel) over its measured duration."""
    algo = ALGO_WORDS[kind] * N * w
    return {"bound": "hbm", "achieved": round(algo / avg_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(algo / avg_s / 1e9 / HBM_PEAK_GBS, 4), "kernel": kind,
            "avg_launch_us": round(avg_s * 1e6, 3), "algorithmic_bytes_per_launch": algo}


def measure(args, p, prec, steps, warmup, transform="auto", breakdown=True):
    """Times `steps` whole solves of problem p on one handle; returns a dict
    of figures and the last restored image (host, float64).

    Kernel durations for the rooflines come from a burst of back-to-back
    launches of each PCG-loop class between two HIP events on the solver's
    stream, with the parameters of the timed solves (tvdeblur_time_kernel);
    the per-class launch counts (which class dominates) from one more,
    untimed solve in which one launch in PROFILE_EVERY of each class carries
    a start/stop event pair on its own dispatch."""
    import torch
    from paper_1011_5964_amd.lib import TVDeblur
    ny, nx = p.v.shape
    dt = torch.float32 if prec == "f32_mixed" else torch.float64
    v = torch.tensor(p.v, dtype=dt, device="cuda")
    h = TVDeblur(ny, nx, prec)
    h.set_psf(p.psf)
    h.set_bc(p.bc)
    h.set_transform(transform)
    stats = []

    def solve():
        u, st = h.solve(v, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")
        stats.append(st)
        return u

    for _ in range(warmup):
        solve()
    torch.cuda.synchronize()
    stats.clear()
    times, u = time_calls(solve, steps, 0)
    timed_stats = list(stats)
    kt = {}
    if breakdown:
        h.set_profiling(PROFILE_EVERY)
        solve()
        torch.cuda.synchronize()
        kt = h.kernel_times()
        h.set_profiling(False)
    stats[:] = timed_stats
    iters = sum(s["total_inner_iters"] for s in stats)
    inner = sum(s["time_inner_s"] for s in stats)
    total = sum(times)
    w = 4 if prec == "f32_mixed" else 8
    N = ny * nx
    res = {"restore_time_s": statistics.median(times), "ms_per_step": 1e3 * total / steps,
           "pcg_iters_per_s": iters / total, "pcg_iters_per_s_inner_loop": iters / inner,
           "pcg_iters_per_solve": iters // steps, "iters_per_step": stats[-1]["inner_iters"],
           "setup_share": sum(s["time_setup_s"] for s in stats) / total}
    # whole-iteration roofline: the method's 13 words per pixel per iteration
    per_iter_s = inner / iters
    res["iteration_roofline"] = {
        "bound": "hbm", "per_iteration_us": round(per_iter_s * 1e6, 3),
        "algorithmic_bytes_per_iteration": ITER_WORDS * N * w,
        "achieved": round(ITER_WORDS * N * w / per_iter_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(ITER_WORDS * N * w / per_iter_s / 1e9 / HBM_PEAK_GBS, 4),
        "frac_with_transposes": round(ITER_WORDS_WITH_TRANSPOSES * N * w / per_iter_s / 1e9 / HBM_PEAK_GBS, 4)}
    res["transform"] = h.transform()
    if res["transform"] == "gemm":
        res["gemm_tile"] = h.gemm_tile()
    loop = {k: x for k, x in kt.items() if k in ALGO_WORDS and x["launches"] > 0}
    burst = {}
    for k in BURST_CLASSES:
        if k in loop:
            burst[k] = h.time_kernel(k, reps=BURST_REPS)
    if burst:
        dom = max(burst, key=lambda k: burst[k] * loop[k]["launches"])
        rl = hbm_roofline(dom, burst[dom] * 1e-6, N, w)
        traffic = None
        if TRAFFIC["source_sha256"] == kernel_source_sha() and prec == "f32_mixed" and (ny, nx) == (512, 512):
            traffic = TRAFFIC["bytes_per_launch"].get(dom)
        rl["traffic"] = traffic
        rl["launches_sampled"] = loop[dom]["launches"]
        rl["duration_source"] = f"burst of {BURST_REPS} launches between HIP events"
        if dom in MFMA_CLASSES:
            # the same launches as dense products on the matrix cores: 2 n^3 flop
            flops = 2.0 * nx * ny * (nx if dom == "transform_gemm" else 1)
            ach = flops / (burst[dom] * 1e-6) / 1e12
            split = prec == "f32_mixed" and res.get("gemm_tile") == 64
            peak = SPLIT_BF16_PEAK_TFLOPS if split else MFMA_PEAK_TFLOPS[prec]
            rl["mfma_view"] = {"algorithmic_flops_per_launch": flops, "achieved_tflops": round(ach, 2),
                               "peak_tflops": peak, "frac": round(ach / peak, 4),
                               "instructions": "bf16, six per FP32 product (split operands)" if split
                               else ("fp32" if prec == "f32_mixed" else "fp64")}
        res["roofline"] = rl
        res["class_rooflines"] = {k: hbm_roofline(k, burst[k] * 1e-6, N, w) for k in burst}
    res["kernel_classes"] = {k: {"launches_sampled": x["launches"],
                                 "avg_us_dispatch_events": round(1e3 * x["total_ms"] / x["launches"], 3),
                                 **({"avg_us_burst": round(burst[k], 3)} if k in burst else {})}
                             for k, x in kt.items() if x["launches"] > 0}
    h.close()
    return res, u.double().cpu().numpy()


def headline(args, p, prec):
    return measure(args, p, prec, args.steps, args.warmup, args.transform)


def fixture(name):
    """The oracle's stored result on a workload (written by
    tests/golden/make_config_fixtures.py from the oracle alone), or None."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "configs", name + ".npz")
    return np.load(path) if os.path.exists(path) else None


CONFIG_RUNS = [("c1", "f64", None), ("c1", "f32_mixed", None),
               ("c2_ar", "f64", "c2_ar_f64"), ("c2_ar", "f32_mixed", "c2_ar_f32"),
               ("c2_r", "f64", "c2_r_f64"), ("c2_r", "f32_mixed", "c2_r_f32"),
               ("c3_gauss", "f32_mixed", "c3_gauss_f32"), ("c3_disk", "f32_mixed", "c3_disk_f32")]


def configs_form(args):
    """The small, mid-size and large single-image workloads (64^2 FP64 and
    FP32-mixed; 256^2 under both BCs and precisions; 1024^2 FP32-mixed with
    the 31x31 Gaussian and the out-of-focus disk): restore time, PCG
    iterations per second, the transform form the handle picked, the HBM
    roofline of each PCG-loop kernel class and of the whole iteration, and
    the relative error against the FP64 oracle's result on the same input
    (stored fixture; the 64^2 one is solved here)."""
    import numpy as np
    from paper_1011_5964_amd import synth
    out = {}
    for name, prec, fx_name in CONFIG_RUNS:
        p = synth.config(name)
        print(f"[bench] config {name} {prec}", file=sys.stderr, flush=True)
        steps = 3 if p.v.shape[0] >= 1024 else 5
        r, u = measure(args, p, prec, steps, 1)
        keep = {k: r[k] for k in ("restore_time_s", "pcg_iters_per_s", "pcg_iters_per_solve", "iters_per_step",
                                  "setup_share", "transform", "iteration_roofline")}
        for k in ("roofline", "class_rooflines"):
            if k in r:
                keep[k] = r[k]
        fx = fixture(fx_name) if fx_name else None
        if fx is not None:
            keep["rel_err_vs_oracle"] = rel2(u, fx["u"].astype(np.float64))
            keep["oracle_iters_per_step"] = [int(c) for c in fx["inner_iters"]]
        elif name == "c1":
            import oracle as O
            vq = p.v.astype(np.float32).astype(np.float64) if prec == "f32_mixed" else p.v
            uo, so = O.fp_solve(vq, p.psf, p.bc, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")
            keep["rel_err_vs_oracle"] = rel2(u, uo)
            keep["oracle_iters_per_step"] = so["inner_iters"]
        out[f"{name}_{prec}"] = keep
    return out


def batch_form(args, p_ref_f64_restore_s):
    """64-image ragged batch (FP32-mixed) against 64 single-image solves of
    the same images (FP32-mixed and FP64; skipped with --no-sequential)."""
    import torch
    from paper_1011_5964_amd import synth
    from paper_1011_5964_amd.lib import TVDeblur, TVDeblurBatch
    probs = synth.config("c4")
    px = sum(p.v.size for p in probs)
    t0 = time.perf_counter()
    b = TVDeblurBatch([p.v.shape for p in probs], [p.psf for p in probs], probs[0].bc, "f32_mixed")
    create_s = time.perf_counter() - t0
    vs = [torch.tensor(p.v, dtype=torch.float32, device="cuda") for p in probs]
    alphas = [p.alpha for p in probs]
    last = {}

    def run():
        # launches issued one by one: graph replay measured 0.5% slower here
        us, st = b.solve(vs, alphas, beta=0.05, max_outer=probs[0].n_outer, inner_tol=1e-6, max_inner=100,
                         precond="x_d", use_graph=False)
        last["u"], last["st"] = us, st
        return us

    times, _ = time_calls(run, max(2, args.steps // 2), 1)
    t_batch = statistics.median(times)
    info = b.info()
    res = {"workload": "64 images, sides U{128,192,256,384,512}, Gaussian PSF odd size 9..21 sigma U[1,4], "
                       "alpha log-uniform [1e-4,1e-2], beta 0.05, AR, X_D, 10 fixed-point steps, FP32-mixed",
           "pixels": px, "batch_solve_s": t_batch, "images_per_s": len(probs) / t_batch,
           "megapixels_per_s": px / t_batch / 1e6, "create_s": create_s,
           "all_converged": all(s["all_converged"] for s in last["st"]),
           "pcg_iters_total": int(sum(s["total_inner_iters"] for s in last["st"])),
           "tuning": {k: info[k] for k in ("line_threads", "tables_in_lds", "from_cache", "candidates",
                                           "candidate_us", "gemm_us", "gemm64_us", "gemm_tile",
                                           "transform")},
           "setup_share": info["time_setup_s"] / t_batch}
    # the batch's PCG loops against the HBM roofline: every image's 13 words
    # per pixel per iteration it ran, over the batch's inner-loop time
    algo = sum(ITER_WORDS * 4 * p.v.size * s["total_inner_iters"] for p, s in zip(probs, last["st"]))
    res["iteration_roofline"] = {"bound": "hbm", "algorithmic_bytes": algo, "inner_loop_s": info["time_inner_s"],
                                 "achieved": round(algo / info["time_inner_s"] / 1e9, 1), "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s",
                                 "frac": round(algo / info["time_inner_s"] / 1e9 / HBM_PEAK_GBS, 4)}
    # 64 single-image solves, one after another, both precisions
    for prec, dt in () if args.no_sequential else (("f32_mixed", torch.float32), ("f64", torch.float64)):
        hs = []
        for p in probs:
            h = TVDeblur(*p.v.shape, prec)
            h.set_psf(p.psf)
            h.set_bc(p.bc)
            hs.append((h, torch.tensor(p.v, dtype=dt, device="cuda"), p))

        def seq():
            for h, v, p in hs:
                h.solve(v, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")

        st, _ = time_calls(seq, 1, 1)
        res[f"sequential_{prec}_s"] = st[0]
        for h, _, _ in hs:
            h.close()
    if not args.no_sequential:
        res["speedup_vs_64_single_f32_mixed"] = res["sequential_f32_mixed_s"] / t_batch
        res["speedup_vs_64_single_f64"] = res["sequential_f64_s"] / t_batch
    b.close()
    return res, probs, last


SWEEP_ALPHAS = [5e-4 * 2.0 ** k for k in range(-5, 5)]   # 1.6e-5 .. 8e-3, the headline alpha included


def sweep_form(args):
    """Alpha sweep (one batched solve over SWEEP_ALPHAS for the headline image)
    under both boundary conditions: the restoration error against the true
    scene per alpha, the best alpha and its error, and the time against the
    same restorations as one-by-one single-image solves (FP32-mixed)."""
    import numpy as np
    import torch
    from paper_1011_5964_amd import synth
    from paper_1011_5964_amd.lib import AlphaSweep, TVDeblur
    p = synth.config("m512")
    v = torch.tensor(p.v, dtype=torch.float32, device="cuda")
    res = {"workload": "the headline 512x512 image, alpha = 5e-4 * 2^k for k = -5..4 (10 values), beta 0.05, "
                       "15 fixed-point steps, X_D, FP32-mixed, one batched solve per boundary condition",
           "alphas": SWEEP_ALPHAS}
    slot = {}
    for bc in ("antireflective", "reflective"):
        sw = AlphaSweep(p.v.shape, p.psf, bc, SWEEP_ALPHAS, "f32_mixed")
        last = {}

        def run():
            us, st = sw.solve(v, beta=p.beta, max_outer=p.n_outer, inner_tol=p.inner_tol, max_inner=p.max_inner)
            last["u"], last["st"] = us, st
            return us

        times, _ = time_calls(run, max(2, args.steps // 2), 1)
        t_sweep = statistics.median(times)
        rre = [rel2(u.double().cpu().numpy(), p.u_true) for u in last["u"]]
        k = int(np.argmin(rre))
        h = TVDeblur(*p.v.shape, "f32_mixed")
        h.set_psf(p.psf)
        h.set_bc(bc)
        h.solve(v, SWEEP_ALPHAS[0], p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for a in SWEEP_ALPHAS:
            h.solve(v, a, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - s0
        h.close()
        res[bc] = {"sweep_s": t_sweep, "restorations_per_s": len(SWEEP_ALPHAS) / t_sweep,
                   "sequential_single_s": t_seq, "speedup_vs_single_solves": t_seq / t_sweep,
                   "transform": sw.info()["transform"],
                   "pcg_iters": [int(st["total_inner_iters"]) for st in last["st"]],
                   "restoration_error": [round(x, 6) for x in rre],
                   "alpha_opt": SWEEP_ALPHAS[k], "restoration_error_at_alpha_opt": round(rre[k], 6)}
        if bc == "antireflective":
            slot["u"] = last["u"][SWEEP_ALPHAS.index(5e-4)].double().cpu().numpy()
        sw.close()
    return res, slot


def reblur_form(args, pcg_iters_per_solve):
    """The reblurring system eq. (fpp) on the headline 512^2 workload with
    PBiCGstab and P_D, FP32-mixed and FP64: restore time, BiCGstab
    iterations (two operator products and two preconditioner solves each)
    and the restoration error against the true scene; the first three steps
    are kept for the comparison with the oracle."""
    import torch
    from paper_1011_5964_amd import synth
    from paper_1011_5964_amd.lib import TVDeblur
    p = synth.config("m512")
    res = {"workload": "the headline 512x512 image (21x21 Gaussian sigma 3, AR, alpha 5e-4, beta 0.05, 15 "
                       "fixed-point steps, PBiCGstab tol 1e-6) on the reblurring system (H'H + alpha L) u = H'v "
                       "with P_D"}
    slot = {}
    for prec in ("f32_mixed", "f64"):
        dt = torch.float32 if prec == "f32_mixed" else torch.float64
        v = torch.tensor(p.v, dtype=dt, device="cuda")
        h = TVDeblur(*p.v.shape, prec)
        h.set_psf(p.psf)
        h.set_bc(p.bc)
        last = {}

        def run():
            u, st = h.solve_reblur(v, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "p_d")
            last["u"], last["st"] = u, st
            return u

        times, _ = time_calls(run, max(2, args.steps // 2), 1)
        t = statistics.median(times)
        st = last["st"]
        its = int(st["total_inner_iters"])
        res[prec] = {"restore_time_s": t, "bicgstab_iters_per_solve": its,
                     "bicgstab_iters_per_s": its / t,
                     "per_iteration_us": 1e6 * st["time_inner_s"] / max(its, 1),
                     "setup_share": st["time_setup_s"] / max(st["time_total_s"], 1e-12),
                     "iters_per_step": st["inner_iters"][:st["outer_steps"]],
                     "all_converged": bool(st["all_converged"]),
                     "operator_products_per_solve": 2 * its,
                     "restoration_error": rel2(last["u"].double().cpu().numpy(), p.u_true)}
        # per-class launch durations from one more, untimed solve with sampled kernel timing
        h.set_profiling(PROFILE_EVERY)
        run()
        torch.cuda.synchronize()
        kt = h.kernel_times()
        h.set_profiling(False)
        res[prec]["kernel_classes"] = {k: {"launches_sampled": v["launches"],
                                           "avg_us": 1e3 * v["total_ms"] / v["launches"]}
                                       for k, v in kt.items() if v["launches"] > 0}
        if prec == "f32_mixed":
            u3, s3 = h.solve_reblur(v, p.alpha, p.beta, 3, p.inner_tol, p.max_inner, "p_d")
            slot["u3"] = u3.double().cpu().numpy()
            slot["iters3"] = s3["inner_iters"][:3]
        h.close()
    if pcg_iters_per_solve:
        res["normal_equations_pcg_iters_per_solve"] = pcg_iters_per_solve
    return res, slot


TABLE_ALPHAS = [1.0, 1e-1, 1e-2, 1e-3, 1e-4]


def tables_form(args):
    """The paper's 2D iteration table on a synthetic image: for each alpha the
    number of fixed-point steps N (stop at a relative change below 1e-4, at
    most 100 steps, beta = 0.01) and the average Krylov iterations per step,
    for PCG on the normal equations under reflective BCs (I, D_R, R_D) and
    anti-reflective BCs (I, D_M, M_D), and PBiCGstab on the reblurring system
    (I, D_P, P_D); FP64.  '*' marks a column where a step hit max_inner."""
    import torch
    from paper_1011_5964_amd import synth
    from paper_1011_5964_amd.lib import TVDeblur
    res = {"workload": "256x256 piecewise-constant phantom (32 shapes, seed of c2), 15x15 Gaussian PSF sigma 2.5, "
                       "1% noise, beta 0.01, FP stop ||u^k - u^{k-1}|| / ||u^k|| < 1e-4, at most 100 FP steps, "
                       "inner tol 1e-6, max_inner 2000, FP64",
           "alphas": TABLE_ALPHAS}
    columns = [("pcg_reflective", "reflective", "solve", ("none", "d_x", "x_d")),
               ("pcg_antireflective", "antireflective", "solve", ("none", "d_x", "x_d")),
               ("pbicgstab_reblur", "antireflective", "solve_reblur", ("none", "d_p", "p_d"))]
    t0 = time.perf_counter()
    for name, bc, fn, precs in columns:
        p = synth.config("c2_r" if bc == "reflective" else "c2_ar")
        v = torch.tensor(p.v, dtype=torch.float64, device="cuda")
        h = TVDeblur(*p.v.shape, "f64")
        h.set_psf(p.psf)
        h.set_bc(bc)
        rows = []
        for a in TABLE_ALPHAS:
            row = {}
            for pc in precs:
                try:
                    _, st = getattr(h, fn)(v, a, 0.01, 100, 1e-6, 2000, pc, fp_tol=1e-4)
                    n = st["outer_steps"]
                    row[pc] = {"N": n, "avg_iters": round(st["total_inner_iters"] / max(n, 1), 1),
                               "converged": bool(st["all_converged"])}
                except Exception as e:  # a breakdown is reported, not fatal
                    row[pc] = {"error": str(e)[:80]}
            rows.append(row)
        res[name] = rows
        h.close()
    res["wall_s"] = time.perf_counter() - t0
    return res


def diff_form(args, f64_restore_s):
    """Forward (with checkpoints) and forward + adjoint on the 512^2
    differentiation workload, FP32-mixed."""
    import torch
    from paper_1011_5964_amd import synth
    from paper_1011_5964_amd.autograd import tv_restore
    from paper_1011_5964_amd.lib import TVDeblur
    p = synth.config("c5")
    n = p.v.shape[0]
    h = TVDeblur(n, n, "f32_mixed")
    h.set_psf(p.psf)
    h.set_bc(p.bc)
    ut = torch.tensor(p.u_true, dtype=torch.float32, device="cuda")
    v0 = torch.tensor(p.v, dtype=torch.float32, device="cuda")

    def fwd():
        with torch.no_grad():
            return tv_restore(v0, p.alpha, p.beta, handle=h, n_outer=p.n_outer)

    def fwd_bwd():
        v = v0.clone().requires_grad_(True)
        a = torch.tensor(p.alpha, dtype=torch.float64, device="cuda", requires_grad=True)
        u = tv_restore(v, a, p.beta, handle=h, n_outer=p.n_outer)
        loss = ((u - ut) ** 2).sum()
        loss.backward()
        return v.grad, a.grad

    tf, _ = time_calls(fwd, 3, 1)
    tb, (gv, ga) = time_calls(fwd_bwd, 3, 1)
    h.close()
    return {"workload": "512x512, 21x21 Gaussian sigma 3, AR, alpha 5e-4, beta 0.05, 15 steps, FP32-mixed, "
                        "loss ||u - u_true||^2, grads w.r.t. v and alpha",
            "forward_s": statistics.median(tf), "forward_backward_s": statistics.median(tb),
            "backward_over_forward": statistics.median(tb) / statistics.median(tf) - 1.0,
            "grad_alpha": float(ga), "grad_v_norm": float(gv.double().norm()),
            "speedup_fwd_bwd_vs_plain_f64_forward": f64_restore_s / statistics.median(tb)}


SIGNAL_ALPHAS = [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6]
SIGNAL_BETAS = [1e-3, 1e-2, 1.0]
SIGNAL_NS = [101, 203, 407, 815, 1631]
SIGNAL_VARIANTS = ["none", "diag", "x", "d_x", "x_d"]


def signals_form(args):
    """The paper's 1D experiments (Section 5.1, Tables 1-2 and the n sweep) on
    synthetic signals, each table one batched launch: n = 203, the out-of-focus
    PSF of eq. (of) with m(n) = round(n/8), 1% noise, FP stop at a relative
    change below 1e-3, PCG tol 1e-6; both BCs x I, D, X, D_X, X_D; the alpha
    sweep at beta 0.1, the beta sweep at alpha 1e-3, and the n sweep at
    alpha 1e-3, beta 0.1.  Reports N and the average PCG iterations per step
    (the trends compare with the paper's; its own signal is not available)
    and the time of each launch; FP64."""
    import numpy as np
    from paper_1011_5964_amd import synth
    from paper_1011_5964_amd.lib import TVDeblurSignals
    res = {"workload": "synthetic piecewise constant / linear signals, out-of-focus PSF m(n) = round(n/8), 1% noise, "
                       "FP stop 1e-3, PCG tol 1e-6, max 1000 (n sweep 4000) iterations, FP64, one launch per table"}

    def run_table(rows, max_inner, system="normal"):
        names = SIGNAL_VARIANTS if system == "normal" else ["none", "diag", "p", "d_p", "p_d"]
        probs = [pr for pr, _ in rows for _ in names]
        variants = [v for _ in rows for v in names]
        sb = TVDeblurSignals([q.v.shape[1] for q in probs], [q.psf for q in probs], [q.bc for q in probs],
                             reblur=[system == "reblur"] * len(probs))
        v = sb.pack([q.v[0] for q in probs])
        alphas = [q.alpha for q in probs]
        betas = [q.beta for q in probs]

        def go():
            return sb.solve(v, alphas, betas=betas, precond=variants, max_outer=100, fp_tol=1e-3, inner_tol=1e-6,
                            max_inner=max_inner, system=system, allow_breakdown=True)

        times, (u, st) = time_calls(go, 3, 1)
        table = []
        for r, (_, label) in enumerate(rows):
            cell = st[5 * r:5 * r + 5]
            table.append({"row": label, "N": [c["outer_steps"] for c in cell],
                          **{vn: round(float(np.mean(c["inner_iters"])), 1) for vn, c in zip(names, cell)},
                          "converged": all(c["all_converged"] for c in cell),
                          "breakdown": [vn for vn, c in zip(names, cell) if c["breakdown"]]})
        sb.close()
        return {"signals": len(probs), "launch_s": statistics.median(times),
                "krylov_iters": int(sum(c["total_inner_iters"] for c in st)), "rows": table}

    for bc, system in (("reflective", "normal"), ("antireflective", "normal"), ("antireflective", "reblur")):
        tag = f"{bc}_pcg" if system == "normal" else "antireflective_reblur_pbicgstab"
        res[f"table1_alpha_{tag}"] = run_table(
            [(synth.signal_problem(203, bc, alpha=a, beta=0.1), f"alpha {a:g}") for a in SIGNAL_ALPHAS], 1000, system)
        res[f"table2_beta_{tag}"] = run_table(
            [(synth.signal_problem(203, bc, alpha=1e-3, beta=b), f"beta {b:g}") for b in SIGNAL_BETAS], 1000, system)
        res[f"n_sweep_{tag}"] = run_table(
            [(synth.signal_problem(n, bc, alpha=1e-3, beta=0.1), f"n {n}") for n in SIGNAL_NS], 4000, system)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--forms", default="all",
                    help="comma list of forms measured beside the headline: f64, batch, diff, sweep, reblur, "
                         "configs, signals ('all' = these seven), tables (2D iteration tables, only when named); "
                         "or 'none'")
    ap.add_argument("--cpu-steps", type=int, default=15,
                    help="fixed-point steps of the oracle CPU sample (0 = skip the oracle)")
    ap.add_argument("--transform", choices=("auto", "fft", "gemm"), default="auto",
                    help="preconditioner transforms of the headline and plain FP64 solves: timed choice (default), "
                         "line transforms, or products on the matrix cores")
    ap.add_argument("--workload", default="m512",
                    help="headline workload (profiling runs): m512 (the metric's), c1, c2_ar, c2_r, c3_gauss, "
                         "c3_disk, c5; any other than m512 makes the line a profiling record, not the metric")
    ap.add_argument("--precision", choices=("f32_mixed", "f64"), default="f32_mixed",
                    help="precision of the headline solves (profiling runs)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batch form without its 64 single-image comparison solves (profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain elementwise copy (y = -x, float32) of this many MiB three times: "
                         "the reference kernel that scales hardware traffic counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (requested --gpus {args.gpus}): this build has no multi-GPU "
              "path; the single-GPU workload is the whole job. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1011_5964_amd import synth

    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        sys.exit(1)

    p = synth.config(args.workload)
    n = p.v.shape[0]
    print(f"[bench] headline {args.precision} {args.workload} {n}x{n}: {args.warmup} warm-up + {args.steps} "
          f"timed solves", file=sys.stderr, flush=True)
    r32, u32 = measure(args, p, args.precision, args.steps, args.warmup, args.transform)
    out = {"metric": "512² AR-BC TV restore time (s) & PCG iters/s at ≤1e-5 rel err vs FP64 oracle",
           "value": round(r32["restore_time_s"], 6), "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(r32["ms_per_step"], 3),
           "restore_time_s": round(r32["restore_time_s"], 6),
           "pcg_iters_per_s": round(r32["pcg_iters_per_s"], 1), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" if args.precision == "f32_mixed" else "f64",
           "precision": ("f32_mixed (FP64 dots, scalars, stopping test)" if args.precision == "f32_mixed"
                         else "f64"),
           "data": "synthetic",
           "config": {"workload": WORKLOAD if args.workload == "m512" else f"profiling record: {args.workload}",
                      "n": n, "psf": f"{p.psf.shape[0]}x{p.psf.shape[1]}", "bc": p.bc,
                      "precond": "x_d", "fixed_point_steps": p.n_outer,
                      "pcg_iters_per_solve": r32["pcg_iters_per_solve"]},
           "roofline": r32["roofline"], "iteration_roofline": r32["iteration_roofline"],
           "transform": r32["transform"],
           "pcg_iters_per_s_inner_loop": round(r32["pcg_iters_per_s_inner_loop"], 1),
           "setup_share": round(r32["setup_share"], 4), "kernel_classes": r32["kernel_classes"]}

    sel = {"all": {"f64", "batch", "diff", "sweep", "reblur", "configs", "signals"}, "none": set()}.get(
        args.forms, set(args.forms.split(",")))
    forms = {}
    u64 = None
    probs = None
    r64_time = None
    if "f64" in sel or "batch" in sel or "diff" in sel:
        # the speedups of every form are against the plain FP64 path
        print("[bench] plain FP64 path", file=sys.stderr, flush=True)
        r64, u64 = headline(args, p, "f64")
        r64_time = r64["restore_time_s"]
        forms["plain_f64"] = {k: r64[k] for k in ("restore_time_s", "pcg_iters_per_s", "pcg_iters_per_s_inner_loop",
                                                  "pcg_iters_per_solve", "setup_share", "transform", "roofline")}
        forms["plain_f64"]["iteration_roofline"] = r64["iteration_roofline"]
        forms["f32_mixed"] = {"restore_time_s": r32["restore_time_s"],
                              "speedup_vs_plain_f64": r64_time / r32["restore_time_s"]}
    if "batch" in sel:
        print("[bench] batching form (64 ragged images)", file=sys.stderr, flush=True)
        rb, probs, last = batch_form(args, r64_time)
        forms["batch"] = rb
    if "diff" in sel:
        print("[bench] differentiation form", file=sys.stderr, flush=True)
        forms["differentiation"] = diff_form(args, r64_time)
    sweep_slot = None
    if "sweep" in sel:
        print("[bench] alpha sweep (both boundary conditions)", file=sys.stderr, flush=True)
        forms["alpha_sweep"], sweep_slot = sweep_form(args)
    if "tables" in sel:
        print("[bench] iteration tables (normal equations and reblurring system)", file=sys.stderr, flush=True)
        forms["tables"] = tables_form(args)
    if "signals" in sel:
        print("[bench] 1D signal tables (one launch per table)", file=sys.stderr, flush=True)
        forms["signals"] = signals_form(args)
    if "configs" in sel:
        forms["configs"] = configs_form(args)
    reblur_slot = None
    if "reblur" in sel:
        print("[bench] reblurring system (PBiCGstab)", file=sys.stderr, flush=True)
        forms["reblur"], reblur_slot = reblur_form(args, r32.get("pcg_iters_per_solve"))

    if args.cpu_steps > 0:
        import scipy.fft
        import threadpoolctl

        import oracle as O
        cores = os.cpu_count() or 1
        k = min(args.cpu_steps, p.n_outer)
        print(f"[bench] oracle on {cores} host cores: {k} fixed-point steps", file=sys.stderr, flush=True)
        with threadpoolctl.threadpool_limits(cores), scipy.fft.set_workers(cores):
            c0 = time.perf_counter()
            uo, so = O.fp_solve(p.v, p.psf, p.bc, p.alpha, p.beta, k, p.inner_tol, p.max_inner, "x_d")
            c1 = time.perf_counter()
        o_iters = int(sum(so["inner_iters"]))
        k1 = min(2, k)
        with threadpoolctl.threadpool_limits(1), scipy.fft.set_workers(1):
            d0 = time.perf_counter()
            _, s1 = O.fp_solve(p.v, p.psf, p.bc, p.alpha, p.beta, k1, p.inner_tol, p.max_inner, "x_d")
            d1 = time.perf_counter()
        out["cpu_baseline"] = {"value": round((c1 - c0) * p.n_outer / k, 3), "unit": "s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"first {k} of {p.n_outer} fixed-point steps of the same 512x512 workload "
                                         f"({o_iters} PCG iterations in {c1 - c0:.1f} s, BLAS and scipy.fft on "
                                         f"{cores} threads), restore time scaled to {p.n_outer} steps",
                               "pcg_iters_per_s": round(o_iters / (c1 - c0), 2),
                               "one_core": {"value": round(sum(s1["inner_iters"]) / (d1 - d0), 2),
                                            "sample": f"first {k1} fixed-point steps on 1 thread "
                                                      f"({sum(s1['inner_iters'])} PCG iterations, "
                                                      f"{d1 - d0:.1f} s)"}}
        if k == p.n_outer:
            out["rel_err_vs_oracle"] = rel2(u32, uo)
            out["gpu_iters_per_step"] = r32["iters_per_step"]
            out["oracle_iters_per_step"] = so["inner_iters"]
            # the rate counting only the iterations the FP64 oracle needs, so
            # that extra iterations caused by FP32 vectors earn nothing
            out["pcg_iters_per_s_oracle_budget"] = round(o_iters / r32["restore_time_s"], 1)
            if u64 is not None:
                forms["plain_f64"]["rel_err_vs_oracle"] = rel2(u64, uo)
            forms.setdefault("f32_mixed", {})["rel_err_vs_oracle"] = out["rel_err_vs_oracle"]
            if sweep_slot is not None:
                # the sweep's alpha = 5e-4 slot is the headline problem
                forms["alpha_sweep"]["rel_err_vs_oracle_alpha_5e-4"] = rel2(sweep_slot["u"], uo)
        if reblur_slot is not None:
            # reblurring system: the first three steps against the oracle's
            from oracle import reblur as RB
            vq = p.v.astype(np.float32).astype(np.float64)
            with threadpoolctl.threadpool_limits(cores), scipy.fft.set_workers(cores):
                ur, sr = RB.fp_solve_reblur(vq, p.psf, p.alpha, p.beta, 3, p.inner_tol, p.max_inner, "p_d")
            forms["reblur"]["first_3_steps_vs_oracle"] = {
                "rel_err": rel2(reblur_slot["u3"], ur), "gpu_iters": reblur_slot["iters3"],
                "oracle_iters": sr["inner_iters"]}
    if probs is not None:
        # per-image error of the batch against the oracle's stored solve of each image
        fx = fixture("c4_f32")
        if fx is not None:
            errs = [rel2(u.double().cpu().numpy(), fx[f"u_{i:02d}"].astype(np.float64))
                    for i, u in enumerate(last["u"])]
            forms["batch"]["rel_err_vs_oracle"] = {"max": max(errs), "median": statistics.median(errs),
                                                   "images": len(errs)}
    if forms:
        out["forms"] = forms
    if args.copy_calibration > 0:
        x = torch.ones(args.copy_calibration * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.neg(x, out=y)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"kernel": "torch.neg float32", "bytes_read": x.numel() * 4,
                                   "bytes_written": y.numel() * 4, "launches": 3}
    out["kernel_source_sha256"] = kernel_source_sha()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
