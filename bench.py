#!/usr/bin/env python
"""Benchmark of the lagged-diffusivity TV deblurring hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one complete tvdeblur_solve of the 512 x 512 anti-reflective
workload (64-shape phantom, 21 x 21 Gaussian PSF sigma 3, 1% noise,
alpha 5e-4, beta 0.05, X_D preconditioner M_D, 15 fixed-point steps, PCG tol
1e-6, at most 100 iterations), FP32-mixed precision, with v already resident
in device memory.  Prints one JSON line: PCG iterations per second over K
timed steps (restore time per step beside it), the roofline of the dominant
kernel (durations from HIP events recorded by the library on its own stream
during the timed steps), the relative error against the FP64 oracle, and the
oracle timed on this host's CPU on a bounded sample of the same workload.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor peak

# Algorithmic HBM bytes per launch of each kernel class, per pixel, in units
# of the element size w (what the kernel must read + write at minimum):
#   band_normal  z, p_old, kappa read; p_new, q written         -> 5
#   row_forward  x, p, q, r, s read; x, r, T1 written           -> 8
#   column       T1, 1/mu read; T2 written                      -> 3
#   row_inverse  T2, s, r read; z written                       -> 4
ALGO_WORDS = {"band_normal": 5, "row_forward": 8, "column": 3, "row_inverse": 4}

WORKLOAD = ("512x512 piecewise-constant phantom (64 rectangles/disks, seed 512), 21x21 Gaussian PSF "
            "sigma 3, 1% noise, anti-reflective BCs, M_D (X_D) DST-I preconditioner, alpha 5e-4, "
            "beta 0.05, 15 fixed-point steps, PCG tol 1e-6, max 100")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="f32_mixed", choices=["f32_mixed", "f64"])
    ap.add_argument("--cpu-steps", type=int, default=15,
                    help="fixed-point steps of the oracle CPU sample (0 = skip the oracle)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (requested --gpus {args.gpus}); the single-GPU "
              "workload is the whole job here. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1011_5964_amd import synth
    from paper_1011_5964_amd.lib import TVDeblur

    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        sys.exit(1)

    p = synth.config("m512")
    n = p.v.shape[0]
    dt = torch.float32 if args.precision == "f32_mixed" else torch.float64
    v = torch.tensor(p.v, dtype=dt, device="cuda")
    h = TVDeblur(n, n, args.precision)
    h.set_psf(p.psf)
    h.set_bc(p.bc)

    def solve():
        return h.solve(v, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    h.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    u = None
    for _ in range(args.steps):
        u, st = solve()
        iters += st["total_inner_iters"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = h.kernel_times()
    h.set_profiling(False)
    elapsed = t1 - t0
    value = iters / elapsed
    ms_per_step = 1e3 * elapsed / args.steps

    # roofline of the dominant kernel class
    w = 4 if args.precision == "f32_mixed" else 8
    N = n * n
    cls = {k: v_ for k, v_ in kt.items() if k in ALGO_WORDS and v_["launches"] > 0}
    dom = max(cls, key=lambda k: cls[k]["total_ms"])
    avg_s = cls[dom]["total_ms"] * 1e-3 / cls[dom]["launches"]
    algo_bytes = ALGO_WORDS[dom] * N * w
    achieved = algo_bytes / avg_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                "avg_launch_us": round(avg_s * 1e6, 3), "algorithmic_bytes_per_launch": algo_bytes}
    kernel_classes = {k: {"launches": v_["launches"], "avg_us": round(1e3 * v_["total_ms"] / v_["launches"], 3),
                          "share_of_step": round(v_["total_ms"] / (1e3 * elapsed), 4)}
                      for k, v_ in kt.items() if v_["launches"] > 0}

    out = {"metric": "512² AR-BC TV restore time (s) & PCG iters/s at ≤1e-5 rel err vs FP64 oracle",
           "value": round(value, 1), "unit": "PCG iters/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
           "restore_time_s": round(ms_per_step / 1e3, 5), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" if args.precision == "f32_mixed" else "f64",
           "precision": args.precision, "data": "synthetic",
           "config": {"workload": WORKLOAD, "n": n, "psf": "gaussian 21x21 sigma 3", "bc": "antireflective",
                      "precond": "x_d", "fixed_point_steps": p.n_outer, "pcg_iters_per_solve": iters // args.steps},
           "roofline": roofline, "kernel_classes": kernel_classes}

    if args.cpu_steps > 0:
        import threadpoolctl

        import oracle as O
        vq = v.double().cpu().numpy()
        k = min(args.cpu_steps, p.n_outer)
        blas = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] + [1])
        c0 = time.perf_counter()
        uo, so = O.fp_solve(vq, p.psf, p.bc, p.alpha, p.beta, k, p.inner_tol, p.max_inner, "x_d")
        c1 = time.perf_counter()
        o_iters = int(sum(so["inner_iters"]))
        out["cpu_baseline"] = {"value": round(o_iters / (c1 - c0), 2), "unit": "PCG iters/s", "cores": blas,
                               "kind": "oracle",
                               "sample": f"first {k} of {p.n_outer} fixed-point steps of the same 512x512 "
                                         f"workload ({o_iters} PCG iterations, {c1 - c0:.1f} s; FFTs and "
                                         f"convolutions single-threaded, matmuls on {blas} BLAS threads)"}
        if k == p.n_outer:
            ug = u.double().cpu().numpy()
        else:
            ug = h.solve(v, p.alpha, p.beta, k, p.inner_tol, p.max_inner, "x_d")[0].double().cpu().numpy()
        out["rel_err_vs_oracle"] = float(np.linalg.norm(ug - uo) / np.linalg.norm(uo))
        out["oracle_fp_steps_compared"] = k
        out["gpu_iters_per_step"] = st["inner_iters"]
        out["oracle_iters_per_step"] = so["inner_iters"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
