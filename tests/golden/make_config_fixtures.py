"""Write the expected results of the full-size workloads with the FP64 oracle.

    python tests/golden/make_config_fixtures.py [case ...]     (default: all)

Each case goes to tests/golden/configs/<case>.npz.  This script imports only
the oracle (oracle/) and the seeded input generator (paper_1011_5964_amd/
synth.py, data only); nothing here comes from the GPU library.  The oracle
runs on the input exactly as a handle of the given precision holds it: the
FP64 cases on v itself, the FP32-mixed cases on v rounded to float32 (round
to nearest even, as torch and the library round it).

Cases (the workloads' parameters are those of synth.config):
  c2_ar_f64, c2_r_f64, c2_ar_f32, c2_r_f32
        256^2, 15x15 Gaussian s=2.5, AR / reflective, X_D, 20 steps;
  c3_gauss_f32, c3_disk_f32
        1024^2, 31x31 Gaussian s=5 / out-of-focus disk r=5, AR, X_D, 20 steps;
  c5_grad_f32
        512^2, 21x21 Gaussian s=3, AR, 15 steps: the forward iterates and the
        FP64 adjoint (vbar, alphabar, betabar) of l = ||u^15 - u_true||^2
        (eq. (fp) differentiated step by step);
  c4_f32
        the 64-image uneven batch, 10 steps per image, X_D.
Stored per case: the restored image(s) (float64 for the FP64 cases, float32
for the FP32-mixed ones, whose 1e-5 bar is far above float32 rounding), the
oracle's PCG iteration counts per step (the GPU replays them where its own
stopping decisions differ) and the fixed-point changes.
"""

import os
import sys
import time
from multiprocessing import Pool

# one BLAS thread per worker process (set before numpy loads its BLAS)
for _var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_var, "1")

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "configs")
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1011_5964_amd import synth  # noqa: E402

VARIANT = "x_d"
C5_ADJ_MAX_INNER = 2000


def held_as(v, prec):
    """The input as a handle of precision prec holds it."""
    return np.asarray(v, dtype=np.float64) if prec == "f64" else np.asarray(v, np.float32).astype(np.float64)


def solve_case(name, prec):
    p = synth.config(name)
    vq = held_as(p.v, prec)
    u, st = O.fp_solve(vq, p.psf, p.bc, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, VARIANT)
    dt = np.float64 if prec == "f64" else np.float32
    return {"u": u.astype(dt), "inner_iters": np.asarray(st["inner_iters"], np.int32),
            "fp_change": np.asarray(st["fp_change"]), "relres": np.asarray(st["relres"])}


def c5_grad():
    p = synth.config("c5")
    vq = held_as(p.v, "f32")
    u, st = O.fp_solve(vq, p.psf, p.bc, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, VARIANT,
                       keep_iterates=True)
    its = st["iterates"]
    vbar, abar, bbar = O.fp_adjoint(p.psf, p.bc, p.alpha, p.beta, its, 2.0 * (its[-1] - p.u_true),
                                    p.inner_tol, C5_ADJ_MAX_INNER, VARIANT)
    return {"u": u.astype(np.float32), "inner_iters": np.asarray(st["inner_iters"], np.int32),
            "vbar": vbar.astype(np.float32), "abar": np.float64(abar), "bbar": np.float64(bbar),
            "adj_max_inner": np.int32(C5_ADJ_MAX_INNER)}


def c4_image(i):
    p = synth.batch_problems(64)[i]
    vq = held_as(p.v, "f32")
    u, st = O.fp_solve(vq, p.psf, p.bc, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, VARIANT)
    return i, u.astype(np.float32), np.asarray(st["inner_iters"], np.int32)


SINGLE = {
    "c2_ar_f64": ("c2_ar", "f64"), "c2_r_f64": ("c2_r", "f64"),
    "c2_ar_f32": ("c2_ar", "f32"), "c2_r_f32": ("c2_r", "f32"),
    "c3_gauss_f32": ("c3_gauss", "f32"), "c3_disk_f32": ("c3_disk", "f32"),
}
ALL = list(SINGLE) + ["c5_grad_f32", "c4_f32"]


def run_single(case):
    t = time.time()
    if case == "c5_grad_f32":
        res = c5_grad()
    else:
        res = solve_case(*SINGLE[case])
    np.savez_compressed(os.path.join(OUT, case + ".npz"), **res)
    print(f"{case}: {time.time() - t:.0f} s, iters {[int(c) for c in res['inner_iters']]}", flush=True)
    return case


def main(cases):
    os.makedirs(OUT, exist_ok=True)
    singles = [c for c in cases if c != "c4_f32"]
    jobs = max(1, min(7, (os.cpu_count() or 2) - 1))
    with Pool(jobs) as pool:
        waiting = [pool.apply_async(run_single, (c,)) for c in singles]
        c4 = [pool.apply_async(c4_image, (i,)) for i in range(64)] if "c4_f32" in cases else []
        for w in waiting:
            w.get()
        if c4:
            res = {}
            iters = np.zeros((64, 10), np.int32)
            for w in c4:
                i, u, it = w.get()
                res[f"u_{i:02d}"] = u
                iters[i, :len(it)] = it
                print(f"c4 image {i} ({u.shape[0]}x{u.shape[1]}) iters {[int(c) for c in it]}", flush=True)
            np.savez_compressed(os.path.join(OUT, "c4_f32.npz"), inner_iters=iters, **res)


if __name__ == "__main__":
    want = sys.argv[1:] or ALL
    bad = [c for c in want if c not in ALL]
    if bad:
        raise SystemExit(f"unknown case(s) {bad}; known: {ALL}")
    main(want)
