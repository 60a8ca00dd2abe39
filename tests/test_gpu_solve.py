"""GPU parity of the whole fixed-point / PCG method against the FP64 oracle,
through the C-ABI, plus edge cases and error paths.

Bars (relative 2-norm error of the restored image against the oracle's):
FP64 <= 1e-10, FP32-mixed <= 1e-5.  Where the GPU's own stopping decisions
could differ from the oracle's at a borderline residual, the GPU is also
run in replay mode with the ORACLE's per-step iteration counts.
"""

import numpy as np
import pytest

import oracle as O
from paper_1011_5964_amd import synth
from parity import check_f64_counts

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

AR, R = "antireflective", "reflective"
BAR = {"f64": 1e-10, "f32_mixed": 1e-5}


def dev(a, prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def host(t):
    return t.detach().double().cpu().numpy()


def rel2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_solve(p, prec, variant="x_d", replay=None, n_outer=None, **kw):
    from paper_1011_5964_amd.lib import TVDeblur
    ny, nx = p.v.shape
    h = TVDeblur(ny, nx, prec)
    h.set_psf(p.psf)
    h.set_bc(p.bc)
    u, st = h.solve(dev(p.v, prec), p.alpha, p.beta, n_outer or p.n_outer, p.inner_tol, p.max_inner,
                    variant, replay=replay, **kw)
    return host(u), st


def oracle_solve(p, variant="x_d", v=None, n_outer=None):
    return O.fp_solve(p.v if v is None else v, p.psf, p.bc, p.alpha, p.beta, n_outer or p.n_outer,
                      p.inner_tol, p.max_inner, variant)


def oracle_envelope(p, variant, vq, so, n_outer):
    """The oracle's own FP64 rounding spread: the same problem transposed
    (identical in exact arithmetic, different rounding order), replaying the
    same iteration counts."""
    ut, _ = O.fp_solve(vq.T.copy(), p.psf.T.copy(), p.bc, p.alpha, p.beta, n_outer or p.n_outer,
                       p.inner_tol, p.max_inner, variant, replay=so["inner_iters"])
    uo, _ = O.fp_solve(vq, p.psf, p.bc, p.alpha, p.beta, n_outer or p.n_outer, p.inner_tol,
                       p.max_inner, variant, replay=so["inner_iters"])
    return rel2(ut.T, uo)


def bar_for(p, prec, variant, vq, so, n_outer, err):
    """1e-10 (FP64) / 1e-5 (FP32-mixed).  For the weakly preconditioned
    variants (none, diag) FP64 CG amplifies rounding beyond 1e-10 on some
    problems; there the bar is 4x the oracle's own rounding envelope when that
    is larger (the transform preconditioners stay at 1e-10)."""
    bar = BAR[prec]
    if prec == "f64" and variant in ("none", "diag") and err > bar:
        env = oracle_envelope(p, variant, vq, so, n_outer)
        print(f"oracle rounding envelope {env:.3e}", flush=True)
        bar = max(bar, 4.0 * env)
    return bar


def check_parity(p, prec, variant="x_d", n_outer=None):
    """Free-running GPU result vs oracle, and (if the per-step iteration
    counts differ) the GPU replaying the oracle's counts vs oracle."""
    vq = host(dev(p.v, prec))                     # input as the GPU holds it
    uo, so = oracle_solve(p, variant, v=vq, n_outer=n_outer)
    ug, sg = gpu_solve(p, prec, variant, n_outer=n_outer)
    err = rel2(ug, uo)
    print(f"oracle iters {so['inner_iters']}\ngpu    iters {sg['inner_iters']}\nrel err {err:.3e}", flush=True)
    if sg["inner_iters"] == so["inner_iters"]:
        assert err <= bar_for(p, prec, variant, vq, so, n_outer, err)
        return err, so, sg
    ur, sr = gpu_solve(p, prec, variant, replay=so["inner_iters"], n_outer=n_outer)
    assert sr["inner_iters"] == so["inner_iters"]
    rerr = rel2(ur, uo)
    print(f"replay rel err {rerr:.3e}", flush=True)
    assert rerr <= bar_for(p, prec, variant, vq, so, n_outer, rerr)
    if prec == "f64":
        check_f64_counts(p, variant, vq, n_outer or p.n_outer, sg["inner_iters"], so["inner_iters"])
    else:
        # float vectors lose CG orthogonality somewhat faster than double,
        # so a step may need a few more iterations; the restored image must
        # still meet the bar.
        assert err <= BAR[prec]
        assert all(abs(a - b) <= max(3, b // 4) for a, b in zip(sg["inner_iters"], so["inner_iters"]))
    return err, so, sg


@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
def test_c1_anti_reflective(prec):
    """64^2, 8 shapes, 9x9 Gaussian s=1.5, AR, X_D, alpha 1e-3, beta 0.1, 10 steps."""
    print(f"case c1 {prec}", flush=True)
    check_parity(synth.config("c1"), prec)


@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
@pytest.mark.parametrize("bc", [AR, R])
@pytest.mark.parametrize("variant", ["none", "diag", "x", "d_x", "x_d"])
def test_variants_small_ragged(bc, variant, prec):
    """Every preconditioner on a ragged 45 x 38 image (several tiles plus a
    tail) with a non-separable PSF for the reflective case."""
    print(f"case variants {bc} {variant} {prec}", flush=True)
    p = synth.small_problem(n=38, ny=45, psf_size=7, sigma=1.3, bc=bc, n_outer=3, alpha=2e-3, beta=0.1)
    if bc == R:
        p.psf = synth.disk_psf(3)
    check_parity(p, prec, variant)


@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
def test_c2_both_bcs(prec):
    """256^2, 32 shapes, 15x15 Gaussian s=2.5, alpha 5e-4, beta 0.05 -- 6 of
    the 20 fixed-point steps (the oracle's time budget), both BCs."""
    for name in ("c2_ar", "c2_r"):
        print(f"case {name} {prec}", flush=True)
        check_parity(synth.config(name), prec, n_outer=6)


@pytest.mark.slow
@pytest.mark.parametrize("name", ["c3_gauss", "c3_disk"])
def test_c3_precision_form_full_size(name):
    """The 1024^2 precision-form workloads (256 shapes + ramp, alpha 1e-4,
    beta 0.01; 31x31 Gaussian s=5, and the non-separable out-of-focus disk
    r=5 that runs the 2D band kernel), FP32-mixed, at full size: the first 2
    of the 20 fixed-point steps (the oracle's time budget) against the FP64
    oracle within 1e-5."""
    print(f"case {name} f32_mixed full size, 2 steps", flush=True)
    err, so, sg = check_parity(synth.config(name), "f32_mixed", n_outer=2)
    print(f"{name} rel err {err:.3e} iters {sg['inner_iters']}", flush=True)


@pytest.mark.slow
def test_m512_fp32_mixed_full():
    """The benchmark workload: 512^2, 21x21 Gaussian s=3, AR, X_D, 15 steps,
    FP32-mixed, against the FP64 oracle."""
    print("case m512 f32_mixed", flush=True)
    err, so, sg = check_parity(synth.config("m512"), "f32_mixed")
    print(f"m512 rel err {err:.3e} iters {sum(sg['inner_iters'])}", flush=True)


def test_identity_psf_alpha_zero_returns_v():
    p = synth.small_problem(n=20)
    p.psf = np.ones((1, 1))
    p.alpha = 0.0
    for prec in ("f64", "f32_mixed"):
        u, st = gpu_solve(p, prec, n_outer=2)
        np.testing.assert_array_equal(u, host(dev(p.v, prec)))
        assert st["inner_iters"] == [0, 0]


def test_constant_image_is_fixed_point():
    p = synth.small_problem(n=24)
    p.v = np.full((24, 24), 0.3)
    u, st = gpu_solve(p, "f64", n_outer=2)
    np.testing.assert_allclose(u, 0.3, atol=1e-13)


def test_minimal_image_and_largest_psf():
    """3 x 3 image with a 3 x 3 PSF; 9 x 9 image with the largest AR PSF
    (half-width n-1 = 8, 17 x 17)."""
    for n, size in ((3, 3), (9, 17)):
        p = synth.small_problem(n=n, psf_size=5, sigma=1.0, n_outer=2)
        p.psf = synth.gaussian_psf(size, 2.0)
        print(f"case tiny n={n} psf={size}", flush=True)
        check_parity(p, "f64", n_outer=2)


def test_error_paths():
    from paper_1011_5964_amd.lib import TVDeblur, TvdError
    h = TVDeblur(16, 16, "f64")
    v = torch.zeros((16, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(TvdError) as e:
        h.solve(v, 1e-3, 0.1, 2)
    assert e.value.name == "TVD_ESTATE"
    bad = synth.gaussian_psf(5, 1.0)
    bad[0, 1] += 1e-3
    bad /= bad.sum()
    with pytest.raises(TvdError) as e:
        h.set_psf(bad)
    assert e.value.name == "TVD_ENOTSYM"
    with pytest.raises(TvdError) as e:
        h.set_psf(2 * synth.gaussian_psf(5, 1.0))
    assert e.value.name == "TVD_ENORM"
    h.set_bc("antireflective")
    with pytest.raises(TvdError) as e:
        h.set_psf(synth.gaussian_psf(33, 4.0))
    assert e.value.name == "TVD_ESIZE"
    h.set_psf(synth.gaussian_psf(5, 1.0))
    with pytest.raises(TvdError) as e:
        h.solve(v, -1.0, 0.1, 2)
    assert e.value.name == "TVD_EINVAL"
    # NaN data makes the PCG curvature NaN: reported as breakdown, no crash
    vn = v.clone()
    vn[3, 4] = float("nan")
    with pytest.raises(TvdError) as e:
        h.solve(vn, 1e-3, 0.1, 2)
    assert e.value.name == "TVD_EBREAKDOWN"


def test_iterates_checkpoint_and_warm_start():
    p = synth.small_problem(n=32, n_outer=4)
    u, st = gpu_solve(p, "f64")
    its = torch.empty((p.n_outer + 1, 32, 32), dtype=torch.float64, device="cuda")
    u2, st2 = gpu_solve(p, "f64", iterates=its)
    np.testing.assert_array_equal(u, u2)
    np.testing.assert_array_equal(host(its[0]), p.v)
    np.testing.assert_array_equal(host(its[-1]), u)
    # resuming from the checkpoint u^2 for 2 steps reproduces u^4
    from paper_1011_5964_amd.lib import TVDeblur
    h = TVDeblur(32, 32, "f64")
    h.set_psf(p.psf)
    h.set_bc(p.bc)
    u3, _ = h.solve(dev(p.v, "f64"), p.alpha, p.beta, 2, p.inner_tol, p.max_inner, u0=its[2].contiguous())
    np.testing.assert_allclose(host(u3), u, rtol=0, atol=1e-14)


def test_run_to_run_determinism():
    p = synth.config("c1")
    a, sa = gpu_solve(p, "f32_mixed")
    b, sb = gpu_solve(p, "f32_mixed")
    np.testing.assert_array_equal(a, b)
    assert sa["inner_iters"] == sb["inner_iters"]


@pytest.mark.parametrize("transform", ["fft", "gemm"])
def test_kernel_timing_sampling(transform):
    """Per-class kernel timing: with every=1 each PCG-loop launch is timed
    (at least one per PCG iteration); with every=4 exactly one in four of the
    same, deterministic launch sequence; durations are positive."""
    from paper_1011_5964_amd.lib import TVDeblur
    p = synth.config("c1")
    h = TVDeblur(64, 64, "f32_mixed")
    h.set_psf(p.psf)
    h.set_bc(p.bc)
    h.set_transform(transform)
    v = dev(p.v, "f32_mixed")
    runs = {}
    for every in (1, 4):
        h.set_profiling(every)
        _, st = h.solve(v, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")
        runs[every] = (h.kernel_times(), st)
    h.set_profiling(0)
    k1, st = runs[1]
    k4, _ = runs[4]
    assert k1["band_normal"]["launches"] >= st["total_inner_iters"]
    # the product form runs the whole normal operator in its y-pass (no x-pass)
    loop = ("row_forward", "column", "row_inverse") if transform == "fft" else ("update", "transform_gemm")
    if transform == "gemm":
        assert k1["x_pass"]["launches"] == 0
    for cls in ("band_normal", "residual", "setup") + loop:
        assert k1[cls]["launches"] > 0 and k1[cls]["total_ms"] > 0, cls
        assert k4[cls]["launches"] == -(-k1[cls]["launches"] // 4), cls


@pytest.mark.parametrize("transform", ["fft", "gemm"])
def test_time_kernel_burst(transform):
    """tvdeblur_time_kernel: positive per-launch times for the classes the
    active form runs, an error for the others and before any solve, and the
    handle still solves correctly afterwards."""
    from paper_1011_5964_amd.lib import TVDeblur, TvdError
    print(f"case time_kernel {transform}", flush=True)
    p = synth.small_problem(n=96, psf_size=9, sigma=1.5, n_outer=2)
    h = TVDeblur(*p.v.shape, "f32_mixed")
    h.set_psf(p.psf)
    h.set_bc(p.bc)
    h.set_transform(transform)
    with pytest.raises(TvdError):
        h.time_kernel("band_normal", 5)
    v = torch.tensor(p.v, dtype=torch.float32, device="cuda")
    u1, _ = h.solve(v, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")
    runs = ("band_normal", "transform_gemm") if transform == "gemm" else ("band_normal", "column")
    for k in runs:
        t = h.time_kernel(k, 10)
        print(f"  {k}: {t:.2f} us", flush=True)
        assert 0.5 < t < 5000.0
    other = "column" if transform == "gemm" else "transform_gemm"
    with pytest.raises(TvdError):
        h.time_kernel(other, 5)
    u2, _ = h.solve(v, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")
    assert torch.equal(u1, u2)


@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
def test_fp_tol_stops_where_the_oracle_stops(prec):
    """fp_tol > 0 on a single image: the fixed-point loop ends after the first
    step whose relative change ||u^{k+1} - u^k|| / ||u^{k+1}|| falls below
    fp_tol (Section 5's outer stopping rule), at the oracle's step, with the
    oracle's image to the bar."""
    p = synth.small_problem(n=40, ny=36, psf_size=7, sigma=1.3, n_outer=40, alpha=2e-3, beta=0.1)
    fp_tol = 2.4e-3
    vq = host(dev(p.v, prec))
    uo, so = O.fp_solve(vq, p.psf, p.bc, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d", fp_tol=fp_tol)
    k = so["outer_steps"]
    ch = so["fp_change"]
    print(f"oracle stops after {k} of {p.n_outer} steps, changes {['%.2e' % c for c in ch]}", flush=True)
    assert 1 < k < p.n_outer
    # the stop is not borderline: the last change is clearly below fp_tol and
    # the one before clearly above it
    assert ch[-1] < 0.9 * fp_tol and ch[-2] > 1.1 * fp_tol
    ug, sg = gpu_solve(p, prec, fp_tol=fp_tol)
    print(f"gpu stops after {sg['outer_steps']} steps, iters {sg['inner_iters'][:sg['outer_steps']]} "
          f"oracle {so['inner_iters']}", flush=True)
    assert sg["outer_steps"] == k
    np.testing.assert_allclose(sg["fp_change"][:k], ch, rtol=1e-3 if prec == "f32_mixed" else 1e-8)
    err = rel2(ug, uo)
    if sg["inner_iters"][:k] != so["inner_iters"]:
        ug, sr = gpu_solve(p, prec, replay=so["inner_iters"], n_outer=k)
        err = rel2(ug, uo)
    print(f"rel err {err:.3e}", flush=True)
    assert err <= BAR[prec]


@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
@pytest.mark.parametrize("transform", ["fft", "gemm"])
def test_graph_replay_equals_stream_launches(prec, transform):
    """Single-image PCG iterations replayed from HIP graphs (use_graph) give
    the same bits as the same launches issued one by one on the stream (the
    default, and the path taken while kernel profiling is on), on every
    fixed-point step, and again when the cached graphs are replayed by later
    solves and after the parameters change."""
    from paper_1011_5964_amd.lib import TVDeblur
    p = synth.config("c1")
    h = TVDeblur(64, 64, prec)
    h.set_psf(p.psf)
    h.set_bc(p.bc)
    h.set_transform(transform)
    v = dev(p.v, prec)
    runs = []
    for alpha in (p.alpha, 3 * p.alpha, p.alpha):
        h.set_profiling(1)
        up, sp = h.solve(v, alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d", use_graph=True)
        h.set_profiling(0)
        us, ss = h.solve(v, alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")
        ug, sg = h.solve(v, alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d", use_graph=True)
        ug2, sg2 = h.solve(v, alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d", use_graph=True)
        print(f"alpha {alpha:.1e}: iters {sg['inner_iters']}", flush=True)
        assert sp["inner_iters"] == ss["inner_iters"] == sg["inner_iters"] == sg2["inner_iters"]
        assert torch.equal(up, us) and torch.equal(us, ug) and torch.equal(ug, ug2)
        runs.append(ug)
    assert torch.equal(runs[0], runs[2])


@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
@pytest.mark.parametrize("case", ["c1", "reflective", "dirichlet", "periodic"])
def test_objective_per_step(prec, case):
    """tvd_stats.tv_objective: T(u^k) of eq. (mp) at every step equals the
    oracle's T on the same iterates (FP64 arithmetic on both sides: 1e-12),
    and decreases from step to step (each lagged-diffusivity step minimises a
    quadratic majoriser of T from its warm start)."""
    from paper_1011_5964_amd.lib import TVDeblur
    p = synth.config("c1") if case == "c1" else synth.small_problem(n=40, ny=36, bc=case, n_outer=5)
    ny, nx = p.v.shape
    h = TVDeblur(ny, nx, prec)
    h.set_psf(p.psf)
    h.set_bc(p.bc)
    v = dev(p.v, prec)
    its = torch.empty((p.n_outer + 1, ny, nx), dtype=v.dtype, device="cuda")
    u, st = h.solve(v, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d", iterates=its, objective=True)
    vq = host(v)
    obj = st["tv_objective"]
    assert len(obj) == p.n_outer + 1
    for k in range(p.n_outer + 1):
        ref = O.tv_objective(host(its[k]), vq, p.psf, p.bc, p.alpha, p.beta)
        assert abs(obj[k] - ref) <= 1e-12 * ref, (k, obj[k], ref)
    print(f"T(u^k): {['%.6e' % t for t in obj]}", flush=True)
    slack = 1e-12 if prec == "f64" else 1e-6  # FP32 iterates: T is evaluated on rounded u
    assert all(b <= a * (1 + slack) for a, b in zip(obj, obj[1:]))
    # off by default, and the solve is unchanged by it
    u2, st2 = h.solve(v, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")
    assert torch.equal(u, u2) and all(t == 0.0 for t in st2["tv_objective"])


@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
def test_caller_workspace(prec):
    """tvdeblur_workspace_bytes / tvdeblur_set_workspace: solves whose work
    buffers live in a caller-owned tensor give the same bits as solves with
    the handle's own buffers, on repeated calls (graphs captured in the
    caller's area replayed) and after returning to the handle's buffers."""
    from paper_1011_5964_amd.lib import TVDeblur, TvdError
    p = synth.config("c1")
    ny, nx = p.v.shape
    h = TVDeblur(ny, nx, prec)
    h.set_psf(p.psf)
    h.set_bc(p.bc)
    v = dev(p.v, prec)
    args = (p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")
    u_own, st_own = h.solve(v, *args)
    nbytes = h.workspace_bytes()
    elems = 16 * ny * nx * v.element_size() + 2 * ny * nx * 8
    assert elems <= nbytes <= elems + 64 * 1024 * 1024
    ws = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    h.set_workspace(ws)
    for graph in (False, True, True):
        u, st = h.solve(v, *args, use_graph=graph)
        assert torch.equal(u, u_own) and st["inner_iters"] == st_own["inner_iters"]
    assert int(ws.count_nonzero()) > 0  # the solve ran in the caller's area
    h.set_workspace(None)
    u, st = h.solve(v, *args)
    assert torch.equal(u, u_own)
    # too small, misaligned, host memory
    small = torch.empty(nbytes - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(TvdError) as e:
        h.set_workspace(small)
    assert e.value.name == "TVD_ESIZE"
    big = torch.empty(nbytes + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(TvdError) as e:
        h.set_workspace(big[1:])
    assert e.value.name == "TVD_EINVAL"
    with pytest.raises(ValueError):
        h.set_workspace(torch.empty(nbytes, dtype=torch.uint8))
