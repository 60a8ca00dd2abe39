"""GPU parity of the batching form (tvdeblur_batch_*): many independent
images of different sizes, PSFs and weights solved together, each checked
against the FP64 oracle run on that image alone.

Bars as for single images: FP64 <= 1e-10, FP32-mixed <= 1e-5 relative
2-norm error of each restored image.  Where an image's own stopping
decisions differ from the oracle's at a borderline residual, the batch is
run again replaying the oracle's per-image iteration counts.
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


# ragged images: (ny, nx, psf size, sigma, alpha, beta, seed); several line
# pairs per block and tails in both directions, one square and one with a
# side below a band tile
RAGGED = [
    (45, 38, 7, 1.3, 2e-3, 0.1, 11),
    (32, 32, 5, 1.0, 1e-3, 0.05, 12),
    (64, 48, 9, 1.5, 5e-4, 0.1, 13),
    (24, 40, 3, 0.8, 4e-3, 0.2, 14),
    (57, 57, 11, 2.0, 1e-3, 0.05, 15),
    (33, 70, 7, 1.7, 2e-4, 0.1, 16),
]


def ragged_problems(bc, n_outer=3):
    out = []
    for ny, nx, size, sig, alpha, beta, seed in RAGGED:
        p = synth.small_problem(n=nx, ny=ny, psf_size=size, sigma=sig, bc=bc, alpha=alpha, beta=beta,
                                n_outer=n_outer, seed=seed, shapes=6)
        out.append(p)
    return out


def split_form(transform):
    """'gemm32' / 'gemm64': the product form with that block tile."""
    if transform.startswith("gemm") and transform != "gemm":
        return "gemm", int(transform[4:])
    return transform, 0


def batch_solve(probs, prec, variant="x_d", replay=None, use_graph=True, fp_tol=0.0, batch=None, transform="auto"):
    from paper_1011_5964_amd.lib import TVDeblurBatch
    b = batch or TVDeblurBatch([p.v.shape for p in probs], [p.psf for p in probs], probs[0].bc, prec)
    vs = [dev(p.v, prec) for p in probs]
    form, tile = split_form(transform)
    us, st = b.solve(vs, [p.alpha for p in probs], betas=[p.beta for p in probs], max_outer=probs[0].n_outer,
                     inner_tol=probs[0].inner_tol, max_inner=probs[0].max_inner, precond=variant,
                     fp_tol=fp_tol, use_graph=use_graph, replay=replay, transform=form, gemm_tile=tile)
    if tile:
        assert b.info()["gemm_tile"] == tile
    return [host(u) for u in us], st, b


def oracle_solves(probs, prec, variant="x_d", fp_tol=0.0):
    res = []
    for p in probs:
        vq = host(dev(p.v, prec))
        res.append(O.fp_solve(vq, p.psf, p.bc, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, variant,
                              fp_tol=fp_tol))
    return res


def check_batch(probs, prec, variant="x_d", use_graph=True, transform="auto"):
    print(f"batch of {len(probs)}: {[p.v.shape for p in probs]} {prec} {variant} graph={use_graph} {transform}",
          flush=True)
    ref = oracle_solves(probs, prec, variant)
    ug, sg, b = batch_solve(probs, prec, variant, use_graph=use_graph, transform=transform)
    if transform != "auto":
        assert b.info()["transform"] == split_form(transform)[0]
    errs = [rel2(u, uo) for u, (uo, _) in zip(ug, ref)]
    same = [s["inner_iters"] == so["inner_iters"] for s, (_, so) in zip(sg, ref)]
    for k, (e, s, (_, so)) in enumerate(zip(errs, sg, ref)):
        print(f"  image {k}: err {e:.3e} gpu {s['inner_iters']} oracle {so['inner_iters']}", flush=True)
    if prec == "f32_mixed":
        for e, s, (_, so) in zip(errs, sg, ref):
            assert e <= BAR[prec]
            assert all(abs(a - c) <= max(3, c // 4) for a, c in zip(s["inner_iters"], so["inner_iters"]))
    if all(same):
        assert max(errs) <= BAR[prec]
        return errs, sg, b
    ur, sr, _ = batch_solve(probs, prec, variant, replay=[so["inner_iters"] for _, so in ref], use_graph=use_graph,
                            batch=b, transform=transform)
    rerrs = [rel2(u, uo) for u, (uo, _) in zip(ur, ref)]
    print(f"  replay errs {[f'{e:.2e}' for e in rerrs]}", flush=True)
    for s, (_, so) in zip(sr, ref):
        assert s["inner_iters"] == so["inner_iters"]
    assert max(rerrs) <= BAR[prec]
    if prec == "f64":
        for p, s, (_, so) in zip(probs, sg, ref):
            check_f64_counts(p, variant, host(dev(p.v, prec)), p.n_outer, s["inner_iters"], so["inner_iters"])
    return errs, sg, b


@pytest.mark.parametrize("transform", ["fft", "gemm32", "gemm64"])
@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
@pytest.mark.parametrize("bc", [AR, R])
def test_ragged_batch_matches_oracle(bc, prec, transform):
    """Six images of different shapes, PSF widths, alphas and betas in one
    batch, with either transform implementation; each against the oracle's
    solve of that image."""
    errs, st, b = check_batch(ragged_problems(bc), prec, transform=transform)
    info = b.info()
    print(f"  tuning {info}", flush=True)
    assert info["line_threads"] in (256, 512, 1024)
    assert all(s["outer_steps"] == 3 and s["all_converged"] for s in st)


@pytest.mark.parametrize("transform", ["fft", "gemm"])
@pytest.mark.parametrize("variant", ["x", "d_x"])
def test_batch_other_transform_variants(variant, transform):
    check_batch(ragged_problems(AR), "f64", variant, transform=transform)


@pytest.mark.parametrize("transform", ["fft", "gemm32", "gemm64"])
def test_graph_replay_equals_stream_launches(transform):
    """The graph-captured PCG loop and plain stream launches run the same
    kernels in the same order: bitwise-identical results and counts."""
    probs = ragged_problems(AR)
    ug, sg, b = batch_solve(probs, "f32_mixed", use_graph=True, transform=transform)
    us, ss, _ = batch_solve(probs, "f32_mixed", use_graph=False, batch=b, transform=transform)
    assert b.info()["graph_launches"] > 0
    for a, c, s1, s2 in zip(ug, us, sg, ss):
        assert np.array_equal(a, c)
        assert s1["inner_iters"] == s2["inner_iters"]


def test_repeated_solves_are_deterministic():
    probs = ragged_problems(R)
    u1, s1, b = batch_solve(probs, "f64")
    u2, s2, _ = batch_solve(probs, "f64", batch=b)
    for a, c in zip(u1, u2):
        assert np.array_equal(a, c)
    assert [s["inner_iters"] for s in s1] == [s["inner_iters"] for s in s2]


@pytest.mark.parametrize("transform", ["fft", "gemm"])
def test_fp_tol_stops_each_image_on_its_own(transform):
    """With a fixed-point tolerance each image stops after its own number of
    steps, as the oracle does for that image alone."""
    probs = ragged_problems(AR, n_outer=12)
    fp_tol = 3e-3
    ref = oracle_solves(probs, "f64", fp_tol=fp_tol)
    ug, sg, _ = batch_solve(probs, "f64", fp_tol=fp_tol, transform=transform)
    steps = [s["outer_steps"] for s in sg]
    print(f"steps gpu {steps} oracle {[len(so['inner_iters']) for _, so in ref]}", flush=True)
    assert len(set(steps)) > 1          # the images really stop at different steps
    for u, s, (uo, so) in zip(ug, sg, ref):
        assert s["outer_steps"] == len(so["inner_iters"])
        assert rel2(u, uo) <= BAR["f64"]


def test_batch_of_one_and_identity_psf():
    """A batch of one image with the identity PSF and alpha = 0 returns v
    (exact recovery, Section 1: H = I, no regularisation)."""
    p = synth.small_problem(n=40, ny=36, psf_size=3, sigma=1.0, bc=AR, alpha=0.0, beta=0.1, n_outer=2)
    p.psf = np.zeros((3, 3))
    p.psf[1, 1] = 1.0
    ug, sg, _ = batch_solve([p], "f64")
    assert rel2(ug[0], p.v) <= 1e-12


def test_batch_matches_single_image_path():
    """Each image of a batch takes the same PCG iteration counts as the
    single-image entry point on the same (line-transform) implementation,
    and agrees with it to rounding."""
    from paper_1011_5964_amd.lib import TVDeblur
    probs = ragged_problems(AR)
    ug, sg, _ = batch_solve(probs, "f64", transform="fft")
    for p, u, s in zip(probs, ug, sg):
        h = TVDeblur(*p.v.shape, "f64")
        h.set_psf(p.psf)
        h.set_bc(p.bc)
        h.set_transform("fft")
        u1, s1 = h.solve(dev(p.v, "f64"), p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")
        assert s1["inner_iters"] == s["inner_iters"]
        assert rel2(u, host(u1)) <= 1e-12


def test_batch_errors():
    from paper_1011_5964_amd.lib import TVDeblurBatch, TvdError
    probs = ragged_problems(AR)[:2]
    # non-separable PSF: not supported by the batched path
    with pytest.raises(TvdError) as e:
        TVDeblurBatch([p.v.shape for p in probs], [synth.disk_psf(3), probs[1].psf], AR, "f32_mixed")
    assert e.value.name == "TVD_EINVAL"
    b = TVDeblurBatch([p.v.shape for p in probs], [p.psf for p in probs], AR, "f32_mixed")
    vs = [dev(p.v, "f32_mixed") for p in probs]
    with pytest.raises(TvdError) as e:
        b.solve(vs, [1e-3, 1e-3], precond="diag")
    assert e.value.name == "TVD_EINVAL"
    with pytest.raises(TvdError) as e:
        b.solve(vs, [1e-3, float("nan")])
    assert e.value.name == "TVD_EINVAL"
    # an output aliasing an input: rejected by the library
    with pytest.raises(TvdError) as e:
        b.solve(vs, [1e-3, 1e-3], outs=[vs[0], torch.empty_like(vs[1])])
    assert e.value.name == "TVD_EINVAL"
    # an output of the wrong shape or type: rejected by the binding before any call
    with pytest.raises(ValueError):
        b.solve(vs, [1e-3, 1e-3], outs=[vs[1], torch.empty_like(vs[1])])
    with pytest.raises(ValueError):
        b.solve(vs, [1e-3, 1e-3], outs=[torch.empty_like(vs[0], dtype=torch.float64), torch.empty_like(vs[1])])
    with pytest.raises(TvdError) as e:
        b.solve(vs, [1e-3, 1e-3], max_outer=0)
    assert e.value.name == "TVD_EINVAL"
    # the batch still works after rejected calls
    us, st = b.solve(vs, [p.alpha for p in probs], max_outer=2)
    assert all(s["outer_steps"] == 2 for s in st)


@pytest.mark.slow
def test_c4_full_batch_sampled_against_oracle():
    """The 64-image batching workload (sides 128..512, own Gaussian PSF of
    size 9..21 and sigma U[1,4], alpha log-uniform in [1e-4, 1e-2], beta
    0.05, AR, 10 steps), FP32-mixed with graph replay as timed by the
    benchmark: every image converges, and the oracle solves one image of each
    of the three smallest sizes on its own, each within 1e-5."""
    probs = synth.config("c4")
    print(f"c4: {len(probs)} images, {sum(p.v.size for p in probs)} px", flush=True)
    ug, sg, b = batch_solve(probs, "f32_mixed")
    print(f"tuning {b.info()}", flush=True)
    assert all(s["outer_steps"] == 10 and s["all_converged"] for s in sg)
    # the other implementation on the same batch gives the same images to the bar
    other = "fft" if b.info()["transform"] == "gemm" else "gemm"
    uo_, so_, _ = batch_solve(probs, "f32_mixed", batch=b, transform=other)
    assert all(s["outer_steps"] == 10 and s["all_converged"] for s in so_)
    picked = {}
    for k, p in enumerate(probs):
        if p.v.shape[0] in (128, 192, 256) and p.v.shape[0] not in picked:
            picked[p.v.shape[0]] = k
    for n, k in sorted(picked.items()):
        p = probs[k]
        uo, so = O.fp_solve(host(dev(p.v, "f32_mixed")), p.psf, p.bc, p.alpha, p.beta, p.n_outer, p.inner_tol,
                            p.max_inner, "x_d")
        e = rel2(ug[k], uo)
        e2 = rel2(uo_[k], uo)
        print(f"image {k} ({n}^2, psf {p.psf.shape[0]}, alpha {p.alpha:.2e}): err {e:.3e} ({other}: {e2:.3e}) "
              f"gpu {sg[k]['inner_iters']} oracle {so['inner_iters']}", flush=True)
        assert e <= BAR["f32_mixed"] and e2 <= BAR["f32_mixed"]
