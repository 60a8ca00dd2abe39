"""GPU parity of the two implementations of the preconditioner's 2D
transforms (Section 3.2): line transforms on the library's FFT in LDS, and
dense products with the n x n basis matrix on the matrix cores.  Both are
checked against the FP64 oracle, as single operator applications and as
whole restorations.

Bars: the preconditioner solve to 1e-12 (FP64) / 1e-5 (FP32-mixed) relative
(max-norm); restorations to 1e-10 / 1e-5 relative 2-norm, with the oracle's
iteration counts replayed where a borderline stopping decision differs.
"""

import numpy as np
import pytest

import oracle as O
from paper_1011_5964_amd import synth
from parity import check_f64_counts

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

AR, R = "antireflective", "reflective"
OP_BAR = {"f64": 1e-12, "f32_mixed": 1e-5}
BAR = {"f64": 1e-10, "f32_mixed": 1e-5}


def dev(a, prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def host(t):
    return t.detach().double().cpu().numpy()


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def handle(shape, psf, bc, prec, transform):
    """transform: 'fft', 'auto', 'gemm' (timed tile), or 'gemm32' / 'gemm64'
    (products with that block tile)."""
    from paper_1011_5964_amd.lib import TVDeblur
    h = TVDeblur(shape[0], shape[1], prec)
    h.set_psf(psf)
    h.set_bc(bc)
    if transform.startswith("gemm") and transform != "gemm":
        h.set_gemm_tile(int(transform[4:]))
        h.set_transform("gemm")
        assert h.gemm_tile() == int(transform[4:])
    else:
        h.set_transform(transform)
    return h


def form(transform):
    return "gemm" if transform.startswith("gemm") else transform


@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
@pytest.mark.parametrize("transform", ["fft", "gemm32", "gemm64"])
@pytest.mark.parametrize("bc", [AR, R])
@pytest.mark.parametrize("variant", ["x", "d_x", "x_d"])
@pytest.mark.parametrize("shape", [(64, 64), (37, 50), (130, 70), (33, 300), (200, 136), (24, 40)])
def test_precond_forms_match_oracle(shape, variant, bc, transform, prec):
    """z = P^{-1} r for both transform implementations on square, ragged and
    elongated images (several 32 x 32 product tiles plus tails in every
    direction; (24, 40): one K slice, so the second K group of the
    single-image 64 x 64 products reads only zeros)."""
    print(f"case precond {shape} {variant} {bc} {transform} {prec}", flush=True)
    rng = np.random.default_rng(11)
    psf = synth.gaussian_psf(7, 1.2)
    p = synth.small_problem(n=max(shape), psf_size=7, sigma=1.2, bc=bc)
    uk = p.v[:shape[0], :shape[1]] + 0.01 * rng.standard_normal(shape)
    alpha, beta = 3e-3, 0.07
    h = handle(shape, psf, bc, prec, transform)
    h.setup(dev(uk, prec), alpha, beta, variant)
    assert h.transform() == form(transform)
    ukq = host(dev(uk, prec))
    ref = O.precond_setup(O.kappa(ukq, beta), alpha, O.psf_symbol_eigenvalues(psf, *shape, bc), bc, variant)
    r = rng.standard_normal(shape)
    z = host(h.precond(dev(r, prec)))
    err = relmax(z, O.precond_apply(host(dev(r, prec)), ref, bc))
    print(f"  rel err {err:.2e}", flush=True)
    assert err < OP_BAR[prec]


def test_auto_choice_is_one_of_the_two():
    h = handle((96, 80), synth.gaussian_psf(5, 1.0), AR, "f32_mixed", "auto")
    assert h.transform() in ("fft", "gemm")


def restore_parity(p, transform, variant="x_d", prec="f32_mixed"):
    vq = host(dev(p.v, prec))
    uo, so = O.fp_solve(vq, p.psf, p.bc, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, variant)
    h = handle(p.v.shape, p.psf, p.bc, prec, transform)
    assert h.transform() == form(transform)
    v = dev(p.v, prec)
    u, st = h.solve(v, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, variant)
    err = rel2(host(u), uo)
    print(f"  {transform} {prec}: gpu {st['inner_iters']} oracle {so['inner_iters']} err {err:.2e}", flush=True)
    if prec == "f64":
        check_f64_counts(p, variant, vq, p.n_outer, st["inner_iters"], so["inner_iters"])
    else:
        assert err <= BAR[prec]
        assert all(abs(a - b) <= max(3, b // 4) for a, b in zip(st["inner_iters"], so["inner_iters"]))
    if st["inner_iters"] != so["inner_iters"]:
        ur, sr = h.solve(v, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, variant, replay=so["inner_iters"])
        assert sr["inner_iters"] == so["inner_iters"]
        err = rel2(host(ur), uo)
    assert err <= BAR[prec]
    return st


@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
@pytest.mark.parametrize("transform", ["fft", "gemm32", "gemm64"])
@pytest.mark.parametrize("variant", ["x", "d_x", "x_d"])
@pytest.mark.parametrize("bc", [AR, R])
def test_restoration_both_forms_small_ragged(bc, variant, transform, prec):
    print(f"case restore {bc} {variant} {transform} {prec}", flush=True)
    p = synth.small_problem(n=38, ny=45, psf_size=7, sigma=1.3, bc=bc, n_outer=3, alpha=2e-3, beta=0.1)
    restore_parity(p, transform, variant, prec)


@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
@pytest.mark.parametrize("transform", ["fft", "gemm32", "gemm64"])
def test_restoration_both_forms_c1(transform, prec):
    print(f"case c1 {transform} {prec}", flush=True)
    restore_parity(synth.config("c1"), transform, prec=prec)


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
def test_restoration_product_form_512(prec):
    """The 512^2 anti-reflective workload (15 steps) with the product form
    and the tile the build-time timing picks."""
    print(f"case m512 gemm {prec}", flush=True)
    restore_parity(synth.config("m512"), "gemm", prec=prec)


def test_restoration_product_form_512_tile64():
    """The 512^2 workload with 64 x 64 product tiles forced (FP32-mixed)."""
    print("case m512 gemm64 f32_mixed", flush=True)
    restore_parity(synth.config("m512"), "gemm64", prec="f32_mixed")


def separable_psf(py, px, sy, sx):
    """py x px quadrantally symmetric Gaussian with its own width per axis."""
    gy = np.exp(-np.arange(-(py // 2), py // 2 + 1) ** 2 / (2.0 * sy * sy))
    gx = np.exp(-np.arange(-(px // 2), px // 2 + 1) ** 2 / (2.0 * sx * sx))
    h = np.outer(gy, gx)
    return h / h.sum()


# Product-form restorations at sizes whose y-pass tiles include interior
# tiles, edge tiles and ragged tails, with band half-widths from 2 to the
# tile halo's limit of 32 (PSF 1x1: the stencil's unit halo only; 21x21: 20;
# 9x17 / 33x5: unequal halos per axis).
FULL_Y_CASES = {
    "gauss21_60x200": ((60, 200), lambda: synth.gaussian_psf(21, 3.0)),
    "rect9x17_97x180": ((97, 180), lambda: separable_psf(9, 17, 1.5, 2.5)),
    "rect33x5_140x77": ((140, 77), lambda: separable_psf(33, 5, 4.0, 1.0)),
    "delta_70x130": ((70, 130), lambda: np.ones((1, 1))),
}


@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
@pytest.mark.parametrize("bc", [AR, R])
@pytest.mark.parametrize("case", sorted(FULL_Y_CASES))
def test_restoration_product_form_whole_operator_ypass(case, bc, prec):
    print(f"case full-y {case} {bc} {prec}", flush=True)
    shape, mk = FULL_Y_CASES[case]
    psf = mk()
    side = max(shape) + psf.shape[0] + psf.shape[1]
    p = synth.make_problem(case, side, 10, psf, bc, 2e-3, 0.1, 3, 0.01, 5)
    p.v = np.ascontiguousarray(p.v[:shape[0], :shape[1]])
    restore_parity(p, "gemm", "x_d", prec)
