"""GPU parity of each operator of the hot path against the FP64 oracle,
called through the C-ABI (libtvdeblur.so).

Tolerances: FP64 handles agree with the oracle to 1e-12 relative (max-norm
over the image); FP32-mixed handles to 2e-6 relative for the linear
operators (float rounding of sums of <= ~500 terms) and 1e-5 for the
preconditioner solve.
"""

import numpy as np
import pytest

import oracle as O
from paper_1011_5964_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

AR, R = "antireflective", "reflective"
TOL = {"f64": 1e-12, "f32_mixed": 2e-6}


def dev(a, prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def host(t):
    return t.detach().double().cpu().numpy()


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def make(shape, psf, bc, prec):
    from paper_1011_5964_amd.lib import TVDeblur
    h = TVDeblur(shape[0], shape[1], prec)
    h.set_psf(psf)
    h.set_bc(bc)
    return h


def nonsep_psf(my, mx, seed):
    rng = np.random.default_rng(seed)
    q = rng.random((my + 1, mx + 1)) + 0.05
    h = np.zeros((2 * my + 1, 2 * mx + 1))
    for a in range(-my, my + 1):
        for b in range(-mx, mx + 1):
            h[a + my, b + mx] = q[abs(a), abs(b)]
    return h / h.sum()


PSFS = {
    "gauss9": synth.gaussian_psf(9, 1.5),
    "disk3": synth.disk_psf(3),
    "rect5x3": nonsep_psf(2, 1, 3),
}
SHAPES = [(64, 64), (37, 50), (130, 70)]


@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
@pytest.mark.parametrize("bc", [AR, R])
@pytest.mark.parametrize("psf", sorted(PSFS))
@pytest.mark.parametrize("shape", SHAPES)
def test_blur_and_adjoint(shape, psf, bc, prec):
    print(f"case blur {shape} {psf} {bc} {prec}", flush=True)
    rng = np.random.default_rng(hash((shape, psf, bc)) % 2**32)
    x = rng.standard_normal(shape)
    h = make(shape, PSFS[psf], bc, prec)
    y = host(h.blur(dev(x, prec)))
    assert relerr(y, O.blur(x, PSFS[psf], bc)) < TOL[prec]
    yt = host(h.blur_adjoint(dev(x, prec)))
    assert relerr(yt, O.blur_adjoint(x, PSFS[psf], bc)) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
@pytest.mark.parametrize("bc", [AR, R])
@pytest.mark.parametrize("variant", ["none", "diag", "x", "d_x", "x_d"])
@pytest.mark.parametrize("shape,psf", [((64, 64), "gauss9"), ((37, 50), "disk3"), ((130, 70), "rect5x3")])
def test_setup_normal_and_precond(shape, psf, bc, variant, prec):
    print(f"case precond {shape} {psf} {bc} {variant} {prec}", flush=True)
    rng = np.random.default_rng(7)
    p = synth.small_problem(n=max(shape), psf_size=5, sigma=1.0, bc=bc)
    uk = p.v[:shape[0], :shape[1]] + 0.01 * rng.standard_normal(shape)
    alpha, beta = 3e-3, 0.07
    h = make(shape, PSFS[psf], bc, prec)
    h.setup(dev(uk, prec), alpha, beta, variant)
    ukq = host(dev(uk, prec))                     # the iterate as the GPU stores it
    kap = O.kappa(ukq, beta)
    lam = O.psf_symbol_eigenvalues(PSFS[psf], shape[0], shape[1], bc)
    ref = O.precond_setup(kap, alpha, lam, bc, variant)
    np.testing.assert_allclose(host(h.export("kappa")), kap, rtol=1e-13)
    np.testing.assert_allclose(host(h.export("lambda_h")), lam, rtol=1e-12, atol=1e-14)
    if "mu" in ref:
        assert relerr(host(h.export("mu")), ref["mu"]) < 1e-11
    if variant in ("d_x", "x_d"):
        assert relerr(host(h.export("s")), ref["s"]) < (1e-14 if prec == "f64" else 1e-7)
    x = rng.standard_normal(shape)
    q = host(h.normal(dev(x, prec)))
    assert relerr(q, O.normal_apply(host(dev(x, prec)), PSFS[psf], bc, kap, alpha)) < TOL[prec]
    r = rng.standard_normal(shape)
    z = host(h.precond(dev(r, prec)))
    zref = O.precond_apply(host(dev(r, prec)), ref, bc)
    assert relerr(z, zref) < (1e-12 if prec == "f64" else 1e-5)


@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
@pytest.mark.parametrize("n,bc,psf", [(512, AR, synth.gaussian_psf(21, 3.0)),
                                      (256, R, synth.gaussian_psf(15, 2.5)),
                                      (1024, AR, synth.disk_psf(5))])
def test_full_size_operators(n, bc, psf, prec):
    """Operators at the full sizes of the benchmark workloads."""
    print(f"case full-size ops {n} {bc} {prec}", flush=True)
    rng = np.random.default_rng(n)
    h = make((n, n), psf, bc, prec)
    uk = rng.random((n, n))
    h.setup(dev(uk, prec), 5e-4, 0.05, "x_d")
    ukq = host(dev(uk, prec))
    kap = O.kappa(ukq, 0.05)
    x = host(dev(rng.standard_normal((n, n)), prec))
    assert relerr(host(h.normal(dev(x, prec))), O.normal_apply(x, psf, bc, kap, 5e-4)) < TOL[prec]
    ref = O.precond_setup(kap, 5e-4, O.psf_symbol_eigenvalues(psf, n, n, bc), bc, "x_d")
    assert relerr(host(h.export("mu")), ref["mu"]) < 1e-11
    z = host(h.precond(dev(x, prec)))
    assert relerr(z, O.precond_apply(x, ref, bc)) < (1e-12 if prec == "f64" else 1e-5)
