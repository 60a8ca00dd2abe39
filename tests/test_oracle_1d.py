"""The oracle on 1D signals (Section 5.1), held as 1 x n images.

Pins: the hand-derived 1D blur matrices of tests/golden; the one-pixel axis
reducing the 2D transforms to the library's 1D DCT-II / DST-I; a textbook
closed form for the reflective preconditioner (constant diffusivity: the
Neumann second-difference matrix is diagonalised by the DCT-II with
eigenvalues 2 - 2 cos(pi k / n), so R equals the system matrix and PCG takes
one step); the 1 x n and n x 1 problems giving the same iterates; PCG against
a dense solve; the out-of-focus PSF of eq. (of)."""

import numpy as np
import pytest
import scipy.fft

import oracle as O
from conftest import load_golden
from paper_1011_5964_amd import synth

AR, R = "antireflective", "reflective"


@pytest.mark.parametrize("name,bc", [("ar_n5_h12321.txt", AR), ("ar_n5_h121.txt", AR), ("refl_n5_h12321.txt", R)])
def test_signal_blur_is_the_hand_derived_matrix(name, bc):
    G = load_golden(name)
    taps = {"ar_n5_h12321.txt": [1, 2, 3, 2, 1], "ar_n5_h121.txt": [1, 2, 1], "refl_n5_h12321.txt": [1, 2, 3, 2, 1]}
    h = np.asarray(taps[name], dtype=np.float64)[None, :]
    h /= h.sum()
    rng = np.random.default_rng(1)
    for _ in range(3):
        x = rng.standard_normal(5)
        np.testing.assert_allclose(O.blur(x[None, :], h, bc)[0], G @ x, rtol=0, atol=1e-14)


@pytest.mark.parametrize("bc", [AR, R])
def test_one_pixel_axis_reduces_to_the_1d_library_transform(bc):
    assert np.array_equal(O.basis_matrix(1, bc), np.ones((1, 1)))
    rng = np.random.default_rng(2)
    x = rng.standard_normal(17)
    y = O.transform_2d(x[None, :], bc)[0]
    if bc == R:
        ref = scipy.fft.dct(x, type=2, norm="ortho")
    else:
        ref = x.copy()
        ref[1:-1] = scipy.fft.dst(x[1:-1], type=1, norm="ortho")
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-14)
    np.testing.assert_allclose(O.inverse_transform_2d(y[None, :], bc)[0], x, rtol=0, atol=1e-13)


@pytest.mark.parametrize("variant", ["x", "d_x", "x_d"])
def test_reflective_constant_diffusivity_closed_form(variant):
    """u^k constant: kappa = 1/beta everywhere, L = (1/beta) D^T D (Neumann),
    A = H^T H + alpha L lies in the DCT-II algebra; mu must be
    lam_H(theta_k)^2 + (alpha/beta)(2 - 2 cos theta_k), theta_k = pi k / n, with
    lam_H(theta) = sum_b h_b cos(b theta) (for X_D with constant D the same
    up to the constant scaling), and PCG must stop after one step."""
    n, alpha, beta = 24, 3e-2, 0.5
    h = synth.out_of_focus_1d(3)
    kap = np.full((1, n), 1.0 / beta)
    lam_h = O.psf_symbol_eigenvalues(h, 1, n, R)
    st = O.precond_setup(kap, alpha, lam_h, R, variant)
    theta = np.pi * np.arange(n) / n
    b = np.arange(-(h.shape[1] // 2), h.shape[1] // 2 + 1)
    sym = np.cos(np.outer(theta, b)) @ h[0]
    lam_l = (2.0 - 2.0 * np.cos(theta)) / beta
    if variant in ("x", "d_x"):
        np.testing.assert_allclose(st["mu"][0], sym ** 2 + alpha * lam_l, rtol=1e-12, atol=1e-14)
    # one PCG step solves A x = b exactly when P = A (X) or a scalar multiple of
    # it (D_X, X_D with constant D away from the two end cells is not exact)
    if variant == "x":
        rng = np.random.default_rng(3)
        rhs = rng.standard_normal((1, n))
        x, info = O.pcg(lambda p: O.normal_apply(p, h, R, kap, alpha), lambda r: O.precond_apply(r, st, R),
                        rhs, np.zeros((1, n)), 1e-12, 10)
        assert info["iters"] == 1


@pytest.mark.parametrize("bc", [AR, R])
@pytest.mark.parametrize("variant", ["none", "diag", "x", "d_x", "x_d"])
def test_row_and_column_signals_agree(bc, variant):
    p = synth.signal_problem(64, bc, alpha=1e-3, n_outer=4, fp_tol=0.0)
    u, st = O.fp_solve(p.v, p.psf, bc, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, variant)
    ut, stt = O.fp_solve(p.v.T.copy(), p.psf.T.copy(), bc, p.alpha, p.beta, p.n_outer, p.inner_tol,
                         p.max_inner, variant)
    assert st["inner_iters"] == stt["inner_iters"]
    np.testing.assert_allclose(u, ut.T, rtol=0, atol=1e-13)


@pytest.mark.parametrize("bc", [AR, R])
def test_signal_pcg_step_is_the_dense_solve(bc):
    p = synth.signal_problem(40, bc, alpha=1e-2, n_outer=1)
    kap = O.kappa(p.v, p.beta)
    A = O.dense_matrix(lambda x: O.normal_apply(x, p.psf, bc, kap, p.alpha), p.v.shape)
    b = O.blur_adjoint(p.v, p.psf, bc).ravel()
    ref = np.linalg.solve(A, b)
    u, st = O.fp_solve(p.v, p.psf, bc, p.alpha, p.beta, 1, 1e-15, 500, "x_d")
    np.testing.assert_allclose(u.ravel(), ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_out_of_focus_psf_and_signal_recipe():
    assert synth.signal_half_width(203) == 25
    h = synth.out_of_focus_1d(25)
    assert h.shape == (1, 49) and np.all(h == h[0, 0]) and abs(h.sum() - 1) < 1e-15
    p = synth.signal_problem(203)
    assert p.v.shape == (1, 203) and p.u_true.shape == (1, 203)
    # the observation is the valid convolution of the scene, so its field of
    # view needs m-1 scene samples on each side
    assert p.fp_tol == 1e-3 and p.inner_tol == 1e-6


@pytest.mark.parametrize("variant", ["p", "d_p", "p_d"])
def test_signal_reblur_preconditioner_is_the_literal_ar_projection(variant):
    """1D reblurring preconditioners (Section 3): the fast eigenvalues (the
    S^ projection of the interior plus the end rule through the weights w)
    equal diag(T^{-1} M T) of the literal matrices built with AR(.) written
    out as in Section 3, and those matrices lie in the algebra."""
    from oracle import reblur as RB
    n, alpha = 23, 5e-2
    p = synth.signal_problem(n, AR, alpha=alpha)
    kap = O.kappa(p.v, p.beta)
    lam_h = O.psf_symbol_eigenvalues(p.psf, 1, n, AR)
    st = RB.reblur_precond_setup(kap, alpha, lam_h, variant)
    Hd = O.dense_matrix(lambda x: O.blur(x, p.psf, AR), (1, n))
    Ld = O.dense_matrix(lambda x: O.tv_apply(kap, x), (1, n))
    T, Ti = RB.ar_transform_matrix(n), RB.ar_transform_inverse_matrix(n)
    D = 1.0 + alpha * np.diag(Ld)
    if variant == "p_d":
        S = np.diag(1.0 / np.sqrt(D))
        AS = RB.ar_projection(S)
        M = Hd @ Hd @ AS @ AS + alpha * RB.ar_projection(S @ Ld @ S)
    else:
        M = Hd @ Hd + alpha * RB.ar_projection(Ld)
    E = Ti @ M @ T
    np.testing.assert_allclose(E - np.diag(np.diag(E)), 0.0, atol=1e-11 * np.abs(E).max())
    np.testing.assert_allclose(st["mu"][0], np.diag(E), rtol=1e-10, atol=1e-13)
    # the solve inverts s^{-1} T diag(mu) T^{-1} s^{-1}
    Mfull = np.diag(1.0 / st["s"][0]) @ T @ np.diag(st["mu"][0]) @ Ti @ np.diag(1.0 / st["s"][0])
    rng = np.random.default_rng(9)
    r = rng.standard_normal((1, n))
    z = RB.reblur_precond_apply(r, st)
    np.testing.assert_allclose(Mfull @ z[0], r[0], rtol=0, atol=1e-10 * np.abs(r).max())


@pytest.mark.parametrize("variant", ["none", "diag", "p", "d_p", "p_d"])
def test_signal_reblur_step_is_the_dense_solve_and_rows_equal_columns(variant):
    from oracle import reblur as RB
    p = synth.signal_problem(40, AR, alpha=1e-2)
    u1, _ = RB.fp_solve_reblur(p.v, p.psf, p.alpha, p.beta, 1, 1e-15, 500, variant)
    kap = O.kappa(p.v, p.beta)
    A = O.dense_matrix(lambda x: RB.reblur_apply(x, p.psf, kap, p.alpha), p.v.shape)
    ref = np.linalg.solve(A, RB.reblur(p.v, p.psf).ravel())
    np.testing.assert_allclose(u1.ravel(), ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    u, st = RB.fp_solve_reblur(p.v, p.psf, p.alpha, p.beta, 5, 1e-6, 500, variant)
    ut, stt = RB.fp_solve_reblur(p.v.T.copy(), p.psf.T.copy(), p.alpha, p.beta, 5, 1e-6, 500, variant)
    assert st["inner_iters"] == stt["inner_iters"]
    np.testing.assert_allclose(u, ut.T, rtol=0, atol=1e-13)
