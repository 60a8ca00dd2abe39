"""Pins of the two classical baseline BCs the paper compares with (Section 1,
Section 2): zero (Dirichlet) ghosts -> Toeplitz blur; periodic ghosts ->
circulant blur.

Independent facts: the library's zero-fill and wrap-around 2D convolutions;
the real Fourier basis is orthonormal and diagonalises every circulant blur of
a quadrantally symmetric PSF with the eigenvalues given by the FFT of its
first column (a textbook closed form); the zero-Dirichlet eigenvalues equal
the dense diag(Q2 H Q2^T) (the optimal cosine-algebra approximation)."""

import numpy as np
import pytest
import scipy.signal

import oracle as O
from paper_1011_5964_amd import synth

DIR, PER = "dirichlet", "periodic"


def psf(my, mx, seed):
    rng = np.random.default_rng(seed)
    q = rng.random((my + 1, mx + 1)) + 0.05
    h = np.zeros((2 * my + 1, 2 * mx + 1))
    for a in range(-my, my + 1):
        for b in range(-mx, mx + 1):
            h[a + my, b + mx] = q[abs(a), abs(b)]
    return h / h.sum()


@pytest.mark.parametrize("bc,boundary", [(DIR, "fill"), (PER, "wrap")])
def test_blur_is_the_library_convolution(bc, boundary):
    rng = np.random.default_rng(4)
    for shape, (my, mx) in (((9, 12), (2, 3)), ((16, 7), (4, 1))):
        u = rng.standard_normal(shape)
        h = psf(my, mx, 5)
        ref = scipy.signal.convolve2d(u, h, mode="same", boundary=boundary)
        np.testing.assert_allclose(O.blur(u, h, bc), ref, rtol=0, atol=1e-14)
        # adjoint = transpose of the dense matrix
        Hd = O.dense_matrix(lambda x: O.blur(x, h, bc), shape)
        w = rng.standard_normal(shape)
        np.testing.assert_allclose(O.blur_adjoint(w, h, bc).ravel(), Hd.T @ w.ravel(), rtol=0, atol=1e-13)


@pytest.mark.parametrize("n", [1, 2, 5, 8, 13])
def test_real_fourier_basis_is_orthonormal(n):
    Q = O.basis_matrix(n, PER)
    np.testing.assert_allclose(Q @ Q.T, np.eye(n), rtol=0, atol=1e-14)


@pytest.mark.parametrize("ny,nx,my,mx", [(8, 11, 2, 3), (9, 6, 1, 2), (12, 12, 3, 3)])
def test_real_fourier_diagonalises_the_periodic_blur(ny, nx, my, mx):
    h = psf(my, mx, 6)
    Hd = O.dense_matrix(lambda x: O.blur(x, h, PER), (ny, nx))
    Q2 = np.kron(O.basis_matrix(ny, PER), O.basis_matrix(nx, PER))
    Dg = Q2 @ Hd @ Q2.T
    np.testing.assert_allclose(Dg - np.diag(np.diag(Dg)), 0.0, rtol=0, atol=1e-13)
    lam = O.psf_symbol_eigenvalues(h, ny, nx, PER)
    np.testing.assert_allclose(np.diag(Dg).reshape(ny, nx), lam, rtol=0, atol=1e-13)
    # the eigenvalues of a circulant are the DFT of its first column: the
    # multiset of lam equals that of fft2 of the wrapped PSF
    col = np.zeros((ny, nx))
    for a in range(-my, my + 1):
        for b in range(-mx, mx + 1):
            col[a % ny, b % nx] += h[a + my, b + mx]
    f = np.fft.fft2(col)
    assert np.max(np.abs(f.imag)) < 1e-13
    np.testing.assert_allclose(np.sort(lam.ravel()), np.sort(f.real.ravel()), rtol=0, atol=1e-13)


@pytest.mark.parametrize("ny,nx,my,mx", [(8, 11, 2, 3), (10, 7, 3, 1)])
def test_dirichlet_eigenvalues_are_the_optimal_cosine_projection(ny, nx, my, mx):
    h = psf(my, mx, 7)
    Hd = O.dense_matrix(lambda x: O.blur(x, h, DIR), (ny, nx))
    Q2 = np.kron(O.basis_matrix(ny, DIR), O.basis_matrix(nx, DIR))
    lam = O.psf_symbol_eigenvalues(h, ny, nx, DIR)
    np.testing.assert_allclose(lam, np.diag(Q2 @ Hd @ Q2.T).reshape(ny, nx), rtol=0, atol=1e-13)
    # the Toeplitz blur is not in the algebra: the off-diagonal part is not 0
    assert np.abs(Q2 @ Hd @ Q2.T - np.diag(np.diag(Q2 @ Hd @ Q2.T))).max() > 1e-4


@pytest.mark.parametrize("bc", [DIR, PER])
@pytest.mark.parametrize("variant", ["x", "d_x", "x_d"])
def test_fp_solve_with_baseline_bcs(bc, variant):
    """One step solves its system; the TV objective decreases; the transform
    preconditioners cut the iterations of none."""
    p = synth.small_problem(n=20, ny=18, psf_size=5, sigma=1.0, bc=bc, n_outer=4)
    u1, st1 = O.fp_solve(p.v, p.psf, bc, p.alpha, p.beta, 1, 1e-14, 1000, variant)
    kap = O.kappa(p.v, p.beta)
    A = O.dense_matrix(lambda x: O.normal_apply(x, p.psf, bc, kap, p.alpha), p.v.shape)
    ref = np.linalg.solve(A, O.blur_adjoint(p.v, p.psf, bc).ravel())
    np.testing.assert_allclose(u1.ravel(), ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    u, st = O.fp_solve(p.v, p.psf, bc, p.alpha, p.beta, 4, 1e-8, 1000, variant, record_objective=True)
    obj = st["objective"]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(obj, obj[1:]))
    _, s0 = O.fp_solve(p.v, p.psf, bc, p.alpha, p.beta, 4, 1e-8, 1000, "none")
    assert sum(st["inner_iters"]) * 2 <= sum(s0["inner_iters"])
