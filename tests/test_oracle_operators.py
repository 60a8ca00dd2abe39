"""Pins of the oracle's blur / adjoint / TV operators against what the paper
and the mathematics fix (not against re-typed copies of the same formulas)."""

import numpy as np
import pytest

import oracle as O
from tests.conftest import load_golden

AR, R = "antireflective", "reflective"


def sym_psf_1d(m, rng):
    a = rng.random(m + 1) + 0.1
    h = np.concatenate([a[:0:-1], a])
    return h / h.sum()


def quad_sym_psf(my, mx, rng):
    q = rng.random((my + 1, mx + 1)) + 0.05
    h = np.zeros((2 * my + 1, 2 * mx + 1))
    for a in range(-my, my + 1):
        for b in range(-mx, mx + 1):
            h[a + my, b + mx] = q[abs(a), abs(b)]
    return h / h.sum()


def blur_matrix_1d(n, h1, bc):
    h = h1[None, :]
    return O.dense_matrix(lambda x: O.blur(x, h, bc), (1, n))


@pytest.mark.parametrize("fname,h,bc", [
    ("ar_n5_h121.txt", np.array([1, 2, 1]) / 4.0, AR),
    ("ar_n5_h12321.txt", np.array([1, 2, 3, 2, 1]) / 9.0, AR),
    ("refl_n5_h12321.txt", np.array([1, 2, 3, 2, 1]) / 9.0, R),
])
def test_blur_matrix_matches_hand_derived_fixture(fname, h, bc):
    """Section 2: the 1D blur matrices worked out by hand from the extension
    rules (tests/golden)."""
    np.testing.assert_allclose(blur_matrix_1d(5, h, bc), load_golden(fname), atol=1e-15)


@pytest.mark.parametrize("n,m", [(5, 1), (7, 3), (9, 4), (8, 7), (12, 5)])
def test_ar_matrix_equals_Tn_Lambda_Tn_inverse(n, m):
    """Section 2: for symmetric h the AR matrix is T_n Lambda T_n^{-1}, with
    the paper's block forms of T_n, T_n^{-1}, p_j = 1 - j/(n-1), and Lambda
    the symbol eq. (symb) sampled on the grid eq. (gridy)."""
    rng = np.random.default_rng(n * 31 + m)
    h = sym_psf_1d(m, rng)
    H = blur_matrix_1d(n, h, AR)
    k = n - 2
    S = np.sqrt(2.0 / (k + 1)) * np.sin(np.outer(np.arange(1, k + 1), np.arange(1, k + 1)) * np.pi / (k + 1))
    p = 1.0 - np.arange(1, k + 1) / (n - 1)
    Jp = p[::-1]
    T = np.zeros((n, n))
    T[0, 0] = T[-1, -1] = 1.0
    T[1:-1, 0] = p
    T[1:-1, 1:-1] = S
    T[1:-1, -1] = Jp
    Ti = np.zeros((n, n))
    Ti[0, 0] = Ti[-1, -1] = 1.0
    Ti[1:-1, 0] = -S @ p
    Ti[1:-1, 1:-1] = S
    Ti[1:-1, -1] = -S @ Jp
    np.testing.assert_allclose(T @ Ti, np.eye(n), atol=1e-13)
    # Lambda = diag(h^(y_j)), eq. (lambda)/(gridy), 1-based y_j=(j-1)pi/(n-1), y_n=0
    y = np.array([(j - 1) * np.pi / (n - 1) for j in range(1, n)] + [0.0])
    a = np.arange(-m, m + 1)
    lam = np.array([np.sum(h * np.exp(1j * a * yy)).real for yy in y])
    np.testing.assert_allclose(H, T @ np.diag(lam) @ Ti, atol=1e-13)
    # the oracle's own symbol-grid eigenvalues agree with the paper's Lambda
    np.testing.assert_allclose(O.psf_symbol_eigenvalues(h[None, :], 1, n, AR)[0], lam, atol=1e-14)


@pytest.mark.parametrize("n", [5, 8, 11])
def test_Tn_functional_form(n):
    """eq. (Tn): T_n = (1 - y/pi, sin y, ..., sin((n-2) y), y/pi) diag(1,
    sqrt(2/(n-1)) I, 1), rows sampled on the uniform grid (i-1) pi/(n-1),
    i = 1..n, equals the block form."""
    k = n - 2
    S = np.sqrt(2.0 / (k + 1)) * np.sin(np.outer(np.arange(1, k + 1), np.arange(1, k + 1)) * np.pi / (k + 1))
    p = 1.0 - np.arange(1, k + 1) / (n - 1)
    T = np.zeros((n, n))
    T[0, 0] = T[-1, -1] = 1.0
    T[1:-1, 0] = p
    T[1:-1, 1:-1] = S
    T[1:-1, -1] = p[::-1]
    y = np.arange(n) * np.pi / (n - 1)
    F = np.column_stack([1 - y / np.pi] + [np.sin(j * y) for j in range(1, n - 1)] + [y / np.pi])
    F = F @ np.diag([1.0] + [np.sqrt(2.0 / (n - 1))] * (n - 2) + [1.0])
    np.testing.assert_allclose(F, T, atol=1e-14)


def test_ar_rows_are_identity_and_structure():
    """Section 2: rows 1 and n of the AR matrix are e_1^T and e_n^T (normalised
    symmetric PSF); interior block H(2:n-1, 2:n-1) lies in tau (Section 3.1)
    with eigenvalues h^(k pi/(n-1))."""
    rng = np.random.default_rng(3)
    n, m = 10, 3
    h = sym_psf_1d(m, rng)
    H = blur_matrix_1d(n, h, AR)
    np.testing.assert_allclose(H[0], np.eye(n)[0], atol=1e-15)
    np.testing.assert_allclose(H[-1], np.eye(n)[-1], atol=1e-15)
    inner = H[1:-1, 1:-1]
    k = n - 2
    S = np.sqrt(2.0 / (k + 1)) * np.sin(np.outer(np.arange(1, k + 1), np.arange(1, k + 1)) * np.pi / (k + 1))
    D = S @ inner @ S
    np.testing.assert_allclose(D - np.diag(np.diag(D)), 0, atol=1e-13)
    a = np.arange(-m, m + 1)
    expect = [np.sum(h * np.cos(a * kk * np.pi / (n - 1))) for kk in range(1, k + 1)]
    np.testing.assert_allclose(np.diag(D), expect, atol=1e-13)


def test_ar_2d_edges_and_corners_literal():
    """Section 2, 2D anti-reflective extension: edge rules and the four
    corner formulas as printed (1-based u_{1-i,1-j} = 4u_{11} - 2u_{1,j+1}
    - 2u_{i+1,1} + u_{i+1,j+1}, etc.)."""
    rng = np.random.default_rng(5)
    n, m = 7, 3
    u = rng.random((n, n))
    E = O.extend(u, m, m, AR)

    def U(i, j):      # 1-based access into u
        return u[i - 1, j - 1]

    def Ut(i, j):     # 1-based access into u~ (indices may be <= 0 or > n)
        return E[i - 1 + m, j - 1 + m]

    for j in range(1, m + 1):
        for phi in range(1, n + 1):
            assert np.isclose(Ut(1 - j, phi), 2 * U(1, phi) - U(j + 1, phi))
            assert np.isclose(Ut(n + j, phi), 2 * U(n, phi) - U(n - j, phi))
            assert np.isclose(Ut(phi, 1 - j), 2 * U(phi, 1) - U(phi, j + 1))
            assert np.isclose(Ut(phi, n + j), 2 * U(phi, n) - U(phi, n - j))
    for i in range(1, m + 1):
        for j in range(1, m + 1):
            assert np.isclose(Ut(1 - i, 1 - j), 4 * U(1, 1) - 2 * U(1, j + 1) - 2 * U(i + 1, 1) + U(i + 1, j + 1))
            assert np.isclose(Ut(1 - i, n + j), 4 * U(1, n) - 2 * U(1, n - j) - 2 * U(i + 1, n) + U(i + 1, n - j))
            assert np.isclose(Ut(n + i, 1 - j), 4 * U(n, 1) - 2 * U(n, j + 1) - 2 * U(n - i, 1) + U(n - i, j + 1))
            assert np.isclose(Ut(n + i, n + j), 4 * U(n, n) - 2 * U(n, n - j) - 2 * U(n - i, n) + U(n - i, n - j))


def test_blur_brute_force_sum():
    """(Hu)_{ij} = sum_ab h_ab u~_{i-a,j-b} by explicit loops on a tiny
    non-square image with a non-square PSF."""
    rng = np.random.default_rng(11)
    u = rng.random((6, 5))
    h = quad_sym_psf(2, 1, rng)
    for bc in (AR, R):
        E = O.extend(u, 2, 1, bc)
        out = np.zeros_like(u)
        for i in range(6):
            for j in range(5):
                for a in range(-2, 3):
                    for b in range(-1, 2):
                        out[i, j] += h[a + 2, b + 1] * E[i - a + 2, j - b + 1]
        np.testing.assert_allclose(O.blur(u, h, bc), out, atol=1e-14)


@pytest.mark.parametrize("bc", [AR, R])
def test_adjoint_is_dense_transpose(bc):
    rng = np.random.default_rng(2)
    shape = (7, 6)
    h = quad_sym_psf(2, 3, rng)
    Hd = O.dense_matrix(lambda x: O.blur(x, h, bc), shape)
    HTd = O.dense_matrix(lambda x: O.blur_adjoint(x, h, bc), shape)
    np.testing.assert_allclose(HTd, Hd.T, atol=1e-14)


def test_reflective_symmetric_and_reproduces_constants():
    rng = np.random.default_rng(4)
    shape = (6, 6)
    h = quad_sym_psf(2, 2, rng)
    Hd = O.dense_matrix(lambda x: O.blur(x, h, R), shape)
    np.testing.assert_allclose(Hd, Hd.T, atol=1e-15)
    np.testing.assert_allclose(O.blur(np.full(shape, 2.5), h, R), 2.5, atol=1e-14)


def test_ar_reproduces_bilinear_images():
    """AR extension of a bilinear image is exact (linear extrapolation), and a
    normalised quadrantally symmetric PSF leaves a bilinear image unchanged,
    so H u = u for u = a + b i + c j + d i j."""
    rng = np.random.default_rng(6)
    ny, nx = 9, 8
    i, j = np.mgrid[0:ny, 0:nx].astype(np.float64)
    u = 0.3 + 0.7 * i - 0.2 * j + 0.05 * i * j
    h = quad_sym_psf(3, 4, rng)
    np.testing.assert_allclose(O.blur(u, h, AR), u, atol=1e-13)


def test_tv_operator_properties():
    rng = np.random.default_rng(8)
    shape = (6, 7)
    u = rng.random(shape)
    kap = O.kappa(u, 0.1)
    Ld = O.dense_matrix(lambda x: O.tv_apply(kap, x), shape)
    np.testing.assert_allclose(Ld, Ld.T, atol=1e-14)
    assert np.linalg.eigvalsh(Ld).min() > -1e-12
    np.testing.assert_allclose(Ld @ np.ones(Ld.shape[0]), 0, atol=1e-13)
    np.testing.assert_allclose(np.diag(Ld).reshape(shape), O.tv_diagonal(kap), atol=1e-14)


def test_tv_gradient_matches_finite_differences():
    """Reading of eq. (mp)/(el)/(fp): with T(u) = 1/2||Hu-v||^2 + alpha TV_beta(u)
    and the cell-centred forward-difference discretisation, the gradient of
    T is exactly H^T(Hu-v) + alpha L(u) u -- the fixed-point map eq. (fp)."""
    rng = np.random.default_rng(9)
    shape = (6, 5)
    u = rng.random(shape)
    v = rng.random(shape)
    h = quad_sym_psf(1, 2, rng)
    alpha, beta = 0.3, 0.2
    for bc in (AR, R):
        g = O.tv_gradient(u, v, h, bc, alpha, beta)
        fd = np.zeros_like(u)
        eps = 1e-6
        for k in range(u.size):
            e = np.zeros(u.size)
            e[k] = eps
            e = e.reshape(shape)
            fd.ravel()[k] = (O.tv_objective(u + e, v, h, bc, alpha, beta)
                             - O.tv_objective(u - e, v, h, bc, alpha, beta)) / (2 * eps)
        np.testing.assert_allclose(g, fd, atol=1e-7)


def test_extension_limits():
    with pytest.raises(ValueError):
        O.extension_matrix(4, 4, AR)
    O.extension_matrix(4, 3, AR)
    O.extension_matrix(4, 4, R)
    with pytest.raises(ValueError):
        O.extension_matrix(4, 5, R)
