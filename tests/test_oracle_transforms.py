"""Pins of the oracle's transforms, symbol eigenvalues and projections
(Section 3) against dense definitions and the paper's structure results."""

import numpy as np
import pytest

import oracle as O

AR, R = "antireflective", "reflective"


def quad_sym_psf(my, mx, rng):
    q = rng.random((my + 1, mx + 1)) + 0.05
    h = np.zeros((2 * my + 1, 2 * mx + 1))
    for a in range(-my, my + 1):
        for b in range(-mx, mx + 1):
            h[a + my, b + mx] = q[abs(a), abs(b)]
    return h / h.sum()


@pytest.mark.parametrize("bc", [AR, R])
@pytest.mark.parametrize("n", [3, 4, 7, 16])
def test_basis_orthogonal_and_library_transform_equals_dense(bc, n):
    Q = O.basis_matrix(n, bc)
    np.testing.assert_allclose(Q @ Q.T, np.eye(n), atol=1e-14)
    rng = np.random.default_rng(n)
    X = rng.random((n, n + 2 if bc == R else n + 1))
    Qx = O.basis_matrix(X.shape[1], bc)
    np.testing.assert_allclose(O.transform_2d(X, bc), Q @ X @ Qx.T, atol=1e-13)
    np.testing.assert_allclose(O.inverse_transform_2d(X, bc), Q.T @ X @ Qx, atol=1e-13)


def test_sine_transform_is_symmetric_involution():
    """Section 3.1: S_n^T = S_n and S_n^2 = I (hence S^ too)."""
    for n in (3, 6, 13):
        Q = O.basis_matrix(n, AR)
        np.testing.assert_allclose(Q, Q.T, atol=1e-15)
        np.testing.assert_allclose(Q @ Q, np.eye(n), atol=1e-14)


def test_dct_orientation_reading():
    """Reflective H is diagonalised by the DCT-II basis with eigenvalues
    h^(pi k / n).  The paper's printed set {C_n^T Lambda C_n} does not contain
    it; {C_n Lambda C_n^T} (columns of C_n as eigenvectors) does."""
    rng = np.random.default_rng(1)
    n, m = 8, 2
    a = rng.random(m + 1) + 0.1
    h = np.concatenate([a[:0:-1], a])
    h = h / h.sum()
    H = O.dense_matrix(lambda x: O.blur(x, h[None, :], R), (1, n))
    i = np.arange(1, n + 1)[:, None]
    j = np.arange(1, n + 1)[None, :]
    Cn = np.sqrt((2.0 - (j == 1)) / n) * np.cos((2 * i - 1) * (j - 1) * np.pi / (2 * n))
    lam = np.array([np.sum(h * np.cos(np.arange(-m, m + 1) * np.pi * k / n)) for k in range(n)])
    np.testing.assert_allclose(H, Cn @ np.diag(lam) @ Cn.T, atol=1e-14)
    assert np.abs(H - Cn.T @ np.diag(lam) @ Cn).max() > 1e-3
    Q = O.basis_matrix(n, R)
    np.testing.assert_allclose(Q.T @ np.diag(lam) @ Q, H, atol=1e-14)


@pytest.mark.parametrize("bc", [AR, R])
def test_symbol_eigenvalues_equal_dense_projection(bc):
    """Eigenvalues of the projected blur diag(Q2 H Q2^T) equal the 2D symbol on
    the boundary condition's grid, for a NON-separable quadrantally symmetric
    PSF on a non-square image."""
    rng = np.random.default_rng(12)
    ny, nx = 7, 6
    h = quad_sym_psf(2, 3, rng)
    Hd = O.dense_matrix(lambda x: O.blur(x, h, bc), (ny, nx))
    Q2 = np.kron(O.basis_matrix(ny, bc), O.basis_matrix(nx, bc))
    P = Q2 @ Hd @ Q2.T
    np.testing.assert_allclose(np.diag(P).reshape(ny, nx), O.psf_symbol_eigenvalues(h, ny, nx, bc), atol=1e-13)
    if bc == R:   # reflective H lies in the algebra: fully diagonalised
        np.testing.assert_allclose(P - np.diag(np.diag(P)), 0, atol=1e-13)


def _tau_generator(B):
    """z with B = T(z) - H(sigma^2 z, J sigma^2 z) from B's first column:
    b_{i1} = z_i - z_{i+2} (zero beyond n)."""
    n = B.shape[0]
    z = np.zeros(n + 2)
    for i in range(n - 1, -1, -1):
        z[i] = B[i, 0] + z[i + 2]
    return z[:n]


def test_tau_toeplitz_minus_hankel_representation():
    """Section 3.1: every B in tau is T(z) - H(sigma^2(z), J sigma^2(z))."""
    rng = np.random.default_rng(3)
    n = 9
    S = O.basis_matrix(n + 2, AR)[1:-1, 1:-1]
    B = S @ np.diag(rng.random(n)) @ S
    z = _tau_generator(B)
    T = np.array([[z[abs(i - j)] for j in range(n)] for i in range(n)])
    s2 = np.concatenate([z[2:], [0.0, 0.0]])          # sigma^2(z)
    first, last = s2, s2[::-1]
    Hk = np.zeros((n, n))                             # Hankel: first col s2, last col J s2
    for i in range(n):
        for j in range(n):
            k = i + j
            Hk[i, j] = first[k] if k < n else last[k - (n - 1)]
    np.testing.assert_allclose(B, T - Hk, atol=1e-13)


def test_proposition_hat_s_projection():
    """Proposition of Section 3.1: s^(A) = blockdiag(A11, s(A(2:n-1,2:n-1)),
    Ann), and it is the Frobenius-nearest element of the hat-tau algebra."""
    rng = np.random.default_rng(4)
    n = 8
    A = rng.random((n, n))
    Sh = O.basis_matrix(n, AR)
    proj = Sh @ np.diag(np.diag(Sh @ A @ Sh)) @ Sh
    S = Sh[1:-1, 1:-1]
    inner = A[1:-1, 1:-1]
    closed = np.zeros((n, n))
    closed[0, 0] = A[0, 0]
    closed[-1, -1] = A[-1, -1]
    closed[1:-1, 1:-1] = S @ np.diag(np.diag(S @ inner @ S)) @ S
    np.testing.assert_allclose(proj, closed, atol=1e-13)
    best = np.linalg.norm(A - proj)
    for _ in range(20):
        lam = np.diag(Sh @ A @ Sh) + 1e-3 * rng.standard_normal(n)
        assert np.linalg.norm(A - Sh @ np.diag(lam) @ Sh) >= best - 1e-14


@pytest.mark.parametrize("bc", [AR, R])
def test_level2_projection_construction(bc):
    """Section 3.2: the level-2 projection Q c1(Q^T c1(A) Q) Q^T (block-wise
    projection, permute, project, permute back) equals the projection onto
    the tensor algebra, Q2^T diag(Q2 A Q2^T) Q2."""
    rng = np.random.default_rng(5)
    n = 5
    A = rng.random((n * n, n * n))
    Q1 = O.basis_matrix(n, bc)

    def c1(M):
        out = np.zeros_like(M)
        for I in range(n):
            for J in range(n):
                blk = M[I * n:(I + 1) * n, J * n:(J + 1) * n]
                out[I * n:(I + 1) * n, J * n:(J + 1) * n] = Q1.T @ np.diag(np.diag(Q1 @ blk @ Q1.T)) @ Q1
        return out

    # permutation with [Q^T A Q]_{i,j;k,l} = [A]_{k,l;i,j}
    P = np.zeros((n * n, n * n))
    for i in range(n):
        for k in range(n):
            P[i * n + k, k * n + i] = 1.0
    lvl2 = P @ c1(P.T @ c1(A) @ P) @ P.T
    Q2 = np.kron(Q1, Q1)
    tensor = Q2.T @ np.diag(np.diag(Q2 @ A @ Q2.T)) @ Q2
    np.testing.assert_allclose(lvl2, tensor, atol=1e-12)
