"""Fast trigonometric transforms that diagonalise the preconditioners, and the
PSF symbol sampled on each boundary condition's grid.

TEST INFRASTRUCTURE (see the package docstring).  Plain FP64 NumPy/SciPy.

basis_matrix(n, bc) returns Q with ROWS equal to the 1D eigenvectors, so the
coefficients of a vector x are Q x and the algebra is {Q^T diag(lam) Q}.
2D: Q2 X = Q_y X Q_x^T (tensor product, Section 3.2).
"""

import numpy as np
import scipy.fft

from .operators import BC_ANTIREFLECTIVE, BC_DIRICHLET, BC_PERIODIC, BC_REFLECTIVE, _check_bc


def basis_matrix(n, bc):
    """Orthogonal 1D transform Q (rows = eigenvectors).

    Reflective, Section 3.1: the DCT-II, [C_n]_{ij} = sqrt((2-delta_{j1})/n)
    cos((2i-1)(j-1)pi/(2n)) with position i and frequency j.  The paper writes
    the algebra as C_n^T Lambda C_n; with this C_n that set does not contain
    the reflective blur, so the eigenvectors are taken to be the COLUMNS of
    C_n, i.e. Q = C_n^T (reading recorded in the design notes).

    Anti-reflective, Section 3.1, eq. (hats): Q = S^ = diag(1, S_{n-2}, 1)
    with S_m = sqrt(2/(m+1)) (sin(ij pi/(m+1)))_{i,j=1..m}, eq. (lambda).

    n = 1 (the one-pixel axis of a 1D signal held as a 1 x n image, Section
    5.1): the axis has only the constant mode, Q = [1] for both BCs (the
    DCT-II formula gives it; for AR the first and last entries coincide).

    Zero-Dirichlet BCs (the Toeplitz blur, not in any fast algebra): the
    same DCT-II, i.e. the cosine-transform preconditioners the paper cites
    for this case (Section 1).  Periodic BCs: the real orthonormal Fourier
    basis 1/sqrt(n); sqrt(2/n) cos(2 pi k i/n), sqrt(2/n) sin(2 pi k i/n) for
    k = 1..ceil(n/2)-1 (in that order, cosine then sine per k); (-1)^i/sqrt(n)
    when n is even.  It diagonalises every symmetric circulant matrix, so the
    periodic blur of a symmetric PSF.
    """
    _check_bc(bc)
    if n == 1:
        return np.ones((1, 1))
    if bc == BC_PERIODIC:
        return _real_fourier(n)
    if bc in (BC_REFLECTIVE, BC_DIRICHLET):
        if n < 2:
            raise ValueError("n >= 1 required")
        i = np.arange(1, n + 1)[:, None]     # position (paper's i)
        j = np.arange(1, n + 1)[None, :]     # frequency (paper's j)
        Cn = np.sqrt((2.0 - (j == 1)) / n) * np.cos((2 * i - 1) * (j - 1) * np.pi / (2 * n))
        return Cn.T.copy()
    if n < 3:
        raise ValueError("n >= 3 required for the anti-reflective transform")
    m = n - 2
    ii = np.arange(1, m + 1)[:, None]
    jj = np.arange(1, m + 1)[None, :]
    S = np.sqrt(2.0 / (m + 1)) * np.sin(ii * jj * np.pi / (m + 1))
    Q = np.zeros((n, n))
    Q[0, 0] = 1.0
    Q[n - 1, n - 1] = 1.0
    Q[1:n - 1, 1:n - 1] = S
    return Q


def _real_fourier(n):
    """Rows: the real orthonormal Fourier basis (see basis_matrix)."""
    i = np.arange(n, dtype=np.float64)
    rows = [np.full(n, 1.0 / np.sqrt(n))]
    for k in range(1, (n + 1) // 2):
        rows.append(np.sqrt(2.0 / n) * np.cos(2.0 * np.pi * k * i / n))
        rows.append(np.sqrt(2.0 / n) * np.sin(2.0 * np.pi * k * i / n))
    if n % 2 == 0:
        rows.append(np.cos(np.pi * i) / np.sqrt(n))
    return np.array(rows)


def _fwd_1d(X, bc, axis):
    if np.shape(X)[axis] == 1:       # one-pixel axis: Q = [1]
        return np.array(X, dtype=np.float64, copy=True)
    if bc == BC_PERIODIC:            # dense product with the real Fourier basis
        return np.moveaxis(np.tensordot(basis_matrix(np.shape(X)[axis], bc), np.asarray(X, dtype=np.float64),
                                        axes=([1], [axis])), 0, axis)
    if bc in (BC_REFLECTIVE, BC_DIRICHLET):
        return scipy.fft.dct(X, type=2, norm="ortho", axis=axis)
    Y = np.array(X, dtype=np.float64, copy=True)
    sl = [slice(None)] * Y.ndim
    sl[axis] = slice(1, Y.shape[axis] - 1)
    Y[tuple(sl)] = scipy.fft.dst(X[tuple(sl)], type=1, norm="ortho", axis=axis)
    return Y


def _inv_1d(Y, bc, axis):
    if np.shape(Y)[axis] == 1:
        return np.array(Y, dtype=np.float64, copy=True)
    if bc == BC_PERIODIC:
        return np.moveaxis(np.tensordot(basis_matrix(np.shape(Y)[axis], bc).T, np.asarray(Y, dtype=np.float64),
                                        axes=([1], [axis])), 0, axis)
    if bc in (BC_REFLECTIVE, BC_DIRICHLET):
        return scipy.fft.idct(Y, type=2, norm="ortho", axis=axis)
    return _fwd_1d(Y, bc, axis)      # S^ is a symmetric involution


def transform_2d(X, bc):
    """Q2 X = Q_y X Q_x^T via library DCT-II / DST-I (orthonormal)."""
    _check_bc(bc)
    X = np.asarray(X, dtype=np.float64)
    return _fwd_1d(_fwd_1d(X, bc, 0), bc, 1)


def inverse_transform_2d(Y, bc):
    """Q2^T Y = Q_y^T Y Q_x."""
    _check_bc(bc)
    Y = np.asarray(Y, dtype=np.float64)
    return _inv_1d(_inv_1d(Y, bc, 0), bc, 1)


def symbol_grid(n, bc):
    """Frequencies at which the PSF symbol gives the eigenvalue of each
    basis vector.

    Reflective (Section 2): theta_k = pi k / n, k = 0..n-1 (DCT-II).
    Anti-reflective, eq. (gridy): y_j = (j-1) pi / (n-1) for j = 1..n-1 and
    y_n = 0; 0-based theta_0 = 0, theta_k = k pi/(n-1) (k = 1..n-2),
    theta_{n-1} = 0.
    Periodic: 2 pi k / n for the cosine and the sine row of frequency k, in
    the order of basis_matrix.  Zero-Dirichlet has no grid (its blur is not
    in the cosine algebra; see psf_symbol_eigenvalues).
    """
    _check_bc(bc)
    k = np.arange(n, dtype=np.float64)
    if n == 1:
        return np.zeros(1)              # a single pixel: only the constant mode
    if bc == BC_DIRICHLET:
        raise ValueError("the zero-Dirichlet blur has no symbol grid")
    if bc == BC_PERIODIC:
        freq = [0] + [kk for kk in range(1, (n + 1) // 2) for _ in (0, 1)] + ([n // 2] if n % 2 == 0 else [])
        return 2.0 * np.pi * np.asarray(freq, dtype=np.float64) / n
    if bc == BC_REFLECTIVE:
        return np.pi * k / n
    th = np.pi * k / (n - 1)
    th[n - 1] = 0.0
    return th


def psf_symbol_eigenvalues(h, ny, nx, bc):
    """lambda_H[k, l] = h^(theta_k, theta_l), the symbol of eq. (symb)
    h^(y, z) = sum_{a,b} h_{ab} exp(i (a y + b z)) sampled on the grid.  For a
    quadrantally symmetric PSF it is real."""
    h = np.asarray(h, dtype=np.float64)
    my, mx = (h.shape[0] - 1) // 2, (h.shape[1] - 1) // 2
    if bc == BC_DIRICHLET:
        return _toeplitz_cosine_projection(h, ny, nx)
    a = np.arange(-my, my + 1, dtype=np.float64)
    b = np.arange(-mx, mx + 1, dtype=np.float64)
    Ey = np.exp(1j * np.outer(symbol_grid(ny, bc), a))
    Ex = np.exp(1j * np.outer(symbol_grid(nx, bc), b))
    lam = Ey @ h @ Ex.T
    return lam.real.copy()


def _toeplitz_cosine_projection(h, ny, nx):
    """Zero-Dirichlet BCs: the eigenvalues of the optimal cosine-algebra
    approximation of the Toeplitz blur (level-2 projection, as Section 3.2
    projects L), diag(Q2 H Q2^T) with Q the DCT-II.  H = sum_{ab} h_ab
    Z_a (x) Z_b with Z_a the shift by a with zero fill, so
    lambda[k, l] = sum_{ab} h_ab c_a[k] c_b[l],  c_a[k] = sum_i phi_k(i) phi_k(i+a)
    over 0 <= i, i+a < n."""
    my, mx = (h.shape[0] - 1) // 2, (h.shape[1] - 1) // 2

    def shifts(n, m):
        Q = basis_matrix(n, BC_DIRICHLET)
        c = np.zeros((2 * m + 1, n))
        for a in range(-m, m + 1):
            lo, hi = max(0, -a), min(n, n - a)
            if lo < hi:
                c[a + m] = np.sum(Q[:, lo:hi] * Q[:, lo + a:hi + a], axis=1)
        return c

    cy, cx = shifts(ny, my), shifts(nx, mx)
    return cy.T @ h @ cx
