"""Blur under reflective / anti-reflective boundary conditions, its adjoint, and
the TV diffusion operator L(u) -- the two operators of the fixed-point system
(H^T H + alpha L(u^k)) u^{k+1} = H^T v  (Section 1, eq. (fp)).

TEST INFRASTRUCTURE (see the package docstring).  Plain FP64 NumPy/SciPy.

Indexing: 0-based, row-major images u[i, j]; i is the first ("x") index and
j the second ("y") index.  Paper index p (1-based) is code index p - 1.
"""

import functools

import numpy as np
import scipy.signal
import scipy.sparse

BC_REFLECTIVE = "reflective"
BC_ANTIREFLECTIVE = "antireflective"
# the two classical BCs the paper compares with (Section 1 and Section 2):
# zero (Dirichlet) ghosts, giving a Toeplitz blur, and periodic ghosts,
# giving a circulant one
BC_DIRICHLET = "dirichlet"
BC_PERIODIC = "periodic"
_BCS = (BC_REFLECTIVE, BC_ANTIREFLECTIVE, BC_DIRICHLET, BC_PERIODIC)


def _check_bc(bc):
    if bc not in _BCS:
        raise ValueError(f"unknown boundary condition {bc!r}")


def extension_matrix(n, m, bc):
    """Dense (n + 2m) x n matrix E with (E u)[t + m] = u~_t for t in [-m, n+m).

    Section 2.  Reflective (Neumann) BCs: u_{1-j} = u_j, u_{n+j} = u_{n+1-j}.
    Anti-reflective BCs, eq. (anti1d): u_{1-j} = 2 u_1 - u_{j+1},
    u_{n+j} = 2 u_n - u_{n-j}, for j = 1..m.  Written here 0-based:
      reflective:      u~[-j] = u[j-1],           u~[n-1+j] = u[n-j]
      anti-reflective: u~[-j] = 2u[0] - u[j],     u~[n-1+j] = 2u[n-1] - u[n-1-j]
    The anti-reflective rule needs u[j] for j <= m, so m <= n-1; the
    reflective rule needs m <= n.
    Zero (Dirichlet) BCs: every ghost is 0 (Toeplitz blur).  Periodic BCs:
    u~[-j] = u[n-j], u~[n-1+j] = u[j-1] (circulant blur), m <= n.
    """
    _check_bc(bc)
    if m < 0:
        raise ValueError("m must be >= 0")
    if bc == BC_ANTIREFLECTIVE and m > n - 1:
        raise ValueError("anti-reflective extension needs m <= n-1")
    if bc in (BC_REFLECTIVE, BC_PERIODIC) and m > n:
        raise ValueError("reflective / periodic extension needs m <= n")
    E = np.zeros((n + 2 * m, n))
    for t in range(n):
        E[t + m, t] = 1.0
    for j in range(1, m + 1):
        lo = m - j            # row of u~[-j]
        hi = m + n - 1 + j    # row of u~[n-1+j]
        if bc == BC_DIRICHLET:
            continue
        if bc == BC_PERIODIC:
            E[lo, n - j] += 1.0
            E[hi, j - 1] += 1.0
        elif bc == BC_REFLECTIVE:
            E[lo, j - 1] += 1.0
            E[hi, n - j] += 1.0
        else:
            E[lo, 0] += 2.0
            E[lo, j] -= 1.0
            E[hi, n - 1] += 2.0
            E[hi, n - 1 - j] -= 1.0
    return E


@functools.lru_cache(maxsize=64)
def _extension_sparse(n, m, bc):
    E = scipy.sparse.csr_matrix(extension_matrix(n, m, bc))
    return E, E.T.tocsr()


def _convolve(a, k, mode):
    """Library 2D convolution; direct summation for small problems, FFT
    (rounding at the 1e-16 relative level) for large ones."""
    method = "direct" if a.size * k.size < 4e7 else "fft"
    return scipy.signal.convolve(a, k, mode=mode, method=method)


def _psf_halfwidths(h):
    h = np.asarray(h, dtype=np.float64)
    if h.ndim != 2 or h.shape[0] % 2 == 0 or h.shape[1] % 2 == 0:
        raise ValueError("PSF must be a 2D array with odd sizes")
    return (h.shape[0] - 1) // 2, (h.shape[1] - 1) // 2


def extend(u, my, mx, bc):
    """Boundary-extended image u~ on [-my, ny+my) x [-mx, nx+mx).

    Section 2, 2D case: the extension is applied first in one direction and
    then in the other (tensor product), which also yields the paper's four
    corner formulas (checked literally in the tests).
    """
    u = np.asarray(u, dtype=np.float64)
    Ey, _ = _extension_sparse(u.shape[0], my, bc)
    Ex, _ = _extension_sparse(u.shape[1], mx, bc)
    return np.asarray((Ex @ (Ey @ u).T).T)


def blur(u, h, bc):
    """H u: (H u)_{ij} = sum_{a,b} h_{ab} u~_{i-a, j-b}.

    Section 2, eq. (blurred1d:matrixform) and its 2D analogue: convolution of
    the PSF with the boundary-extended image, restricted to the n x n field.
    Library primitive: scipy.signal.convolve in 'valid' mode.
    """
    h = np.asarray(h, dtype=np.float64)
    my, mx = _psf_halfwidths(h)
    ext = extend(u, my, mx, bc)
    return _convolve(ext, h, "valid")


def blur_adjoint(w, h, bc):
    """H^T w, with H = C E (C = valid convolution, E = extension).

    C^T w is the full convolution of w with the 180-degree-rotated PSF over the
    extended domain; E^T then folds every ghost value back onto the pixels it
    was built from, with the extension weights (+1 / +2 / -1).
    """
    h = np.asarray(h, dtype=np.float64)
    my, mx = _psf_halfwidths(h)
    w = np.asarray(w, dtype=np.float64)
    y = _convolve(w, h[::-1, ::-1], "full")
    _, EyT = _extension_sparse(w.shape[0], my, bc)
    _, ExT = _extension_sparse(w.shape[1], mx, bc)
    return np.asarray((ExT @ (EyT @ y).T).T)


def forward_diff(u):
    """Zero-Neumann forward differences (reading of "centred finite
    differences of order two" in Section 1 with a cell-centred diffusivity):
      (D_x u)_{ij} = u_{i+1,j} - u_{ij} for i < ny-1, 0 on the last row;
      (D_y u)_{ij} = u_{i,j+1} - u_{ij} for j < nx-1, 0 on the last column.
    """
    u = np.asarray(u, dtype=np.float64)
    dx = np.zeros_like(u)
    dy = np.zeros_like(u)
    dx[:-1, :] = u[1:, :] - u[:-1, :]
    dy[:, :-1] = u[:, 1:] - u[:, :-1]
    return dx, dy


def forward_diff_adjoint(gx, gy):
    """D_x^T gx + D_y^T gy (transpose of forward_diff)."""
    gx = np.asarray(gx, dtype=np.float64)
    gy = np.asarray(gy, dtype=np.float64)
    out = np.zeros_like(gx)
    out[:-1, :] -= gx[:-1, :]
    out[1:, :] += gx[:-1, :]
    out[:, :-1] -= gy[:, :-1]
    out[:, 1:] += gy[:, :-1]
    return out


def kappa(u, beta):
    """Diffusivity 1 / sqrt(|grad u|^2 + beta^2) per cell (Section 1, the
    coefficient of the operator L_u in eq. (el))."""
    dx, dy = forward_diff(u)
    return 1.0 / np.sqrt(dx * dx + dy * dy + beta * beta)


def tv_apply(kap, y):
    """L(u^k) y = D_x^T (kappa o D_x y) + D_y^T (kappa o D_y y).

    The discrete -div(kappa grad y) with zero-Neumann BCs (Section 1,
    operator L_u; Section 3 imposes Neumann BCs on L).  Symmetric PSD,
    L 1 = 0.
    """
    dx, dy = forward_diff(y)
    return forward_diff_adjoint(kap * dx, kap * dy)


def tv_diagonal(kap):
    """diag(L(u^k)) as an image: kappa_{ij}([i<ny-1] + [j<nx-1])
    + kappa_{i-1,j}[i>0] + kappa_{i,j-1}[j>0]."""
    kap = np.asarray(kap, dtype=np.float64)
    d = np.zeros_like(kap)
    d[:-1, :] += kap[:-1, :]
    d[:, :-1] += kap[:, :-1]
    d[1:, :] += kap[:-1, :]
    d[:, 1:] += kap[:, :-1]
    return d


def tv_objective(u, v, h, bc, alpha, beta):
    """T(u) = 1/2 ||H u - v||^2 + alpha sum sqrt(|grad u|^2 + beta^2).

    Section 1, eq. (mp), read with the fidelity term squared and halved, the
    form whose Euler-Lagrange map is the fixed-point system eq. (fp).
    """
    res = blur(u, h, bc) - v
    dx, dy = forward_diff(u)
    return 0.5 * float(np.sum(res * res)) + alpha * float(np.sum(np.sqrt(dx * dx + dy * dy + beta * beta)))


def tv_gradient(u, v, h, bc, alpha, beta):
    """g(u) = H^T (H u - v) + alpha L(u) u  (Section 1, eq. (el), with the
    sign and argument of the L term read as in eq. (fp))."""
    kap = kappa(u, beta)
    return blur_adjoint(blur(u, h, bc) - v, h, bc) + alpha * tv_apply(kap, u)


def normal_apply(p, h, bc, kap, alpha):
    """A p = H^T H p + alpha L(u^k) p, the matrix of eq. (fp)."""
    return blur_adjoint(blur(p, h, bc), h, bc) + alpha * tv_apply(kap, p)


def dense_matrix(f, shape):
    """Dense matrix of a linear map on images of `shape`, column k = f(e_k)
    flattened row-major.  Test helper for tiny sizes."""
    n = shape[0] * shape[1]
    cols = []
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        cols.append(np.asarray(f(e.reshape(shape)), dtype=np.float64).ravel())
    return np.stack(cols, axis=1)
