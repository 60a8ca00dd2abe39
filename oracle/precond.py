"""Fast-transform preconditioners for the fixed-point system, eq. (fp).

TEST INFRASTRUCTURE (see the package docstring).  Plain FP64 NumPy.

Variants (columns of the paper's Tables 1-3):
  'none'  I                    no preconditioner
  'diag'  D = I + alpha diag(L(u^k))            eq. (D) ("D" column)
  'x'     R (reflective, eq. (R)/(R2)) or M (anti-reflective, eq. (M))
          = Q2^T (lam_H^2 + alpha lam_L) Q2
  'd_x'   D_X = D^{1/2} X D^{1/2}                eq. (DR2), D_M
  'x_d'   X_D for the scaled system eq. (scalesys), R_D / M_D of Section 3.2:
          Q2^T (lam_H^2 lam_D^2 + alpha lam_Lt) Q2, applied to (fp) as
          D^{1/2} X_D D^{1/2}

Each eigenvalue array is the diagonal of Q2 A Q2^T (the optimal Frobenius
projection onto the transform algebra, Section 3; level-2 projection of
Section 3.2), with Q2 = Q_y (x) Q_x, Q from basis_matrix().
"""

import numpy as np

from .operators import blur, dense_matrix, tv_apply, tv_diagonal
from .transforms import basis_matrix, inverse_transform_2d, psf_symbol_eigenvalues, transform_2d

VARIANTS = ("none", "diag", "x", "d_x", "x_d")


def weighted_laplacian_eigs(kap, s, bc):
    """diag(Q2 (S L S) Q2^T) with S = diag(s), L = L(u^k) of the TV operator.

    For a basis image phi_kl = phi_k(i) phi_l(j) the diagonal entry is
      sum_ij kappa_ij [ (D_x(s o phi_kl))_ij^2 + (D_y(s o phi_kl))_ij^2 ].
    Expanding the squares makes every term a product  P^T X W  of an
    elementwise array X (kappa and shifted s) with squared / shifted basis
    matrices, evaluated here with dense matmuls.  s = 1 gives lam_L.
    """
    kap = np.asarray(kap, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    ny, nx = kap.shape
    Py = basis_matrix(ny, bc).T          # Py[i, k] = phi_k(i)
    Px = basis_matrix(nx, bc).T
    Wy, Wx = Py * Py, Px * Px

    def shifted(P):
        up = np.zeros_like(P)
        up[:-1] = P[1:]                  # phi_k(i+1), 0 on the last position
        lo = P.copy()
        lo[-1] = 0.0                     # phi_k(i), masked where D is zero
        return up, lo

    Pyu, Pyl = shifted(Py)
    Pxu, Pxl = shifted(Px)

    s_dn = np.zeros_like(s)
    s_dn[:-1, :] = s[1:, :]              # s_{i+1, j}
    s_rt = np.zeros_like(s)
    s_rt[:, :-1] = s[:, 1:]              # s_{i, j+1}
    row_mask = np.ones_like(s)
    row_mask[-1, :] = 0.0
    col_mask = np.ones_like(s)
    col_mask[:, -1] = 0.0

    A1 = kap * s_dn * s_dn
    A2 = kap * s_dn * s
    A3 = kap * s * s * row_mask
    lam_x = (Pyu * Pyu).T @ A1 @ Wx - 2.0 * (Pyu * Pyl).T @ A2 @ Wx + (Pyl * Pyl).T @ A3 @ Wx

    B1 = kap * s_rt * s_rt
    B2 = kap * s_rt * s
    B3 = kap * s * s * col_mask
    lam_y = Wy.T @ B1 @ (Pxu * Pxu) - 2.0 * Wy.T @ B2 @ (Pxu * Pxl) + Wy.T @ B3 @ (Pxl * Pxl)
    return lam_x + lam_y


def diagonal_eigs(s, bc):
    """diag(Q2 diag(s) Q2^T)[k, l] = sum_ij s_ij phi_k(i)^2 phi_l(j)^2."""
    s = np.asarray(s, dtype=np.float64)
    Wy = basis_matrix(s.shape[0], bc).T ** 2
    Wx = basis_matrix(s.shape[1], bc).T ** 2
    return Wy.T @ s @ Wx


def precond_setup(kap, alpha, lam_h, bc, variant="x_d"):
    """Per fixed-point-step setup: scaling s and eigenvalues mu (Section 3.2).

    lam_h: eigenvalues of the projected blur (psf_symbol_eigenvalues).
    Returns a dict used by precond_apply.
    """
    if variant not in VARIANTS:
        raise ValueError(f"unknown preconditioner {variant!r}")
    kap = np.asarray(kap, dtype=np.float64)
    out = {"variant": variant}
    if variant == "none":
        return out
    D = 1.0 + alpha * tv_diagonal(kap)                     # eq. (D)
    if variant == "diag":
        out["d"] = D
        return out
    ones = np.ones_like(kap)
    if variant == "x":
        out["s"] = ones
        out["mu"] = lam_h * lam_h + alpha * weighted_laplacian_eigs(kap, ones, bc)
        return out
    s = 1.0 / np.sqrt(D)                                    # D^{-1/2}
    out["s"] = s
    if variant == "d_x":
        out["mu"] = lam_h * lam_h + alpha * weighted_laplacian_eigs(kap, ones, bc)
    else:  # x_d
        lam_d = diagonal_eigs(s, bc)
        out["mu"] = lam_h * lam_h * lam_d * lam_d + alpha * weighted_laplacian_eigs(kap, s, bc)
    return out


def precond_setup_dense(kap, alpha, h, bc, variant="x_d"):
    """Same as precond_setup, every projection formed from dense matrices
    diag(Q2 A Q2^T) (tiny sizes only; used to pin the fast formulas)."""
    kap = np.asarray(kap, dtype=np.float64)
    ny, nx = kap.shape
    Q2 = np.kron(basis_matrix(ny, bc), basis_matrix(nx, bc))   # row-major vec
    Hd = dense_matrix(lambda x: blur(x, h, bc), (ny, nx))
    Ld = dense_matrix(lambda x: tv_apply(kap, x), (ny, nx))

    def proj(A):
        return np.diag(Q2 @ A @ Q2.T).reshape(ny, nx)

    out = {"variant": variant}
    if variant == "none":
        return out
    D = 1.0 + alpha * np.diag(Ld).reshape(ny, nx)
    if variant == "diag":
        out["d"] = D
        return out
    lam_h = proj(Hd)
    if variant in ("x", "d_x"):
        out["s"] = np.ones_like(kap) if variant == "x" else 1.0 / np.sqrt(D)
        out["mu"] = lam_h ** 2 + alpha * proj(Ld)
        return out
    s = 1.0 / np.sqrt(D)
    S = np.diag(s.ravel())
    out["s"] = s
    out["mu"] = lam_h ** 2 * proj(S) ** 2 + alpha * proj(S @ Ld @ S)
    return out


def precond_apply(r, setup, bc):
    """z = P^{-1} r.  Transform variants: z = s o Q2^T[(Q2(s o r)) / mu]."""
    v = setup["variant"]
    r = np.asarray(r, dtype=np.float64)
    if v == "none":
        return r.copy()
    if v == "diag":
        return r / setup["d"]
    s = setup["s"]
    return s * inverse_transform_2d(transform_2d(s * r, bc) / setup["mu"], bc)


def lambda_h(h, ny, nx, bc):
    """Convenience alias of psf_symbol_eigenvalues."""
    return psf_symbol_eigenvalues(h, ny, nx, bc)
