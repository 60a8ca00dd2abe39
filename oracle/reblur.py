"""The reblurring system and the anti-reflective algebra (Section 3, eq. (fpp),
eq. (ARalg), the operator AR(.) and the preconditioners P, D_P, P_D; their
two-dimensional forms AR_1, AR_2 at the end of Section 3.2), solved by
preconditioned BiCGstab (van der Vorst 1992, the method the paper cites for
the nonsymmetric system).

TEST INFRASTRUCTURE (see the package docstring).  Plain FP64 NumPy/SciPy.

Setting: anti-reflective BCs for H with a symmetric PSF, and zero-Neumann
BCs for L(u^k) -- the setting in which Section 3 defines P, D_P and P_D.
The reblurring matrix H' is H built from the PSF rotated by 180 degrees,
which for a symmetric PSF equals H, so the system matrix H'H + alpha L(u^k)
is not symmetric (H is not), hence BiCGstab.

Transform: T_n of Section 2 (columns (1, p, 0), (0, S_{n-2}, 0), (0, Jp, 1)
with p_j = 1 - j/(n-1)), T_n = S^(I + U), T_n^{-1} = (I - U) S^ (Remark in
Section 3).  2D: T2 = T_y (x) T_x acting as T_y X T_x^T on images.
"""

import numpy as np
import scipy.fft

from .operators import BC_ANTIREFLECTIVE, blur, dense_matrix, kappa, tv_apply, tv_diagonal
from .precond import diagonal_eigs, weighted_laplacian_eigs
from .transforms import psf_symbol_eigenvalues

REBLUR_VARIANTS = ("p", "d_p", "p_d")
# with the plain preconditioners of the paper's tables (I and D)
REBLUR_ALL_VARIANTS = ("none", "diag") + REBLUR_VARIANTS


def _sine_matrix(m):
    """S_m = sqrt(2/(m+1)) (sin(ij pi/(m+1)))_{i,j=1..m}, eq. (lambda)."""
    i = np.arange(1, m + 1)[:, None]
    j = np.arange(1, m + 1)[None, :]
    return np.sqrt(2.0 / (m + 1)) * np.sin(i * j * np.pi / (m + 1))


def _ramp(n):
    """p of T_n: samples of 1 - x at x = j/(n-1), interior j = 1..n-2."""
    j = np.arange(1, n - 1, dtype=np.float64)
    return 1.0 - j / (n - 1)


def ar_transform_matrix(n):
    """T_n (Section 2, the transform that diagonalises anti-reflective BC
    matrices of a symmetric PSF)."""
    if n < 3:
        raise ValueError("n >= 3 required")
    p = _ramp(n)
    T = np.zeros((n, n))
    T[0, 0] = 1.0
    T[n - 1, n - 1] = 1.0
    T[1:n - 1, 0] = p
    T[1:n - 1, 1:n - 1] = _sine_matrix(n - 2)
    T[1:n - 1, n - 1] = p[::-1]
    return T


def ar_transform_inverse_matrix(n):
    """T_n^{-1} as printed in Section 2: interior rows (-S p, S, -S J p)."""
    if n < 3:
        raise ValueError("n >= 3 required")
    p = _ramp(n)
    S = _sine_matrix(n - 2)
    Ti = np.zeros((n, n))
    Ti[0, 0] = 1.0
    Ti[n - 1, n - 1] = 1.0
    Ti[1:n - 1, 0] = -S @ p
    Ti[1:n - 1, 1:n - 1] = S
    Ti[1:n - 1, n - 1] = -S @ p[::-1]
    return Ti


def _ar_inv_1d(X, axis):
    """T^{-1} along one axis: keep the two end values, DST-I (library,
    orthonormal) of the interior minus the linear interpolant of the ends.
    A one-pixel axis (a 1D signal held as a 1 x n image) is left as it is."""
    X = np.moveaxis(np.asarray(X, dtype=np.float64), axis, 0)
    n = X.shape[0]
    if n == 1:
        return np.moveaxis(X.copy(), 0, axis)
    p = _ramp(n).reshape((-1,) + (1,) * (X.ndim - 1))
    Y = X.copy()
    Y[1:n - 1] = scipy.fft.dst(X[1:n - 1] - p * X[0] - p[::-1] * X[n - 1], type=1, norm="ortho", axis=0)
    return np.moveaxis(Y, 0, axis)


def _ar_fwd_1d(Y, axis):
    """T along one axis: interior = DST-I of the interior + ends times p, Jp."""
    Y = np.moveaxis(np.asarray(Y, dtype=np.float64), axis, 0)
    n = Y.shape[0]
    if n == 1:
        return np.moveaxis(Y.copy(), 0, axis)
    p = _ramp(n).reshape((-1,) + (1,) * (Y.ndim - 1))
    X = Y.copy()
    X[1:n - 1] = scipy.fft.dst(Y[1:n - 1], type=1, norm="ortho", axis=0) + p * Y[0] + p[::-1] * Y[n - 1]
    return np.moveaxis(X, 0, axis)


def ar_coefficients_2d(X):
    """T2^{-1} X = T_y^{-1} X T_x^{-T} (coefficients in the AR algebra)."""
    return _ar_inv_1d(_ar_inv_1d(X, 0), 1)


def ar_synthesis_2d(Y):
    """T2 Y = T_y Y T_x^T."""
    return _ar_fwd_1d(_ar_fwd_1d(Y, 0), 1)


def tau_generator(tau):
    """z with tau = T(z) - H(sigma^2(z), J sigma^2(z)) (Section 3): the first
    column c of a tau matrix is c_k = z_k - z_{k+2} (z beyond its length is
    zero), so z follows by recursion from the last entry."""
    c = np.asarray(tau, dtype=np.float64)[:, 0]
    m = c.size
    z = np.zeros(m + 2)
    for k in range(m - 1, -1, -1):
        z[k] = c[k] + z[k + 2]
    return z[:m]


def ar_projection(A):
    """AR(A) of an n x n matrix, written out as in Section 3: the interior
    block is s(A(2:n-1, 2:n-1)), the optimal tau approximation S diag(S A S) S
    of the inner block; its generator z gives the first column
    (z_1 + 2 sum_{k>=2} z_k, z_2 + 2 sum_{k>=3} z_k, ..., z_{n-2}, 0) and the
    last column is the first one flipped; the first and last rows are zero
    apart from their corner."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    if n < 3:
        raise ValueError("n >= 3 required")
    S = _sine_matrix(n - 2)
    mu = np.diag(S @ A[1:n - 1, 1:n - 1] @ S)
    tau = S @ np.diag(mu) @ S
    z = tau_generator(tau)
    col = np.zeros(n)
    tails = np.cumsum(z[::-1])[::-1]          # tails[k] = sum_{t >= k} z_t
    col[:n - 2] = z + 2.0 * (tails - z)
    B = np.zeros((n, n))
    B[1:n - 1, 1:n - 1] = tau
    B[:, 0] = col
    B[:, n - 1] = col[::-1]
    return B


def ar_projection_level1(A, n_outer, n_inner):
    """AR_1(A): AR(.) applied to every n_inner x n_inner block of A
    (n_outer x n_outer blocks), Section 3.2."""
    A = np.asarray(A, dtype=np.float64)
    B = np.zeros_like(A)
    for i in range(n_outer):
        for j in range(n_outer):
            blk = A[i * n_inner:(i + 1) * n_inner, j * n_inner:(j + 1) * n_inner]
            B[i * n_inner:(i + 1) * n_inner, j * n_inner:(j + 1) * n_inner] = ar_projection(blk)
    return B


def _shuffle(ny, nx):
    """Permutation Q with Q^T vec_row(X) = vec_row(X^T): it swaps the
    Kronecker order (y, x) -> (x, y)."""
    Q = np.zeros((ny * nx, ny * nx))
    for i in range(ny):
        for j in range(nx):
            Q[i * nx + j, j * ny + i] = 1.0
    return Q


def ar_projection_level2(A, ny, nx):
    """AR_2(A) = Q AR_1(Q^T AR_1(A) Q) Q^T (Section 3.2) for an operator on
    ny x nx images in row-major order."""
    Q = _shuffle(ny, nx)
    inner = ar_projection_level1(A, ny, nx)
    return Q @ ar_projection_level1(Q.T @ inner @ Q, nx, ny) @ Q.T


def ar_end_weights(n):
    """w with lambda_end = sum_j w_j mu_j: the eigenvalue of AR(A) at y = 0
    (its corner entry z_1 + 2 sum z_k) as a linear function of the interior
    eigenvalues mu = diag(S A_in S).  Built column by column from
    tau_generator, i.e. from the definition."""
    m = n - 2
    S = _sine_matrix(m)
    w = np.zeros(m)
    for j in range(m):
        tau = np.outer(S[:, j], S[:, j])       # S diag(e_j) S
        z = tau_generator(tau)
        w[j] = z[0] + 2.0 * np.sum(z[1:])
    return w


def ar_extend_eigs(lam_in, ny, nx):
    """Eigenvalues of AR_2(A) on the full ny x nx grid from the interior
    ones: E_y lam_in E_x^T with E = [w^T; I; w^T].  The grid is that of
    eq. (gridy): index 0 and n-1 are the two y = 0 columns of T_n.  A
    one-pixel axis (1D signals, ny = 1) has no ends: E = [1] and lam_in keeps
    that axis whole."""
    def ext(n):
        if n == 1:
            return np.ones((1, 1))
        E = np.zeros((n, n - 2))
        E[1:n - 1] = np.eye(n - 2)
        w = ar_end_weights(n)
        E[0] = w
        E[n - 1] = w
        return E
    return ext(ny) @ np.asarray(lam_in, dtype=np.float64) @ ext(nx).T


def ar_extend_rows_cols(u):
    """u on [-1, ny] x [-1, nx]: one ghost line on every side by the
    anti-reflection of Section 2 (u_{-1} = 2u_0 - u_1, u_n = 2u_{n-1} - u_{n-2}),
    rows first, then columns (the tensor-product order of the 2D extension)."""
    u = np.asarray(u, dtype=np.float64)
    r = np.vstack([2 * u[:1] - u[1:2], u, 2 * u[-1:] - u[-2:-1]])
    return np.hstack([2 * r[:, :1] - r[:, 1:2], r, 2 * r[:, -1:] - r[:, -2:-1]])


def kappa_ar(u, beta):
    """Diffusivity of L(u^k) under anti-reflective BCs (reading, not written out
    in the paper): the forward differences of the anti-reflectively extended
    u^k on every face of the image, the ghost faces included.  Returns
    (kx, ky): kx[i+1, j] sits on the face between rows i and i+1 (i = -1..ny-1),
    ky[i, j+1] on the face between columns j and j+1 (j = -1..nx-1)."""
    e = ar_extend_rows_cols(u)
    ny, nx = np.asarray(u).shape
    gx = e[1:, 1:-1] - e[:-1, 1:-1]            # (ny+1) x nx, row faces
    gy = e[1:-1, 1:] - e[1:-1, :-1]            # ny x (nx+1), column faces
    # the other component on each face: the forward difference of the cell
    # below / left of the face along the other axis (as the Neumann kappa)
    gy_on_x = e[:-1, 2:] - e[:-1, 1:-1]        # row faces: d/dy of the upper cell
    gx_on_y = e[2:, :-1] - e[1:-1, :-1]        # column faces: d/dx of the left cell
    gy_on_x = gy_on_x[:, :nx]
    gx_on_y = gx_on_y[:ny, :]
    kx = 1.0 / np.sqrt(gx * gx + gy_on_x * gy_on_x + beta * beta)
    ky = 1.0 / np.sqrt(gy * gy + gx_on_y * gx_on_y + beta * beta)
    return kx, ky


def tv_apply_ar(kx, ky, y):
    """L(u^k) y under anti-reflective BCs (reading): the flux divergence over
    all faces of every pixel, y extended by the anti-reflection on the ghost
    side of the boundary faces.  Not symmetric."""
    e = ar_extend_rows_cols(y)
    fx = kx * (e[1:, 1:-1] - e[:-1, 1:-1])     # fluxes on row faces
    fy = ky * (e[1:-1, 1:] - e[1:-1, :-1])     # fluxes on column faces
    return -(fx[1:] - fx[:-1]) - (fy[:, 1:] - fy[:, :-1])


def reblur(w, h):
    """H' w: blur with the PSF rotated by 180 degrees under anti-reflective
    BCs (Section 3, the reblurring matrix)."""
    h = np.asarray(h, dtype=np.float64)
    return blur(w, h[::-1, ::-1], BC_ANTIREFLECTIVE)


def reblur_apply(p, h, kap, alpha):
    """A' p = H' H p + alpha L(u^k) p, the matrix of eq. (fpp)."""
    return reblur(blur(p, h, BC_ANTIREFLECTIVE), h) + alpha * tv_apply(kap, p)


def reblur_precond_setup(kap, alpha, lam_h, variant="p_d"):
    """Setup of the preconditioner: 'none' (I) and 'diag' (D = I + alpha
    diag(L), eq. (D)) as in the paper's tables, or the scaling s and
    eigenvalues mu of P, D_P or P_D (Section 3 and the end of Section 3.2),
    all in the algebra of T2:
      'p'    P   = H'H + alpha AR_2(L):            s = 1,      mu = lam_H^2 + alpha lam_L
      'd_p'  D_P = D^{1/2} P D^{1/2}:              s = D^{-1/2}, mu as P
      'p_d'  P_D for the scaled system (scalereb): s = D^{-1/2},
             mu = lam_H^2 lam_D^2 + alpha lam_Lt, lam_D of AR_2(D^{-1/2}),
             lam_Lt of AR_2(D^{-1/2} L D^{-1/2}); applied to (fpp) as
             D^{1/2} P_D D^{1/2}.
    The interior eigenvalues of AR_2(.) are those of the level-2 tau
    projection of the operator's inner block, which equal the interior
    entries of the S^-projection (S^ is zero off the interior there)."""
    if variant not in REBLUR_ALL_VARIANTS:
        raise ValueError(f"unknown reblurring preconditioner {variant!r}")
    kap = np.asarray(kap, dtype=np.float64)
    ny, nx = kap.shape
    D = 1.0 + alpha * tv_diagonal(kap)
    ones = np.ones_like(kap)
    if variant == "none":                     # I
        return {"variant": variant}
    if variant == "diag":                     # D = I + alpha diag(L), eq. (D)
        return {"variant": variant, "d": D}

    def inner(n):
        return slice(0, 1) if n == 1 else slice(1, n - 1)

    def ar2(lam_hat):
        return ar_extend_eigs(lam_hat[inner(ny), inner(nx)], ny, nx)

    if variant in ("p", "d_p"):
        s = ones if variant == "p" else 1.0 / np.sqrt(D)
        mu = lam_h * lam_h + alpha * ar2(weighted_laplacian_eigs(kap, ones, BC_ANTIREFLECTIVE))
        return {"variant": variant, "s": s, "mu": mu}
    s = 1.0 / np.sqrt(D)
    lam_d = ar2(diagonal_eigs(s, BC_ANTIREFLECTIVE))
    mu = lam_h * lam_h * lam_d * lam_d + alpha * ar2(weighted_laplacian_eigs(kap, s, BC_ANTIREFLECTIVE))
    return {"variant": variant, "s": s, "mu": mu}


def reblur_precond_setup_dense(kap, alpha, h, variant="p_d"):
    """Same eigenvalues from dense matrices and the literal AR_2(.)
    (tiny sizes only; pins the fast formulas)."""
    kap = np.asarray(kap, dtype=np.float64)
    ny, nx = kap.shape
    T2 = np.kron(ar_transform_matrix(ny), ar_transform_matrix(nx))
    T2i = np.kron(ar_transform_inverse_matrix(ny), ar_transform_inverse_matrix(nx))
    Hd = dense_matrix(lambda x: blur(x, h, BC_ANTIREFLECTIVE), (ny, nx))
    Ld = dense_matrix(lambda x: tv_apply(kap, x), (ny, nx))

    def eig(A):
        return np.diag(T2i @ A @ T2).reshape(ny, nx)

    lam_h = eig(Hd)
    D = 1.0 + alpha * np.diag(Ld).reshape(ny, nx)
    if variant in ("p", "d_p"):
        s = np.ones_like(kap) if variant == "p" else 1.0 / np.sqrt(D)
        return {"variant": variant, "s": s,
                "mu": lam_h ** 2 + alpha * eig(ar_projection_level2(Ld, ny, nx))}
    s = 1.0 / np.sqrt(D)
    S = np.diag(s.ravel())
    lam_d = eig(ar_projection_level2(S, ny, nx))
    return {"variant": variant, "s": s,
            "mu": lam_h ** 2 * lam_d ** 2 + alpha * eig(ar_projection_level2(S @ Ld @ S, ny, nx))}


def reblur_precond_apply(r, setup):
    """z = M^{-1} r: r (I), r / D (D), or s o T2[(T2^{-1}(s o r)) / mu]."""
    if setup["variant"] == "none":
        return np.array(r, dtype=np.float64, copy=True)
    if setup["variant"] == "diag":
        return np.asarray(r, dtype=np.float64) / setup["d"]
    s = setup["s"]
    return s * ar_synthesis_2d(ar_coefficients_2d(s * np.asarray(r, dtype=np.float64)) / setup["mu"])


def _dot(a, b):
    return float(np.dot(np.ravel(a), np.ravel(b)))


def pbicgstab(apply_a, apply_pinv, b, x0, tol, max_iter, replay_iters=None):
    """Preconditioned BiCGstab (van der Vorst 1992), preconditioner applied
    to the search directions (x = x + alpha M^{-1}p + omega M^{-1}s).

    Shadow residual r^ = r_0.  Convergence is tested once per iteration, on
    the updated residual: ||r_k|| / ||r_0|| < tol (strict, as the PCG
    loop).  One iteration = two products with A.  rho = <r^, r> = 0 or
    <r^, v> = 0 ends the loop with breakdown=True.  <t, t> = 0 (s = 0) sets
    omega = 0, which leaves x = x + alpha M^{-1}p and r = s.  With
    replay_iters the loop runs exactly that many iterations and skips the
    test.
    """
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - apply_a(x)
    r0 = np.sqrt(_dot(r, r))
    info = {"iters": 0, "r0": r0, "relres": 0.0 if r0 == 0.0 else 1.0,
            "breakdown": False, "converged": r0 == 0.0}
    if r0 == 0.0:
        return x, info
    limit = max_iter if replay_iters is None else replay_iters
    rhat = r.copy()
    rho_old = alpha = omega = 1.0
    p = np.zeros_like(r)
    v = np.zeros_like(r)
    it = 0
    while it < limit:
        rho = _dot(rhat, r)
        if rho == 0.0:
            info["breakdown"] = True
            break
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        phat = apply_pinv(p)
        v = apply_a(phat)
        sigma = _dot(rhat, v)
        if sigma == 0.0:
            info["breakdown"] = True
            break
        alpha = rho / sigma
        s = r - alpha * v
        shat = apply_pinv(s)
        t = apply_a(shat)
        tt = _dot(t, t)
        omega = _dot(t, s) / tt if tt > 0.0 else 0.0
        x += alpha * phat + omega * shat
        r = s - omega * t
        it += 1
        rn = np.sqrt(_dot(r, r))
        info["relres"] = rn / r0
        if replay_iters is None and rn < tol * r0:
            info["converged"] = True
            break
        if omega == 0.0:
            info["breakdown"] = rn > 0.0
            break
        rho_old = rho
    info["iters"] = it
    return x, info


def fp_solve_reblur(v, h, alpha, beta, n_outer, inner_tol=1e-6, max_inner=100,
                    variant="p_d", fp_tol=0.0, u0=None, replay=None, l_bc="neumann"):
    """Lagged-diffusivity fixed point on the reblurring system, eq. (fpp):
        (H'H + alpha L(u^k)) u^{k+1} = H' v,   u^0 = v,
    each step by PBiCGstab warm-started at u^k with I, D, P, D_P or P_D built
    from kappa(u^k).  Stopping and replay as fp_solve.

    l_bc = 'antireflective' takes L(u^k) under anti-reflective BCs
    (kappa_ar / tv_apply_ar, a reading).  Its inner block equals the Neumann
    operator's, so AR_2(L) and the eigenvalues of P, D_P, P_D are unchanged;
    D keeps eq. (D) with the Neumann diagonal (the anti-reflective diagonal
    is a difference of face diffusivities at the edges and need not be
    positive)."""
    if l_bc not in ("neumann", "antireflective"):
        raise ValueError(f"unknown BC for L: {l_bc!r}")
    v = np.asarray(v, dtype=np.float64)
    ny, nx = v.shape
    lam_h = psf_symbol_eigenvalues(h, ny, nx, BC_ANTIREFLECTIVE)
    b = reblur(v, h)
    u = v.copy() if u0 is None else np.array(u0, dtype=np.float64, copy=True)
    stats = {"inner_iters": [], "relres": [], "fp_change": [], "breakdown": False}
    for k in range(n_outer):
        kap = kappa(u, beta)
        setup = reblur_precond_setup(kap, alpha, lam_h, variant)
        if l_bc == "antireflective":
            kx, ky = kappa_ar(u, beta)

            def apply_a(p, kx=kx, ky=ky):
                return reblur(blur(p, h, BC_ANTIREFLECTIVE), h) + alpha * tv_apply_ar(kx, ky, p)
        else:
            def apply_a(p, kap=kap):
                return reblur_apply(p, h, kap, alpha)

        def apply_pinv(r, setup=setup):
            return reblur_precond_apply(r, setup)

        rp = None if replay is None else int(replay[k])
        u_new, info = pbicgstab(apply_a, apply_pinv, b, u, inner_tol, max_inner, rp)
        change = np.linalg.norm(u_new - u) / max(np.linalg.norm(u_new), 1e-300)
        u = u_new
        stats["inner_iters"].append(info["iters"])
        stats["relres"].append(info["relres"])
        stats["fp_change"].append(change)
        if info["breakdown"]:
            stats["breakdown"] = True
            break
        if fp_tol > 0.0 and change < fp_tol:
            break
    stats["outer_steps"] = len(stats["inner_iters"])
    return u, stats
