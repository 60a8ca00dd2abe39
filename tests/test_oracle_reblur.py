"""Pins of the oracle's reblurring system, anti-reflective algebra and
PBiCGstab (Section 3, eq. (fpp), eq. (ARalg), AR(.), AR_2(.); Section 2's
transform T_n)."""

import numpy as np
import pytest
import scipy.linalg

import oracle as O
from oracle import reblur as RB

AR = "antireflective"


def ar_blur_1d(g, n):
    """Dense 1D anti-reflective blur matrix: valid convolution of the
    extension (extension_matrix is pinned in the operator tests)."""
    m = len(g) // 2
    E = O.extension_matrix(n, m, AR)
    C = np.zeros((n, n + 2 * m))
    for i in range(n):
        for a in range(-m, m + 1):
            C[i, i - a + m] += g[a + m]
    return C @ E


def sym_1d(m, rng):
    q = rng.random(m + 1) + 0.05
    g = np.concatenate([q[:0:-1], q])
    return g / g.sum()


def quad_sym_psf(my, mx, rng):
    q = rng.random((my + 1, mx + 1)) + 0.05
    h = np.zeros((2 * my + 1, 2 * mx + 1))
    for a in range(-my, my + 1):
        for b in range(-mx, mx + 1):
            h[a + my, b + mx] = q[abs(a), abs(b)]
    return h / h.sum()


@pytest.mark.parametrize("n", range(3, 11))
def test_printed_inverse_of_T(n):
    """Section 2 prints T_n^{-1} in closed form; it is the inverse of T_n."""
    T = RB.ar_transform_matrix(n)
    np.testing.assert_allclose(RB.ar_transform_inverse_matrix(n) @ T, np.eye(n), atol=1e-14)
    np.testing.assert_allclose(np.linalg.inv(T), RB.ar_transform_inverse_matrix(n), atol=1e-13)


@pytest.mark.parametrize("n", [4, 7, 10])
def test_T_factorises_as_in_the_remark(n):
    """T_n = S^(I + U), T_n^{-1} = (I - U) S^ with U zero except its
    interior rows (S p, 0, S J p) (Remark in Section 3); S^ is the pinned
    anti-reflective basis of the M preconditioners."""
    Sh = O.basis_matrix(n, AR)
    S = Sh[1:n - 1, 1:n - 1]
    p = 1.0 - np.arange(1, n - 1) / (n - 1)
    U = np.zeros((n, n))
    U[1:n - 1, 0] = S @ p
    U[1:n - 1, n - 1] = S @ p[::-1]
    np.testing.assert_allclose(Sh @ (np.eye(n) + U), RB.ar_transform_matrix(n), atol=1e-14)
    np.testing.assert_allclose((np.eye(n) - U) @ Sh, RB.ar_transform_inverse_matrix(n), atol=1e-14)


@pytest.mark.parametrize("n,m", [(7, 1), (9, 2), (12, 3), (8, 5)])
def test_T_diagonalises_antireflective_blur(n, m):
    """Section 2: for a symmetric PSF the anti-reflective matrix is
    T_n Lambda T_n^{-1}, Lambda = the symbol sampled on the grid of
    eq. (gridy) (y = 0 at both ends)."""
    g = sym_1d(m, np.random.default_rng(n + m))
    H = ar_blur_1d(g, n)
    D = RB.ar_transform_inverse_matrix(n) @ H @ RB.ar_transform_matrix(n)
    np.testing.assert_allclose(D - np.diag(np.diag(D)), 0.0, atol=1e-14)
    y = O.symbol_grid(n, AR)
    a = np.arange(-m, m + 1)
    sym = np.cos(np.outer(y, a)) @ g
    np.testing.assert_allclose(np.diag(D), sym, atol=1e-14)


def test_T2_diagonalises_2d_blur_with_symbol_eigenvalues():
    """2D: T2^{-1} H T2 = diag(lambda_H) with the non-separable symmetric
    PSF symbol of psf_symbol_eigenvalues."""
    rng = np.random.default_rng(3)
    ny, nx = 6, 7
    h = quad_sym_psf(1, 2, rng)
    Hd = O.dense_matrix(lambda x: O.blur(x, h, AR), (ny, nx))
    T2 = np.kron(RB.ar_transform_matrix(ny), RB.ar_transform_matrix(nx))
    T2i = np.kron(RB.ar_transform_inverse_matrix(ny), RB.ar_transform_inverse_matrix(nx))
    D = T2i @ Hd @ T2
    np.testing.assert_allclose(D - np.diag(np.diag(D)), 0.0, atol=1e-14)
    np.testing.assert_allclose(np.diag(D).reshape(ny, nx), O.psf_symbol_eigenvalues(h, ny, nx, AR),
                               atol=1e-14)


@pytest.mark.parametrize("m", [4, 6, 9])
def test_tau_generator_inverts_toeplitz_minus_hankel(m):
    """tau(z) = T(z) - H(sigma^2 z, J sigma^2 z) built with the library
    Toeplitz / Hankel constructors: tau_generator returns z, and the
    eigenvalues of tau(z) are z_1 + 2 sum_k z_k cos((k-1) j pi/(m+1))."""
    rng = np.random.default_rng(m)
    z = rng.standard_normal(m)
    s2 = np.concatenate([z[2:], [0.0, 0.0]])
    tau = scipy.linalg.toeplitz(z) - scipy.linalg.hankel(s2, s2[::-1])
    np.testing.assert_allclose(RB.tau_generator(tau), z, atol=1e-14)
    S = RB._sine_matrix(m)
    j = np.arange(1, m + 1)
    k = np.arange(1, m + 1)
    lam = z[0] + 2.0 * np.cos(np.outer(j, k[1:] - 1) * np.pi / (m + 1)) @ z[1:]
    np.testing.assert_allclose(S @ tau @ S, np.diag(lam), atol=1e-12)


@pytest.mark.parametrize("n,m", [(7, 1), (9, 2), (11, 4)])
def test_AR_of_an_antireflective_matrix_is_itself(n, m):
    """AR(.) written out from Section 3 reproduces every anti-reflective
    blur matrix of a symmetric PSF (they lie in the algebra)."""
    H = ar_blur_1d(sym_1d(m, np.random.default_rng(40 + n)), n)
    np.testing.assert_allclose(RB.ar_projection(H), H, atol=1e-14)


@pytest.mark.parametrize("sym", [True, False])
@pytest.mark.parametrize("n", [5, 8])
def test_AR_lies_in_the_algebra(sym, n):
    """AR(A) is in the algebra of T_n (Section 3): T^{-1} AR(A) T is
    diagonal, interior eigenvalues diag(S A_in S), both end eigenvalues
    the corner z_1 + 2 sum z_k = w . mu (ar_end_weights)."""
    rng = np.random.default_rng(50 + n)
    A = rng.standard_normal((n, n))
    if sym:
        A = A + A.T
    B = RB.ar_projection(A)
    D = RB.ar_transform_inverse_matrix(n) @ B @ RB.ar_transform_matrix(n)
    np.testing.assert_allclose(D - np.diag(np.diag(D)), 0.0, atol=1e-13)
    S = RB._sine_matrix(n - 2)
    mu = np.diag(S @ A[1:n - 1, 1:n - 1] @ S)
    np.testing.assert_allclose(np.diag(D)[1:n - 1], mu, atol=1e-13)
    end = RB.ar_end_weights(n) @ mu
    np.testing.assert_allclose(np.diag(D)[[0, n - 1]], [end, end], atol=1e-13)
    np.testing.assert_allclose(B[0, 0], end, atol=1e-13)


@pytest.mark.parametrize("n", [5, 9, 40, 130])
def test_end_weights_reproduce_constants(n):
    """AR(.) of the identity is the identity (the identity is in the algebra),
    so the end eigenvalue of mu = 1 is 1: the weights sum to 1.  They
    extrapolate to y = 0 and alternate, with absolute sum n - 2."""
    w = RB.ar_end_weights(n)
    assert abs(w.sum() - 1.0) < 1e-12
    # the generator recursion and the corner sum accumulate O(n^2) roundings
    np.testing.assert_allclose(RB.ar_projection(np.eye(n)), np.eye(n), atol=2 * n * n * np.finfo(float).eps)
    assert abs(np.abs(w).sum() - (n - 2)) < 1e-9 * n


@pytest.mark.parametrize("n", [3, 4, 9, 40, 130, 300])
def test_end_weights_closed_form(n):
    """The corner of AR(.) counts each entry c_k of the tau matrix's first
    column k times (z_k = sum_t c_{k+2t}, corner z_1 + 2 sum_{k>=2} z_k), so
    w_j = S_1j sum_k k S_kj; summing the series at theta_j = j pi/(n-1) gives
    w_j = (-1)^(j+1) (1 + cos theta_j).  The recursion of the definition
    rounds at O(n^2) eps."""
    m = n - 2
    j = np.arange(1, m + 1)
    closed = (-1.0) ** (j + 1) * (1.0 + np.cos(j * np.pi / (m + 1)))
    np.testing.assert_allclose(RB.ar_end_weights(n), closed, rtol=0, atol=2 * n * n * np.finfo(float).eps)


def test_level2_projection_is_in_the_2d_algebra():
    """AR_2(L) = Q AR_1(Q^T AR_1(L) Q) Q^T (Section 3.2) is diagonalised by
    T2, with the eigenvalues of ar_extend_eigs on the interior S^-projection."""
    rng = np.random.default_rng(5)
    ny, nx = 5, 6
    kap = O.kappa(rng.random((ny, nx)), 0.2)
    Ld = O.dense_matrix(lambda x: O.tv_apply(kap, x), (ny, nx))
    B = RB.ar_projection_level2(Ld, ny, nx)
    T2 = np.kron(RB.ar_transform_matrix(ny), RB.ar_transform_matrix(nx))
    T2i = np.kron(RB.ar_transform_inverse_matrix(ny), RB.ar_transform_inverse_matrix(nx))
    D = T2i @ B @ T2
    np.testing.assert_allclose(D - np.diag(np.diag(D)), 0.0, atol=1e-13)
    lam_hat = O.precond.weighted_laplacian_eigs(kap, np.ones_like(kap), AR)
    fast = RB.ar_extend_eigs(lam_hat[1:ny - 1, 1:nx - 1], ny, nx)
    np.testing.assert_allclose(np.diag(D).reshape(ny, nx), fast, atol=1e-13)


@pytest.mark.parametrize("variant", RB.REBLUR_VARIANTS)
def test_fast_reblur_setup_equals_literal_definitions(variant):
    """mu of P, D_P, P_D from the fast formulas equals the eigenvalues of the
    literal dense H'H + alpha AR_2(.) forms (non-square, non-separable PSF)."""
    rng = np.random.default_rng(6)
    ny, nx = 6, 7
    kap = O.kappa(rng.random((ny, nx)), 0.15)
    h = quad_sym_psf(1, 2, rng)
    alpha = 0.07
    fast = RB.reblur_precond_setup(kap, alpha, O.psf_symbol_eigenvalues(h, ny, nx, AR), variant)
    dense = RB.reblur_precond_setup_dense(kap, alpha, h, variant)
    np.testing.assert_allclose(fast["s"], dense["s"], rtol=1e-14)
    np.testing.assert_allclose(fast["mu"], dense["mu"], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("variant", RB.REBLUR_VARIANTS)
def test_preconditioner_solve_inverts_its_matrix(variant):
    """reblur_precond_apply is the inverse of s^{-1} T2 diag(mu) T2^{-1} s^{-1}
    built densely."""
    rng = np.random.default_rng(7)
    ny, nx = 5, 6
    kap = O.kappa(rng.random((ny, nx)), 0.1)
    h = quad_sym_psf(1, 1, rng)
    st = RB.reblur_precond_setup(kap, 0.05, O.psf_symbol_eigenvalues(h, ny, nx, AR), variant)
    T2 = np.kron(RB.ar_transform_matrix(ny), RB.ar_transform_matrix(nx))
    T2i = np.kron(RB.ar_transform_inverse_matrix(ny), RB.ar_transform_inverse_matrix(nx))
    Si = np.diag(1.0 / st["s"].ravel())
    P = Si @ T2 @ np.diag(st["mu"].ravel()) @ T2i @ Si
    Pi = O.dense_matrix(lambda r: RB.reblur_precond_apply(r, st), (ny, nx))
    np.testing.assert_allclose(Pi @ P, np.eye(ny * nx), atol=1e-11)


def test_fast_transforms_equal_dense_T():
    rng = np.random.default_rng(8)
    X = rng.standard_normal((7, 9))
    Ty, Tx = RB.ar_transform_matrix(7), RB.ar_transform_matrix(9)
    Tyi, Txi = RB.ar_transform_inverse_matrix(7), RB.ar_transform_inverse_matrix(9)
    np.testing.assert_allclose(RB.ar_coefficients_2d(X), Tyi @ X @ Txi.T, atol=1e-14)
    np.testing.assert_allclose(RB.ar_synthesis_2d(X), Ty @ X @ Tx.T, atol=1e-14)
    np.testing.assert_allclose(RB.ar_synthesis_2d(RB.ar_coefficients_2d(X)), X, atol=1e-13)


def test_reblurring_matrix_and_nonsymmetric_system():
    """H' (rotated PSF) equals H for a symmetric PSF; H'H + alpha L is not
    symmetric under anti-reflective BCs (why the paper uses BiCGstab), and
    differs from H^T H only through the boundary corrections."""
    rng = np.random.default_rng(9)
    ny, nx = 7, 8
    h = quad_sym_psf(1, 2, rng)
    kap = O.kappa(rng.random((ny, nx)), 0.1)
    x = rng.standard_normal((ny, nx))
    np.testing.assert_allclose(RB.reblur(x, h), O.blur(x, h, AR), atol=1e-15)
    A = O.dense_matrix(lambda p: RB.reblur_apply(p, h, kap, 0.05), (ny, nx))
    assert np.abs(A - A.T).max() > 1e-3
    N = O.dense_matrix(lambda p: O.normal_apply(p, h, AR, kap, 0.05), (ny, nx))
    inner = np.zeros((ny, nx), bool)
    inner[3:-3, 3:-3] = True          # rows and columns the boundary corrections of H never meet in HH
    k = np.flatnonzero(inner.ravel())
    np.testing.assert_allclose(A[np.ix_(k, k)], N[np.ix_(k, k)], atol=1e-15)


def test_pbicgstab_solves_a_nonsymmetric_system():
    rng = np.random.default_rng(10)
    n = 14
    A = 4.0 * np.eye(n) + 0.6 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    x, info = RB.pbicgstab(lambda p: A @ p, lambda r: r, b, np.zeros(n), 1e-12, 200)
    assert info["converged"] and not info["breakdown"]
    np.testing.assert_allclose(x, np.linalg.solve(A, b), atol=1e-11)
    # the exact preconditioner ends it in one iteration
    x1, info1 = RB.pbicgstab(lambda p: A @ p, lambda r: np.linalg.solve(A, r), b, np.zeros(n), 1e-12, 50)
    assert info1["iters"] == 1
    np.testing.assert_allclose(x1, np.linalg.solve(A, b), atol=1e-12)
    # replay runs exactly the requested count
    _, info3 = RB.pbicgstab(lambda p: A @ p, lambda r: r, b, np.zeros(n), 1e-12, 200, replay_iters=3)
    assert info3["iters"] == 3
    # zero residual at the start: no iteration
    x0 = np.linalg.solve(A, b)
    _, info0 = RB.pbicgstab(lambda p: A @ p, lambda r: r, A @ x0, x0, 1e-6, 10)
    assert info0["iters"] == 0 and info0["converged"]


def test_pbicgstab_recurrence_matches_true_residual():
    """The recurred residual r = s - omega t equals b - A x (rounding only)
    after each replayed count."""
    rng = np.random.default_rng(11)
    n = 20
    A = 3.0 * np.eye(n) + 0.5 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    M = np.diag(np.diag(A))
    for k in (1, 2, 5):
        x, info = RB.pbicgstab(lambda p: A @ p, lambda r: np.linalg.solve(M, r), b, np.zeros(n), 0.0, 50,
                               replay_iters=k)
        rn = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        assert abs(rn - info["relres"]) < 1e-13


def test_reblur_fixed_point_recovers_noise_free_image_at_alpha_zero():
    """alpha = 0: the system is H'H u = H'v; with v = H u_true and an
    invertible H every step returns u_true (well-conditioned PSF)."""
    rng = np.random.default_rng(12)
    n = 12
    g = np.array([0.1, 0.8, 0.1])
    h = np.outer(g, g)
    u_true = rng.random((n, n))
    v = O.blur(u_true, h, AR)
    u, st = RB.fp_solve_reblur(v, h, 0.0, 0.1, 2, inner_tol=1e-13, max_inner=200, variant="p")
    assert st["inner_iters"][0] > 0
    np.testing.assert_allclose(u, u_true, atol=1e-11)


def test_reblur_identity_psf_alpha_zero_is_exact():
    """Identity PSF and alpha = 0: A' = I and H'v = v, so u^0 = v is
    already the solution (zero initial residual, no iteration)."""
    v = np.random.default_rng(13).random((9, 10))
    u, st = RB.fp_solve_reblur(v, np.ones((1, 1)), 0.0, 0.1, 2)
    assert st["inner_iters"] == [0, 0]
    np.testing.assert_array_equal(u, v)


def test_reblur_fixed_point_steps_solve_their_systems():
    """Each fixed-point step's result satisfies eq. (fpp) to the inner
    tolerance: ||H'v - A'(u^k) u^{k+1}|| <= tol ||H'v - A'(u^k) u^k||."""
    rng = np.random.default_rng(14)
    ny, nx = 10, 11
    h = quad_sym_psf(1, 1, rng)
    v = O.blur(rng.random((ny, nx)), h, AR) + 0.01 * rng.standard_normal((ny, nx))
    alpha, beta, tol = 0.02, 0.1, 1e-8
    u1, st1 = RB.fp_solve_reblur(v, h, alpha, beta, 1, inner_tol=tol, max_inner=300)
    u2, st2 = RB.fp_solve_reblur(v, h, alpha, beta, 2, inner_tol=tol, max_inner=300)
    kap = O.kappa(u1, beta)
    b = RB.reblur(v, h)
    r_end = np.linalg.norm(b - RB.reblur_apply(u2, h, kap, alpha))
    r_start = np.linalg.norm(b - RB.reblur_apply(u1, h, kap, alpha))
    assert st2["inner_iters"][1] > 0 and r_end < tol * r_start


def test_plain_preconditioners_of_the_tables():
    """I and D of the tables: I leaves r, D divides by 1 + alpha diag(L)
    (diag(L) from the dense operator); PBiCGstab with D on the reblurring
    system matches a direct solve."""
    rng = np.random.default_rng(15)
    ny, nx = 6, 7
    kap = O.kappa(rng.random((ny, nx)), 0.1)
    alpha = 0.05
    r = rng.standard_normal((ny, nx))
    st_i = RB.reblur_precond_setup(kap, alpha, None, "none")
    np.testing.assert_array_equal(RB.reblur_precond_apply(r, st_i), r)
    st_d = RB.reblur_precond_setup(kap, alpha, None, "diag")
    Ld = O.dense_matrix(lambda x: O.tv_apply(kap, x), (ny, nx))
    np.testing.assert_allclose(RB.reblur_precond_apply(r, st_d), r / (1 + alpha * np.diag(Ld).reshape(ny, nx)),
                               rtol=1e-14)
    h = quad_sym_psf(1, 1, rng)
    A = O.dense_matrix(lambda p: RB.reblur_apply(p, h, kap, alpha), (ny, nx))
    b = rng.standard_normal(ny * nx)
    x, info = RB.pbicgstab(lambda p: RB.reblur_apply(p, h, kap, alpha),
                           lambda q: RB.reblur_precond_apply(q, st_d), b.reshape(ny, nx), np.zeros((ny, nx)),
                           1e-12, 200)
    assert info["converged"]
    np.testing.assert_allclose(x.ravel(), np.linalg.solve(A, b), atol=1e-10)


@pytest.mark.parametrize("variant", RB.REBLUR_ALL_VARIANTS)
def test_one_reblur_step_equals_a_dense_solve(variant):
    """One fixed-point step (tight tolerance) equals the direct solution of
    the dense system (H'H + alpha L(v)) u = H'v built from the blur and the
    TV operator, for every preconditioner."""
    rng = np.random.default_rng(16)
    ny, nx = 7, 9
    h = quad_sym_psf(1, 1, rng)
    v = O.blur(rng.random((ny, nx)), h, AR) + 0.01 * rng.standard_normal((ny, nx))
    alpha, beta = 0.03, 0.1
    u, st = RB.fp_solve_reblur(v, h, alpha, beta, 1, inner_tol=1e-13, max_inner=500, variant=variant)
    kap = O.kappa(v, beta)
    Hd = O.dense_matrix(lambda x: O.blur(x, h, AR), (ny, nx))
    Ld = O.dense_matrix(lambda x: O.tv_apply(kap, x), (ny, nx))
    ref = np.linalg.solve(Hd @ Hd + alpha * Ld, (Hd @ v.ravel()))
    assert st["inner_iters"][0] > 0
    np.testing.assert_allclose(u.ravel(), ref, rtol=0, atol=1e-10 * np.abs(ref).max())


def test_ar_bc_operator_constant_diffusivity_in_the_algebra():
    """With constant diffusivity, L under anti-reflective BCs lies in the
    algebra of T_n (x) T_n with symbol (2 - 2cos y) + (2 - 2cos z): a linear
    extension has zero second difference, so the edge rows carry no extra
    term (the corner 0 of AR(.) for the Laplacian)."""
    ny, nx = 6, 7
    kx, ky = np.ones((ny + 1, nx)), np.ones((ny, nx + 1))
    L = O.dense_matrix(lambda y: RB.tv_apply_ar(kx, ky, y), (ny, nx))
    T2 = np.kron(RB.ar_transform_matrix(ny), RB.ar_transform_matrix(nx))
    T2i = np.kron(RB.ar_transform_inverse_matrix(ny), RB.ar_transform_inverse_matrix(nx))
    D = T2i @ L @ T2
    np.testing.assert_allclose(D - np.diag(np.diag(D)), 0.0, atol=1e-13)
    sym = (2 - 2 * np.cos(O.symbol_grid(ny, AR)))[:, None] + (2 - 2 * np.cos(O.symbol_grid(nx, AR)))[None, :]
    np.testing.assert_allclose(np.diag(D).reshape(ny, nx), sym, atol=1e-13)


def test_ar_bc_operator_inner_block_and_projection_equal_neumann():
    """Variable diffusivity: the anti-reflective L annihilates constants, is
    not symmetric, and differs from the Neumann L only in the rows and columns
    of edge pixels, so AR_2 of the two operators coincide (the reblurring
    preconditioners do not change); its face diffusivities equal the Neumann
    kappa wherever the Neumann differences are not cut at the far edges."""
    rng = np.random.default_rng(17)
    ny, nx = 6, 7
    u = rng.random((ny, nx))
    beta = 0.2
    kx, ky = RB.kappa_ar(u, beta)
    kap = O.kappa(u, beta)
    np.testing.assert_allclose(kx[1:ny, :nx - 1], kap[:ny - 1, :nx - 1], rtol=1e-14)
    np.testing.assert_allclose(ky[:ny - 1, 1:nx], kap[:ny - 1, :nx - 1], rtol=1e-14)
    Lar = O.dense_matrix(lambda y: RB.tv_apply_ar(kx, ky, y), (ny, nx))
    Ln = O.dense_matrix(lambda y: O.tv_apply(kap, y), (ny, nx))
    np.testing.assert_allclose(Lar @ np.ones(ny * nx), 0.0, atol=1e-12)
    assert np.abs(Lar - Lar.T).max() > 1e-3
    inner = np.zeros((ny, nx), bool)
    inner[1:-1, 1:-1] = True
    k = np.flatnonzero(inner.ravel())
    np.testing.assert_allclose(Lar[np.ix_(k, k)], Ln[np.ix_(k, k)], atol=1e-13)
    np.testing.assert_allclose(RB.ar_projection_level2(Lar, ny, nx), RB.ar_projection_level2(Ln, ny, nx),
                               atol=1e-12)


def test_reblur_with_ar_bc_operator_solves_its_systems():
    """The fixed point with L under anti-reflective BCs: each step solves its
    (nonsymmetric) system to the tolerance; the preconditioner still helps."""
    rng = np.random.default_rng(18)
    ny, nx = 12, 13
    h = quad_sym_psf(1, 1, rng)
    v = O.blur(rng.random((ny, nx)), h, AR) + 0.01 * rng.standard_normal((ny, nx))
    alpha, beta, tol = 0.02, 0.1, 1e-8
    u1, _ = RB.fp_solve_reblur(v, h, alpha, beta, 1, tol, 400, "p_d", l_bc="antireflective")
    u2, st = RB.fp_solve_reblur(v, h, alpha, beta, 2, tol, 400, "p_d", l_bc="antireflective")
    kx, ky = RB.kappa_ar(u1, beta)
    b = RB.reblur(v, h)

    def A(p):
        return RB.reblur(O.blur(p, h, AR), h) + alpha * RB.tv_apply_ar(kx, ky, p)

    assert np.linalg.norm(b - A(u2)) < tol * np.linalg.norm(b - A(u1))
    _, st_none = RB.fp_solve_reblur(v, h, alpha, beta, 2, 1e-6, 400, "none", l_bc="antireflective")
    _, st_pd = RB.fp_solve_reblur(v, h, alpha, beta, 2, 1e-6, 400, "p_d", l_bc="antireflective")
    assert sum(st_pd["inner_iters"]) < sum(st_none["inner_iters"])
    with pytest.raises(ValueError):
        RB.fp_solve_reblur(v, h, alpha, beta, 1, l_bc="dirichlet")
