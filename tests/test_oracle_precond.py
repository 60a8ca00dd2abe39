"""Pins of the oracle's preconditioner setup and application (Section 3)."""

import numpy as np
import pytest

import oracle as O

AR, R = "antireflective", "reflective"
DIR, PER = "dirichlet", "periodic"  # the two classical baseline BCs


def quad_sym_psf(my, mx, rng):
    q = rng.random((my + 1, mx + 1)) + 0.05
    h = np.zeros((2 * my + 1, 2 * mx + 1))
    for a in range(-my, my + 1):
        for b in range(-mx, mx + 1):
            h[a + my, b + mx] = q[abs(a), abs(b)]
    return h / h.sum()


@pytest.mark.parametrize("bc", [AR, R, DIR, PER])
@pytest.mark.parametrize("variant", ["diag", "x", "d_x", "x_d"])
def test_fast_setup_equals_dense_projection(bc, variant):
    """The GEMM-form eigenvalues (lam_L, lam_D, lam_Lt) equal diag(Q2 A Q2^T)
    of the dense matrices (level-2 optimal projection, Section 3.2), on a
    non-square image with a non-separable PSF."""
    rng = np.random.default_rng(21)
    ny, nx = 6, 7
    u = rng.random((ny, nx))
    kap = O.kappa(u, 0.15)
    h = quad_sym_psf(1, 2, rng)
    alpha = 0.07
    fast = O.precond_setup(kap, alpha, O.psf_symbol_eigenvalues(h, ny, nx, bc), bc, variant)
    dense = O.precond_setup_dense(kap, alpha, h, bc, variant)
    for key in ("d", "s", "mu"):
        if key in dense:
            np.testing.assert_allclose(fast[key], dense[key], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("bc", [AR, R, DIR, PER])
@pytest.mark.parametrize("variant", ["diag", "x", "d_x", "x_d"])
def test_preconditioner_spd_and_preconditioned_spectrum(bc, variant):
    """PCG needs an SPD preconditioner (Section 1): P^{-1} is symmetric
    positive definite and eig(P^{-1} A) are real and positive."""
    rng = np.random.default_rng(22)
    shape = (6, 6)
    u = rng.random(shape)
    kap = O.kappa(u, 0.1)
    h = quad_sym_psf(1, 1, rng)
    alpha = 0.05
    st = O.precond_setup(kap, alpha, O.psf_symbol_eigenvalues(h, *shape, bc), bc, variant)
    if "mu" in st:
        assert st["mu"].min() > 0
    Pi = O.dense_matrix(lambda r: O.precond_apply(r, st, bc), shape)
    np.testing.assert_allclose(Pi, Pi.T, atol=1e-13)
    assert np.linalg.eigvalsh(0.5 * (Pi + Pi.T)).min() > 0
    A = O.dense_matrix(lambda p: O.normal_apply(p, h, bc, kap, alpha), shape)
    ev = np.linalg.eigvals(Pi @ A)
    assert np.abs(ev.imag).max() < 1e-9 and ev.real.min() > 0


def test_x_d_preconditioner_is_scaled_system_preconditioner():
    """eq. (scalesys): applying X_D to the scaled system A~ = D^{-1/2} A
    D^{-1/2} is P = D^{1/2} X_D D^{1/2} on the original system; with s = 1
    (alpha -> diag L vanishing is not needed) X_D reduces to X when D = I."""
    rng = np.random.default_rng(23)
    shape = (5, 6)
    kap = O.kappa(rng.random(shape), 0.2)
    h = quad_sym_psf(1, 1, rng)
    lam = O.psf_symbol_eigenvalues(h, *shape, AR)
    # alpha = 0 makes D = I: every transform variant collapses to lam_H^2
    for v in ("x", "d_x", "x_d"):
        st = O.precond_setup(kap, 0.0, lam, AR, v)
        np.testing.assert_allclose(st["mu"], lam ** 2, atol=1e-14)
        np.testing.assert_allclose(st["s"], 1.0, atol=0)
    st = O.precond_setup(kap, 0.3, lam, AR, "x_d")
    Xd_inv = O.dense_matrix(lambda r: O.inverse_transform_2d(O.transform_2d(r, AR) / st["mu"], AR), shape)
    S = np.diag(st["s"].ravel())
    Pi = O.dense_matrix(lambda r: O.precond_apply(r, st, AR), shape)
    np.testing.assert_allclose(Pi, S @ Xd_inv @ S, atol=1e-13)


@pytest.mark.parametrize("bc", [AR, R, DIR, PER])
@pytest.mark.parametrize("variant", ["none", "diag", "x", "d_x", "x_d"])
def test_preconditioner_solve_inverts_its_matrix(bc, variant):
    """precond_apply is the inverse of the preconditioner matrix the paper
    defines, formed densely and independently of the fast formulas:
      I;  D = I + alpha diag(L)                       (eq. (D));
      X   = Q2^T diag(mu) Q2                          (eqs. (R), (M); Section 3.2);
      D_X = D^{1/2} Q2^T diag(mu) Q2 D^{1/2}          (eq. (DR2));
      X_D = Q2^T diag(mu) Q2 for the scaled system (eq. (scalesys)), which
            acts on eq. (fp) as D^{1/2} X_D D^{1/2},
    with mu taken from precond_setup_dense (dense diag(Q2 A Q2^T) of dense H
    and L, pinned to the fast setup above) and Q2 the Kronecker product of
    the dense 1D bases.  A wrong power of lambda_H, a missing scaling or a
    transposed transform in precond_apply fails here."""
    rng = np.random.default_rng(24)
    ny, nx = 6, 5
    kap = O.kappa(rng.random((ny, nx)), 0.12)
    h = quad_sym_psf(1, 2, rng)
    alpha = 0.04
    dense = O.precond_setup_dense(kap, alpha, h, bc, variant)
    Ld = O.dense_matrix(lambda x: O.tv_apply(kap, x), (ny, nx))
    D = np.eye(ny * nx) + alpha * np.diag(np.diag(Ld))
    if variant == "none":
        P = np.eye(ny * nx)
    elif variant == "diag":
        P = D
    else:
        Q2 = np.kron(O.basis_matrix(ny, bc), O.basis_matrix(nx, bc))
        X = Q2.T @ np.diag(dense["mu"].ravel()) @ Q2
        Dh = np.sqrt(D)
        P = X if variant == "x" else Dh @ X @ Dh
    fast = O.precond_setup(kap, alpha, O.psf_symbol_eigenvalues(h, ny, nx, bc), bc, variant)
    Pi = O.dense_matrix(lambda r: O.precond_apply(r, fast, bc), (ny, nx))
    np.testing.assert_allclose(Pi @ P, np.eye(ny * nx), atol=1e-11)
