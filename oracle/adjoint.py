"""Reverse-mode derivative of K lagged-diffusivity steps.

TEST INFRASTRUCTURE (see the package docstring).  Plain FP64 NumPy.

Derivation (from eq. (fp), assuming each linear system is solved exactly):
u^{k+1} = A_k^{-1} H^T v with A_k = H^T H + alpha L(u^k), L = D^T K D and
K = diag(kappa), kappa = (|D u^k|^2 + beta^2)^{-1/2}.  With ubar = dl/du^{k+1}
and lam = A_k^{-1} ubar (A_k symmetric):
    vbar     += H lam                         (from the right-hand side H^T v)
    e         = D_x lam o D_x u^{k+1} + D_y lam o D_y u^{k+1}
    alphabar -= sum kappa o e                 (= <lam, L u^{k+1}>)
    betabar  += alpha beta sum kappa^3 o e    (d kappa/d beta = -beta kappa^3)
    ubar^k    = alpha [D_x^T(kappa^3 e o D_x u^k) + D_y^T(kappa^3 e o D_y u^k)]
and finally vbar += ubar^0 because u^0 = v.
"""

import numpy as np

from .operators import (blur, blur_adjoint, dense_matrix, forward_diff,
                        forward_diff_adjoint, kappa, normal_apply, tv_apply)
from .precond import precond_apply, precond_setup
from .solver import pcg
from .transforms import psf_symbol_eigenvalues


def _adjoint_sweep(h, bc, alpha, beta, iterates, ubar_k, solve):
    K = len(iterates) - 1
    ubar = np.array(ubar_k, dtype=np.float64, copy=True)
    vbar = np.zeros_like(ubar)
    abar = 0.0
    bbar = 0.0
    for k in range(K - 1, -1, -1):
        uk, uk1 = iterates[k], iterates[k + 1]
        kap = kappa(uk, beta)
        lam = solve(k, kap, ubar)
        vbar += blur(lam, h, bc)
        dxl, dyl = forward_diff(lam)
        dxu1, dyu1 = forward_diff(uk1)
        e = dxl * dxu1 + dyl * dyu1
        abar -= float(np.sum(kap * e))
        k3e = kap ** 3 * e
        bbar += alpha * beta * float(np.sum(k3e))
        dxu, dyu = forward_diff(uk)
        ubar = alpha * forward_diff_adjoint(k3e * dxu, k3e * dyu)
    vbar += ubar
    return vbar, abar, bbar


def fp_adjoint(h, bc, alpha, beta, iterates, ubar_k, inner_tol=1e-12,
               max_inner=1000, variant="x_d"):
    """Gradients (vbar, alphabar, betabar) of a loss l(u^K) given
    ubar_k = dl/du^K and the forward iterates u^0..u^K.  Each adjoint system
    A_k lam = ubar is solved by the same PCG and preconditioner as the
    forward step, from lam = 0."""
    ny, nx = np.shape(iterates[0])
    lam_h = psf_symbol_eigenvalues(h, ny, nx, bc)

    def solve(k, kap, rhs):
        setup = precond_setup(kap, alpha, lam_h, bc, variant)
        x, _ = pcg(lambda p: normal_apply(p, h, bc, kap, alpha),
                   lambda r: precond_apply(r, setup, bc),
                   rhs, np.zeros_like(rhs), inner_tol, max_inner)
        return x

    return _adjoint_sweep(h, bc, alpha, beta, iterates, ubar_k, solve)


def fp_forward_dense(v, h, bc, alpha, beta, n_outer):
    """Exact fixed-point iterates u^0..u^K with dense solves (tiny sizes)."""
    v = np.asarray(v, dtype=np.float64)
    shape = v.shape
    Hd = dense_matrix(lambda x: blur(x, h, bc), shape)
    b = blur_adjoint(v, h, bc).ravel()
    its = [v.copy()]
    u = v.copy()
    for _ in range(n_outer):
        kap = kappa(u, beta)
        Ld = dense_matrix(lambda x, kap=kap: tv_apply(kap, x), shape)
        u = np.linalg.solve(Hd.T @ Hd + alpha * Ld, b).reshape(shape)
        its.append(u.copy())
    return its


def fp_adjoint_dense(h, bc, alpha, beta, iterates, ubar_k):
    """Same recurrence as fp_adjoint with dense numpy.linalg.solve."""
    shape = np.shape(iterates[0])

    def solve(k, kap, rhs):
        A = dense_matrix(lambda x: normal_apply(x, h, bc, kap, alpha), shape)
        return np.linalg.solve(A, rhs.ravel()).reshape(shape)

    return _adjoint_sweep(h, bc, alpha, beta, iterates, ubar_k, solve)
