"""Pins of the oracle's reverse-mode derivative of K fixed-point steps."""

import numpy as np
import pytest
import torch

import oracle as O
from oracle.adjoint import fp_adjoint_dense, fp_forward_dense
from paper_1011_5964_amd import synth

AR = "antireflective"


def _loss(v, alpha, beta, h, K, u_true, bc=AR):
    its = fp_forward_dense(v, h, bc, alpha, beta, K)
    return float(np.sum((its[-1] - u_true) ** 2)), its


@pytest.mark.parametrize("bc", [AR, "reflective"])
def test_dense_adjoint_matches_central_differences(bc):
    p = synth.small_problem(n=6, psf_size=3, sigma=0.8, ny=5, bc=bc)
    K, alpha, beta = 2, 0.05, 0.3
    l0, its = _loss(p.v, alpha, beta, p.psf, K, p.u_true, bc)
    vbar, abar, bbar = fp_adjoint_dense(p.psf, bc, alpha, beta, its, 2 * (its[-1] - p.u_true))
    eps = 1e-6
    fd_v = np.zeros_like(p.v)
    for k in range(p.v.size):
        e = np.zeros(p.v.size)
        e[k] = eps
        e = e.reshape(p.v.shape)
        fd_v.ravel()[k] = (_loss(p.v + e, alpha, beta, p.psf, K, p.u_true, bc)[0]
                           - _loss(p.v - e, alpha, beta, p.psf, K, p.u_true, bc)[0]) / (2 * eps)
    np.testing.assert_allclose(vbar, fd_v, rtol=1e-6, atol=1e-9)
    fa = (_loss(p.v, alpha + eps, beta, p.psf, K, p.u_true, bc)[0]
          - _loss(p.v, alpha - eps, beta, p.psf, K, p.u_true, bc)[0]) / (2 * eps)
    fb = (_loss(p.v, alpha, beta + eps, p.psf, K, p.u_true, bc)[0]
          - _loss(p.v, alpha, beta - eps, p.psf, K, p.u_true, bc)[0]) / (2 * eps)
    assert abs(abar - fa) <= 1e-6 * max(1.0, abs(fa))
    assert abs(bbar - fb) <= 1e-6 * max(1.0, abs(fb))


def test_dense_adjoint_matches_torch_autograd():
    """Independent check: torch float64 autograd through K unrolled dense
    solves (CPU), sharing no code with the hand-written recurrence."""
    p = synth.small_problem(n=5, psf_size=3, sigma=0.7)
    K, alpha, beta = 3, 0.04, 0.25
    shape = p.v.shape
    Hd = torch.tensor(O.dense_matrix(lambda x: O.blur(x, p.psf, AR), shape))
    v = torch.tensor(p.v.ravel(), requires_grad=True)
    a = torch.tensor(alpha, dtype=torch.float64, requires_grad=True)
    b = torch.tensor(beta, dtype=torch.float64, requires_grad=True)
    ny, nx = shape
    N = ny * nx
    Dx = torch.zeros(N, N, dtype=torch.float64)
    Dy = torch.zeros(N, N, dtype=torch.float64)
    for i in range(ny):
        for j in range(nx):
            k = i * nx + j
            if i < ny - 1:
                Dx[k, k] = -1
                Dx[k, k + nx] = 1
            if j < nx - 1:
                Dy[k, k] = -1
                Dy[k, k + 1] = 1
    u = v
    for _ in range(K):
        kap = 1.0 / torch.sqrt((Dx @ u) ** 2 + (Dy @ u) ** 2 + b * b)
        L = Dx.T @ torch.diag(kap) @ Dx + Dy.T @ torch.diag(kap) @ Dy
        u = torch.linalg.solve(Hd.T @ Hd + a * L, Hd.T @ v)
    loss = torch.sum((u - torch.tensor(p.u_true.ravel())) ** 2)
    loss.backward()
    its = fp_forward_dense(p.v, p.psf, AR, alpha, beta, K)
    vbar, abar, bbar = fp_adjoint_dense(p.psf, AR, alpha, beta, its, 2 * (its[-1] - p.u_true))
    np.testing.assert_allclose(vbar.ravel(), v.grad.numpy(), rtol=1e-9, atol=1e-12)
    assert abs(abar - a.grad.item()) < 1e-9 * max(1, abs(abar))
    assert abs(bbar - b.grad.item()) < 1e-9 * max(1, abs(bbar))


def test_pcg_adjoint_matches_dense_adjoint():
    p = synth.small_problem(n=10, psf_size=5, sigma=1.0)
    K, alpha, beta = 3, 1e-2, 0.2
    u, st = O.fp_solve(p.v, p.psf, AR, alpha, beta, K, inner_tol=1e-13, max_inner=2000, keep_iterates=True)
    its = st["iterates"]
    ubar = 2 * (its[-1] - p.u_true)
    g1 = O.fp_adjoint(p.psf, AR, alpha, beta, its, ubar, inner_tol=1e-13, max_inner=2000)
    g2 = fp_adjoint_dense(p.psf, AR, alpha, beta, its, ubar)
    np.testing.assert_allclose(g1[0], g2[0], rtol=1e-8, atol=1e-10)
    assert abs(g1[1] - g2[1]) < 1e-8 * max(1, abs(g2[1]))
    assert abs(g1[2] - g2[2]) < 1e-8 * max(1, abs(g2[2]))
