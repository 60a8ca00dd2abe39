"""Pins of the oracle's PCG and lagged-diffusivity loop (Section 1, eq. (fp);
Section 5 set-up)."""

import numpy as np
import pytest

import oracle as O
from paper_1011_5964_amd import synth

AR, R = "antireflective", "reflective"
DIR, PER = "dirichlet", "periodic"  # the two classical baseline BCs


def test_pcg_matches_dense_solve():
    rng = np.random.default_rng(1)
    M = rng.random((30, 30))
    A = M @ M.T + 30 * np.eye(30)
    b = rng.random(30)
    x, info = O.pcg(lambda p: A @ p, lambda r: r / np.diag(A), b, np.zeros(30), 1e-14, 500)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-12)
    assert info["converged"]


def test_pcg_terminates_in_distinct_eigenvalue_count():
    """CG in exact arithmetic terminates in at most (number of distinct
    eigenvalues) steps; A = I takes one step; P = A^{-1} takes one step."""
    rng = np.random.default_rng(2)
    Qm, _ = np.linalg.qr(rng.standard_normal((20, 20)))
    A = Qm @ np.diag([1.0] * 7 + [3.0] * 7 + [10.0] * 6) @ Qm.T
    b = rng.random(20)
    x, info = O.pcg(lambda p: A @ p, lambda r: r, b, np.zeros(20), 1e-10, 100)
    assert info["iters"] == 3
    x, info = O.pcg(lambda p: p, lambda r: r, b, np.zeros(20), 1e-12, 100)
    assert info["iters"] == 1
    Ai = np.linalg.inv(A)
    x, info = O.pcg(lambda p: A @ p, lambda r: Ai @ r, b, np.zeros(20), 1e-10, 100)
    assert info["iters"] == 1


def test_pcg_zero_residual_start_and_replay():
    A = np.diag([1.0, 2.0, 3.0])
    b = np.array([1.0, 2.0, 3.0])
    x, info = O.pcg(lambda p: A @ p, lambda r: r, b, np.ones(3), 1e-6, 10)
    assert info["iters"] == 0 and info["converged"]
    x, info = O.pcg(lambda p: A @ p, lambda r: r, b, np.zeros(3), 1e-30, 10, replay_iters=2)
    assert info["iters"] == 2


@pytest.mark.parametrize("bc", [AR, R, DIR, PER])
@pytest.mark.parametrize("variant", ["none", "x", "x_d"])
def test_fixed_point_objective_decreases_monotonically(bc, variant):
    """The lagged-diffusivity step minimises a quadratic majoriser of T at
    u^k and warm-started PCG only lowers that quadratic, so
    T(u^{k+1}) <= T(u^k) (fixed-point method of Vogel-Oman, eq. (fp))."""
    p = synth.small_problem(n=20, psf_size=5, sigma=1.0, bc=bc, n_outer=6)
    u, st = O.fp_solve(p.v, p.psf, bc, p.alpha, p.beta, 6, variant=variant, record_objective=True)
    obj = np.asarray(st["objective"])
    assert np.all(obj[1:] <= obj[:-1] * (1 + 1e-13))
    assert obj[-1] < obj[0]


def test_identity_psf_alpha_zero_recovers_v_exactly():
    p = synth.small_problem(n=16)
    h = np.ones((1, 1))
    u, st = O.fp_solve(p.v, h, AR, 0.0, 0.1, 1)
    np.testing.assert_array_equal(u, p.v)
    assert st["inner_iters"] == [0]


@pytest.mark.parametrize("bc", [AR, R, PER])   # zero ghosts do not reproduce constants
def test_constant_image_is_a_fixed_point(bc):
    p = synth.small_problem(n=12)
    v = np.full((12, 12), 0.4)
    u, st = O.fp_solve(v, p.psf, bc, 1e-2, 0.1, 2)
    np.testing.assert_allclose(u, v, atol=1e-14)


@pytest.mark.parametrize("bc", [AR, R, DIR, PER])
def test_fixed_point_limit_solves_euler_lagrange(bc):
    """Converged FP iterates satisfy g(u) = 0 (eq. (el)) to the solver
    tolerance."""
    p = synth.small_problem(n=12, psf_size=3, sigma=0.8, bc=bc, beta=0.5, alpha=1e-2)
    u, st = O.fp_solve(p.v, p.psf, bc, p.alpha, p.beta, 60, inner_tol=1e-13,
                       max_inner=500, fp_tol=1e-13)
    g = O.tv_gradient(u, p.v, p.psf, bc, p.alpha, p.beta)
    assert np.linalg.norm(g) < 1e-9 * np.linalg.norm(O.blur_adjoint(p.v, p.psf, bc))


def test_pcg_solution_of_one_step_matches_dense_solve():
    p = synth.small_problem(n=10, psf_size=5, sigma=1.0)
    its = O.adjoint.fp_forward_dense(p.v, p.psf, AR, p.alpha, p.beta, 1)
    u, st = O.fp_solve(p.v, p.psf, AR, p.alpha, p.beta, 1, inner_tol=1e-14, max_inner=1000)
    np.testing.assert_allclose(u, its[1], rtol=1e-11, atol=1e-12)


def test_preconditioners_reduce_iterations():
    """Soft trend of Tables 1-3: transform preconditioners need far fewer
    iterations than none; X_D is never much worse than X."""
    p = synth.small_problem(n=32, psf_size=7, sigma=1.5, n_outer=3, alpha=1e-3)
    counts = {}
    for v in ("none", "x", "x_d"):
        _, st = O.fp_solve(p.v, p.psf, AR, p.alpha, p.beta, 3, variant=v)
        counts[v] = np.mean(st["inner_iters"])
    assert counts["x"] < 0.6 * counts["none"]
    assert counts["x_d"] <= 1.2 * counts["x"]
