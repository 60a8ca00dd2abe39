"""Preconditioned conjugate gradients and the lagged-diffusivity fixed-point
loop (Section 1, eq. (fp); Section 5 set-up).

TEST INFRASTRUCTURE (see the package docstring).  Plain FP64 NumPy.
"""

import numpy as np

from .operators import blur_adjoint, kappa, normal_apply, tv_objective
from .precond import precond_apply, precond_setup
from .transforms import psf_symbol_eigenvalues


def _dot(a, b):
    return float(np.dot(np.ravel(a), np.ravel(b)))


def pcg(apply_a, apply_pinv, b, x0, tol, max_iter, replay_iters=None):
    """PCG of Golub & Van Loan, Algorithm 10.3.1 (cited in Section 1).

    Starts from x0 (Section 5: the previous fixed-point iterate), stops when
    ||r_k|| / ||r_0|| < tol (strict, Section 5) or after max_iter products
    A p.  The returned count is the number of A p products.  If r_0 = 0 the
    start is returned with 0 iterations.  A non-positive curvature p^T A p
    ends the loop with breakdown=True.  With replay_iters the loop runs
    exactly that many iterations and skips the stopping test.
    """
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - apply_a(x)
    r0 = np.sqrt(_dot(r, r))
    info = {"iters": 0, "r0": r0, "relres": 0.0 if r0 == 0.0 else 1.0,
            "breakdown": False, "converged": r0 == 0.0}
    if r0 == 0.0:
        return x, info
    limit = max_iter if replay_iters is None else replay_iters
    z = apply_pinv(r)
    rho = _dot(r, z)
    p = z.copy()
    it = 0
    while it < limit:
        q = apply_a(p)
        gamma = _dot(p, q)
        it += 1
        if not gamma > 0.0:
            info["breakdown"] = True
            it -= 1
            break
        a = rho / gamma
        x += a * p
        r -= a * q
        rn = np.sqrt(_dot(r, r))
        info["relres"] = rn / r0
        if replay_iters is None and rn < tol * r0:
            info["converged"] = True
            break
        if it == limit:
            break
        z = apply_pinv(r)
        rho_new = _dot(r, z)
        p = z + (rho_new / rho) * p
        rho = rho_new
    info["iters"] = it
    return x, info


def fp_solve(v, h, bc, alpha, beta, n_outer, inner_tol=1e-6, max_inner=100,
             variant="x_d", fp_tol=0.0, u0=None, replay=None,
             record_objective=False, keep_iterates=False):
    """Lagged-diffusivity fixed point, eq. (fp):
        (H^T H + alpha L(u^k)) u^{k+1} = H^T v,   u^0 = v (Section 5).

    Each linear system is solved by PCG warm-started at u^k with the chosen
    preconditioner built from kappa(u^k).  Runs n_outer steps, or stops early
    when fp_tol > 0 and ||u^{k+1} - u^k|| / ||u^{k+1}|| < fp_tol.
    replay: optional per-step iteration counts (run exactly those).
    """
    v = np.asarray(v, dtype=np.float64)
    ny, nx = v.shape
    lam_h = psf_symbol_eigenvalues(h, ny, nx, bc)
    b = blur_adjoint(v, h, bc)
    u = v.copy() if u0 is None else np.array(u0, dtype=np.float64, copy=True)
    stats = {"inner_iters": [], "relres": [], "fp_change": [], "objective": [],
             "breakdown": False, "iterates": [u.copy()] if keep_iterates else None}
    if record_objective:
        stats["objective"].append(tv_objective(u, v, h, bc, alpha, beta))
    for k in range(n_outer):
        kap = kappa(u, beta)
        setup = precond_setup(kap, alpha, lam_h, bc, variant)

        def apply_a(p, kap=kap):
            return normal_apply(p, h, bc, kap, alpha)

        def apply_pinv(r, setup=setup):
            return precond_apply(r, setup, bc)

        rp = None if replay is None else int(replay[k])
        u_new, info = pcg(apply_a, apply_pinv, b, u, inner_tol, max_inner, rp)
        change = np.linalg.norm(u_new - u) / max(np.linalg.norm(u_new), 1e-300)
        u = u_new
        stats["inner_iters"].append(info["iters"])
        stats["relres"].append(info["relres"])
        stats["fp_change"].append(change)
        if keep_iterates:
            stats["iterates"].append(u.copy())
        if record_objective:
            stats["objective"].append(tv_objective(u, v, h, bc, alpha, beta))
        if info["breakdown"]:
            stats["breakdown"] = True
            break
        if fp_tol > 0.0 and change < fp_tol:
            break
    stats["outer_steps"] = len(stats["inner_iters"])
    return u, stats
