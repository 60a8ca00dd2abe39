"""Differentiable TV restoration: torch.autograd.Function over
tvdeblur_solve / tvdeblur_solve_adjoint.

Forward runs the K lagged-diffusivity steps on the GPU and keeps the iterates
u^0..u^K as checkpoints; backward recomputes kappa(u^k) and the
preconditioner from each checkpoint and solves the adjoint systems with the
same PCG (all in libtvdeblur's kernels), returning dl/dv, dl/dalpha and
dl/dbeta.  The gradient is that of the exact fixed-point map; pass a tight
inner_tol for gradient checks.
"""

import torch

from .lib import TVDeblur


class TVRestore(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, alpha, beta, handle, n_outer, inner_tol, max_inner, precond):
        a, b = float(alpha), float(beta)
        its = torch.empty((n_outer + 1,) + tuple(v.shape), dtype=v.dtype, device=v.device)
        u, st = handle.solve(v.detach().contiguous(), a, b, n_outer, inner_tol, max_inner, precond, iterates=its)
        K = st["outer_steps"]
        ctx.save_for_backward(its[:K + 1])
        ctx.cfg = (handle, a, b, K, inner_tol, max_inner, precond)
        ctx.alpha_meta = (alpha.dtype, alpha.device) if torch.is_tensor(alpha) else None
        ctx.beta_meta = (beta.dtype, beta.device) if torch.is_tensor(beta) else None
        return u

    @staticmethod
    def backward(ctx, ubar):
        (its,) = ctx.saved_tensors
        handle, a, b, K, inner_tol, max_inner, precond = ctx.cfg
        vbar, abar, bbar, _ = handle.solve_adjoint(its, K, ubar.contiguous(), a, b, inner_tol, max_inner, precond)
        ga = torch.tensor(abar, dtype=ctx.alpha_meta[0], device=ctx.alpha_meta[1]) if ctx.alpha_meta else None
        gb = torch.tensor(bbar, dtype=ctx.beta_meta[0], device=ctx.beta_meta[1]) if ctx.beta_meta else None
        return vbar, ga, gb, None, None, None, None, None


def tv_restore(v, alpha, beta, handle=None, psf=None, bc="antireflective", n_outer=15, inner_tol=1e-6,
               max_inner=100, precond="x_d"):
    """u = TV restoration of v (differentiable in v, alpha, beta).  Either
    pass a configured TVDeblur handle or psf (+ bc) to build one; the
    handle's precision follows v's dtype (float64 -> f64, float32 ->
    f32_mixed)."""
    if handle is None:
        prec = "f64" if v.dtype == torch.float64 else "f32_mixed"
        handle = TVDeblur(v.shape[0], v.shape[1], prec)
        handle.set_psf(psf)
        handle.set_bc(bc)
    return TVRestore.apply(v, alpha, beta, handle, n_outer, inner_tol, max_inner, precond)
