"""Misfit of BDDC-preconditioned solutions and its gradient with respect to
element log10-coefficients, as a ``torch.autograd.Function``.

With K(theta) = sum_e 10^theta_e Khat_e, x_k = K^{-1} f_k and
J = 1/2 sum_k ||x_k - x_obs,k||^2, the adjoint lambda_k = K^{-1}(x_k - x_obs,k)
(K is symmetric) gives

    dJ/dtheta_e = -ln(10) sum_k lambda_k,e^T K_e x_k,e,   K_e = 10^theta_e Khat_e.

Forward runs the library's set-up from theta (coefficients computed on the
device), the multilevel BDDC-PCG solve and the misfit kernel; backward reuses
the same handle (same hierarchy, same preconditioner) for the adjoint solve
and assembles the element gradient in the library.  If the handle was set up
again between forward and backward (another forward, a finite-difference
probe), backward first repeats the set-up at the forward's theta, so the
adjoint solve and the element matrices always belong to the theta the
gradient is taken at.  The argument tensors stay on the GPU; no step runs on
the host.
"""
from __future__ import annotations

import torch


class BddcMisfit(torch.autograd.Function):
    """J(theta) = 1/2 sum_k ||K(theta)^{-1} f_k - x_obs,k||^2.

    Arguments of ``apply``: theta (float64 CUDA tensor [n_elems]), handle
    (``paper_1301_0191_amd.Handle`` of the mesh), F (float64 CUDA tensor
    [nrhs, n_free], row k = right-hand side k), x_obs (same shape as F),
    rtol and maxit of the two PCG solves.  Returns J as a 0-d tensor.
    """

    @staticmethod
    def forward(ctx, theta, handle, F, x_obs, rtol=1e-10, maxit=1000):
        th = theta.detach().contiguous().clone()
        handle.setup_log10(th)
        X = handle.solve(F, rtol=rtol, maxit=maxit).x
        J, R = handle.misfit(X, x_obs)
        ctx.save_for_backward(X, R, th)
        ctx.handle = handle
        ctx.setup_count = handle.setup_count
        ctx.rtol = rtol
        ctx.maxit = maxit
        return theta.new_tensor(J)

    @staticmethod
    def backward(ctx, grad_J):
        X, R, th = ctx.saved_tensors
        h = ctx.handle
        if h.setup_count != ctx.setup_count:
            # the handle now holds another set-up: restore the forward's
            h.setup_log10(th)
            ctx.setup_count = h.setup_count
        Lam = h.solve(R, rtol=ctx.rtol, maxit=ctx.maxit).x
        g = h.element_gradient(X, Lam)
        return g * grad_J, None, None, None, None, None


def misfit(theta, handle, F, x_obs, rtol=1e-10, maxit=1000):
    """J(theta) with autograd support (see ``BddcMisfit``)."""
    return BddcMisfit.apply(theta, handle, F, x_obs, rtol, maxit)
