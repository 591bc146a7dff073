"""Gradient of a least-squares misfit w.r.t. element log10-coefficients (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Not part of the paper: K(theta) = sum_e 10^theta_e K_hat_e, x_k = K^{-1} f_k,
J = 1/2 sum_k ||x_k - x_obs,k||^2.  The adjoint lambda_k = K^{-1}(x_k - x_obs,k)
(K symmetric) gives dJ/dtheta_e = -ln(10) 10^theta_e sum_k lambda_k,e^T K_hat_e x_k,e,
where the element vectors carry zeros at Dirichlet DOFs.  Direct sparse
solves are used, so this is the exact-arithmetic gradient.
"""
from __future__ import annotations

import numpy as np

from . import fem
from .bddc import direct_solve


def misfit_gradient(prob, theta, x_obs, F=None):
    """Return (J, grad, X, Lam) for element log-coefficients theta."""
    kappa = 10.0 ** np.asarray(theta, dtype=np.float64)
    Ke = fem.element_matrices(prob, kappa)
    F = prob.rhs if F is None else F
    X = direct_solve(prob, F, Ke)
    Rm = X - x_obs
    J = 0.5 * float(np.sum(Rm * Rm))
    Lam = direct_solve(prob, Rm, Ke)
    fmap = fem.free_map(prob)
    ed = fmap[fem.elem_dof_ids(prob)]
    nrhs = X.shape[1]
    Xf = np.vstack([X, np.zeros((1, nrhs))])      # index -1 -> zero row
    Lf = np.vstack([Lam, np.zeros((1, nrhs))])
    xe = Xf[ed]                                    # (ne, m, nrhs)
    le = Lf[ed]
    g = -np.log(10.0) * np.einsum("emk,emn,enk->e", le, Ke, xe)
    return J, g, X, Lam
