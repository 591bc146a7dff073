"""Pins of the oracle's misfit gradient.

* central finite differences of J in single element log-coefficients;
* the scaling identity: K(theta + c) = 10^c K(theta) gives
  sum_e dJ/dtheta_e = -ln(10) sum_k (x_k - x_obs,k)^T x_k exactly.
"""
import numpy as np
import pytest

import workloads as W
from oracle.adjoint import misfit_gradient
from oracle.bddc import direct_solve
from oracle import fem


@pytest.fixture(scope="module")
def adj_case():
    prob = W.make_problem((6, 6, 6), (2, 2, 2), seed=21)
    rng = np.random.default_rng(21)
    theta = rng.normal(0.5, 0.7, prob.n_elems)
    nfree = prob.n_free
    F = np.zeros((nfree, 3))
    F[rng.choice(nfree, 3, replace=False), np.arange(3)] = 1.0
    theta_obs = theta + 0.1 * rng.standard_normal(prob.n_elems)
    x_obs = direct_solve(prob, F, fem.element_matrices(prob, 10.0 ** theta_obs))
    return prob, theta, x_obs, F


def test_gradient_central_differences(adj_case):
    prob, theta, x_obs, F = adj_case
    J, g, X, Lam = misfit_gradient(prob, theta, x_obs, F)
    h = 1e-4
    for e in np.random.default_rng(0).choice(prob.n_elems, 8, replace=False):
        tp = theta.copy(); tp[e] += h
        tm = theta.copy(); tm[e] -= h
        Jp = misfit_gradient(prob, tp, x_obs, F)[0]
        Jm = misfit_gradient(prob, tm, x_obs, F)[0]
        fd = (Jp - Jm) / (2 * h)
        assert fd == pytest.approx(g[e], rel=1e-5, abs=1e-8 * np.abs(g).max())


def test_gradient_scaling_identity(adj_case):
    prob, theta, x_obs, F = adj_case
    J, g, X, Lam = misfit_gradient(prob, theta, x_obs, F)
    expect = -np.log(10.0) * np.sum((X - x_obs) * X)
    assert g.sum() == pytest.approx(expect, rel=1e-10)
