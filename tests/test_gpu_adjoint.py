"""GPU adjoint gradient (autograd.Function over the library) against the
FP64 oracle, central finite differences and the scaling identity.

Workload C5: Poisson 32^3, 4x4x4 subdomains, theta ~ N(2,1) per element,
8 unit point sources; x_obs from the perturbed theta_obs by the oracle's
direct solve.  Tolerances: J and the gradient within 1e-8 (relative to
max|g|) of the oracle's direct-solve gradient (PCG at rtol 1e-11), with the FP64 preconditioner
and with its operators stored in FP32 (PCG on FP64 residuals refines the
solutions to the same accuracy); central
differences (h = 1e-4, the GPU solver at rtol 1e-11) within 1e-4 relative
plus 1e-6 max|g| absolute; the scaling identity
sum_e g_e = -ln10 sum_k (x_k - x_obs,k)^T x_k, exact since
K(theta + c) = 10^c K(theta), within 1e-9 relative.
"""
import numpy as np
import pytest

import workloads as W
import oracle as O
from gpu_common import torch_cuda

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


_CASES = {}


def _case(name):
    if name in _CASES:
        return _CASES[name]
    if name == "c5":
        prob = W.CONFIGS["c5"](0)
        theta = prob.extra["theta"]
        theta_obs = prob.extra["theta_obs"]
        fd = prob.extra["fd_elems"]
    else:
        prob = W.make_problem((8, 8, 8), (2, 2, 2), seed=21)
        rng = np.random.default_rng(21)
        theta = rng.normal(0.5, 0.7, prob.n_elems)
        theta_obs = theta + 0.1 * rng.standard_normal(prob.n_elems)
        F = np.zeros((prob.n_free, 3))
        F[rng.choice(prob.n_free, 3, replace=False), np.arange(3)] = 1.0
        prob.rhs = F
        fd = rng.choice(prob.n_elems, 8, replace=False)
    from oracle import fem
    x_obs = O.direct_solve(prob, prob.rhs, fem.element_matrices(prob, 10.0 ** theta_obs))
    J, g, X, Lam = O.misfit_gradient(prob, theta, x_obs, prob.rhs)
    _CASES[name] = (prob, theta, x_obs, fd, J, g, X)
    return _CASES[name]


def _gpu(prob, precision=0):
    torch = torch_cuda()
    from paper_1301_0191_amd import Handle
    h = Handle.from_problem(prob, precision=precision)
    dev = torch.device("cuda:0")
    F = torch.from_numpy(np.ascontiguousarray(prob.rhs.T)).to(dev)
    return torch, h, dev, F


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", ["tiny", "c5"])
def test_autograd_gradient_matches_oracle(name, precision):
    log("CASE adjoint vs oracle", name, "precision", precision)
    prob, theta, x_obs, fd, J_or, g_or, X_or = _case(name)
    torch, h, dev, F = _gpu(prob, precision)
    from paper_1301_0191_amd.adjoint import misfit
    th = torch.from_numpy(theta).to(dev).requires_grad_(True)
    xo = torch.from_numpy(np.ascontiguousarray(x_obs.T)).to(dev)
    J = misfit(th, h, F, xo, rtol=1e-11)
    J.backward()
    g = th.grad.cpu().numpy()
    log("  J", float(J.detach()), J_or, " max|g|", np.abs(g_or).max())
    assert float(J) == pytest.approx(J_or, rel=1e-9)
    assert np.abs(g - g_or).max() <= 1e-8 * np.abs(g_or).max()
    h.close()


def test_gradient_central_differences_c5():
    log("CASE adjoint finite differences c5")
    prob, theta, x_obs, fd, J_or, g_or, X_or = _case("c5")
    torch, h, dev, F = _gpu(prob)
    from paper_1301_0191_amd.adjoint import misfit
    xo = torch.from_numpy(np.ascontiguousarray(x_obs.T)).to(dev)
    th = torch.from_numpy(theta).to(dev).requires_grad_(True)
    J = misfit(th, h, F, xo, rtol=1e-11)
    J.backward()
    g = th.grad.cpu().numpy()
    gmax = np.abs(g).max()
    step = 1e-4
    for e in fd:
        tp = theta.copy()
        tp[e] += step
        tm = theta.copy()
        tm[e] -= step
        Jp = float(misfit(torch.from_numpy(tp).to(dev), h, F, xo, rtol=1e-11))
        Jm = float(misfit(torch.from_numpy(tm).to(dev), h, F, xo, rtol=1e-11))
        d = (Jp - Jm) / (2 * step)
        assert abs(d - g[e]) <= 1e-4 * abs(g[e]) + 1e-6 * gmax, (e, d, g[e])
    h.close()


def test_gradient_scaling_identity_c5():
    log("CASE adjoint scaling identity c5")
    prob, theta, x_obs, fd, J_or, g_or, X_or = _case("c5")
    torch, h, dev, F = _gpu(prob)
    xo = torch.from_numpy(np.ascontiguousarray(x_obs.T)).to(dev)
    h.setup_log10(torch.from_numpy(theta).to(dev))
    X = h.solve(F, rtol=1e-11).x
    J, R = h.misfit(X, xo)
    Lam = h.solve(R, rtol=1e-11).x
    g = h.element_gradient(X, Lam).cpu().numpy()
    Xh, Rh = X.cpu().numpy(), R.cpu().numpy()
    assert np.abs(Rh - (Xh - x_obs.T)).max() == 0.0
    assert J == pytest.approx(0.5 * float(np.sum(Rh * Rh)), rel=1e-12)
    rhs = -np.log(10.0) * float(np.sum(Rh * Xh))
    assert float(np.sum(g)) == pytest.approx(rhs, rel=1e-9)
    h.close()


def test_backward_after_another_forward_on_the_same_handle():
    """The handle is set up at theta2 between forward(theta1) and backward:
    the gradient must still be the one at theta1."""
    log("CASE adjoint, interleaved forward")
    prob, theta, x_obs, fd, J_or, g_or, X_or = _case("tiny")
    torch, h, dev, F = _gpu(prob)
    from paper_1301_0191_amd.adjoint import misfit
    xo = torch.from_numpy(np.ascontiguousarray(x_obs.T)).to(dev)
    th1 = torch.from_numpy(theta).to(dev).requires_grad_(True)
    J1 = misfit(th1, h, F, xo, rtol=1e-11)
    th2 = torch.from_numpy(theta + 0.3).to(dev).requires_grad_(True)
    J2 = misfit(th2, h, F, xo, rtol=1e-11)
    J1.backward()
    g = th1.grad.cpu().numpy()
    assert float(J1) == pytest.approx(J_or, rel=1e-9)
    assert float(J2) != pytest.approx(J_or, rel=1e-3)
    assert np.abs(g - g_or).max() <= 1e-8 * np.abs(g_or).max()
    h.close()
