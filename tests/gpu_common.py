"""Helpers shared by the GPU tests: run a workload through the C ABI and
compare with the oracle (test infrastructure)."""
import numpy as np
import pytest


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def gpu_handle(prob, **kw):
    torch = torch_cuda()
    from paper_1301_0191_amd import Handle
    h = Handle.from_problem(prob, **kw)
    dev = torch.device("cuda:0")
    coeff = torch.from_numpy(np.ascontiguousarray(prob.coeff)).to(dev)
    nu = None if prob.nu is None else torch.from_numpy(np.ascontiguousarray(prob.nu)).to(dev)
    h.setup(coeff, nu)
    return h


def gpu_solve(h, rhs, rtol=1e-10, maxit=2000):
    torch = torch_cuda()
    r = torch.from_numpy(np.ascontiguousarray(np.asarray(rhs).reshape(rhs.shape[0], -1).T)).to("cuda:0")
    res = h.solve(r, rtol=rtol, maxit=maxit)
    torch.cuda.synchronize()
    return res.x.cpu().numpy().T, res.iterations, res.cond


def subspace_gap(A, B):
    """Sine of the largest principal angle between the row spaces of A and B."""
    if A.shape[0] == 0 and B.shape[0] == 0:
        return 0.0
    qa, _ = np.linalg.qr(A.T)
    qb, _ = np.linalg.qr(B.T)
    s = np.linalg.svd(qa.T @ qb, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - s.min() ** 2)))
