"""Failure handling of the library through the C ABI.  Every case runs a
fixed code path whose kernels finish normally; the error is detected on the
host from what they computed (or from the allocation), never by a fault.

* E_ASSUMPTION: a subdomain made of two disconnected blocks (the spurious
  mechanisms Section 8 warns about) whose blocks each touch one edge: every
  constrained Neumann problem is nonsingular, but on the pair of that
  subdomain with a clamped neighbour the pair coarse matrix keeps the
  constant of the block the neighbour does not touch as a null vector, so
  Assumption 1 (Section 4) fails.  The oracle agrees (its pair problem has a
  singular B there), and the message names the pair.
* E_INVALID_ARG for a coefficient that is not a number, or a Poisson ratio
  of 1/2, naming the element.
* LOBPCG stopped at one iteration: not an error; the unconverged pairs are
  counted and the set-up still gives a preconditioner with which PCG
  converges.
* E_OOM: a two-subdomain problem whose dense subdomain blocks would need
  over a terabyte; the handle is not created and the library stays usable.
"""
import numpy as np
import pytest

import workloads as W
from oracle.adaptive import pair_eigenproblem
from oracle.substructure import build_level, level1_input
from gpu_common import gpu_handle, gpu_solve, torch_cuda

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


def disconnected_problem():
    """6 x 4 x 1 elements: the bottom row of 2 x 2 blocks is subdomains
    0 | 1 | 0 (subdomain 0 in two pieces), the top row 2 | 3 | 4, clamped on
    the top face."""
    prob = W.make_problem((6, 4, 1), None, cuts=[[0, 2, 4, 6], [0, 2, 4], [0, 1]], seed=1)
    remap = np.array([0, 1, 0, 2, 3, 4])
    e2s = remap[prob.elem_to_sub].astype(np.int32)
    dm = W.dirichlet_face(prob.coords, 1, 1, 1.0)
    nfree = int(np.count_nonzero(dm == 0))
    return W._finish("disconnected", prob.shape, prob.coords, prob.elem_nodes, 1, prob.coeff,
                     None, e2s, [], dm, np.ones((nfree, 1)), levels=2, tau=10.0)


def test_assumption_failure_is_reported():
    log("CASE E_ASSUMPTION")
    torch = torch_cuda()
    from paper_1301_0191_amd import AmbddcError, Handle
    prob = disconnected_problem()
    L = build_level(level1_input(prob))
    with pytest.raises(AssertionError, match="Assumption 1"):
        s, t, g = L.pairs[1]
        assert (s, t) == (0, 2)
        pair_eigenproblem(L, s, t, L.globs[g], prob.tau, prob.nev_max)
    h = Handle.from_problem(prob)
    with pytest.raises(AmbddcError, match=r"E_ASSUMPTION.*pair \(0,[24]\)"):
        h.setup(torch.from_numpy(prob.coeff).to("cuda:0"))
    # the same handle without adaptivity: no pair problems, no error
    h.close()
    h = gpu_handle(prob, tau=0.0)
    X, its, cond = gpu_solve(h, prob.rhs, rtol=1e-10)
    assert its[0] > 0
    h.close()


def test_bad_coefficients_are_rejected():
    log("CASE E_INVALID_ARG coefficients")
    torch = torch_cuda()
    from paper_1301_0191_amd import AmbddcError, Handle
    prob = W.tiny_poisson(shape=(4, 4, 4), subs=(2, 2, 2), seed=0)
    h = Handle.from_problem(prob)
    c = prob.coeff.copy()
    c[5] = np.nan
    with pytest.raises(AmbddcError, match="E_INVALID_ARG.*element 5 "):
        h.setup(torch.from_numpy(c).to("cuda:0"))
    c = prob.coeff.copy()
    c[7] = np.inf
    with pytest.raises(AmbddcError, match="E_INVALID_ARG.*element 7 "):
        h.setup(torch.from_numpy(c).to("cuda:0"))
    h.setup(torch.from_numpy(prob.coeff).to("cuda:0"))
    h.close()
    pe = W.tiny_elasticity(shape=(4, 4, 4), subs=(2, 2, 2), seed=1)
    h = Handle.from_problem(pe)
    nu = pe.nu.copy()
    nu[3] = 0.5
    with pytest.raises(AmbddcError, match="E_INVALID_ARG.*element 3 "):
        h.setup(torch.from_numpy(pe.coeff).to("cuda:0"), torch.from_numpy(nu).to("cuda:0"))
    h.close()


def test_lobpcg_iteration_cap_counts_unconverged_pairs():
    log("CASE LOBPCG maxit 1")
    prob = W.tiny_poisson(shape=(8, 8, 8), subs=(2, 2, 2), seed=1)
    h = gpu_handle(prob, lobpcg_maxit=1)
    st = h.stats()
    log("  stats", st["n_unconverged"], st["lobpcg_iters"], st["n_adaptive"])
    assert st["lobpcg_iters"][0] == 1
    assert st["n_unconverged"][0] > 0
    conv = [h.pair_result(0, p)["converged"] for p in range(st["n_pairs"][0])]
    assert sum(not c for c in conv) == st["n_unconverged"][0]
    X, its, cond = gpu_solve(h, prob.rhs, rtol=1e-10)
    import oracle as O
    xd = O.direct_solve(prob)
    assert np.linalg.norm(X - xd) <= 1e-8 * np.linalg.norm(xd)
    h.close()


def test_oversized_problem_reports_oom():
    log("CASE E_OOM")
    torch_cuda()
    from paper_1301_0191_amd import AmbddcError, Handle
    prob = W.make_problem((120, 60, 60), (2, 1, 1), seed=0)   # 2 x 412 GB dense blocks
    with pytest.raises(AmbddcError, match="E_OOM"):
        Handle.from_problem(prob)
    # the library is still usable afterwards
    small = W.tiny_poisson(shape=(4, 4, 4), subs=(2, 2, 2), seed=0)
    h = gpu_handle(small)
    X, its, cond = gpu_solve(h, small.rhs, rtol=1e-10)
    assert its[0] > 0
    h.close()
