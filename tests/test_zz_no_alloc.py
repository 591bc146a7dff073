"""ambddc_solve_noalloc (the solve whose scratch is a fixed device array)
against ambddc_solve through the C ABI: the same kernels in the same order,
so the iterations, condition estimates and true residuals are identical and
the solutions agree to rounding (1e-13 relative, far inside the 1e-10 bar).
Two calls in a row share the array, the second with a smaller problem; the
limits are rejected with E_INVALID_ARG."""
import numpy as np
import pytest

import workloads as W
from gpu_common import gpu_handle, torch_cuda

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


def _rhs(torch, prob):
    return torch.from_numpy(np.ascontiguousarray(prob.rhs.T)).to("cuda:0")


def _compare(a, b):
    assert a.iterations == b.iterations
    np.testing.assert_allclose(a.cond, b.cond, rtol=1e-12)
    np.testing.assert_allclose(a.true_residual, b.true_residual, rtol=1e-6, atol=1e-15)
    xa, xb = a.x.cpu().numpy(), b.x.cpu().numpy()
    assert np.abs(xa - xb).max() <= 1e-13 * np.abs(xb).max()


def test_noalloc_solve_matches_solve():
    log("CASE no-alloc solve")
    torch = torch_cuda()
    from paper_1301_0191_amd import AmbddcError
    big = W.tiny_poisson(shape=(8, 8, 8), subs=(2, 2, 2), seed=3, rhs="normal", nrhs=3)
    small = W.tiny_elasticity(shape=(4, 4, 4), subs=(2, 2, 2), seed=4)
    assert small.n_free * 1 < big.n_free * 3
    ha = gpu_handle(big)
    hb = gpu_handle(small)
    Fa, Fb = _rhs(torch, big), _rhs(torch, small)
    # before the handle has a 3-column workspace
    with pytest.raises(AmbddcError, match="E_INVALID_ARG.*workspace"):
        ha.solve_noalloc(Fa, torch.empty_like(Fa), rtol=1e-10)
    ref_a = ha.solve(Fa, rtol=1e-10)          # prepares three columns
    got_a = ha.solve_noalloc(Fa, torch.empty_like(Fa), rtol=1e-10)
    log("  a: its", got_a.iterations, "cond", got_a.cond)
    _compare(got_a, ref_a)
    got_b = hb.solve_noalloc(Fb, torch.empty_like(Fb), rtol=1e-10)
    ref_b = hb.solve(Fb, rtol=1e-10)
    log("  b: its", got_b.iterations, "cond", got_b.cond)
    _compare(got_b, ref_b)
    # and once more on the first handle after the smaller call
    again = ha.solve_noalloc(Fa, torch.empty_like(Fa), rtol=1e-10)
    _compare(again, ref_a)
    with pytest.raises(AmbddcError, match="E_INVALID_ARG.*1 to 3"):
        F4 = torch.cat([Fa, Fa[:1]], 0)
        ha.solve_noalloc(F4, torch.empty_like(F4))
    with pytest.raises(AmbddcError, match="E_INVALID_ARG.*bytes of scratch"):
        ha.solve_noalloc(Fa, torch.empty_like(Fa), maxit=10_000_000)
    ha.close()
    hb.close()
