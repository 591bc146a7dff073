"""GPU parity of the FP32 forms against the FP64 oracle: precision 1 (the
PCG preconditioner's dense subdomain operators stored in FP32, widened to
FP64 on load) and precision 2 (also the pair LOBPCG's operator products in
FP32 with FP32 MFMA accumulation until each pair reaches residual 1e-5,
then FP64 polish to the FP64 tolerance).

Every result the oracle fixes keeps the FP64 bar: pair eigenvalues 1e-6 relative, identical selected counts and
constraint spans (the adaptive set-up is FP64 in both modes), solution 1e-10
relative to a direct solve after PCG to rtol 1e-10 on the true residual,
which the library recomputes before it stops.  The PCG iteration count and condition estimate follow the
oracle's FP64 preconditioner within 2 iterations and 1e-3 relative (the FP32
rounding perturbs the preconditioner by about 6e-8 of its norm).
"""
import numpy as np
import pytest

import workloads as W
import oracle as O
from gpu_common import gpu_handle, gpu_solve, residual_floor
from test_gpu_parity import TINY, check_pairs, oracle_hierarchy

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("precision", [1, 2])
@pytest.mark.parametrize("case", ["poisson_ragged", "elasticity", "c1", "c2"])
def test_fp32_preconditioner_parity(case, precision):
    log("CASE precision", precision, case)
    prob = TINY[case]() if case in TINY else W.CONFIGS[case](0)
    h = gpu_handle(prob, precision=precision)
    assert h.precision == precision
    H = oracle_hierarchy(case, prob)
    st = h.stats()
    assert st["n_adaptive"][0] == H.stats["n_adaptive"][0]
    assert st["n_coarse"][0] == H.stats["n_coarse"][0]
    assert st["omega_tilde"][0] == pytest.approx(H.stats["omega"][0], rel=1e-6)
    check_pairs(h, prob, H)
    log("  LOBPCG iterations", st["lobpcg_iters"], "of them with FP32 products",
        st["lobpcg_iters_fp32"])
    if precision == 2:
        assert st["lobpcg_iters_fp32"][0] > 0
    else:
        assert st["lobpcg_iters_fp32"][0] == 0
    torch = pytest.importorskip("torch")
    F = torch.from_numpy(np.ascontiguousarray(prob.rhs.reshape(prob.rhs.shape[0], -1).T)).to("cuda:0")
    res = h.solve(F, rtol=1e-10, raise_on_noconv=False)
    X = res.x.cpu().numpy().T
    Xo, ito, co, _ = O.solve_problem(prob, rtol=1e-10, H=H, start="interior")
    xd = O.direct_solve(prob).reshape(X.shape)
    err = np.linalg.norm(X - xd) / np.linalg.norm(xd)
    log("  its", res.iterations, "oracle", ito, "cond", res.cond, co, "err", err,
        "true residual", res.true_residual)
    if h.stats()["pcg_stalled"]:
        # rtol below what FP64 attains on this system (C1): within 2x of the
        # true residual of the oracle's direct solution, and the error
        # between two FP64 solutions of so ill-conditioned a system
        assert max(res.true_residual) <= 2 * residual_floor(case, prob)
        assert err <= 3e-10
        h.close()
        return
    assert err <= 1e-10
    assert max(res.true_residual) <= 1e-10
    assert abs(res.iterations[0] - ito[0]) <= 2
    assert res.cond[0] == pytest.approx(co[0], rel=1e-3)
    h.close()


@pytest.mark.parametrize("nrhs", [1, 3, 4, 16])
def test_fp32_preconditioner_multiple_rhs(nrhs):
    """GEMV (nrhs < 4) and MFMA GEMM (nrhs >= 4) applications of the FP32
    operators, three levels, lockstep columns against a single solve."""
    log("CASE precision 1 multi-rhs", nrhs)
    prob = W.make_problem((8, 8, 8), (4, 4, 4), group=(2, 2, 2), coeff="lognormal", seed=11,
                          rhs="normal", nrhs=nrhs)
    h = gpu_handle(prob, precision=1)
    X, its, cond = gpu_solve(h, prob.rhs, rtol=1e-10)
    xd = O.direct_solve(prob).reshape(X.shape)
    for j in range(nrhs):
        assert np.linalg.norm(X[:, j] - xd[:, j]) <= 1e-10 * np.linalg.norm(xd[:, j]), j
    # a single solve applies the operators as GEMVs, the lockstep solve from 4
    # columns on as MFMA GEMMs: the same FP32 operands, FP64 sums in another
    # order, so the stopping test may fall one iteration apart
    x1, it1, c1 = gpu_solve(h, prob.rhs.reshape(prob.rhs.shape[0], -1)[:, -1:], rtol=1e-10)
    assert abs(it1[0] - its[-1]) <= 1
    assert np.linalg.norm(X[:, -1] - x1[:, 0]) <= 1e-10 * np.linalg.norm(x1)
    h.close()


def test_fp32_and_fp64_handles_agree():
    """Both precisions on one workload: identical adaptive selection, the same
    solution to 1e-10, iteration counts within 1."""
    log("CASE precision 0 vs 1")
    prob = W.tiny_poisson(shape=(8, 8, 8), subs=(2, 2, 2), seed=7, rhs="normal", nrhs=2)
    h0 = gpu_handle(prob, precision=0)
    h1 = gpu_handle(prob, precision=1)
    s0, s1 = h0.stats(), h1.stats()
    assert s0["n_adaptive"] == s1["n_adaptive"]
    assert s0["n_coarse"] == s1["n_coarse"]
    X0, its0, _ = gpu_solve(h0, prob.rhs, rtol=1e-10)
    X1, its1, _ = gpu_solve(h1, prob.rhs, rtol=1e-10)
    assert np.linalg.norm(X1 - X0) <= 1e-10 * np.linalg.norm(X0)
    assert max(abs(a - b) for a, b in zip(its0, its1)) <= 1
    h0.close()
    h1.close()
