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


def gpu_solve(h, rhs, rtol=1e-10, maxit=2000, raise_on_noconv=True):
    torch = torch_cuda()
    r = torch.from_numpy(np.ascontiguousarray(np.asarray(rhs).reshape(rhs.shape[0], -1).T)).to("cuda:0")
    res = h.solve(r, rtol=rtol, maxit=maxit, raise_on_noconv=raise_on_noconv)
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


def check_pair(h, level, p, L, r, prob, log=None, **okw):
    """One pair eigenproblem of the library against the oracle's dense solve
    ``r`` (pair_eigenproblem on the oracle level ``L``; ``okw`` are the
    options it was solved with: keep_edges, fixed).

    * the first nsel+1 eigenvalues: 1e-6 relative (eigenvalues that vanish in
      exact arithmetic, i.e. pairs with few shared DOFs, are rounding noise on
      both sides and compared to 1e-10 lambda_1; every eigenvalue within a
      decade of tau, which decides the selection, strictly relative);
    * the selected count and the first unselected eigenvalue;
    * the constraint rows: the support DOFs are identical, the rows
      orthonormal, and their span equals the oracle's (sine of the largest
      principal angle <= 1e-6, or 1e-7 / gap when the relative eigenvalue
      gap at the cut is below 0.1: the eigenvectors of a residual-1e-7
      LOBPCG are only that accurate), times the amplification
      ||c|| / sigma_min(face rows of c) of the face restriction, times 10 on
      level >= 2 (operators built from level-1 results).  Where the selection cuts a cluster of
      eigenvalues (relative gap <= 1e-3 at the cut) only the span of the
      whole cluster is fixed: then the rows must lie inside the span of the
      oracle's rows built from every eigenvector up to the cluster's end.
    Returns the selected count."""
    from oracle.adaptive import pair_eigenproblem
    s, t, g = L.pairs[p]
    assert h.pair_info(level, p)[:2] == (s, t)
    gp = h.pair_result(level, p)
    assert gp["converged"], (level, p, gp["resid"])
    nsel = okw.get("fixed") or prob.nev_max
    kk = min(nsel + 1, len(r["lam"]))
    lam_o = r["lam"][:kk]
    err = np.abs(gp["lam"][:kk] - lam_o)
    ok = err <= np.maximum(1e-6 * np.abs(lam_o), 1e-10 * abs(lam_o[0]))
    assert ok.all(), (level, p, err, lam_o)
    near = lam_o >= 0.1 * prob.tau
    if near.any() and not okw.get("fixed"):
        strict = np.abs(gp["lam"][:kk] - lam_o)[near] / lam_o[near]
        assert strict.max() <= 1e-6, (level, p, strict.max())
    assert gp["k"] == len(r["rows"]), (level, p, gp["k"], len(r["rows"]))
    if r["lam_next"] > 0:
        assert gp["lam_next"] == pytest.approx(r["lam_next"], rel=1e-6)
    if gp["k"] > 0:
        rows, fd = h.face_constraints(level, p, gp["k"])
        np.testing.assert_array_equal(fd, r["face_dofs"])
        np.testing.assert_allclose(rows @ rows.T, np.eye(gp["k"]), atol=1e-10)
        lam = r["lam"]
        k = r["k"]
        gap = (lam[k - 1] - lam[k]) / lam[k - 1] if k < len(lam) else 1.0
        if gap > 1e-3:
            # an eigenvector converged to relative residual 1e-7 is accurate
            # to about 1e-7 / gap: the spans agree to 1e-6 unless the gap at
            # the cut is below 0.1.  On level >= 2 the pair operators are
            # assembled from level-1 coarse matrices whose constraint rows
            # agree with the oracle's to 1e-6, ten times that.
            # The rows span the face restriction F of the vectors c_l: an error
            # e ||c|| in c turns the span by about e ||c|| / sigma_min(F).
            from oracle.adaptive import pair_operators
            Gs = pair_operators(L, s, t)["Gs"]
            F = r["c_full"][np.searchsorted(Gs, r["face_dofs"])]
            sv = np.linalg.svd(F, compute_uv=False)
            amp = max(1.0, np.linalg.norm(r["c_full"], 2) / max(sv[len(r["rows"]) - 1], 1e-300))
            tol = max(1e-6, 1e-7 / gap) * (10.0 if level > 0 else 1.0) * amp
            sg = subspace_gap(rows, r["rows"])
            if amp > 10 and log:
                log(f"  pair {p}: face rows amplify errors of c by {amp:.1e}; span tolerance {tol:.1e}")
            assert sg <= tol, (level, p, gap, sg, amp)
        else:
            j = k
            while j < len(lam) and lam[j - 1] - lam[j] <= 1e-3 * lam[j - 1]:
                j += 1
            rc = pair_eigenproblem(L, s, t, L.globs[g], prob.tau, prob.nev_max, span_upto=j,
                                   **okw)
            Q = rc["span_rows"]
            out = rows.T - Q.T @ (Q @ rows.T)
            if log:
                log(f"  pair {p}: selection cuts a cluster (gap {gap:.1e}), rows checked "
                    f"against the span of {j} eigenvectors")
            assert np.abs(out).max() <= 1e-6, (level, p, np.abs(out).max())
    return gp["k"]


_FLOORS = {}


def residual_floor(key, prob):
    """||f - K x|| / ||f|| (FP64, per column, max) of the oracle's sparse direct
    solution: what an FP64 solution of this system attains, as measured by
    the same residual formula the tests use."""
    if key not in _FLOORS:
        import oracle as O
        from oracle import fem
        K = fem.assemble_global(prob)
        xd = O.direct_solve(prob)
        f = prob.rhs
        _FLOORS[key] = float((np.linalg.norm(f - K @ xd.reshape(f.shape), axis=0) /
                              np.linalg.norm(f, axis=0)).max())
    return _FLOORS[key]
