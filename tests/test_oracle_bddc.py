"""Pins of the oracle's pair eigenproblems, multilevel BDDC and PCG.

* Two subdomains that both touch the Dirichlet boundary share one face and
  nothing else, so the pair problem *is* the global problem (Section 4):
  by Cor. 1 and Lemma 1 the largest eigenvalue of the BDDC-preconditioned
  operator equals the largest pair eigenvalue, and after adding the k
  adaptive constraints it equals lambda_{k+1}.
* Lemma 1: kappa <= prod_i omega_i with omega_i from eq. def-omega,
  computed here by brute force on the whole level (not per pair).
* Pair problem: lambda >= 0, lambda_max >= 1 (norm of a nontrivial
  projection), null(B) inside null(A), Prop. 1 (the constraint row is
  [c^s, -c^s] supported on Gamma^st), and the eigenvalues agree with an
  independent regularised-pencil computation that never forms null(D).
* PCG with BDDC: solution equals the direct solve, lambda_min(M K) >= 1,
  one subdomain gives the exact inverse, the Lanczos estimate agrees with
  the dense spectrum of M K.
* PCG from the level-1 interior solution x0 = [K_II^-1 f_I; 0]: the residual
  is zero on the interiors, Alg. 1 maps it to a discrete harmonic correction
  (K z zero on the interiors, Section 2) without a pre-correction, every
  PCG residual stays zero there, the solution equals the direct solve, the
  iteration count is that of x0 = 0 within two, the Lanczos estimate is a
  lower bound of the dense spectrum's condition number within 1%, and one
  subdomain needs no iteration (x0 is the solution).
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import fem
from oracle.adaptive import enrich_level, pair_eigenproblem, pair_operators, pair_rigid
from oracle.bddc import (bddc_apply, direct_solve, interior_solution, lanczos_cond, pcg,
                         setup_hierarchy, solve_problem)
from oracle.substructure import build_level, level1_input, coarse_basis


def dense_preconditioned(H):
    K = H.levels[0].Kglob.toarray()
    n = K.shape[0]
    M = np.column_stack([bddc_apply(H, e) for e in np.eye(n)])
    M = 0.5 * (M + M.T)
    ev = np.sort(np.real(sla.eigvals(M @ K)))
    return K, M, ev


def global_omega(L):
    """sup over W~ of ||(I-P) E w||_a^2 / ||w||_a^2 on one level (brute force)."""
    nsub = L.inp.n_sub
    offs = np.cumsum([0] + L.n_G)
    m = offs[-1]
    n = L.inp.n_dof
    Sb = np.zeros((m, m))
    RE = np.zeros((m, m))
    Rt = np.zeros((m, n))
    Ew = np.zeros((n, m))
    for s in range(nsub):
        G = L.sub_dofs[s][L.n_I[s]:]
        sl = slice(offs[s], offs[s + 1])
        Sb[sl, sl] = L.S[s]
        Rt[offs[s] + np.arange(len(G)), G] = 1.0
        Ew[G, offs[s] + np.arange(len(G))] = L.weights[s]
    RE = Rt @ Ew
    # W~: coarse DOFs agree between all subdomains sharing them
    rows = []
    for cid in range(L.n_coarse):
        owners = [(s, np.flatnonzero(L.Rc[s] == cid)[0]) for s in range(nsub)
                  if np.any(L.Rc[s] == cid)]
        s0, r0 = owners[0]
        for s1, r1 in owners[1:]:
            row = np.zeros(m)
            row[offs[s0]:offs[s0 + 1]] += L.C[s0][r0]
            row[offs[s1]:offs[s1 + 1]] -= L.C[s1][r1]
            rows.append(row)
    Q = sla.null_space(np.array(rows)) if rows else np.eye(m)
    A = Q.T @ RE.T @ Sb @ RE @ Q
    B = Q.T @ Sb @ Q
    return float(sla.eigh(0.5 * (A + A.T), 0.5 * (B + B.T), eigvals_only=True)[-1])


@pytest.fixture(scope="module")
def two_sub():
    return W.make_problem((6, 8, 5), (1, 2, 1), coeff="lognormal", seed=4, tau=2.0)


def test_two_subdomains_cor1_equality(two_sub):
    prob = two_sub
    # non-adaptive: lambda_max(MK) = lambda_1 of the (global = pair) problem
    H0 = setup_hierarchy(prob, adaptive=False)
    L0 = H0.levels[0]
    assert len(L0.pairs) == 1 and L0.n_coarse == 0
    s, t, g = L0.pairs[0]
    res = pair_eigenproblem(L0, s, t, L0.globs[g], prob.tau, prob.nev_max)
    _, _, ev0 = dense_preconditioned(H0)
    assert ev0[0] >= 1.0 - 1e-9
    assert ev0[-1] == pytest.approx(res["lam"][0], rel=1e-8)
    # adaptive: k constraints -> lambda_max(MK) = lambda_{k+1}
    H = setup_hierarchy(prob, adaptive=True)
    r = H.levels[0].adaptive["results"][0]
    assert r["k"] >= 1 and len(r["rows"]) == r["k"]
    _, _, ev = dense_preconditioned(H)
    assert ev[0] >= 1.0 - 1e-9
    assert ev[-1] == pytest.approx(max(r["lam_next"], 1.0), rel=1e-8)
    np.testing.assert_allclose(r["lam"], res["lam"], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("maker", [
    lambda: W.tiny_poisson(shape=(6, 6, 6), subs=(2, 2, 2), seed=5),
    lambda: W.tiny_elasticity(shape=(4, 4, 4), subs=(2, 2, 2), seed=6),
])
def test_lemma1_bound_two_level(maker):
    prob = maker()
    for adaptive in (False, True):
        H = setup_hierarchy(prob, adaptive=adaptive)
        _, _, ev = dense_preconditioned(H)
        omega = global_omega(H.levels[0])
        kappa = ev[-1] / ev[0]
        assert ev[0] >= 1.0 - 1e-9
        assert kappa <= omega * (1 + 1e-8)
        # BDDC attains the bound: lambda_max(MK) = omega
        assert ev[-1] == pytest.approx(omega, rel=1e-7)


def test_lemma1_bound_three_level():
    prob = W.make_problem((8, 8, 8), (4, 4, 4), group=(2, 2, 2), coeff="lognormal", seed=7)
    H = setup_hierarchy(prob, adaptive=True)
    assert len(H.levels) == 2
    _, _, ev = dense_preconditioned(H)
    assert ev[0] >= 1.0 - 1e-9
    om = [global_omega(L) for L in H.levels]
    assert ev[-1] / ev[0] <= om[0] * om[1] * (1 + 1e-8)


@pytest.fixture(scope="module")
def mixed_level():
    prob = W.tiny_elasticity(shape=(4, 4, 4), subs=(2, 2, 2), seed=8)
    L = build_level(level1_input(prob))
    return prob, L


def test_pair_problem_properties(mixed_level):
    prob, L = mixed_level
    seen_float = False
    for (s, t, g) in L.pairs:
        res = pair_eigenproblem(L, s, t, L.globs[g], 0.0, 10)
        lam = res["lam"]
        assert lam[-1] >= -1e-9 * lam[0]
        assert lam[0] >= 1.0 - 1e-10
        ops = pair_operators(L, s, t)
        A = ops["IE"].T @ ops["S"] @ ops["IE"]
        # Prop. 1: c = [c^s, -c^s] on Gamma^st, zero elsewhere
        c = res["c_full"]
        ns = ops["ns"]
        mask_s = np.zeros(ns, bool)
        mask_s[ops["is_"]] = True
        mask_t = np.zeros(ops["nt"], bool)
        mask_t[ops["it_"]] = True
        scale = np.abs(c).max()
        assert np.abs(c[:ns][~mask_s]).max(initial=0) <= 1e-12 * scale
        assert np.abs(c[ns:][~mask_t]).max(initial=0) <= 1e-12 * scale
        np.testing.assert_allclose(c[:ns][ops["is_"]], -c[ns:][ops["it_"]], atol=1e-10 * scale)
        if res["both_floating"]:
            seen_float = True
            R = pair_rigid(L, s, t, ops)
            # rigid modes: continuous coarse DOFs, energy free, A-null
            assert np.abs(ops["D"] @ R).max() < 1e-12
            assert np.abs(ops["S"] @ R).max() < 1e-9 * np.abs(ops["S"]).max()
            assert np.abs(A @ R).max() < 1e-9 * np.abs(ops["S"]).max()
        # independent pencil: (Pi A Pi, Pi S Pi + D^T D + R R^T) without null(D)
        D = ops["D"]
        n = A.shape[0]
        Pi = np.eye(n) - D.T @ np.linalg.solve(D @ D.T, D)
        Breg = Pi @ ops["S"] @ Pi + D.T @ D * np.abs(ops["S"]).max()
        if res["both_floating"]:
            R = sla.orth(pair_rigid(L, s, t, ops))
            Breg += (R @ R.T) * np.abs(ops["S"]).max()
        ev = np.sort(sla.eigh(Pi @ A @ Pi, 0.5 * (Breg + Breg.T), eigvals_only=True))[::-1]
        np.testing.assert_allclose(ev[:12], lam[:12], rtol=1e-7, atol=1e-10)
    assert seen_float


@pytest.mark.parametrize("maker,levels", [
    (lambda: W.tiny_poisson(shape=(8, 8, 8), subs=(2, 2, 2), seed=9), 2),
    (lambda: W.tiny_elasticity(shape=(4, 4, 4), subs=(2, 2, 2), seed=10), 2),
    (lambda: W.make_problem((8, 8, 8), (4, 4, 4), group=(2, 2, 2), coeff="lognormal",
                            seed=11, rhs="normal"), 3),
])
def test_pcg_solution_matches_direct(maker, levels):
    prob = maker()
    X, its, conds, H = solve_problem(prob, rtol=1e-12)
    xd = direct_solve(prob)
    assert np.linalg.norm(X - xd) / np.linalg.norm(xd) < 1e-9
    assert len(H.levels) == levels - 1


def test_adaptivity_lowers_condition():
    prob = W.tiny_poisson(shape=(8, 8, 8), subs=(2, 2, 2), seed=12, coeff="blocks")
    _, its_a, cond_a, Ha = solve_problem(prob, rtol=1e-10)
    _, its_n, cond_n, _ = solve_problem(prob, rtol=1e-10, adaptive=False)
    assert cond_a[0] < cond_n[0] and its_a[0] <= its_n[0]
    assert Ha.stats["omega"][0] <= prob.tau


def test_single_subdomain_is_exact():
    prob = W.make_problem((4, 4, 4), (1, 1, 1), coeff="lognormal", seed=13)
    X, its, conds, H = solve_problem(prob, rtol=1e-12)
    assert its[0] == 1
    np.testing.assert_allclose(X, direct_solve(prob), rtol=1e-10)


def test_lanczos_estimate_matches_dense_spectrum():
    prob = W.tiny_poisson(shape=(6, 6, 6), subs=(2, 2, 2), seed=14, coeff="blocks")
    H = setup_hierarchy(prob, adaptive=False)
    K, M, ev = dense_preconditioned(H)
    f = np.random.default_rng(0).standard_normal(K.shape[0])
    x, it, al, be, _ = pcg(H.levels[0].Kglob, f, lambda v: bddc_apply(H, v), 1e-14, 500)
    cond, lmin, lmax = lanczos_cond(al, be)
    assert lmin >= ev[0] * (1 - 1e-8) and lmax <= ev[-1] * (1 + 1e-8)
    assert cond == pytest.approx(ev[-1] / ev[0], rel=1e-3)


def _interior_mask(H):
    L = H.levels[0]
    m = np.zeros(L.inp.n_dof, dtype=bool)
    for s in range(L.inp.n_sub):
        m[L.sub_dofs[s][:L.n_I[s]]] = True
    return m


@pytest.mark.parametrize("maker", [
    lambda: W.tiny_poisson(shape=(8, 8, 8), subs=(2, 2, 2), seed=9),
    lambda: W.tiny_elasticity(shape=(4, 4, 4), subs=(2, 2, 2), seed=10),
    lambda: W.make_problem((8, 8, 8), (4, 4, 4), group=(2, 2, 2), coeff="lognormal",
                           seed=11, rhs="normal"),
])
def test_interior_start_keeps_residuals_harmonic(maker):
    prob = maker()
    H = setup_hierarchy(prob)
    K = H.levels[0].Kglob
    f = prob.rhs.reshape(prob.rhs.shape[0], -1)[:, 0]
    nf = np.linalg.norm(f)
    mI = _interior_mask(H)
    assert mI.any() and not mI.all()
    x = interior_solution(H, f)
    r = f - K @ x
    assert np.linalg.norm(r[mI]) <= 1e-12 * nf
    # Alg. 1 of a residual that is zero on the interiors: no pre-correction,
    # a discrete harmonic result
    z = bddc_apply(H, r)
    rc = r.copy()
    rc[mI] = 0.0
    np.testing.assert_allclose(bddc_apply(H, rc), z, rtol=0, atol=1e-12 * np.linalg.norm(z))
    Kz = K @ z
    assert np.linalg.norm(Kz[mI]) <= 1e-10 * np.linalg.norm(Kz)
    # CG recurrences (written out): the residuals stay zero on the interiors
    p = z.copy()
    rz = r @ z
    for _ in range(8):
        q = K @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        assert np.linalg.norm(r[mI]) <= 1e-10 * max(np.linalg.norm(r), 1e-300)
        z = bddc_apply(H, r)
        rzn = r @ z
        p = z + (rzn / rz) * p
        rz = rzn
    # the whole solve from this start
    X, its, _, _ = solve_problem(prob, rtol=1e-12, H=H, start="interior")
    xd = direct_solve(prob)
    assert np.linalg.norm(X - xd) / np.linalg.norm(xd) < 1e-9
    _, its0, _, _ = solve_problem(prob, rtol=1e-12, H=H)
    assert abs(its[0] - its0[0]) <= 2


def test_interior_start_lanczos_and_single_subdomain():
    prob = W.tiny_poisson(shape=(6, 6, 6), subs=(2, 2, 2), seed=14, coeff="blocks")
    H = setup_hierarchy(prob, adaptive=False)
    K, M, ev = dense_preconditioned(H)
    f = np.random.default_rng(0).standard_normal(K.shape[0])
    x0 = interior_solution(H, f)
    x, it, al, be, _ = pcg(H.levels[0].Kglob, f, lambda v: bddc_apply(H, v), 1e-14, 500, x0=x0)
    cond, lmin, lmax = lanczos_cond(al, be)
    assert lmin >= ev[0] * (1 - 1e-8) and lmax <= ev[-1] * (1 + 1e-8)
    assert ev[-1] / ev[0] * (1 - 1e-2) <= cond <= ev[-1] / ev[0] * (1 + 1e-8)
    one = W.make_problem((4, 4, 4), (1, 1, 1), coeff="lognormal", seed=13)
    X, its, _, _ = solve_problem(one, rtol=1e-12, start="interior")
    assert its[0] == 0
    np.testing.assert_allclose(X, direct_solve(one), rtol=1e-10)


def _explicit_alg1(H, dtype):
    """Alg. 1 on a two-level hierarchy with every subdomain operator formed
    explicitly (K_II^-1, K_GI K_II^-1, the interface block Z of the saddle
    inverse, Psi) and rounded through ``dtype``; the coarsest solve stays FP64.
    Test code: the reading that storing the PCG preconditioner's operators in
    FP32 leaves the FP64 PCG solution and iteration count unchanged."""
    L = H.levels[0]
    ops = []
    for s in range(L.inp.n_sub):
        nI = L.n_I[s]
        K = L.K[s]
        Ki = np.linalg.inv(K[:nI, :nI])
        S = K[nI:, nI:] - K[nI:, :nI] @ Ki @ K[:nI, nI:]
        C = L.C[s]
        nG, nc = S.shape[0], C.shape[0]
        M = np.zeros((nG + nc, nG + nc))
        M[:nG, :nG] = S
        M[:nG, nG:] = C.T
        M[nG:, :nG] = C
        Mi = np.linalg.inv(M)
        rnd = lambda X: X.astype(dtype).astype(np.float64)
        ops.append((rnd(Ki), rnd(K[nI:, :nI] @ Ki), rnd(Mi[:nG, :nG]), rnd(Mi[:nG, nG:]),
                    rnd(Ki @ K[:nI, nI:])))

    def apply(r):
        u = np.zeros_like(r)
        rB = r.copy()
        for s, (Ki, GKi, Z, Psi, KiIG) in enumerate(ops):
            d, nI = L.sub_dofs[s], L.n_I[s]
            u[d[:nI]] += Ki @ r[d[:nI]]
            rB[d[nI:]] -= GKi @ r[d[:nI]]
        rc = np.zeros(L.n_coarse)
        fs = []
        for s, (Ki, GKi, Z, Psi, KiIG) in enumerate(ops):
            d, nI = L.sub_dofs[s], L.n_I[s]
            f = L.weights[s] * rB[d[nI:]]
            fs.append(f)
            np.add.at(rc, L.Rc[s], Psi.T @ f)
        uc = sla.cho_solve(H.top_chol, rc)
        uB = np.zeros_like(r)
        for s, (Ki, GKi, Z, Psi, KiIG) in enumerate(ops):
            d, nI = L.sub_dofs[s], L.n_I[s]
            np.add.at(uB, d[nI:], L.weights[s] * (Z @ fs[s] + Psi @ uc[L.Rc[s]]))
        for s, (Ki, GKi, Z, Psi, KiIG) in enumerate(ops):
            d, nI = L.sub_dofs[s], L.n_I[s]
            u[d[:nI]] -= KiIG @ uB[d[nI:]]
        return u + uB
    return apply


def test_fp32_stored_preconditioner_keeps_fp64_pcg():
    prob = W.tiny_poisson(shape=(8, 8, 8), subs=(2, 2, 2), seed=4, coeff="blocks", rhs="normal")
    H = setup_hierarchy(prob)
    K = H.levels[0].Kglob
    f = prob.rhs[:, 0]
    xd = direct_solve(prob)[:, 0]
    # the explicit FP64 operators reproduce the oracle's Alg. 1
    r = np.random.default_rng(0).standard_normal(f.shape[0])
    np.testing.assert_allclose(_explicit_alg1(H, np.float64)(r), bddc_apply(H, r),
                               rtol=0, atol=1e-9 * np.abs(bddc_apply(H, r)).max())
    x0, it0, *_ = pcg(K, f, _explicit_alg1(H, np.float64), 1e-12, 500)
    x1, it1, *_ = pcg(K, f, _explicit_alg1(H, np.float32), 1e-12, 500)
    assert abs(it1 - it0) <= 1
    assert np.linalg.norm(x1 - xd) <= 1e-9 * np.linalg.norm(xd)
    assert np.linalg.norm(x0 - xd) <= 1e-9 * np.linalg.norm(xd)
