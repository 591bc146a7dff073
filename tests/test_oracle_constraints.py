"""Pins of the oracle's adaptive constraint rows and of its level >= 2 input
for elasticity (CPU only).

* Courant-Fischer at pair level.  The constraint rows of eq. d-def are
  c_l = Pi A Pi w_l = lambda_l Pi B Pi w_l, so on the factor space c_l^T w = 0
  says w is B-orthogonal to the eigenvector w_l.  Adding the k rows
  [c^s, -c^s] (kept on all of Gamma^st, Prop. 1) to D therefore leaves a
  pair problem whose largest eigenvalue is exactly lambda_{k+1}.  The check
  builds the enriched pair problem itself, from the pair operators, with
  its own null-space basis; a wrong weight, sign, index, half or mask in
  the row construction changes that eigenvalue.
* The default rows (Section 7: entries on the shared edges and corners set
  to zero) are the pinned rows above with that mask applied, then
  orthonormalised; they are supported on the face DOFs only, and as a
  weaker constraint leave lambda_max >= lambda_{k+1}.
* "3eigv" (Section 8.2): a fixed count of three rows per face, whatever tau.
* Three-level elasticity: the level-2 "elements" are the level-1 coarse
  matrices K_c^s, whose null space for a floating subdomain is C^s applied
  to the six rigid-body modes (Section 3, Section 5); the level-2 rigid modes
  the oracle passes on (coarse values of the level-1 modes) must therefore be
  exactly the null space of every floating level-2 subdomain matrix and of
  its coarse matrix; Lemma 1's product bound holds at three levels, and PCG
  reproduces the direct solve.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle.adaptive import pair_eigenproblem, pair_operators, pair_rigid
from oracle.bddc import direct_solve, setup_hierarchy, solve_problem
from oracle.substructure import build_level, level1_input
from test_oracle_bddc import dense_preconditioned, global_omega

CASES = {
    "poisson": lambda: W.tiny_poisson(shape=(6, 6, 6), subs=(2, 2, 2), seed=31),
    "poisson_ragged": lambda: W.make_problem((7, 6, 5), None, coeff="lognormal", seed=32,
                                             cuts=[[0, 2, 7], [0, 4, 6], [0, 3, 5]]),
    "elasticity": lambda: W.tiny_elasticity(shape=(4, 4, 4), subs=(2, 2, 2), seed=33),
    "elasticity_3x2x2": lambda: W.tiny_elasticity(shape=(6, 4, 4), subs=(3, 2, 2), seed=34),
}

_LEVELS = {}


def level(case):
    if case not in _LEVELS:
        prob = CASES[case]()
        _LEVELS[case] = (prob, build_level(level1_input(prob)))
    return _LEVELS[case]


def constrained_lambda_max(L, s, t, rows, support):
    """Largest eigenvalue of the pair problem with extra rows [r, -r] in D.

    rows: (k, len(support)) values of the s-half on the level DOFs `support`
    (a subset of Gamma^st); the t-half carries the opposite sign."""
    ops = pair_operators(L, s, t)
    ns = ops["ns"]
    n = ns + ops["nt"]
    ps = np.searchsorted(ops["Gs"], support)
    pt = ns + np.searchsorted(ops["Gt"], support)
    assert np.array_equal(ops["Gs"][ps], support) and np.array_equal(ops["Gt"][pt - ns], support)
    extra = np.zeros((rows.shape[0], n))
    extra[:, ps] = rows
    extra[:, pt] = -rows
    D = np.vstack([ops["D"], extra]) if ops["D"].shape[0] else extra
    Q = sla.null_space(D)
    if L.inp.sub_floating[s] and L.inp.sub_floating[t]:
        Y = Q.T @ pair_rigid(L, s, t, ops)
        Q = Q @ sla.null_space(Y.T)
    A = ops["IE"].T @ ops["S"] @ ops["IE"]
    Ah = Q.T @ A @ Q
    Bh = Q.T @ ops["S"] @ Q
    return float(sla.eigh(0.5 * (Ah + Ah.T), 0.5 * (Bh + Bh.T), eigvals_only=True)[-1])


@pytest.mark.parametrize("case", sorted(CASES))
def test_keep_edge_rows_courant_fischer(case):
    prob, L = level(case)
    checked = 0
    for (s, t, g) in L.pairs:
        ops = pair_operators(L, s, t)
        # a threshold that selects a few eigenvectors of this pair
        r0 = pair_eigenproblem(L, s, t, L.globs[g], 0.0, 10)
        lam = r0["lam"]
        if len(lam) < 3 or lam[2] <= 1e-6 * lam[0]:
            continue   # lambda_3 is a rounding zero: nothing to pin
        tau = 0.5 * (lam[1] + lam[2])
        r = pair_eigenproblem(L, s, t, L.globs[g], tau, 10, keep_edges=True)
        k = r["k"]
        assert k == 2
        np.testing.assert_array_equal(r["face_dofs"], ops["shared"])
        assert len(r["rows"]) == k
        np.testing.assert_allclose(r["rows"] @ r["rows"].T, np.eye(k), atol=1e-12)
        lmax = constrained_lambda_max(L, s, t, r["rows"], r["face_dofs"])
        assert lmax == pytest.approx(r["lam_next"], rel=1e-8), (s, t)
        assert r["lam_next"] == pytest.approx(lam[2], rel=1e-10)
        checked += 1
    assert checked >= 3


@pytest.mark.parametrize("case", sorted(CASES))
def test_default_rows_are_the_face_mask_of_the_pinned_rows(case):
    prob, L = level(case)
    for (s, t, g) in L.pairs:
        face = L.globs[g]["dofs"]
        r0 = pair_eigenproblem(L, s, t, L.globs[g], 0.0, 10)
        lam = r0["lam"]
        if len(lam) < 4 or lam[3] <= 1e-6 * lam[0]:
            continue
        tau = 0.5 * (lam[2] + lam[3])
        rk = pair_eigenproblem(L, s, t, L.globs[g], tau, 10, keep_edges=True)
        rd = pair_eigenproblem(L, s, t, L.globs[g], tau, 10)
        assert rk["k"] == rd["k"] == 3
        np.testing.assert_array_equal(rd["face_dofs"], face)
        # same c_l; the default keeps the s-half on the face positions only
        np.testing.assert_allclose(rd["c_full"], rk["c_full"], rtol=0, atol=0)
        ops = pair_operators(L, s, t)
        F = rk["c_full"][np.searchsorted(ops["Gs"], face)]
        Qf = sla.orth(F)
        P = rd["rows"].T - Qf @ (Qf.T @ rd["rows"].T)
        assert np.abs(P).max() <= 1e-10
        assert Qf.shape[1] == len(rd["rows"])
        # the face is a proper subset of Gamma^st whenever edges exist, and
        # the masked (weaker) constraint cannot push lambda_max below lambda_4
        if len(face) < len(ops["shared"]):
            lmax = constrained_lambda_max(L, s, t, rd["rows"], face)
            assert lmax >= rk["lam_next"] * (1 - 1e-8)


def test_fixed_three_per_face():
    prob, L = level("elasticity")
    for (s, t, g) in L.pairs:
        r = pair_eigenproblem(L, s, t, L.globs[g], 1e300, 10, fixed=3)
        assert r["k"] == 3 and len(r["rows"]) == 3
        assert r["lam_next"] == pytest.approx(r["lam"][3], rel=1e-12)
        lmax = constrained_lambda_max(L, s, t, r["rows"], r["face_dofs"])
        assert lmax >= r["lam"][3] * (1 - 1e-8)


@pytest.fixture(scope="module")
def elasticity_3level():
    prob = W.make_problem((8, 8, 8), (4, 4, 4), dof_per_node=3, coeff="lognormal",
                          dirichlet_axis=2, group=(2, 2, 2), seed=35, rhs="normal")
    H = setup_hierarchy(prob)
    return prob, H


def test_three_level_elasticity_rigid_modes(elasticity_3level):
    prob, H = elasticity_3level
    assert len(H.levels) == 2
    L2 = H.levels[1]
    inp = L2.inp
    assert inp.rigid.shape[1] == 6
    nfloat = 0
    for s in range(inp.n_sub):
        dofs = L2.sub_dofs[s]
        K = L2.K[s]
        Rs = inp.rigid[dofs]
        scale = np.abs(K).max()
        ev = np.linalg.eigvalsh(0.5 * (K + K.T))
        if inp.sub_floating[s]:
            nfloat += 1
            # the level-2 subdomain matrix annihilates the coarse rigid modes ...
            assert np.linalg.matrix_rank(Rs, tol=1e-10 * np.abs(Rs).max()) == 6
            assert np.abs(K @ Rs).max() <= 1e-9 * scale * np.abs(Rs).max()
            # ... and has no other null vectors
            assert ev[5] <= 1e-9 * ev[-1] and ev[6] > 1e-7 * ev[-1], ev[:8] / ev[-1]
            # its coarse matrix: null space = C^s applied to those modes
            nI = L2.n_I[s]
            CR = L2.C[s] @ Rs[nI:]
            Kc = L2.Kc[s]
            assert np.abs(Kc @ CR).max() <= 1e-8 * np.abs(Kc).max() * np.abs(CR).max()
            evc = np.linalg.eigvalsh(0.5 * (Kc + Kc.T))
            assert evc[5] <= 1e-8 * evc[-1] and evc[6] > 1e-8 * evc[-1]
        else:
            assert ev[0] > 1e-9 * ev[-1]
    assert nfloat == 4


def test_three_level_elasticity_lemma1_and_direct(elasticity_3level):
    prob, H = elasticity_3level
    _, _, ev = dense_preconditioned(H)
    assert ev[0] >= 1.0 - 1e-9
    om = [global_omega(L) for L in H.levels]
    assert ev[-1] / ev[0] <= om[0] * om[1] * (1 + 1e-8)
    X, its, conds, _ = solve_problem(prob, rtol=1e-12, H=H)
    xd = direct_solve(prob)
    assert np.linalg.norm(X - xd) <= 1e-10 * np.linalg.norm(xd)
