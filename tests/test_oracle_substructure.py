"""Pins of the oracle's substructuring layer.

* Glob counts against the paper's weak-scaling table (Tabs. 1-2: elasticity
  cube, H/h = 16, N = 8, 64 and 512 cubic subdomains; n, n_Gamma and n_f
  are printed rounded) and the first-level pair count of Tab. 5 (4096
  subdomains), both from fixtures under tests/golden/, and against the
  box-decomposition counts of the workloads (3(B-1)B^2 faces, 3B(B-1)^2
  edges, (B-1)^3 corners).
* Schur complements: symmetric PSD, constants (Poisson) or rigid modes
  (elasticity) in the null space of floating subdomains, minimal energy
  among interior extensions, and the assembled interface problem
  reproduces the direct solution on the interface.
* Averaging: the weights form a partition of unity, E is a projection that
  leaves continuous functions unchanged (Section 2).
* Coarse basis: C Psi = I and Psi^T S Psi = -mu (Section 5).
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import fem
from oracle.substructure import (build_level, classify, coarse_basis, level1_input,
                                 saddle_inverse)
from oracle.bddc import direct_solve


def _glob_counts(prob):
    inp = level1_input(prob, Ke=False)
    _, globs = classify(inp)
    types = [g["type"] for g in globs]
    n_iface_dofs = len(np.unique(np.concatenate([g["dofs"] for g in globs])))
    return types.count("corner"), types.count("edge"), types.count("face"), n_iface_dofs


GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _printed(v):
    """Parse a rounded figure as the paper prints it: '9.5k', '0.1M', '12'."""
    scale = {"k": 1e3, "M": 1e6}.get(v[-1], 1.0)
    digits = v[:-1] if v[-1] in "kM" else v
    return float(digits), scale, (len(digits.split(".")[1]) if "." in digits else 0)


def _matches_printed(x, v):
    val, scale, nd = _printed(v)
    return round(x / scale, nd) == val


def _golden_rows(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line.split())
    return rows


@pytest.mark.parametrize("row", _golden_rows("cube_weak_scaling_counts.txt")[:2],
                         ids=lambda r: "N" + r[0])
def test_glob_counts_match_paper_weak_scaling_table(row):
    N = int(row[0])
    B = round(N ** (1.0 / 3.0))
    n = 16 * B
    prob = W.make_problem((n, n, n), (B, B, B), dof_per_node=3, dirichlet_axis=None)
    nc, ne, nf, n_gamma = _glob_counts(prob)
    assert _matches_printed(prob.n_dofs_total, row[1])
    assert _matches_printed(n_gamma, row[2])
    assert _matches_printed(nf, row[3])
    # exact structural counts behind the rounded figures
    assert nf == 3 * (B - 1) * B * B
    assert n_gamma == 3 * ((n + 1) ** 3 - (n + 2 - B) ** 3)


@pytest.mark.slow
def test_glob_counts_match_paper_weak_scaling_table_n512():
    row = _golden_rows("cube_weak_scaling_counts.txt")[2]
    B = 8
    n = 16 * B
    prob = W.make_problem((n, n, n), (B, B, B), dof_per_node=3, dirichlet_axis=None)
    nc, ne, nf, n_gamma = _glob_counts(prob)
    assert _matches_printed(prob.n_dofs_total, row[1])
    assert _matches_printed(n_gamma, row[2])
    assert _matches_printed(nf, row[3])


def test_first_level_pairs_of_the_4096_subdomain_cube():
    g = dict((k, int(v)) for k, v in _golden_rows("cube_4096_pairs.txt"))
    prob = W.make_problem((64, 64, 64), (16, 16, 16), dof_per_node=3, dirichlet_axis=None)
    nc, ne, nf, _ = _glob_counts(prob)
    assert nf == g["pairs_level1"]
    # the second level groups 4^3 first-level subdomains: a 4 x 4 x 4 box of
    # subdomains has 3 * 3 * 4^2 faces
    assert 3 * 3 * 4 * 4 == g["pairs_level2"]
    assert prob.n_dofs_total - g["unknowns_printed"] == 3


@pytest.mark.parametrize("cfg,expect", [("c1", (1, 6, 12)), ("c2", (27, 108, 144))])
def test_glob_counts_workloads(cfg, expect):
    prob = W.CONFIGS[cfg](0)
    nc, ne, nf, _ = _glob_counts(prob)
    assert (nc, ne, nf) == expect


@pytest.fixture(scope="module")
def poisson_level():
    prob = W.tiny_poisson(shape=(8, 8, 8), subs=(2, 2, 2), seed=1)
    return prob, build_level(level1_input(prob))


@pytest.fixture(scope="module")
def elast_level():
    prob = W.tiny_elasticity(shape=(4, 4, 4), subs=(2, 2, 2), seed=2)
    return prob, build_level(level1_input(prob))


def test_schur_symmetric_psd_and_null_space(poisson_level, elast_level):
    for (prob, L), rb in ((poisson_level, 1), (elast_level, 6)):
        n_float = 0
        for s in range(L.inp.n_sub):
            S = L.S[s]
            assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
            ev = np.linalg.eigvalsh(S)
            assert ev[0] >= -1e-11 * ev[-1]
            if L.inp.sub_floating[s]:
                n_float += 1
                G = L.sub_dofs[s][L.n_I[s]:]
                R = L.inp.rigid[G]
                assert R.shape[1] == rb
                assert np.abs(S @ R).max() <= 1e-10 * np.abs(S).max()
                assert np.count_nonzero(ev < 1e-10 * ev[-1]) == rb
            else:
                assert ev[0] > 1e-10 * ev[-1]
        assert n_float > 0


def test_schur_energy_minimal_extension(poisson_level):
    prob, L = poisson_level
    rng = np.random.default_rng(0)
    s = 3
    K, nI = L.K[s], L.n_I[s]
    uG = rng.standard_normal(L.n_G[s])
    # harmonic extension minimises the energy; any other interior is worse
    uI = -np.linalg.solve(K[:nI, :nI], K[:nI, nI:] @ uG)
    u = np.concatenate([uI, uG])
    assert u @ K @ u == pytest.approx(uG @ L.S[s] @ uG, rel=1e-12)
    for _ in range(3):
        v = u.copy()
        v[:nI] += 1e-3 * rng.standard_normal(nI)
        assert v @ K @ v > u @ K @ u


def test_interface_problem_reproduces_direct_solution(poisson_level):
    prob, L = poisson_level
    n = L.inp.n_dof
    x = direct_solve(prob)[:, 0]
    f = prob.rhs[:, 0]
    Sg = np.zeros((n, n))
    g = np.zeros(n)
    for s in range(L.inp.n_sub):
        nI = L.n_I[s]
        I, G = L.sub_dofs[s][:nI], L.sub_dofs[s][nI:]
        K = L.K[s]
        Sg[np.ix_(G, G)] += L.S[s]
        # interface right-hand side: f_G - K_GI K_II^{-1} f_I (f split once)
        g[G] -= K[nI:, :nI] @ np.linalg.solve(K[:nI, :nI], f[I])
    iface = np.unique(np.concatenate([L.sub_dofs[s][L.n_I[s]:] for s in range(L.inp.n_sub)]))
    g[iface] += f[iface]
    xs = np.linalg.solve(Sg[np.ix_(iface, iface)], g[iface])
    np.testing.assert_allclose(xs, x[iface], rtol=1e-9, atol=1e-12 * np.abs(x).max())


def test_weights_partition_of_unity_and_E_projection(poisson_level):
    prob, L = poisson_level
    n = L.inp.n_dof
    tot = np.zeros(n)
    cnt = np.zeros(n)
    for s in range(L.inp.n_sub):
        G = L.sub_dofs[s][L.n_I[s]:]
        np.add.at(tot, G, L.weights[s])
        np.add.at(cnt, G, 1)
        assert np.all(L.weights[s] > 0)
    np.testing.assert_allclose(tot[cnt > 0], 1.0, rtol=1e-14)
    # E: stacked interface vectors -> weighted average, restricted back
    offs = np.cumsum([0] + L.n_G)
    m = offs[-1]
    Rt = np.zeros((m, n))
    Dw = np.zeros(m)
    for s in range(L.inp.n_sub):
        G = L.sub_dofs[s][L.n_I[s]:]
        Rt[offs[s] + np.arange(len(G)), G] = 1.0
        Dw[offs[s]:offs[s + 1]] = L.weights[s]
    E = Rt @ (Rt.T * Dw[None, :])
    np.testing.assert_allclose(E @ E, E, atol=1e-13)
    u = np.random.default_rng(1).standard_normal(n)
    np.testing.assert_allclose(E @ (Rt @ u), Rt @ u, atol=1e-13)


def test_initial_constraints_and_coarse_basis(poisson_level, elast_level):
    for prob, L in (poisson_level, elast_level):
        coarse_basis(L)
        for s in range(L.inp.n_sub):
            C, Psi, S = L.C[s], L.Psi[s], L.S[s]
            np.testing.assert_allclose(C @ Psi, np.eye(C.shape[0]), atol=1e-10)
            Kc = Psi.T @ S @ Psi
            np.testing.assert_allclose(Kc, L.Kc[s], rtol=1e-8, atol=1e-10 * np.abs(Kc).max())
            # Z maps into the constrained space and inverts S there
            Z = L.Z[s]
            assert np.abs(C @ Z).max() < 1e-9 * max(1.0, np.abs(Z).max())
            # floating subdomains: coarse matrix null space = coarse values of rigid modes
            if L.inp.sub_floating[s]:
                G = L.sub_dofs[s][L.n_I[s]:]
                r = C @ L.inp.rigid[G]
                assert np.abs(L.Kc[s] @ r).max() < 1e-8 * np.abs(L.Kc[s]).max()


def test_edge_average_rows_per_component(elast_level):
    prob, L = elast_level
    for c in L.constraints:
        gl = L.globs[c["glob"]]
        comps = L.inp.dof_comp[c["dofs"]]
        assert np.all(comps == comps[0])
        if gl["type"] == "edge":
            np.testing.assert_allclose(c["w"], 1.0 / len(c["dofs"]))
        else:
            assert gl["type"] == "corner" and len(c["dofs"]) == 1
