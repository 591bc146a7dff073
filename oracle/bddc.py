"""Multilevel BDDC, its adaptive set-up and PCG (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``setup_hierarchy`` follows Alg. 3: per level, build substructures and
  initial constraints, solve the pair problems and add adaptive face
  constraints, set up the BDDC structures, then recurse with the coarse
  problem as the next level's problem; the top coarse problem is solved
  directly.
* ``bddc_apply`` is Alg. 1 (Multilevel BDDC) written in the full
  subdomain spaces: interior pre-correction, residual update, substructure
  correction and coarse problem with the weighted test functions E z,
  recursion, averaging, interior post-correction, combination.
* ``pcg`` is plain preconditioned CG from x0 = 0 with the stopping test on
  the relative residual (Section 8), and ``lanczos_cond`` the condition
  estimate from the CG coefficients.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import fem
from .substructure import (build_level, coarse_basis, level1_input, next_level_input,
                           assemble_level_matrix)
from .adaptive import enrich_level


@dataclass
class Hierarchy:
    levels: list = field(default_factory=list)
    Ktop: np.ndarray = None
    top_chol: tuple = None
    stats: dict = field(default_factory=dict)


def _prepare_full_space(L):
    """Factorisations of the full-space subdomain problems used by Alg. 1."""
    L.KII_chol, L.sadd_lu, L.Phi = [], [], []
    for s in range(L.inp.n_sub):
        nI = L.n_I[s]
        K = L.K[s]
        L.KII_chol.append(sla.cho_factor(K[:nI, :nI], lower=True) if nI else None)
        n = K.shape[0]
        nc = L.C[s].shape[0]
        Cbar = np.zeros((nc, n))
        Cbar[:, nI:] = L.C[s]
        A = np.zeros((n + nc, n + nc))
        A[:n, :n] = K
        A[:n, n:] = Cbar.T
        A[n:, :n] = Cbar
        lu = sla.lu_factor(A)
        L.sadd_lu.append(lu)
        rhs = np.zeros((n + nc, nc))
        rhs[n:, :] = np.eye(nc)
        L.Phi.append(sla.lu_solve(lu, rhs)[:n] if nc else np.zeros((n, 0)))
    L.Kglob = assemble_level_matrix(L.inp) if L.Kglob is None else L.Kglob


def setup_hierarchy(prob, adaptive=True, tau=None, nev_max=None, face_averages=False,
                    Ke=None, pair_subset=None, keep_edges=False, fixed=0, corners_only=False):
    """Adaptive-Multilevel BDDC set-up (Alg. 3) for ``prob.levels`` levels.
    keep_edges / fixed: see adaptive.pair_eigenproblem; corners_only /
    face_averages select the initial constraints 'c' / 'c+e+f'."""
    tau = prob.tau if tau is None else tau
    nev_max = prob.nev_max if nev_max is None else nev_max
    H = Hierarchy()
    inp = level1_input(prob, Ke)
    nlev = prob.levels
    for i in range(nlev - 1):
        L = build_level(inp, face_averages=face_averages, corners_only=corners_only)
        if i == 0:
            L.Kglob = fem.assemble_global(prob, None if Ke is None else Ke)
        if adaptive and (np.isfinite(tau) or fixed > 0):
            enrich_level(L, tau, nev_max, pairs=pair_subset if i == 0 else None,
                         keep_edges=keep_edges, fixed=fixed)
        coarse_basis(L)
        _prepare_full_space(L)
        H.levels.append(L)
        if i < nlev - 2:
            inp = next_level_input(L, np.asarray(prob.parents[i]))
    Lt = H.levels[-1]
    nC = Lt.n_coarse
    Ktop = np.zeros((nC, nC))
    for s in range(Lt.inp.n_sub):
        r = Lt.Rc[s]
        Ktop[np.ix_(r, r)] += Lt.Kc[s]
    H.Ktop = Ktop
    H.top_chol = sla.cho_factor(Ktop, lower=True) if nC else None
    H.stats = dict(
        omega=[L.adaptive.get("omega", 0.0) for L in H.levels],
        n_adaptive=[L.adaptive.get("n_added", 0) for L in H.levels],
        n_pairs=[len(L.pairs) for L in H.levels],
        n_coarse=[L.n_coarse for L in H.levels])
    return H


def bddc_apply(H, r, i=0):
    """One application of Multilevel BDDC (Alg. 1) on level i (0-based)."""
    L = H.levels[i]
    nsub = L.inp.n_sub
    r = np.asarray(r, dtype=np.float64)
    # interior pre-correction
    uI = np.zeros_like(r)
    for s in range(nsub):
        nI = L.n_I[s]
        if nI:
            I = L.sub_dofs[s][:nI]
            uI[I] = sla.cho_solve(L.KII_chol[s], r[I])
    # updated residual r_B = r - K u_I
    rB = r - L.Kglob @ uI
    # substructure corrections and coarse right-hand side
    rc = np.zeros(L.n_coarse)
    wD = []
    for s in range(nsub):
        nI = L.n_I[s]
        dofs = L.sub_dofs[s]
        n = len(dofs)
        nc = L.C[s].shape[0]
        f = np.zeros(n)
        f[nI:] = L.weights[s] * rB[dofs[nI:]]     # <r_B, E z>
        rhs = np.concatenate([f, np.zeros(nc)])
        w = sla.lu_solve(L.sadd_lu[s], rhs)[:n]
        wD.append(w)
        if nc:
            np.add.at(rc, L.Rc[s], L.Phi[s].T @ f)
    # coarse problem: direct at the top, one BDDC application otherwise
    if i == len(H.levels) - 1:
        uc = sla.cho_solve(H.top_chol, rc) if L.n_coarse else rc
    else:
        uc = bddc_apply(H, rc, i + 1)
    # averaging u_B = E (w_Delta + u_{i+1})
    uB = np.zeros_like(r)
    for s in range(nsub):
        nI = L.n_I[s]
        dofs = L.sub_dofs[s]
        w = wD[s] + (L.Phi[s] @ uc[L.Rc[s]] if L.C[s].shape[0] else 0.0)
        uB[dofs[:nI]] = w[:nI]
        np.add.at(uB, dofs[nI:], L.weights[s] * w[nI:])
    # interior post-correction v_I: a(v_I, z_I) = a(u_B, z_I)
    KuB = L.Kglob @ uB
    vI = np.zeros_like(r)
    for s in range(nsub):
        nI = L.n_I[s]
        if nI:
            I = L.sub_dofs[s][:nI]
            vI[I] = sla.cho_solve(L.KII_chol[s], KuB[I])
    return uI + uB - vI


def lanczos_cond(alphas, betas):
    """Extreme eigenvalues of the CG Lanczos tridiagonal and their ratio."""
    k = len(alphas)
    if k == 0:
        return 1.0, 1.0, 1.0
    d = np.empty(k)
    e = np.empty(max(k - 1, 0))
    d[0] = 1.0 / alphas[0]
    for j in range(1, k):
        d[j] = 1.0 / alphas[j] + betas[j - 1] / alphas[j - 1]
        e[j - 1] = np.sqrt(betas[j - 1]) / alphas[j - 1]
    ev = sla.eigvalsh_tridiagonal(d, e) if k > 1 else d
    return float(ev[-1] / ev[0]), float(ev[0]), float(ev[-1])


def pcg(K, f, M, rtol=1e-10, maxit=1000, x0=None):
    """Preconditioned CG from x0 (default 0); stops when ||f - K x|| / ||f||
    <= rtol (recursive residual).  Returns x, iterations, alphas, betas,
    history."""
    f = np.asarray(f, dtype=np.float64)
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    r = f - K @ x if x0 is not None else f.copy()
    nf = np.linalg.norm(f)
    if nf == 0:
        return x, 0, [], [], [0.0]
    if np.linalg.norm(r) <= rtol * nf:
        return x, 0, [], [], [np.linalg.norm(r) / nf]
    z = M(r)
    p = z.copy()
    rz = r @ z
    alphas, betas, hist = [], [], [1.0]
    it = 0
    for it in range(1, maxit + 1):
        q = K @ p
        a = rz / (p @ q)
        alphas.append(a)
        x += a * p
        r -= a * q
        rel = np.linalg.norm(r) / nf
        hist.append(rel)
        if rel <= rtol:
            break
        z = M(r)
        rz_new = r @ z
        b = rz_new / rz
        betas.append(b)
        rz = rz_new
        p = z + b * p
    return x, it, alphas, betas, hist


def direct_solve(prob, rhs=None, Ke=None):
    K = fem.assemble_global(prob, Ke).tocsc()
    rhs = prob.rhs if rhs is None else rhs
    lu = spla.splu(K)
    return lu.solve(np.asarray(rhs, dtype=np.float64))


def interior_solution(H, f):
    """x = [K_II^-1 f_I; 0] on level 1: every subdomain's interior problem
    solved with the right-hand side's interior values, zero on the interface.
    f - K x is then zero on the interiors, i.e. the residual of a discrete
    harmonic correction problem (the splitting U = U_I + W^ of Section 2), so
    PCG from this x0 runs on the interface problem of the Schur complement,
    which BDDC preconditions (Section 5)."""
    L = H.levels[0]
    x = np.zeros_like(np.asarray(f, dtype=np.float64))
    for s in range(L.inp.n_sub):
        nI = L.n_I[s]
        if nI:
            I = L.sub_dofs[s][:nI]
            x[I] = sla.cho_solve(L.KII_chol[s], f[I])
    return x


def solve_problem(prob, rtol=1e-10, maxit=1000, adaptive=True, H=None, rhs=None,
                  start="zero", **kw):
    """Set up the hierarchy and run PCG for every right-hand-side column, from
    x0 = 0 (start="zero") or from the level-1 interior solution
    (start="interior", see interior_solution)."""
    if H is None:
        H = setup_hierarchy(prob, adaptive=adaptive, **kw)
    K = H.levels[0].Kglob
    F = prob.rhs if rhs is None else rhs
    F = F.reshape(F.shape[0], -1)
    X = np.zeros_like(F)
    its, conds = [], []
    for j in range(F.shape[1]):
        x0 = interior_solution(H, F[:, j]) if start == "interior" else None
        x, it, al, be, _ = pcg(K, F[:, j], lambda v: bddc_apply(H, v), rtol, maxit, x0=x0)
        X[:, j] = x
        its.append(it)
        conds.append(lanczos_cond(al, be)[0])
    return X, its, conds, H
