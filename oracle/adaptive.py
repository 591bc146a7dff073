"""Adaptive coarse degrees of freedom from pair eigenproblems (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 4: for every pair of subdomains s, t sharing a face, the localized
generalized eigenproblem (eq. eig-matrix)

    Pi (I-E^st)^T S^st (I-E^st) Pi w = lambda Pi S^st Pi w

is solved on the factor space modulo null(Pi S^st Pi).  Eigenvectors with
lambda above the threshold tau give the constraint rows (eq. d-def)
c_l = w_l^T Pi (I-E)^T S (I-E) Pi, whose two halves are equal up to sign
(Prop. 1).  One half, restricted to the face DOFs (edge and corner entries
dropped, Section 7), is orthonormalised by a reduced QR and added to both
C^s and C^t.  Alg. 2 picks, per pair, the smallest k with
lambda_{k+1} <= tau, capped at nev_max (Section 8 uses at most 10).

Readings: D = [C^s_shared, -C^t_shared] (one row per shared initial coarse
DOF: the coarse DOFs of s and t agree); with keep_edges the rows stay on all
of Gamma^st and are applied to s and t only (a coarse DOF of the pair, not
of the other subdomains on the shared edges); the pair weights are the
stiffness-scaling weights renormalised over {s, t}; when both subdomains
are floating, the pair-continuous rigid modes (in null D and null S^st)
are removed from the factor space; the QR rank tolerance is 1e-10 max|R_jj|.

The solve here is a dense generalized eigendecomposition of the deflated
pair problem (brute force); the GPU library uses LOBPCG for the same
eigenpairs.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

QR_RANK_TOL = 1e-10
ZERO_EIG = 1e-9       # pair eigenvalues below ZERO_EIG max(1, lambda_1) are rounding zeros


def pair_operators(L, s, t):
    """Dense pair operators on [Gamma^s; Gamma^t].

    Returns dict with S (block diagonal), IE (= I - E^st), D, and index data.
    """
    nIs, nIt = L.n_I[s], L.n_I[t]
    Gs = L.sub_dofs[s][nIs:]
    Gt = L.sub_dofs[t][nIt:]
    ns, nt = len(Gs), len(Gt)
    n = ns + nt
    S = np.zeros((n, n))
    S[:ns, :ns] = L.S[s]
    S[ns:, ns:] = L.S[t]
    shared, is_, it_ = np.intersect1d(Gs, Gt, return_indices=True)
    ks = np.diag(L.K[s])[nIs:][is_]
    kt = np.diag(L.K[t])[nIt:][it_]
    ds = ks / (ks + kt)
    dt = 1.0 - ds
    # E^st: weighted average on Gamma^st, identity elsewhere
    E = np.eye(n)
    a = is_
    b = ns + it_
    E[a, a] = ds
    E[a, b] = dt
    E[b, a] = ds
    E[b, b] = dt
    IE = np.eye(n) - E
    # D: shared initial coarse DOFs must agree
    common = np.intersect1d(L.Rc[s], L.Rc[t])
    rows = []
    for cid in common:
        rs = np.flatnonzero(L.Rc[s] == cid)[0]
        rt = np.flatnonzero(L.Rc[t] == cid)[0]
        rows.append(np.concatenate([L.C[s][rs], -L.C[t][rt]]))
    D = np.array(rows).reshape(len(rows), n)
    return dict(S=S, IE=IE, D=D, Gs=Gs, Gt=Gt, ns=ns, nt=nt, shared=shared,
                is_=is_, it_=it_, ds=ds)


def pair_rigid(L, s, t, ops):
    """Pair-continuous rigid modes restricted to [Gamma^s; Gamma^t]."""
    R = L.inp.rigid
    return np.vstack([R[ops["Gs"]], R[ops["Gt"]]])


def pair_eigenproblem(L, s, t, face_glob, tau, nev_max, keep_edges=False, fixed=0,
                      span_upto=0):
    """Dense solution of the pair eigenproblem and the resulting constraints.

    The rows follow eq. d-def: c_l = Pi (I-E)^T S (I-E) Pi w_l for the k
    selected eigenvectors, supported on the shared DOFs Gamma^st with
    halves [c^s, -c^s] (Prop. 1).  The s-half is kept on all of Gamma^st
    (keep_edges, the form the theory asks for) or, by default, restricted to
    the face DOFs, i.e. the entries on the shared edges and corners are set
    to zero (Section 7); then a reduced QR orthonormalises them.

    k is min(#{lambda > tau}, nev_max) (Alg. 2), or, with fixed > 0, the
    fixed count min(fixed, #{lambda > rounding zero}) regardless of tau (the "3eigv" runs of
    Section 8.2: three eigenvector constraints per face in place of the
    face averages).  span_upto > 0 also returns, as "span_rows", the
    orthonormalised rows of the first span_upto eigenvectors (used to check
    a selection that cuts a cluster of equal eigenvalues, where only the
    span of the whole cluster is fixed)."""
    ops = pair_operators(L, s, t)
    n = ops["ns"] + ops["nt"]
    D = ops["D"]
    QD = sla.null_space(D) if D.shape[0] else np.eye(n)
    Q = QD
    both_floating = bool(L.inp.sub_floating[s] and L.inp.sub_floating[t])
    if both_floating:
        Y = QD.T @ pair_rigid(L, s, t, ops)
        Q = QD @ sla.null_space(Y.T)
    Afull = ops["IE"].T @ ops["S"] @ ops["IE"]
    Ah = Q.T @ Afull @ Q
    Bh = Q.T @ ops["S"] @ Q
    Ah = 0.5 * (Ah + Ah.T)
    Bh = 0.5 * (Bh + Bh.T)
    bev = np.linalg.eigvalsh(Bh)
    if bev[0] <= 1e-11 * bev[-1]:
        raise AssertionError(f"Assumption 1 violated on pair ({s},{t}): "
                             f"min eig(B) / max = {bev[0] / bev[-1]:.3e}")
    lam, W = sla.eigh(Ah, Bh)
    lam = lam[::-1]
    W = W[:, ::-1]
    if fixed > 0:
        # an eigenvalue that is zero up to rounding gives c = A w = 0: no
        # constraint, so the fixed count never takes one
        k = int(min(fixed, np.count_nonzero(lam > ZERO_EIG * max(1.0, lam[0]))))
    else:
        k = int(min(np.count_nonzero(lam > tau), nev_max))
    lam_next = float(lam[k]) if k < len(lam) else 0.0
    # support of the rows: Gamma^st (keep_edges) or the face DOFs only
    face = ops["shared"] if keep_edges else face_glob["dofs"]
    pos = np.searchsorted(ops["Gs"], face)
    PiD = QD @ QD.T

    def rows_of(j):
        """Orthonormal rows from the first j eigenvectors (eq. d-def, then
        the restriction to `face`, then reduced QR with the rank test)."""
        if j == 0:
            return np.zeros((0, len(face))), None
        c = PiD @ Afull @ (Q @ W[:, :j])         # eq. d-def, columns c_l
        F = c[pos, :]                             # s-half on the kept DOFs
        Qr, Rr = np.linalg.qr(F, mode="reduced")
        dR = np.abs(np.diag(Rr))
        keep = dR > QR_RANK_TOL * dR.max() if dR.size else np.zeros(0, bool)
        r = Qr[:, keep].T
        # canonical sign of each row: its largest-magnitude entry (first on
        # ties) positive; only the span is fixed by the method
        for x in r:
            if x[np.argmax(np.abs(x))] < 0:
                x *= -1.0
        return r, c

    rows, c_full = rows_of(k)
    out = dict(s=s, t=t, lam=lam, k=k, lam_next=lam_next, rows=rows, face_dofs=face,
               c_full=c_full, n=n, n_factor=Q.shape[1], both_floating=both_floating,
               Q=Q, Ah=Ah, Bh=Bh)
    if span_upto > 0:
        out["span_rows"] = rows_of(min(span_upto, len(lam)))[0]
    return out


def enrich_level(L, tau, nev_max, pairs=None, keep_edges=False, fixed=0):
    """Alg. 2 on one level: solve every pair problem and append the adaptive
    face constraints to C^s and C^t.  Records omega_i (max lambda_{k+1}).
    keep_edges and fixed as in pair_eigenproblem."""
    from .substructure import rebuild_constraint_matrices
    results = []
    sel = range(len(L.pairs)) if pairs is None else pairs
    for p in sel:
        s, t, g = L.pairs[p]
        res = pair_eigenproblem(L, s, t, L.globs[g], tau, nev_max, keep_edges=keep_edges,
                                fixed=fixed)
        res["pair"] = p
        results.append(res)
    for res in results:
        g = L.pairs[res["pair"]][2]
        for r in res["rows"]:
            L.glob_cons[g].append(len(L.constraints))
            L.constraints.append(dict(glob=g, dofs=res["face_dofs"], w=r.copy(), adaptive=True))
    rebuild_constraint_matrices(L)
    omega = max([r["lam_next"] for r in results], default=0.0)
    L.adaptive = dict(results=results, omega=omega,
                      n_added=int(sum(len(r["rows"]) for r in results)))
    return L.adaptive
