"""Substructuring components on one level (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Section 2 (interface, faces/edges/corners, discrete harmonic
extension, coarse degrees of freedom, averaging E), Section 3 (levels:
level-(i-1) substructures are level-i elements, level-(i-1) coarse DOFs
are level-i DOFs), Section 5 (local saddle point problem for the coarse
basis, coarse matrix = -mu) and Section 7 (stiffness scaling, corners plus
edge averages as initial constraints).

Readings where the paper leaves details open:
* globs are classified on all nodes, Dirichlet DOFs removed afterwards;
  a corner is an edge glob that has exactly one node;
* an edge average is taken per displacement component;
* at level >= 2 a "node" is a level-(i-1) glob carrying its coarse DOFs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem


@dataclass
class LevelInput:
    """A level's 'mesh': elements with dense matrices over level DOFs."""
    n_dof: int
    n_node: int
    elem_dofs: list            # per element: global DOF ids (-1 = fixed/removed)
    elem_mats: list            # per element: dense matrix matching elem_dofs
    elem_nodes: list           # per element: node ids (for glob classification)
    elem_sub: np.ndarray       # element -> subdomain
    n_sub: int
    node_dofs: list            # per node: its free DOF ids
    dof_comp: np.ndarray       # per DOF: component (0..d-1) or -1
    rigid: np.ndarray          # (n_dof, n_rb) rigid-body modes at this level
    sub_floating: np.ndarray   # per subdomain: no Dirichlet DOF touches it
    dof_per_node: int = 1


@dataclass
class Level:
    inp: LevelInput
    sub_dofs: list = field(default_factory=list)      # [I..., G...] global ids
    n_I: list = field(default_factory=list)
    n_G: list = field(default_factory=list)
    K: list = field(default_factory=list)             # dense subdomain matrices
    globs: list = field(default_factory=list)         # dict(type, subs, nodes, dofs)
    pairs: list = field(default_factory=list)         # (s, t, face glob id)
    weights: list = field(default_factory=list)       # delta^s over Gamma^s
    S: list = field(default_factory=list)
    constraints: list = field(default_factory=list)   # dict(glob, dofs, w)
    glob_cons: list = field(default_factory=list)     # glob -> coarse ids
    C: list = field(default_factory=list)             # dense (n_c, n_G)
    Rc: list = field(default_factory=list)            # coarse ids of C rows
    Psi: list = field(default_factory=list)
    Kc: list = field(default_factory=list)
    Z: list = field(default_factory=list)
    n_coarse: int = 0
    Kglob: Optional[sp.csr_matrix] = None
    adaptive: dict = field(default_factory=dict)      # filled by adaptive.enrich_level


def level1_input(prob, Ke=None):
    """Level-1 input from a problem description (FE elements, mesh nodes)."""
    d = prob.dof_per_node
    if Ke is None:
        Ke = fem.element_matrices(prob)
    elif Ke is False:          # structure only (glob classification)
        Ke = [None] * prob.n_elems
    fmap = fem.free_map(prob)
    edofs = fmap[fem.elem_dof_ids(prob)]
    n_nodes = prob.n_nodes
    full = np.arange(n_nodes * d).reshape(n_nodes, d)
    ff = fmap[full]
    node_dofs = [row[row >= 0] for row in ff]
    dof_comp = np.tile(np.arange(d), n_nodes)[prob.dirichlet == 0]
    free_nodes_rb = fem.rigid_modes(prob.coords, d)[prob.dirichlet == 0]
    n_sub = prob.n_sub
    touches = np.zeros(n_sub, dtype=bool)
    fixed_elem = (edofs < 0).any(axis=1)
    touches[prob.elem_to_sub[fixed_elem]] = True
    return LevelInput(
        n_dof=prob.n_free, n_node=n_nodes,
        elem_dofs=list(edofs), elem_mats=list(Ke), elem_nodes=list(prob.elem_nodes.astype(np.int64)),
        elem_sub=prob.elem_to_sub.astype(np.int64), n_sub=n_sub, node_dofs=node_dofs,
        dof_comp=dof_comp, rigid=free_nodes_rb, sub_floating=~touches, dof_per_node=d)


def _node_subdomain_sets(inp):
    """For each node, the sorted tuple of subdomains whose elements contain it."""
    pairs = set()
    en = inp.elem_nodes
    es = inp.elem_sub
    sets = [set() for _ in range(inp.n_node)]
    for e in range(len(en)):
        s = int(es[e])
        for n in en[e]:
            sets[int(n)].add(s)
    return [tuple(sorted(x)) for x in sets]


def _node_subdomain_sets_fast(inp):
    en = inp.elem_nodes
    lens = np.array([len(x) for x in en])
    if np.all(lens == lens[0]):
        nodes = np.concatenate(en).astype(np.int64)
        subs = np.repeat(inp.elem_sub.astype(np.int64), lens)
        key = np.unique(nodes * (inp.n_sub + 1) + subs)
        nn = key // (inp.n_sub + 1)
        ss = key % (inp.n_sub + 1)
        out = [()] * inp.n_node
        starts = np.searchsorted(nn, np.arange(inp.n_node + 1))
        for n in range(inp.n_node):
            a, b = starts[n], starts[n + 1]
            out[n] = tuple(ss[a:b].tolist())
        return out
    return _node_subdomain_sets(inp)


def classify(inp):
    """Interface globs: face = nodes shared by the same two subdomains, edge =
    nodes shared by the same set of more than two, corner = an edge of one
    node (Section 2).  Returns (node_sets, globs)."""
    node_sets = _node_subdomain_sets_fast(inp)
    groups = {}
    for n, key in enumerate(node_sets):
        if len(key) >= 2:
            groups.setdefault(key, []).append(n)
    globs = []
    for key in sorted(groups.keys(), key=lambda k: (groups[k][0], k)):
        nodes = groups[key]
        dofs = np.sort(np.concatenate([inp.node_dofs[n] for n in nodes]).astype(np.int64)) \
            if nodes else np.zeros(0, np.int64)
        if len(dofs) == 0:
            continue
        if len(key) == 2:
            typ = "face"
        elif len(nodes) == 1:
            typ = "corner"
        else:
            typ = "edge"
        globs.append(dict(type=typ, subs=key, nodes=np.array(nodes), dofs=dofs))
    return node_sets, globs


def build_level(inp, face_averages=False, corners_only=False, only=None):
    """Subdomain matrices, globs, weights, initial constraints and Schur
    complements of one level (initial constraints = corners + edge averages,
    Section 7; optionally face averages as well ('c+e+f'), or corners alone
    ('c'), the variants of Section 8.2's tables).

    only: None, or a collection of subdomains: then the dense matrices and
    Schur complements are formed for those subdomains alone (the others get
    None) and the global weights are skipped; the structure (globs, DOF
    sets, constraints, pairs) is always complete.  Used to time a sample of
    a large workload; the pair problem of two sampled subdomains is exact."""
    L = Level(inp=inp)
    node_sets, globs = classify(inp)
    L.globs = globs
    n_sub = inp.n_sub
    # subdomain DOF sets
    sub_all = [set() for _ in range(n_sub)]
    for e in range(len(inp.elem_dofs)):
        s = int(inp.elem_sub[e])
        dd = inp.elem_dofs[e]
        sub_all[s].update(int(x) for x in dd[dd >= 0])
    dof_node = np.empty(inp.n_dof, dtype=np.int64)
    for n, dl in enumerate(inp.node_dofs):
        dof_node[dl] = n
    is_iface = np.array([len(node_sets[dof_node[j]]) >= 2 for j in range(inp.n_dof)], dtype=bool)
    for s in range(n_sub):
        a = np.array(sorted(sub_all[s]), dtype=np.int64)
        I = a[~is_iface[a]]
        G = a[is_iface[a]]
        L.sub_dofs.append(np.concatenate([I, G]))
        L.n_I.append(len(I))
        L.n_G.append(len(G))
    # dense subdomain matrices
    sub_elems = [[] for _ in range(n_sub)]
    for e in range(len(inp.elem_dofs)):
        sub_elems[int(inp.elem_sub[e])].append(e)
    for s in range(n_sub):
        if only is not None and s not in only:
            L.K.append(None)
            continue
        dofs = L.sub_dofs[s]
        loc = {int(g): i for i, g in enumerate(dofs)}
        n = len(dofs)
        K = np.zeros((n, n))
        for e in sub_elems[s]:
            dd = inp.elem_dofs[e]
            keep = np.flatnonzero(dd >= 0)
            li = np.array([loc[int(dd[k])] for k in keep])
            K[np.ix_(li, li)] += inp.elem_mats[e][np.ix_(keep, keep)]
        L.K.append(K)
    # stiffness-scaling weights: delta_j^s = K^s_jj / sum_r K^r_jj
    if only is None:
        diag_sum = np.zeros(inp.n_dof)
        for s in range(n_sub):
            nI = L.n_I[s]
            G = L.sub_dofs[s][nI:]
            np.add.at(diag_sum, G, np.diag(L.K[s])[nI:])
        for s in range(n_sub):
            nI = L.n_I[s]
            G = L.sub_dofs[s][nI:]
            L.weights.append(np.diag(L.K[s])[nI:] / diag_sum[G])
    # Schur complements S^s = K_GG - K_GI K_II^{-1} K_IG
    for s in range(n_sub):
        L.S.append(None if L.K[s] is None else schur(L.K[s], L.n_I[s]))
    # initial constraints
    cons = []
    glob_cons = []
    for g, gl in enumerate(globs):
        ids = []
        if gl["type"] == "corner":
            for j in gl["dofs"]:
                ids.append(len(cons))
                cons.append(dict(glob=g, dofs=np.array([j]), w=np.array([1.0])))
        elif (gl["type"] == "edge" and not corners_only) or \
                (gl["type"] == "face" and face_averages):
            comps = inp.dof_comp[gl["dofs"]]
            for c in np.unique(comps):
                dd = gl["dofs"][comps == c]
                ids.append(len(cons))
                cons.append(dict(glob=g, dofs=dd, w=np.full(len(dd), 1.0 / len(dd))))
        glob_cons.append(ids)
    L.constraints = cons
    L.glob_cons = glob_cons
    L.pairs = [(gl["subs"][0], gl["subs"][1], g) for g, gl in enumerate(globs)
               if gl["type"] == "face"]
    rebuild_constraint_matrices(L)
    return L


def schur(K, nI):
    """Schur complement of the leading nI x nI block (dense Cholesky)."""
    if nI == 0:
        return K.copy()
    KII = K[:nI, :nI]
    KIG = K[:nI, nI:]
    cf = sla.cho_factor(KII, lower=True)
    return K[nI:, nI:] - KIG.T @ sla.cho_solve(cf, KIG)


def rebuild_constraint_matrices(L):
    """Dense C^s over the local interface and its coarse-id map R_c^s."""
    n_sub = L.inp.n_sub
    L.C, L.Rc = [], []
    L.n_coarse = len(L.constraints)
    for s in range(n_sub):
        nI = L.n_I[s]
        G = L.sub_dofs[s][nI:]
        loc = {int(g): i for i, g in enumerate(G)}
        rows, ids = [], []
        for g, gl in enumerate(L.globs):
            if s not in gl["subs"]:
                continue
            for cid in L.glob_cons[g]:
                c = L.constraints[cid]
                r = np.zeros(len(G))
                for j, w in zip(c["dofs"], c["w"]):
                    r[loc[int(j)]] = w
                rows.append(r)
                ids.append(cid)
        order = np.argsort(ids, kind="stable")
        C = np.array(rows).reshape(len(rows), len(G))[order] if rows else np.zeros((0, len(G)))
        L.C.append(C)
        L.Rc.append(np.array(ids, dtype=np.int64)[order])


def saddle_inverse(S, C):
    """Blocks of [[S, C^T], [C, 0]]^{-1} = [[Z, Psi], [Psi^T, mu]] (Section 5).

    Z is the constrained Neumann solution operator, Psi the coarse basis
    (C Psi = I, minimal energy), mu gives the coarse matrix Psi^T S Psi = -mu.
    """
    n, nc = S.shape[0], C.shape[0]
    A = np.zeros((n + nc, n + nc))
    A[:n, :n] = S
    A[:n, n:] = C.T
    A[n:, :n] = C
    inv = sla.solve(A, np.eye(n + nc), assume_a="sym")
    inv = 0.5 * (inv + inv.T)
    return inv[:n, :n], inv[:n, n:], inv[n:, n:]


def coarse_basis(L):
    """Coarse basis Psi^s, coarse element matrices K_c^s = -mu^s and the
    constrained Neumann operators Z^s for every subdomain."""
    L.Psi, L.Kc, L.Z = [], [], []
    for s in range(L.inp.n_sub):
        Z, Psi, mu = saddle_inverse(L.S[s], L.C[s])
        L.Z.append(Z)
        L.Psi.append(Psi)
        L.Kc.append(-mu)


def assemble_level_matrix(inp):
    """Global matrix of a level assembled from its elements (sparse)."""
    rows, cols, vals = [], [], []
    for dd, M in zip(inp.elem_dofs, inp.elem_mats):
        keep = np.flatnonzero(dd >= 0)
        d = dd[keep]
        rows.append(np.repeat(d, len(d)))
        cols.append(np.tile(d, len(d)))
        vals.append(M[np.ix_(keep, keep)].ravel())
    n = inp.n_dof
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def next_level_input(L, parent):
    """Level-(i+1) input: level-i subdomains become elements with matrices
    K_c^s over the level-i coarse DOFs; each level-i glob that carries coarse
    DOFs becomes a node (Section 3)."""
    globs_with = [g for g in range(len(L.globs)) if len(L.glob_cons[g]) > 0]
    node_of_glob = {g: k for k, g in enumerate(globs_with)}
    node_dofs = [np.array(L.glob_cons[g], dtype=np.int64) for g in globs_with]
    dof_comp = -np.ones(L.n_coarse, dtype=np.int64)
    inp = L.inp
    for cid, c in enumerate(L.constraints):
        comps = inp.dof_comp[c["dofs"]]
        gl = L.globs[c["glob"]]
        if gl["type"] in ("corner", "edge") and np.all(comps == comps[0]):
            dof_comp[cid] = comps[0]
    elem_nodes = []
    for s in range(inp.n_sub):
        elem_nodes.append(np.array(sorted({node_of_glob[L.constraints[c]["glob"]]
                                           for c in L.Rc[s]}), dtype=np.int64))
    # coarse values of the level-i rigid modes
    rigid = np.zeros((L.n_coarse, inp.rigid.shape[1]))
    for cid, c in enumerate(L.constraints):
        rigid[cid] = c["w"] @ inp.rigid[c["dofs"]]
    n_parent = int(parent.max()) + 1
    floating = np.ones(n_parent, dtype=bool)
    for s in range(inp.n_sub):
        if not inp.sub_floating[s]:
            floating[parent[s]] = False
    return LevelInput(
        n_dof=L.n_coarse, n_node=len(globs_with), elem_dofs=[r.copy() for r in L.Rc],
        elem_mats=[k.copy() for k in L.Kc], elem_nodes=elem_nodes,
        elem_sub=np.asarray(parent, dtype=np.int64), n_sub=n_parent, node_dofs=node_dofs,
        dof_comp=dof_comp, rigid=rigid, sub_floating=floating,
        dof_per_node=inp.dof_per_node)
