"""Seeded synthetic inputs for Adaptive-Multilevel BDDC runs.

This module only *describes* problems: a structured hexahedral mesh of the
unit cube, per-element material data, a box decomposition into subdomains
(and the grouping of subdomains into higher-level subdomains), the
Dirichlet mask and the right-hand sides.  It holds none of the solver's
arithmetic: no element matrices, no assembly, no solves.  Both the FP64
oracle (test infrastructure) and the GPU library consume these arrays.

Conventions shared by every consumer
------------------------------------
* Nodes are numbered x-fastest: node (i, j, k) -> i + (nx+1)*(j + (ny+1)*k).
* Elements are numbered x-fastest as well; the 8 local nodes of an element
  are in lexicographic order: local index a + 2*b + 4*c is the node at
  offset (a, b, c) from the element's lowest corner.
* Degrees of freedom: ``dof_per_node`` (1 for Poisson, 3 for elasticity)
  per node, DOF id = node*dof_per_node + component before Dirichlet
  removal.  Free DOFs keep that order with the Dirichlet DOFs removed.
* Right-hand sides are given over the free DOFs, shape (n_free, nrhs).

Workload recipes follow the synthetic stand-ins for the paper's
engineering problems (jumping coefficients, many subdomains, two or three
levels; Section 8 of the paper describes the original problems).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "Problem", "box_mesh", "box_decomposition", "make_problem",
    "config_c1", "config_c2", "config_c3", "config_c4", "config_c5", "cube_tab5",
    "tiny_poisson", "tiny_elasticity", "CONFIGS",
]


@dataclass
class Problem:
    name: str
    shape: tuple                     # (nx, ny, nz) elements
    coords: np.ndarray               # (n_nodes, 3) float64
    elem_nodes: np.ndarray           # (n_elems, 8) int32
    dof_per_node: int                # 1 Poisson, 3 elasticity
    coeff: np.ndarray                # (n_elems,) kappa (Poisson) or Young modulus E
    nu: Optional[np.ndarray]         # (n_elems,) Poisson ratio or None
    elem_to_sub: np.ndarray          # (n_elems,) int32 level-1 subdomain
    parents: list                    # level-i subdomain -> level-(i+1) subdomain, i = 1..L-2
    dirichlet: np.ndarray            # (n_nodes*dof_per_node,) uint8, 1 = fixed to zero
    rhs: np.ndarray                  # (n_free, nrhs) float64, Fortran order
    levels: int = 2
    tau: float = 10.0
    nev_max: int = 10
    extra: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return self.coords.shape[0]

    @property
    def n_elems(self) -> int:
        return self.elem_nodes.shape[0]

    @property
    def n_dofs_total(self) -> int:
        return self.n_nodes * self.dof_per_node

    @property
    def free_dofs(self) -> np.ndarray:
        return np.flatnonzero(self.dirichlet == 0).astype(np.int64)

    @property
    def n_free(self) -> int:
        return int(np.count_nonzero(self.dirichlet == 0))

    @property
    def n_sub(self) -> int:
        return int(self.elem_to_sub.max()) + 1


# --------------------------------------------------------------------------
# geometry and decomposition
# --------------------------------------------------------------------------

def box_mesh(nx: int, ny: int, nz: int):
    """Unit-cube structured hex mesh: coordinates and element connectivity."""
    xs = np.linspace(0.0, 1.0, nx + 1)
    ys = np.linspace(0.0, 1.0, ny + 1)
    zs = np.linspace(0.0, 1.0, nz + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    coords = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    base = (i + (nx + 1) * (j + (ny + 1) * k)).ravel()
    off = []
    for c in range(2):
        for b in range(2):
            for a in range(2):
                off.append(a + (nx + 1) * (b + (ny + 1) * c))
    # local index a + 2b + 4c
    order = [0] * 8
    idx = 0
    for c in range(2):
        for b in range(2):
            for a in range(2):
                order[a + 2 * b + 4 * c] = off[idx]
                idx += 1
    elem_nodes = (base[:, None] + np.asarray(order)[None, :]).astype(np.int32)
    return coords, elem_nodes


def element_ijk(nx: int, ny: int, nz: int):
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def box_decomposition(shape, cuts):
    """Box decomposition of an (nx, ny, nz) element grid.

    ``cuts`` = (cx, cy, cz), each an increasing list of cut positions in
    element units including 0 and n.  Subdomain index is x-fastest.
    Returns (elem_to_sub int32, (bx, by, bz)).
    """
    nx, ny, nz = shape
    i, j, k = element_ijk(nx, ny, nz)
    cx, cy, cz = (np.asarray(c) for c in cuts)
    bi = np.searchsorted(cx, i, side="right") - 1
    bj = np.searchsorted(cy, j, side="right") - 1
    bk = np.searchsorted(cz, k, side="right") - 1
    bx, by, bz = len(cx) - 1, len(cy) - 1, len(cz) - 1
    return (bi + bx * (bj + by * bk)).astype(np.int32), (bx, by, bz)


def group_boxes(nboxes, group):
    """Parent map grouping a (bx,by,bz) box grid into blocks of ``group`` boxes."""
    bx, by, bz = nboxes
    gx, gy, gz = group
    assert bx % gx == 0 and by % gy == 0 and bz % gz == 0
    k, j, i = np.meshgrid(np.arange(bz), np.arange(by), np.arange(bx), indexing="ij")
    px, py = bx // gx, by // gy
    parent = (i // gx) + px * ((j // gy) + py * (k // gz))
    return parent.ravel().astype(np.int32), (bx // gx, by // gy, bz // gz)


def uniform_cuts(n, parts):
    assert n % parts == 0
    return list(range(0, n + 1, n // parts))


def dirichlet_face(coords, dof_per_node, axis, value=0.0):
    on = np.isclose(coords[:, axis], value)
    mask = np.repeat(on, dof_per_node).astype(np.uint8)
    return mask


def _finish(name, shape, coords, elem_nodes, dof, coeff, nu, elem_to_sub, parents,
            dirichlet, rhs, levels, tau, nev_max=10, extra=None):
    rhs = np.asfortranarray(np.asarray(rhs, dtype=np.float64).reshape(rhs.shape[0], -1))
    return Problem(name=name, shape=tuple(shape), coords=coords, elem_nodes=elem_nodes,
                   dof_per_node=dof, coeff=np.ascontiguousarray(coeff, dtype=np.float64),
                   nu=None if nu is None else np.ascontiguousarray(nu, dtype=np.float64),
                   elem_to_sub=elem_to_sub.astype(np.int32), parents=parents,
                   dirichlet=dirichlet.astype(np.uint8), rhs=rhs, levels=levels,
                   tau=tau, nev_max=nev_max, extra=extra or {})


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def config_c1(seed: int = 0) -> Problem:
    """Poisson 16^3, 2x2x2 subdomains of 8^3, three high-conductivity channels.

    kappa = 1 with three axis-aligned channels (one per axis, full length,
    2x2-element cross-section at seeded transverse offsets) of kappa = 1e6;
    f = 1 at every free node, u = 0 on x = 0, tau = 10, two levels.
    """
    rng = np.random.default_rng(seed)
    n = 16
    coords, elem_nodes = box_mesh(n, n, n)
    i, j, k = element_ijk(n, n, n)
    ijk = [i, j, k]
    kappa = np.ones(n ** 3)
    for d in range(3):
        t1, t2 = [ax for ax in range(3) if ax != d]
        lo = rng.integers(0, 15, 2)
        inside = ((ijk[t1] >= lo[0]) & (ijk[t1] < lo[0] + 2) &
                  (ijk[t2] >= lo[1]) & (ijk[t2] < lo[1] + 2))
        kappa[inside] = 1e6
    e2s, _ = box_decomposition((n, n, n), [uniform_cuts(n, 2)] * 3)
    dmask = dirichlet_face(coords, 1, 0)
    nfree = int(np.count_nonzero(dmask == 0))
    rhs = np.ones((nfree, 1))
    return _finish("c1_poisson16_channels", (n, n, n), coords, elem_nodes, 1, kappa, None,
                   e2s, [], dmask, rhs, levels=2, tau=10.0)


def config_c2(seed: int = 0) -> Problem:
    """Poisson 32^3, 4x4x4 subdomains of 8^3, kappa = 10^U per 2x2x2 block.

    U is discrete-uniform on {0,...,6}, drawn per 2x2x2 element block; the
    right-hand side is N(0,1) per free DOF; u = 0 on x = 0; tau = 10.
    """
    rng = np.random.default_rng(seed)
    n = 32
    coords, elem_nodes = box_mesh(n, n, n)
    i, j, k = element_ijk(n, n, n)
    U = rng.integers(0, 7, size=(16, 16, 16))   # indexed [bk, bj, bi]
    kappa = 10.0 ** U[k // 2, j // 2, i // 2]
    e2s, _ = box_decomposition((n, n, n), [uniform_cuts(n, 4)] * 3)
    dmask = dirichlet_face(coords, 1, 0)
    nfree = int(np.count_nonzero(dmask == 0))
    rhs = rng.standard_normal((nfree, 1))
    return _finish("c2_poisson32_jumps", (n, n, n), coords, elem_nodes, 1, kappa, None,
                   e2s, [], dmask, rhs, levels=2, tau=10.0)


def _random_widths(rng, total, parts, lo, hi):
    while True:
        w = rng.integers(lo, hi + 1, size=parts)
        if int(w.sum()) == total:
            return w


def config_c3(seed: int = 0) -> Problem:
    """Elasticity 48^3, 6x6x6 uneven boxes (sides 5..11), stiff spherical inclusions.

    E = 1 with spheres (centre ~ U[0,48]^3, radius ~ U[2,4] element units)
    of E = 1e3 added until at least 15% of element centroids are inside;
    nu = 0.3; clamped on z = 0; unit body force (0,0,-1) as a consistent
    nodal load (each element gives volume/8 to each of its nodes).
    """
    rng = np.random.default_rng(seed)
    n = 48
    coords, elem_nodes = box_mesh(n, n, n)
    cuts = []
    for _ in range(3):
        w = _random_widths(rng, n, 6, 5, 11)
        cuts.append([0] + list(np.cumsum(w)))
    i, j, k = element_ijk(n, n, n)
    cen = np.stack([i + 0.5, j + 0.5, k + 0.5], axis=1)
    inside = np.zeros(n ** 3, dtype=bool)
    target = int(np.ceil(0.15 * n ** 3))
    while np.count_nonzero(inside) < target:
        c = rng.uniform(0.0, n, size=3)
        r = rng.uniform(2.0, 4.0)
        inside |= np.sum((cen - c) ** 2, axis=1) <= r * r
    E = np.where(inside, 1e3, 1.0)
    nu = np.full(n ** 3, 0.3)
    e2s, _ = box_decomposition((n, n, n), cuts)
    dmask = dirichlet_face(coords, 3, 2)
    vol = (1.0 / n) ** 3
    load = np.zeros((coords.shape[0], 3))
    np.add.at(load[:, 2], elem_nodes.ravel(), -vol / 8.0)
    rhs = load.ravel()[dmask == 0][:, None]
    return _finish("c3_elasticity48_inclusions", (n, n, n), coords, elem_nodes, 3, E, nu,
                   e2s, [], dmask, rhs, levels=2, tau=10.0,
                   extra={"cuts": cuts, "inclusion_fraction": float(inside.mean())})


def config_c4(seed: int = 0) -> Problem:
    """Poisson 64^3, three levels: 8^3 subdomains of 8^3, grouped 4^3 -> 2^3.

    kappa = 10^U with U ~ U[0,5) per element; 16 right-hand sides N(0,1).
    """
    rng = np.random.default_rng(seed)
    n = 64
    coords, elem_nodes = box_mesh(n, n, n)
    kappa = 10.0 ** rng.uniform(0.0, 5.0, size=n ** 3)
    e2s, nb = box_decomposition((n, n, n), [uniform_cuts(n, 8)] * 3)
    parent, _ = group_boxes(nb, (4, 4, 4))
    dmask = dirichlet_face(coords, 1, 0)
    nfree = int(np.count_nonzero(dmask == 0))
    rhs = rng.standard_normal((nfree, 16))
    return _finish("c4_poisson64_3level", (n, n, n), coords, elem_nodes, 1, kappa, None,
                   e2s, [parent], dmask, rhs, levels=3, tau=10.0)


def config_c5(seed: int = 0) -> Problem:
    """Adjoint workload: Poisson 32^3, 4x4x4, theta ~ N(2,1), 8 point sources.

    kappa = 10^theta per element.  ``extra['theta_obs']`` is theta perturbed
    by 0.1*N(0,1); the observations x_obs are the solutions for theta_obs.
    ``extra['fd_elems']`` are 32 seeded elements for finite-difference checks.
    """
    rng = np.random.default_rng(seed)
    n = 32
    coords, elem_nodes = box_mesh(n, n, n)
    theta = rng.normal(2.0, 1.0, size=n ** 3)
    e2s, _ = box_decomposition((n, n, n), [uniform_cuts(n, 4)] * 3)
    dmask = dirichlet_face(coords, 1, 0)
    nfree = int(np.count_nonzero(dmask == 0))
    src = rng.choice(nfree, size=8, replace=False)
    rhs = np.zeros((nfree, 8))
    rhs[src, np.arange(8)] = 1.0
    theta_obs = theta + 0.1 * rng.standard_normal(n ** 3)
    fd = rng.choice(n ** 3, size=32, replace=False)
    return _finish("c5_poisson32_adjoint", (n, n, n), coords, elem_nodes, 1, 10.0 ** theta,
                   None, e2s, [], dmask, rhs, levels=2, tau=10.0,
                   extra={"theta": theta, "theta_obs": theta_obs, "sources": src,
                          "fd_elems": fd})


def cube_tab5(tau2: float = 4.0, n: int = 64, sub: int = 4, group: int = 4,
              seed: int = 0) -> Problem:
    """Homogeneous elasticity cube of Section 8.1's level comparison (Tab. 5).

    n^3 Q1 elements (64^3: 823,875 nodal DOFs), cubic level-1 subdomains of
    sub^3 elements (4,096 of 4^3), grouped group^3 per level-2 subdomain (64);
    E = 1, nu = 0.3 (the paper does not state them), body force (0, 0, -1)
    as a consistent nodal load (own weight).  Support: the vertical face
    x = 0 is clamped (the paper fixes one vertical edge; fixing a line alone
    leaves the rotation about it free).  Three levels; tau = sqrt(tau2) on
    both substructured levels, so that the indicator target of the product
    is tau2.  The random generator is not used (the problem is fixed).
    """
    del seed
    coords, elem_nodes = box_mesh(n, n, n)
    e2s, nb = box_decomposition((n, n, n), [uniform_cuts(n, n // sub)] * 3)
    parent, _ = group_boxes(nb, (group, group, group))
    dmask = dirichlet_face(coords, 3, 0)
    vol = (1.0 / n) ** 3
    load = np.zeros((coords.shape[0], 3))
    np.add.at(load[:, 2], elem_nodes.ravel(), -vol / 8.0)
    rhs = load.ravel()[dmask == 0][:, None]
    ne = n ** 3
    return _finish(f"tab5_elasticity{n}_tau2_{tau2:g}", (n, n, n), coords, elem_nodes, 3,
                   np.ones(ne), np.full(ne, 0.3), e2s, [parent], dmask, rhs, levels=3,
                   tau=float(np.sqrt(tau2)), extra={"tau2": tau2})


CONFIGS = {"c1": config_c1, "c2": config_c2, "c3": config_c3, "c4": config_c4,
           "c5": config_c5}


# --------------------------------------------------------------------------
# small problems for tests
# --------------------------------------------------------------------------

def make_problem(shape, subs, dof_per_node=1, coeff=None, nu=0.3, dirichlet_axis=0,
                 group=None, rhs="ones", nrhs=1, tau=10.0, nev_max=10, seed=0,
                 cuts=None, name="tiny", levels=None):
    """Generic box problem used by the tests.

    ``subs`` = subdomains per axis (uniform cuts) unless ``cuts`` is given;
    ``coeff`` = None (all ones), an array per element, or "lognormal"
    (10^N(0,1.5)) / "blocks" (10^{0..6} per element, seeded).
    ``dirichlet_axis`` None gives no Dirichlet boundary (singular system);
    ``group`` = boxes per level-2 subdomain per axis.
    """
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    coords, elem_nodes = box_mesh(nx, ny, nz)
    ne = nx * ny * nz
    if coeff is None:
        c = np.ones(ne)
    elif isinstance(coeff, str):
        if coeff == "lognormal":
            c = 10.0 ** rng.normal(0.0, 1.5, size=ne)
        elif coeff == "blocks":
            c = 10.0 ** rng.integers(0, 7, size=ne).astype(float)
        else:
            raise ValueError(coeff)
    else:
        c = np.asarray(coeff, dtype=np.float64)
    if cuts is None:
        cuts = [uniform_cuts(nx, subs[0]), uniform_cuts(ny, subs[1]), uniform_cuts(nz, subs[2])]
    e2s, nb = box_decomposition(shape, cuts)
    parents = []
    if group is not None:
        p, _ = group_boxes(nb, group)
        parents = [p]
    if dirichlet_axis is None:
        dmask = np.zeros(coords.shape[0] * dof_per_node, dtype=np.uint8)
    else:
        dmask = dirichlet_face(coords, dof_per_node, dirichlet_axis)
    nfree = int(np.count_nonzero(dmask == 0))
    if rhs == "ones":
        r = np.ones((nfree, nrhs))
    else:
        r = rng.standard_normal((nfree, nrhs))
    nuv = np.full(ne, nu) if dof_per_node == 3 else None
    if levels is None:
        levels = 2 + len(parents)
    return _finish(name, shape, coords, elem_nodes, dof_per_node, c, nuv, e2s, parents,
                   dmask, r, levels=levels, tau=tau, nev_max=nev_max)


def tiny_poisson(seed=0, shape=(8, 8, 8), subs=(2, 2, 2), coeff="lognormal", **kw):
    return make_problem(shape, subs, 1, coeff=coeff, seed=seed, name="tiny_poisson", **kw)


def tiny_elasticity(seed=0, shape=(6, 6, 6), subs=(2, 2, 2), coeff="lognormal", **kw):
    kw.setdefault("dirichlet_axis", 2)
    return make_problem(shape, subs, 3, coeff=coeff, seed=seed, name="tiny_elasticity", **kw)
