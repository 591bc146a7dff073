"""Q1 hexahedral finite elements and global assembly (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's setting (Section 2) is a conforming FE discretisation with one
DOF per node for the scalar problem and three displacement DOFs per node
for linear elasticity; its examples use tri-linear hexahedra (Section 8).
Element matrices here use the trilinear map and 2x2x2 Gauss quadrature,
which integrates the Q1 stiffness exactly on parallelepipeds.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# reference node positions, local index a + 2b + 4c  ->  (xi, eta, zeta)
_REF = np.array([[(-1.0 if a == 0 else 1.0), (-1.0 if b == 0 else 1.0), (-1.0 if c == 0 else 1.0)]
                 for c in range(2) for b in range(2) for a in range(2)])
_G = 1.0 / np.sqrt(3.0)
_GAUSS = np.array([[x, y, z] for z in (-_G, _G) for y in (-_G, _G) for x in (-_G, _G)])


def _shape_grads(xi):
    """Derivatives of the 8 trilinear shape functions at reference point xi: (8, 3)."""
    d = np.empty((8, 3))
    for n in range(8):
        r = _REF[n]
        f = [(1.0 + r[q] * xi[q]) for q in range(3)]
        d[n, 0] = 0.125 * r[0] * f[1] * f[2]
        d[n, 1] = 0.125 * f[0] * r[1] * f[2]
        d[n, 2] = 0.125 * f[0] * f[1] * r[2]
    return d


_DN = np.stack([_shape_grads(g) for g in _GAUSS])   # (8 gauss, 8 nodes, 3)


def _physical_grads(xe):
    """Physical shape gradients and Jacobian determinants at the Gauss points.

    xe: (8, 3) node coordinates.  Returns (grads (8g, 8n, 3), detJ (8g,)).
    """
    grads = np.empty((8, 8, 3))
    dets = np.empty(8)
    for g in range(8):
        J = _DN[g].T @ xe            # J[i, j] = d x_j / d xi_i
        dets[g] = np.linalg.det(J)
        grads[g] = np.linalg.solve(J, _DN[g].T).T
    return grads, dets


def element_matrix_poisson(xe, kappa=1.0):
    """K_e[a, b] = kappa * integral grad N_a . grad N_b over the element."""
    grads, dets = _physical_grads(np.asarray(xe, dtype=np.float64))
    K = np.zeros((8, 8))
    for g in range(8):
        K += dets[g] * grads[g] @ grads[g].T
    return kappa * K


def lame(E, nu):
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def element_matrix_elasticity(xe, E=1.0, nu=0.3):
    """24x24 isotropic linear-elastic stiffness, DOF order 3*node + component.

    Strain in Voigt order (xx, yy, zz, yz, xz, xy) with engineering shears;
    D = lambda * m m^T + mu * diag(2, 2, 2, 1, 1, 1).
    """
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D += np.diag([2 * mu, 2 * mu, 2 * mu, mu, mu, mu])
    grads, dets = _physical_grads(np.asarray(xe, dtype=np.float64))
    K = np.zeros((24, 24))
    for g in range(8):
        B = np.zeros((6, 24))
        for n in range(8):
            dx, dy, dz = grads[g, n]
            c = 3 * n
            B[0, c] = dx
            B[1, c + 1] = dy
            B[2, c + 2] = dz
            B[3, c + 1] = dz
            B[3, c + 2] = dy
            B[4, c] = dz
            B[4, c + 2] = dx
            B[5, c] = dy
            B[5, c + 1] = dx
        K += dets[g] * B.T @ D @ B
    return K


def element_matrices(prob, coeff=None):
    """All element matrices of a problem, (n_elems, ne, ne).

    Elements of a structured box mesh that are translates of each other
    share the unit-coefficient matrix; it is computed per distinct shape.
    """
    coeff = prob.coeff if coeff is None else coeff
    xe_all = prob.coords[prob.elem_nodes]              # (ne, 8, 3)
    rel = xe_all - xe_all[:, :1, :]
    key = np.round(rel.reshape(len(rel), -1), 12)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    inv = inv.ravel()
    d = prob.dof_per_node
    out = np.empty((prob.n_elems, 8 * d, 8 * d))
    for u in range(len(uniq)):
        sel = np.flatnonzero(inv == u)
        xe = xe_all[sel[0]]
        if d == 1:
            Kref = element_matrix_poisson(xe, 1.0)
            out[sel] = coeff[sel, None, None] * Kref[None]
        else:
            # elasticity stiffness is linear in E for fixed nu
            nus = prob.nu[sel]
            for nu in np.unique(nus):
                s2 = sel[nus == nu]
                Kref = element_matrix_elasticity(xe, 1.0, float(nu))
                out[s2] = coeff[s2, None, None] * Kref[None]
    return out


def elem_dof_ids(prob):
    """Global DOF ids (before Dirichlet removal) of every element, (ne, 8*d)."""
    d = prob.dof_per_node
    en = prob.elem_nodes.astype(np.int64)
    return (en[:, :, None] * d + np.arange(d)[None, None, :]).reshape(len(en), 8 * d)


def free_map(prob):
    """Map full DOF id -> free DOF id (-1 for Dirichlet)."""
    fm = -np.ones(prob.n_dofs_total, dtype=np.int64)
    free = np.flatnonzero(prob.dirichlet == 0)
    fm[free] = np.arange(len(free))
    return fm


def assemble_global(prob, Ke=None, coeff=None):
    """Global stiffness on the free DOFs as a CSR matrix."""
    if Ke is None:
        Ke = element_matrices(prob, coeff)
    dofs = free_map(prob)[elem_dof_ids(prob)]
    ne, m = dofs.shape
    rows = np.repeat(dofs, m, axis=1).ravel()
    cols = np.tile(dofs, (1, m)).ravel()
    vals = Ke.reshape(ne, m * m).ravel()
    keep = (rows >= 0) & (cols >= 0)
    n = prob.n_free
    return sp.csr_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n, n))


def rigid_modes(coords, dof_per_node):
    """Rigid-body modes evaluated at nodes, (n_nodes*d, n_rb).

    Poisson: the constant.  Elasticity: 3 translations and 3 rotations about
    the centroid of ``coords``.
    """
    n = coords.shape[0]
    if dof_per_node == 1:
        return np.ones((n, 1))
    x = coords - coords.mean(axis=0)
    R = np.zeros((n, 3, 6))
    for c in range(3):
        R[:, c, c] = 1.0
    # rotation about x: (0, -z, y); about y: (z, 0, -x); about z: (-y, x, 0)
    R[:, 1, 3] = -x[:, 2]
    R[:, 2, 3] = x[:, 1]
    R[:, 0, 4] = x[:, 2]
    R[:, 2, 4] = -x[:, 0]
    R[:, 0, 5] = -x[:, 1]
    R[:, 1, 5] = x[:, 0]
    return R.reshape(n * 3, 6)
