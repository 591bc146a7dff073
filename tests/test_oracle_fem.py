"""Pins of the oracle's finite-element layer against closed forms.

The Q1 Laplacian on a cube of side h has the element matrix h*Khat with
Khat = 1/3 on the diagonal, 0 between nodes that differ in one coordinate
and -1/12 between nodes that differ in two or three; a trilinear element
reproduces linear displacement fields exactly, so its strain energy for a
homogeneous strain is volume * (lambda tr(eps)^2 + 2 mu eps:eps).
"""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import fem


def _cube(h=1.0, origin=(0.0, 0.0, 0.0)):
    return np.array([[origin[0] + a * h, origin[1] + b * h, origin[2] + c * h]
                     for c in range(2) for b in range(2) for a in range(2)])


def _lattice(i):
    return np.array([i & 1, (i >> 1) & 1, (i >> 2) & 1])


@pytest.mark.parametrize("h", [1.0, 0.25, 1.0 / 16])
def test_poisson_element_closed_form(h):
    K = fem.element_matrix_poisson(_cube(h, (0.3, -1.0, 2.0)), kappa=1.0)
    expect = {0: 1.0 / 3.0, 1: 0.0, 2: -1.0 / 12.0, 3: -1.0 / 12.0}
    for a, b in itertools.product(range(8), range(8)):
        d = int(np.sum(_lattice(a) != _lattice(b)))
        assert K[a, b] == pytest.approx(h * expect[d], abs=1e-14)


def test_poisson_element_scales_with_kappa():
    K1 = fem.element_matrix_poisson(_cube(0.5), 1.0)
    K7 = fem.element_matrix_poisson(_cube(0.5), 7.0)
    np.testing.assert_allclose(K7, 7.0 * K1, rtol=1e-15)


def test_global_poisson_stencil_and_row_sums():
    prob = W.make_problem((6, 6, 6), (1, 1, 1), dirichlet_axis=None)
    K = fem.assemble_global(prob).toarray()
    h = 1.0 / 6
    np.testing.assert_allclose(K.sum(axis=1), 0.0, atol=1e-13)
    # interior node (3,3,3): 27-point stencil
    n = lambda i, j, k: i + 7 * (j + 7 * k)
    c = n(3, 3, 3)
    expect = {0: 8.0 / 3.0, 1: 0.0, 2: -1.0 / 6.0, 3: -1.0 / 12.0}
    for di, dj, dk in itertools.product((-1, 0, 1), repeat=3):
        d = abs(di) + abs(dj) + abs(dk)
        assert K[c, n(3 + di, 3 + dj, 3 + dk)] == pytest.approx(h * expect[d], abs=1e-14)
    assert np.count_nonzero(np.abs(K[c]) > 1e-15) == 1 + 12 + 8


def _strain_energy_dense(E, nu, G, vol):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    eps = 0.5 * (G + G.T)
    return vol * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))


def test_elasticity_element_homogeneous_strain_energy():
    rng = np.random.default_rng(3)
    h = 0.5
    xe = _cube(h, (0.1, 0.2, -0.3))
    E, nu = 2.5, 0.27
    K = fem.element_matrix_elasticity(xe, E, nu)
    for _ in range(5):
        G = rng.standard_normal((3, 3))
        u = (xe @ G.T).ravel()          # u(x) = G x, DOF order 3*node + comp
        assert u @ K @ u == pytest.approx(_strain_energy_dense(E, nu, G, h ** 3), rel=1e-12)


def test_elasticity_element_rigid_modes_and_rank():
    xe = _cube(1.0 / 48)
    K = fem.element_matrix_elasticity(xe, 1.0, 0.3)
    np.testing.assert_allclose(K, K.T, atol=1e-15)
    R = fem.rigid_modes(xe, 3)
    assert np.abs(K @ R).max() < 1e-13 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert np.count_nonzero(ev > 1e-10 * ev[-1]) == 18
    assert ev[0] > -1e-12 * ev[-1]


def test_elasticity_global_rigid_null_space():
    prob = W.make_problem((3, 2, 2), (1, 1, 1), dof_per_node=3, dirichlet_axis=None)
    K = fem.assemble_global(prob).toarray()
    R = fem.rigid_modes(prob.coords, 3)
    assert np.abs(K @ R).max() < 1e-12 * np.abs(K).max()


def test_dirichlet_system_is_spd():
    prob = W.tiny_elasticity(shape=(2, 2, 2), subs=(1, 1, 1))
    K = fem.assemble_global(prob).toarray()
    assert np.linalg.eigvalsh(K)[0] > 0
