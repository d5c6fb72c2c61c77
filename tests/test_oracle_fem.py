"""Pins of the oracle's discretisation (Sec. 2 eq. system_finest, Sec. 6.1).

Each test checks the oracle against something other than itself: closed-form
stencils, the P1 cotangent formula, polynomial consistency identities that any
correct Galerkin discretisation satisfies, exact reproduction of polynomial
solutions, and counting identities of the DOF map.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from oracle.fem import DofMap, assemble, assemble_full, element_matrices
from tests.meshes_util import tiny_cube, tiny_square


def _cot(u, v):
    return np.dot(u, v) / abs(u[0] * v[1] - u[1] * v[0])


def test_p1_triangle_matches_cotangent_formula():
    rng = np.random.default_rng(3)
    for _ in range(20):
        x = rng.uniform(-1, 1, size=(3, 2))
        if np.linalg.det(np.stack([x[1] - x[0], x[2] - x[0]])) < 0:
            x = x[[0, 2, 1]]
        Ke, _ = element_matrices(x, np.array([[0, 1, 2]]), 1)
        K = Ke[0]
        for i in range(3):
            for j in range(3):
                if i == j:
                    continue
                k = 3 - i - j
                expect = -0.5 * _cot(x[i] - x[k], x[j] - x[k])
                assert abs(K[i, j] - expect) <= 1e-12 * (1 + abs(expect))


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_stiffness_annihilates_constants_and_is_symmetric(degree):
    dm, K, M = assemble_full(tiny_square(5, seed=degree), degree)
    one = np.ones(dm.n_dofs)
    assert np.max(np.abs(K @ one)) < 1e-12
    assert abs(K - K.T).max() < 1e-13
    assert abs(one @ (M @ one) - 1.0) < 1e-13           # |Omega| = 1


@pytest.mark.parametrize("degree", [1, 2])
def test_stiffness_annihilates_constants_3d(degree):
    dm, K, M = assemble_full(tiny_cube(2, seed=degree), degree)
    one = np.ones(dm.n_dofs)
    assert np.max(np.abs(K @ one)) < 1e-12
    assert abs(one @ (M @ one) - 1.0) < 1e-13


def test_unjittered_square_gives_five_point_stencil():
    n = 6
    mesh = tiny_square(n, jitter=0.0, diagonal="right")
    dm, K, _ = assemble_full(mesh, 1)
    for v in range(dm.n_dofs):
        i, j = v % (n + 1), v // (n + 1)
        if 0 < i < n and 0 < j < n:
            row = K[v].toarray().ravel()
            assert abs(row[v] - 4.0) < 1e-12
            for nb in (v - 1, v + 1, v - (n + 1), v + (n + 1)):
                assert abs(row[nb] + 1.0) < 1e-12
            others = np.delete(row, [v, v - 1, v + 1, v - n - 1, v + n + 1])
            assert np.max(np.abs(others)) < 1e-12


def test_unjittered_kuhn_cube_gives_seven_point_stencil():
    n = 3
    h = 1.0 / n
    mesh = tiny_cube(n, jitter=0.0)
    dm, K, _ = assemble_full(mesh, 1)
    m = n + 1
    v = 1 + m * 1 + m * m * 1    # interior vertex (1,1,1)
    row = K[v].toarray().ravel()
    assert K[v].nnz == 15                       # Kuhn vertex has 14 neighbours
    assert abs(row[v] - 6 * h) < 1e-12
    for nb in (v - 1, v + 1, v - m, v + m, v - m * m, v + m * m):
        assert abs(row[nb] + h) < 1e-12
    rest = np.delete(row, [v, v - 1, v + 1, v - m, v + m, v - m * m, v + m * m])
    assert np.max(np.abs(rest)) < 1e-12


def _interior_dofs(dm):
    """DOFs whose basis support does not touch the domain boundary."""
    on_bnd_vertex = np.any((dm.coords < 1e-12) | (dm.coords > 1 - 1e-12), axis=1)
    bad_cells = np.any(on_bnd_vertex[dm.cells], axis=1)
    touched = np.unique(dm.cell_dofs[bad_cells])
    keep = np.ones(dm.n_dofs, dtype=bool)
    keep[touched] = False
    return np.flatnonzero(keep)


_POLYS_2D = {
    1: (lambda x, y: 0.3 + 2 * x - 1.5 * y, lambda x, y: 0 * x),
    2: (lambda x, y: x * x - 3 * x * y + 0.5 * y * y + x,
        lambda x, y: -(2 - 0 + 1.0) + 0 * x),          # -Laplace = -(2 + 1)
    3: (lambda x, y: x ** 3 - 2 * x * y * y + y ** 2,
        lambda x, y: -(6 * x - 4 * x + 2)),             # -Laplace
}


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_polynomial_consistency_2d(degree):
    """For q of degree <= p: (K I(q))_i = int(-Lap q) phi_i = (M I(-Lap q))_i
    on DOFs whose support avoids the boundary (Green's formula, exact)."""
    dm, K, M = assemble_full(tiny_square(8, seed=11 + degree), degree)
    q, f = _POLYS_2D[degree]
    X, Y = dm.nodes[:, 0], dm.nodes[:, 1]
    lhs = K @ q(X, Y)
    rhs = M @ f(X, Y)
    inner = _interior_dofs(dm)
    assert inner.size > 10
    assert np.max(np.abs(lhs[inner] - rhs[inner])) < 1e-11


@pytest.mark.parametrize("degree", [1, 2])
def test_polynomial_consistency_3d(degree):
    dm, K, M = assemble_full(tiny_cube(4, seed=5 + degree), degree)
    X, Y, Z = dm.nodes.T
    if degree == 1:
        q, f = 1 + X - 2 * Y + 0.5 * Z, 0 * X
    else:
        q, f = X * Y + Z * Z - X * X + 0.25 * Y * Y, -(2 - 2 + 0.5) + 0 * X
    inner = _interior_dofs(dm)
    assert inner.size > 0
    assert np.max(np.abs((K @ q - M @ f)[inner])) < 1e-11


@pytest.mark.parametrize("degree,dim", [(2, 2), (3, 2), (2, 3)])
def test_exact_solution_is_reproduced(degree, dim):
    """u = x(1-x) (P2) or x - x^3 (P3) with u = 0 on x = 0, 1 and zero flux
    elsewhere lies in V_h, so the discrete solution equals its interpolant."""
    if dim == 2:
        mesh = tiny_square(6, seed=7, dirichlet=("x0", "x1"))
    else:
        mesh = tiny_cube(3, seed=7, dirichlet=("x0", "x1"))
    dm, A, Mf = assemble(mesh, degree)
    X = dm.nodes[:, 0]
    if degree == 2:
        u_exact, f = X * (1 - X), 2.0 + 0 * X
    else:
        u_exact, f = X - X ** 3, 6 * X
    u = spla.spsolve(A.tocsc(), Mf @ f)
    assert np.max(np.abs(u - u_exact[dm.free])) < 1e-11


def test_reduced_operator_is_spd():
    for degree in (1, 2, 3):
        dm, A, _ = assemble(tiny_square(4, seed=degree), degree)
        Ad = A.toarray()
        assert np.allclose(Ad, Ad.T, atol=1e-14)
        assert np.linalg.eigvalsh(Ad).min() > 0


def test_dof_counts():
    n = 7
    for degree, expect in ((1, (n + 1) ** 2), (2, (2 * n + 1) ** 2), (3, (3 * n + 1) ** 2)):
        dm = DofMap(tiny_square(n, seed=1), degree)
        assert dm.n_dofs == expect
    mesh = tiny_cube(3, seed=1)
    assert DofMap(mesh, 2).n_dofs == 7 ** 3
    # every DOF node is inside the unit square / cube
    dm = DofMap(tiny_square(n, seed=2), 3)
    assert np.all(dm.nodes >= -1e-15) and np.all(dm.nodes <= 1 + 1e-15)


def test_dirichlet_dofs_lie_on_dirichlet_sides():
    mesh = tiny_square(6, seed=3, dirichlet=("y0", "y1"))
    for degree in (2, 3):
        dm = DofMap(mesh, degree)
        y = dm.nodes[:, 1]
        on = (y < 1e-12) | (y > 1 - 1e-12)
        assert np.array_equal(dm.dirichlet, on)
    mesh = tiny_cube(3, seed=3, dirichlet=("x0", "x1"))
    dm = DofMap(mesh, 2)
    x = dm.nodes[:, 0]
    assert np.array_equal(dm.dirichlet, (x < 1e-12) | (x > 1 - 1e-12))


def test_p3_edge_nodes_follow_low_to_high_vertex():
    dm = DofMap(tiny_square(3, seed=4), 3)
    nv = dm.coords.shape[0]
    # each edge DOF pair: first node closer to the lower-id vertex
    cells = dm.cells
    for c in range(cells.shape[0]):
        for k, (a, b) in enumerate(oracle.fem.LOCAL_EDGES[2]):
            ga, gb = cells[c, a], cells[c, b]
            lo, hi = min(ga, gb), max(ga, gb)
            d1, d2 = dm.cell_dofs[c, 3 + 2 * k], dm.cell_dofs[c, 4 + 2 * k]
            first = min(d1, d2)
            assert first >= nv and (first - nv) % 2 == 0
            assert np.allclose(dm.nodes[first], (2 * dm.coords[lo] + dm.coords[hi]) / 3)
