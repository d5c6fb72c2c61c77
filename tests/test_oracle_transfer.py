"""Pins of the oracle's non-nested transfers and Galerkin operators (Sec. 2)."""
import numpy as np
import pytest

import oracle
from oracle.fem import DofMap, assemble
from oracle.transfer import barycentric, galerkin, locate, prolongation
from tests.meshes_util import red_refine, tiny_cube, tiny_square


def _brute_force_locate(points, coords, cells):
    out = []
    allc = np.arange(cells.shape[0])
    for p in points:
        lam = barycentric(coords, cells, allc, np.repeat(p[None], cells.shape[0], 0))
        m = lam.min(axis=1)
        inside = np.flatnonzero(m >= -1e-12)
        if inside.size:
            out.append(inside.min())
        else:
            best = np.flatnonzero(m == m.max())
            out.append(best.min())
    return np.array(out)


def test_locate_matches_brute_force_2d():
    fine = tiny_square(9, seed=1)
    coarse = tiny_square(4, seed=2)
    dmf = DofMap(fine, 3)
    got = locate(dmf.nodes, coarse["coords"], coarse["cells"])
    want = _brute_force_locate(dmf.nodes, coarse["coords"], coarse["cells"].astype(np.int64))
    assert np.array_equal(got, want)


def test_locate_matches_brute_force_3d():
    fine = tiny_cube(4, seed=1)
    coarse = tiny_cube(2, seed=2)
    dmf = DofMap(fine, 2)
    got = locate(dmf.nodes, coarse["coords"], coarse["cells"])
    want = _brute_force_locate(dmf.nodes, coarse["coords"], coarse["cells"].astype(np.int64))
    assert np.array_equal(got, want)


def test_locate_tie_takes_lowest_cell_id():
    coarse = tiny_square(2, seed=0, jitter=0.0, diagonal="right")
    centre = np.array([[0.5, 0.5]])        # vertex shared by six cells
    cells = coarse["cells"].astype(np.int64)
    sharing = np.flatnonzero(np.any(cells == 4, axis=1))
    assert locate(centre, coarse["coords"], cells)[0] == sharing.min()


def test_locate_rejects_points_outside():
    coarse = tiny_square(2, seed=0)
    with pytest.raises(oracle.LocateError):
        locate(np.array([[1.5, 0.5]]), coarse["coords"], coarse["cells"])


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_prolongation_reproduces_polynomials_2d(degree):
    fine = tiny_square(8, seed=3, dirichlet=())
    coarse = tiny_square(4, seed=4, dirichlet=())
    dmf, dmc = DofMap(fine, degree), DofMap(coarse, degree)
    P, _ = prolongation(dmf, dmc)
    assert np.max(np.abs(P @ np.ones(dmc.n_free) - 1.0)) < 1e-13     # partition of unity
    qs = {1: lambda x, y: 1 + 2 * x - y,
          2: lambda x, y: x * y - x * x + 0.3 * y,
          3: lambda x, y: x ** 3 - x * y * y + y}
    q = qs[degree]
    assert np.max(np.abs(P @ q(*dmc.nodes.T) - q(*dmf.nodes.T))) < 1e-12


@pytest.mark.parametrize("degree", [1, 2])
def test_prolongation_reproduces_polynomials_3d(degree):
    fine = tiny_cube(4, seed=3, dirichlet=())
    coarse = tiny_cube(2, seed=4, dirichlet=())
    dmf, dmc = DofMap(fine, degree), DofMap(coarse, degree)
    P, _ = prolongation(dmf, dmc)
    assert np.max(np.abs(P @ np.ones(dmc.n_free) - 1.0)) < 1e-13
    q = (lambda x, y, z: x - 2 * y + z) if degree == 1 else (lambda x, y, z: x * z - y * y + x)
    assert np.max(np.abs(P @ q(*dmc.nodes.T) - q(*dmf.nodes.T))) < 1e-12


def test_prolongation_with_dirichlet_drops_boundary_columns():
    fine = tiny_square(8, seed=3)
    coarse = tiny_square(4, seed=4)
    dmf, dmc = DofMap(fine, 2), DofMap(coarse, 2)
    P, _ = prolongation(dmf, dmc)
    assert P.shape == (dmf.n_free, dmc.n_free)
    # a coarse function vanishing on the boundary: x(1-x)y(1-y) is not in P2,
    # but the interpolant of a P2 function that is zero on the boundary nodes
    # must be reproduced: use the coarse basis expansion directly
    rng = np.random.default_rng(0)
    uc = rng.normal(size=dmc.n_free)
    full = np.zeros(dmc.n_dofs)
    full[dmc.free] = uc
    # evaluate the coarse FE function at fine nodes by barycentric interpolation
    cell = locate(dmf.nodes[dmf.free], dmc.coords, dmc.cells)
    lam = barycentric(dmc.coords, dmc.cells, cell, dmf.nodes[dmf.free])
    basis, _ = oracle.local_basis(2, 2)
    vals = np.stack([oracle.fem.poly_eval(p, lam) for p in basis], axis=1)
    want = np.sum(vals * full[dmc.cell_dofs[cell]], axis=1)
    assert np.max(np.abs(P @ uc - want)) < 1e-13


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_nested_galerkin_equals_rediscretisation(degree):
    """If the fine mesh is a uniform refinement of the coarse one, the coarse
    space is a subspace, P is the exact embedding and P^T A_f P equals the
    coarse stiffness matrix."""
    coarse = tiny_square(3, seed=6)
    fine = red_refine(coarse)
    dmf, Af, _ = assemble(fine, degree)
    dmc, Ac, _ = assemble(coarse, degree)
    P, _ = prolongation(dmf, dmc)
    G = galerkin(Af, P)
    assert abs(G - Ac).max() < 1e-12 * abs(Ac).max()


def test_galerkin_is_symmetric_and_annihilates_constants_on_neumann_rows():
    fine = tiny_square(8, seed=1, dirichlet=("x0",))
    coarse = tiny_square(4, seed=2, dirichlet=("x0",))
    dmf, Af, _ = assemble(fine, 2)
    dmc = DofMap(coarse, 2)
    P, _ = prolongation(dmf, dmc)
    G = galerkin(Af, P)
    assert abs(G - G.T).max() < 1e-13
    # rows of coarse DOFs whose support is away from x = 0: G . 1 = 0
    far = dmc.nodes[dmc.free][:, 0] > 0.6
    assert np.max(np.abs((G @ np.ones(dmc.n_free))[far])) < 1e-12
    assert np.linalg.eigvalsh(G.toarray()).min() > 0
