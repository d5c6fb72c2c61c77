"""Pins of the oracle's linear elasticity (paper Sec. 6.2): rigid motions span
the kernel of the unconstrained stiffness, the discrete operator reproduces
-div sigma(u) exactly for displacements in the element space, the clamped
system is symmetric positive definite, and multigrid-preconditioned CG on it
behaves like the paper's (global-local smoothing keeps the reference count)."""
import numpy as np
import pytest

import meshgen
import oracle
from oracle import elasticity as el
from oracle.multigrid import Hierarchy, Options


def _meshes(dim):
    if dim == 2:
        return meshgen.square_mesh(5, 1, n_single=1, single_depth=1e-2)
    return meshgen.cube_mesh(3, 2, slivers=1)


def _rigid_modes(nodes):
    dim = nodes.shape[1]
    modes = []
    for c in range(dim):
        u = np.zeros_like(nodes)
        u[:, c] = 1.0
        modes.append(u)
    if dim == 2:
        modes.append(np.stack([-nodes[:, 1], nodes[:, 0]], axis=1))
    else:
        for w in np.eye(3):
            modes.append(np.cross(w, nodes))
    return [m.ravel() for m in modes]


@pytest.mark.parametrize("dim,degree", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_rigid_motions_are_the_kernel(dim, degree):
    dm, K, _ = el.assemble_full(_meshes(dim), degree, young=2.5, nu=0.3)
    scale = abs(K).max()
    for r in _rigid_modes(dm.nodes):
        assert np.abs(K @ r).max() <= 1e-11 * scale * np.abs(r).max()
    # and nothing else: dim (dim + 1) / 2 zero eigenvalues
    ev = np.linalg.eigvalsh(K.toarray())
    nz = dim * (dim + 1) // 2
    assert np.all(np.abs(ev[:nz]) < 1e-10 * ev[-1]) and ev[nz] > 1e-8 * ev[-1]


def _quadratic_field(nodes, rng):
    """u_c(x) = sum_kl a_ckl x_k x_l + b_ck x_k + c_c and -div sigma(u)."""
    dim = nodes.shape[1]
    a = rng.normal(size=(dim, dim, dim))
    a = 0.5 * (a + a.transpose(0, 2, 1))
    b = rng.normal(size=(dim, dim))
    c = rng.normal(size=dim)
    u = np.einsum("ckl,nk,nl->nc", a, nodes, nodes) + nodes @ b.T + c
    return a, u


@pytest.mark.parametrize("dim", [2, 3])
def test_p2_reproduces_minus_div_sigma(dim):
    """For u in P2, -div sigma(u) = -(mu lap u + (mu + lambda) grad div u) is
    constant, and K I(u) = (M (x) I) I(f) holds on every interior vector DOF."""
    rng = np.random.default_rng(dim)
    young, nu = 3.0, 0.27
    mu, lam = el.lame(young, nu)
    dm, K, M = el.assemble_full(_meshes(dim), 2, young, nu)
    a, u = _quadratic_field(dm.nodes, rng)
    lap = 2.0 * np.einsum("ckk->c", a)                  # lap u_c
    graddiv = 2.0 * np.einsum("kkl->l", a)              # d_l (div u)
    f = -(mu * lap + (mu + lam) * graddiv)
    fvec = np.tile(f, dm.n_dofs)
    from oracle.fem import _facets
    facets, bd = _facets(dm.cells)
    bverts = np.unique(facets[bd])
    boundary = np.zeros(dm.n_dofs, dtype=bool)
    # interior DOFs: vertices off the boundary, and P2 edge DOFs with at least
    # one end off the boundary (conservative: such an edge is not on a
    # boundary facet)
    boundary[bverts] = True
    if dm.n_edges:
        le = oracle.fem.LOCAL_EDGES[dim]
        for cell in range(dm.cells.shape[0]):
            for k, (p, q) in enumerate(le):
                e = dm.cell_dofs[cell, dim + 1 + k]
                if boundary[dm.cells[cell, p]] and boundary[dm.cells[cell, q]]:
                    boundary[e] = True
    interior = el.vector_ids(np.flatnonzero(~boundary), dim)
    lhs = (K @ u.ravel())[interior]
    rhs = (M @ fvec)[interior]
    assert interior.size > 0
    assert np.abs(lhs - rhs).max() <= 1e-9 * np.abs(rhs).max()


def test_p1_patch_test():
    """Linear displacements have constant stress: zero force on interior DOFs."""
    rng = np.random.default_rng(5)
    dm, K, _ = el.assemble_full(_meshes(3), 1, young=1.0, nu=0.3)
    B = rng.normal(size=(3, 3))
    u = dm.nodes @ B.T + rng.normal(size=3)
    from oracle.fem import _facets
    facets, bd = _facets(dm.cells)
    inner = np.setdiff1d(np.arange(dm.n_dofs), np.unique(facets[bd]))
    r = (K @ u.ravel())[el.vector_ids(inner, 3)]
    assert inner.size > 0 and np.abs(r).max() <= 1e-11 * abs(K).max() * np.abs(u).max()


def test_clamped_system_is_spd_and_scales_with_young():
    m = _meshes(3)
    dm, A = el.assemble(m, 1, young=2.0, nu=0.25)
    _, A2 = el.assemble(m, 1, young=6.0, nu=0.25)
    D = A.toarray()
    assert np.allclose(D, D.T, atol=1e-12 * np.abs(D).max())
    assert np.linalg.eigvalsh(D).min() > 0
    assert np.allclose(A2.toarray(), 3.0 * D)
    assert A.shape[0] == 3 * dm.n_free


def test_lattice_global_local_recovers_reference_iterations():
    """Sec. 6.2 (lattice): with low-quality cells the plain smoother needs more
    CG iterations than the reference mesh, the global-local smoother does not."""
    low = meshgen.hierarchy("lattice", seed=0, scale=4)
    ref = meshgen.hierarchy("lattice", seed=0, scale=4, case="ref")
    its = {}
    for name, meshes, local in (("gl", low, True), ("plain", low, False), ("ref", ref, True)):
        H = Hierarchy(meshes, tau=0.1, layers=1,
                      opts=Options(degree=1, local_correction=local, adjusted_eig=local, problem="elasticity"))
        b = meshgen.random_rhs(H.levels[0].A.shape[0], 2)
        _, it, conv, _ = H.pcg(b, 1e-8, 300)
        assert conv
        its[name] = it
    assert its["gl"] <= its["ref"] + 1
    assert its["plain"] >= its["gl"] + 3
