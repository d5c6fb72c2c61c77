"""Pins of the oracle's V-cycle (Algorithm alg:mg) and MG-preconditioned CG
(Sec. 6.2): brute-force dense multigrid operators on tiny meshes, exact
coarse solves, and the paper's qualitative claims on iteration counts."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import meshgen
import oracle
from oracle.multigrid import Hierarchy, Options


def _tiny_hierarchy(degree=1, sides=(8, 4), nu=2, k=2, local=True, seed=0, n_single=2):
    meshes = [meshgen.square_mesh(sides[0], seed, n_single=n_single, single_depth=1e-3)]
    meshes += [meshgen.square_mesh(s, seed + 10 + i) for i, s in enumerate(sides[1:])]
    return Hierarchy(meshes, tau=0.1, layers=1,
                     opts=Options(degree=degree, nu=nu, cheb_degree=k, local_correction=local))


def _dense_smoother(H, l):
    lev = H.levels[l]
    n = lev.A.shape[0]
    return np.stack([H.smooth(l, e, np.zeros(n), 1) for e in np.eye(n)], axis=1)


def _dense_B(H, l):
    """Brute-force V-cycle operator B_l (u = B_l b from u = 0):
    E_l = (I - S A)^nu (I - P B_(l+1) P^T A) (I - S A)^nu,  B_l = (I - E_l) A^-1."""
    lev = H.levels[l]
    Ad = lev.A.toarray()
    if l == len(H.levels) - 1:
        return np.linalg.inv(Ad)
    n = Ad.shape[0]
    S = _dense_smoother(H, l)
    I = np.eye(n)
    P = lev.P.toarray()
    Esm = np.linalg.matrix_power(I - S @ Ad, H.opts.nu)
    E = Esm @ (I - P @ _dense_B(H, l + 1) @ P.T @ Ad) @ Esm
    return (I - E) @ np.linalg.inv(Ad)


@pytest.mark.parametrize("sides,degree", [((8, 4), 1), ((6, 3), 2), ((10, 5, 3), 1)])
def test_vcycle_equals_brute_force_operator(sides, degree):
    H = _tiny_hierarchy(degree=degree, sides=sides)
    n = H.levels[0].A.shape[0]
    V = np.stack([H.vcycle(e) for e in np.eye(n)], axis=1)
    B = _dense_B(H, 0)
    assert np.allclose(V, B, atol=1e-9 * np.abs(B).max())
    # symmetric positive definite preconditioner
    assert np.allclose(V, V.T, atol=1e-9 * np.abs(V).max())
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0


def test_vcycle_with_nonzero_initial_guess_is_affine():
    H = _tiny_hierarchy(sides=(8, 4))
    n = H.levels[0].A.shape[0]
    rng = np.random.default_rng(2)
    b, u = rng.normal(size=n), rng.normal(size=n)
    B = _dense_B(H, 0)
    A = H.levels[0].A
    assert np.allclose(H.vcycle(b, u), u + B @ (b - A @ u), atol=1e-10)


def test_stationary_solver_is_the_iteration_of_the_dense_operator():
    """x_(k+1) = x_k + B (b - A x_k) with the brute-force B: after k cycles the
    error is (I - B A)^k e_0, and the residual history is that of the dense
    iteration."""
    H = _tiny_hierarchy(sides=(8, 4))
    A = H.levels[0].A
    n = A.shape[0]
    b = np.random.default_rng(3).normal(size=n)
    B = _dense_B(H, 0)
    x, it, conv, hist = H.mg_solve(b, 1e-300, 6)
    assert it == 6 and not conv and len(hist) == 7
    xs = np.zeros(n)
    for k in range(6):
        xs = xs + B @ (b - A @ xs)
        assert abs(hist[k + 1] - np.linalg.norm(b - A @ xs) / np.linalg.norm(b)) < 1e-9
    assert np.allclose(x, xs, atol=1e-9 * np.abs(xs).max())
    u = np.linalg.solve(A.toarray(), b)
    E = np.eye(n) - B @ A.toarray()
    assert np.allclose(u - x, np.linalg.matrix_power(E, 6) @ u, atol=1e-9 * np.abs(u).max())
    # convergence to the direct solution; zero right-hand side
    x, it, conv, _ = H.mg_solve(b, 1e-10, 100)
    assert conv and np.linalg.norm(x - u) <= 1e-8 * np.linalg.norm(u)
    assert H.mg_solve(np.zeros(n), 1e-8, 10)[1] == 0


def test_galerkin_coarse_operator_in_hierarchy():
    H = _tiny_hierarchy(sides=(8, 4))
    l0, l1 = H.levels
    want = (l0.P.T @ l0.A @ l0.P).toarray()
    assert np.allclose(l1.A.toarray(), want, atol=1e-14)


def test_single_level_pcg_converges_in_one_iteration():
    mesh = meshgen.square_mesh(6, 0)
    H = Hierarchy([mesh], opts=Options(degree=2))
    b = meshgen.random_rhs(H.levels[0].A.shape[0], 0)
    x, it, conv, _ = H.pcg(b, 1e-12, 10)
    assert conv and it == 1
    assert np.allclose(x, spla.spsolve(H.levels[0].A.tocsc(), b), rtol=1e-10)


def test_pcg_solution_matches_direct_solve():
    H = _tiny_hierarchy(degree=2, sides=(10, 5))
    A = H.levels[0].A
    b = meshgen.random_rhs(A.shape[0], 3)
    x, it, conv, hist = H.pcg(b, 1e-12, 100)
    assert conv
    assert np.linalg.norm(b - A @ x) <= 1.01e-12 * np.linalg.norm(b)
    assert np.allclose(x, spla.spsolve(A.tocsc(), b), rtol=1e-8, atol=1e-12)
    assert all(h2 < 10 * h1 for h1, h2 in zip(hist, hist[1:]))


def test_pcg_zero_rhs():
    H = _tiny_hierarchy(sides=(6, 3))
    n = H.levels[0].A.shape[0]
    x, it, conv, _ = H.pcg(np.zeros(n), 1e-10, 10)
    assert conv and it == 0 and np.all(x == 0)


def test_rhs_from_nodal_is_mass_times_nodal_values():
    mesh = meshgen.square_mesh(6, 0, dirichlet=("y0", "y1"))
    H = Hierarchy([mesh], opts=Options(degree=2))
    dm = H.levels[0].dofmap
    f = np.ones(dm.n_dofs)
    b = H.rhs_from_nodal(f)
    # sum over free rows of int phi_i = area minus the Dirichlet share
    _, _, M = oracle.assemble_full(mesh, 2)
    assert np.allclose(b, (M @ f)[dm.free])


def test_global_local_recovers_reference_iterations():
    """Table number_struct / Sec. 6: with the local correction and adjusted
    eigenvalue, CG iterations return to the high-quality reference count
    (within one), while the plain smoother needs many more."""
    low = meshgen.hierarchy("square_p1_4k", seed=0)
    ref = meshgen.hierarchy("square_p1_4k", seed=0, case="ref")
    its = {}
    for name, meshes, local in (("gl", low, True), ("plain", low, False), ("ref", ref, True)):
        H = Hierarchy(meshes, tau=0.1, layers=2,
                      opts=Options(degree=1, local_correction=local, adjusted_eig=local))
        b = meshgen.random_rhs(H.levels[0].A.shape[0], 1)
        _, it, conv, _ = H.pcg(b, 1e-10, 200)
        assert conv
        its[name] = it
    assert abs(its["gl"] - its["ref"]) <= 1
    assert its["plain"] >= its["gl"] + 4


def test_sgs_vcycle_equals_brute_force_operator():
    """Symmetric Gauss-Seidel as S_g: the cycle is the dense multigrid operator
    built from the smoother's own dense matrix, and symmetric positive definite."""
    meshes = [meshgen.square_mesh(8, 0, n_single=2, single_depth=1e-3), meshgen.square_mesh(4, 10)]
    H = Hierarchy(meshes, tau=0.1, layers=1, opts=Options(degree=1, global_smoother="sgs"))
    n = H.levels[0].A.shape[0]
    V = np.stack([H.vcycle(e) for e in np.eye(n)], axis=1)
    B = _dense_B(H, 0)
    assert np.allclose(V, B, atol=1e-9 * np.abs(B).max())
    assert np.allclose(V, V.T, atol=1e-9 * np.abs(V).max())
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0


def test_sgs_global_local_recovers_reference_cycles():
    """Sec. 3.2 / Sec. 6.1 with symmetric Gauss-Seidel as the global smoother
    (multigrid as a stationary solver, as in the paper): the local correction
    restores the reference mesh's cycle count, the plain smoother does not."""
    low = meshgen.hierarchy("square_p1_4k", seed=0)
    ref = meshgen.hierarchy("square_p1_4k", seed=0, case="ref")
    cyc = {}
    for name, meshes, local in (("gl", low, True), ("plain", low, False), ("ref", ref, True)):
        H = Hierarchy(meshes, tau=0.1, layers=2,
                      opts=Options(degree=1, local_correction=local, adjusted_eig=local, global_smoother="sgs",
                                   nu=1))
        b = meshgen.random_rhs(H.levels[0].A.shape[0], 1)
        _, it, conv, _ = H.mg_solve(b, 1e-8, 300)
        assert conv
        cyc[name] = it
    assert cyc["gl"] <= cyc["ref"] + 2
    assert cyc["plain"] >= 2 * cyc["gl"]


def test_given_prolongations_and_intervals_reproduce_the_hierarchy():
    """The large-size checks build the oracle from given transfer operators
    and Chebyshev intervals; given the oracle's own, the cycle is unchanged."""
    meshes = meshgen.hierarchy("square_1025", seed=0, scale=32)
    opts = Options(degree=2)
    H = Hierarchy(meshes, tau=0.1, layers=1, opts=opts)
    G = Hierarchy(meshes, tau=0.1, layers=1, opts=opts,
                  prolongations=[lev.P for lev in H.levels[:-1]],
                  intervals=[(lev.lo, lev.hi) for lev in H.levels[:-1]])
    for a, b in zip(H.levels, G.levels):
        assert (a.A != b.A).nnz == 0
    n = H.levels[0].A.shape[0]
    b = meshgen.random_rhs(n, 3)
    assert np.array_equal(H.vcycle(b), G.vcycle(b))
    # a different interval changes the cycle (the option is really used)
    W = Hierarchy(meshes, tau=0.1, layers=1, opts=opts, prolongations=[lev.P for lev in H.levels[:-1]],
                  intervals=[(lev.lo, 1.5 * lev.hi) for lev in H.levels[:-1]])
    assert not np.allclose(H.vcycle(b), W.vcycle(b), rtol=1e-6, atol=0)


def test_replaced_coarse_operators():
    """Given its own Galerkin products, the cycle is unchanged; given perturbed
    coarse operators, it changes."""
    meshes = meshgen.hierarchy("square_1025", seed=0, scale=32)
    H = Hierarchy(meshes, tau=0.1, layers=1, opts=Options(degree=2))
    n = H.levels[0].A.shape[0]
    b = meshgen.random_rhs(n, 3)
    x = H.vcycle(b)
    H.replace_coarse_operators([lev.A.copy() for lev in H.levels[1:]])
    assert np.array_equal(x, H.vcycle(b))
    H.replace_coarse_operators([1.01 * lev.A for lev in H.levels[1:]])
    assert not np.allclose(x, H.vcycle(b), rtol=1e-6, atol=0)
