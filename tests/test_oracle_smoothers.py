"""Pins of the oracle's smoothers (Sec. 3.2, 4.1, 4.2, 5)."""
import numpy as np
import pytest
import scipy.linalg as sla
from numpy.polynomial import chebyshev as C

import meshgen
import oracle
from oracle.fem import DofMap, assemble
from oracle.patches import MERGE, OVERLAP, colour, patches
from oracle.smoothers import LocalCorrection, chebyshev, lanczos_lmax, sandwich, start_vector
from tests.meshes_util import tiny_cube, tiny_square


def _system(n=8, seed=3, degree=1, n_single=2, dirichlet=("x0", "x1", "y0", "y1")):
    mesh = meshgen.square_mesh(n, seed, n_single=n_single, single_depth=1e-3, dirichlet=dirichlet)
    dm, A, _ = assemble(mesh, degree)
    return mesh, dm, A


def _cheb_factor(t, k, lo, hi):
    """T_k((theta - t)/delta) / T_k(theta/delta)."""
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    ck = np.zeros(k + 1)
    ck[k] = 1
    return C.chebval((theta - t) / delta, ck) / C.chebval(theta / delta, ck)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_chebyshev_error_polynomial(k):
    _, _, A = _system()
    Ad = A.toarray()
    D = np.diag(np.diag(Ad))
    t, V = sla.eigh(Ad, D)               # D^-1 A v = t v
    hi = t.max() * 1.02
    lo = hi / 10
    dinv = 1.0 / np.diag(Ad)
    for j in (0, len(t) // 3, len(t) - 1):
        v = V[:, j]
        x = chebyshev(A, dinv, np.zeros_like(v), v.copy(), k, lo, hi)
        assert np.allclose(x, _cheb_factor(t[j], k, lo, hi) * v, atol=1e-12)


def test_lanczos_matches_closed_form_square():
    """5-point Dirichlet grid with n cells per side: lambda_max(D^-1 A) = 1 + cos(pi/n)."""
    n = 12
    mesh = tiny_square(n, jitter=0.0, diagonal="right")
    _, A, _ = assemble(mesh, 1)
    lam, its = lanczos_lmax(A, None, 1e-10, 400)
    assert abs(lam - (1 + np.cos(np.pi / n))) < 1e-9


def test_lanczos_matches_closed_form_cube():
    n = 6
    mesh = tiny_cube(n, jitter=0.0, dirichlet=("x0", "x1", "y0", "y1", "z0", "z1"))
    _, A, _ = assemble(mesh, 1)
    lam, _ = lanczos_lmax(A, None, 1e-10, 400)
    assert abs(lam - (1 + np.cos(np.pi / n))) < 1e-9


@pytest.mark.parametrize("degree", [1, 2])
def test_lanczos_and_adjusted_match_dense_eigensolver(degree):
    mesh, dm, A = _system(n=10, seed=5, degree=degree, n_single=3)
    gamma = oracle.radius_ratio(mesh["coords"], mesh["cells"])
    _, pd = patches(dm.cells, dm.coords.shape[0], gamma, 0.1, 1, MERGE, dm.cell_dofs, dm.free_index)
    assert pd
    Ad = A.toarray()
    lam, _ = lanczos_lmax(A, None, 1e-10, 500)
    want = sla.eigh(Ad, np.diag(np.diag(Ad)), eigvals_only=True).max()
    assert abs(lam - want) < 1e-8 * want
    g = np.ones(A.shape[0], dtype=bool)
    for B in pd:
        g[B] = False
    lam_adj, _ = lanczos_lmax(A, g, 1e-10, 500)
    Agg = Ad[np.ix_(g, g)]
    want_adj = sla.eigh(Agg, np.diag(np.diag(Agg)), eigvals_only=True).max()
    assert abs(lam_adj - want_adj) < 1e-8 * want_adj
    # Sec. 5 / table eig_cube: the adjusted value is well below the unadjusted one
    assert lam_adj < lam


def test_start_vector_is_splitmix64():
    """First outputs of SplitMix64 from seeds 0, 1 (published reference values
    for state 0: 0xE220A8397B1DCDAF)."""
    z = oracle.splitmix64(np.array([0], dtype=np.uint64))[0]
    assert int(z) == 0xE220A8397B1DCDAF
    v = start_vector(4)
    assert np.all(np.abs(v) < 1)
    assert v[0] == (0xE220A8397B1DCDAF >> 11) * 2.0 ** -53 * 2 - 1


def _local(A, pd, policy_colours=None):
    cols = colour(pd) if policy_colours is None else policy_colours
    return LocalCorrection(A, pd, cols)


def test_local_correction_is_patch_direct_solve():
    mesh, dm, A = _system(n=10, seed=7, degree=2, n_single=3)
    gamma = oracle.radius_ratio(mesh["coords"], mesh["cells"])
    _, pd = patches(dm.cells, dm.coords.shape[0], gamma, 0.1, 1, MERGE, dm.cell_dofs, dm.free_index)
    L = _local(A, pd)
    rng = np.random.default_rng(0)
    b, u = rng.normal(size=A.shape[0]), rng.normal(size=A.shape[0])
    out = L.apply(A, b, u)
    r = b - A @ u
    want = u.copy()
    Ad = A.toarray()
    for B in pd:                        # eq. local / local_update, dense solves
        want[B] += np.linalg.solve(Ad[np.ix_(B, B)], r[B])
    assert np.allclose(out, want, rtol=1e-10, atol=1e-12)


def test_single_patch_correction_is_a_projection():
    mesh, dm, A = _system(n=10, seed=8, degree=1, n_single=1)
    gamma = oracle.radius_ratio(mesh["coords"], mesh["cells"])
    _, pd = patches(dm.cells, dm.coords.shape[0], gamma, 0.1, 1, MERGE, dm.cell_dofs, dm.free_index)
    assert len(pd) == 1
    L = _local(A, pd)
    n = A.shape[0]
    # dense S_c from unit right-hand sides with u = 0
    Sc = np.stack([L.apply(A, e, np.zeros(n)) for e in np.eye(n)], axis=1)
    Ad = A.toarray()
    ScA = Sc @ Ad
    assert np.allclose(ScA @ ScA, ScA, atol=1e-10)
    rng = np.random.default_rng(1)
    b, u = rng.normal(size=n), rng.normal(size=n)
    u2 = L.apply(A, b, u)
    assert np.max(np.abs((b - A @ u2)[pd[0]])) < 1e-10


def _dense_Sg(Ad, k, lo, hi):
    """x <- x + S_g (b - A x) for the Chebyshev smoother, from the spectral
    decomposition: 1 - t q(t) = T_k((theta-t)/delta)/T_k(theta/delta)."""
    D = np.diag(np.diag(Ad))
    t, V = sla.eigh(Ad, D)           # V^T D V = I
    q = (1 - _cheb_factor(t, k, lo, hi)) / t
    return V @ np.diag(q) @ V.T       # = V q(T) V^-1 D^-1 with V^-1 = V^T D


@pytest.mark.parametrize("policy", [MERGE, OVERLAP])
def test_sandwich_equals_paper_formula_and_is_symmetric(policy):
    """S_gc = 2 S_c - S_c A S_c + (I - S_c A) S_g (I - A S_c)  (Sec. 4.2)."""
    mesh, dm, A = _system(n=9, seed=4, degree=2, n_single=2)
    gamma = oracle.radius_ratio(mesh["coords"], mesh["cells"])
    _, pd = patches(dm.cells, dm.coords.shape[0], gamma, 0.1, 1, policy, dm.cell_dofs, dm.free_index)
    cols = colour(pd)
    if policy == MERGE:
        assert np.all(cols == 0)
    L = LocalCorrection(A, pd, cols)
    Ad = A.toarray()
    n = A.shape[0]
    dinv = 1 / np.diag(Ad)
    hi = 1.05 * sla.eigh(Ad, np.diag(np.diag(Ad)), eigvals_only=True).max()
    lo = hi / 10
    Sgc = np.stack([sandwich(A, dinv, e, np.zeros(n), L, 2, lo, hi) for e in np.eye(n)], axis=1)
    Sg = _dense_Sg(Ad, 2, lo, hi)
    I = np.eye(n)
    if np.all(cols == 0):
        Sc = np.zeros((n, n))
        for B in pd:
            Sc[np.ix_(B, B)] += np.linalg.inv(Ad[np.ix_(B, B)])
        want = 2 * Sc - Sc @ Ad @ Sc + (I - Sc @ Ad) @ Sg @ (I - Ad @ Sc)
        assert np.allclose(Sgc, want, atol=1e-9 * np.abs(want).max())
    assert np.allclose(Sgc, Sgc.T, atol=1e-10 * np.abs(Sgc).max())


def test_smoother_error_localises_at_low_quality_cells():
    """Sec. 3.2: after a few smoothing steps from a high-frequency guess the
    remaining error concentrates around the low-quality cells; with the local
    correction the error there drops."""
    mesh = meshgen.square_mesh(24, 3, n_single=1, single_depth=1e-4)
    dm, A, _ = assemble(mesh, 1)
    gamma = oracle.radius_ratio(mesh["coords"], mesh["cells"])
    _, pd = patches(dm.cells, dm.coords.shape[0], gamma, 0.1, 1, MERGE, dm.cell_dofs, dm.free_index)
    x, y = dm.nodes[dm.free].T
    u0 = np.sin(10 * np.pi * x) * np.sin(10 * np.pi * y)
    b = np.zeros_like(u0)
    dinv = 1 / A.diagonal()
    lam, _ = lanczos_lmax(A, None, 1e-8, 200)
    u = u0.copy()
    for _ in range(5):
        u = chebyshev(A, dinv, b, u, 2, lam / 10, lam)
    inside = np.zeros(u.size, dtype=bool)
    inside[pd[0]] = True
    share_before = np.abs(u0[inside]).max() / np.abs(u0).max()
    share_after = np.abs(u[inside]).max() / np.abs(u).max()
    assert share_after > share_before
    assert np.abs(u[inside]).max() > 2 * np.abs(u[~inside]).max()
    L = _local(A, pd)
    v = u0.copy()
    for _ in range(5):
        v = sandwich(A, dinv, b, v, L, 2, lam / 10, lam)
    assert np.abs(v[inside]).max() < 0.05 * np.abs(u[inside]).max()


# --- symmetric Gauss-Seidel as the global smoother --------------------------

def _sgs_problem(degree=2):
    m = meshgen.square_mesh(6, 3, n_single=2, single_depth=1e-3)
    _, A, _ = oracle.assemble(m, degree)
    return A.tocsr()


def test_matrix_colouring_is_proper_and_greedy():
    A = _sgs_problem()
    col = oracle.matrix_colouring(A)
    C = A.tocoo()
    d = np.sqrt(A.diagonal())
    coupled = (C.row != C.col) & (np.abs(C.data) > 1e-12 * d[C.row] * d[C.col])
    weak = (C.row != C.col) & ~coupled
    assert np.all(np.abs(C.data[weak]) < 1e-12 * np.abs(C.data).max())   # dropped entries are rounding noise
    assert np.all(col[C.row[coupled]] != col[C.col[coupled]])            # proper
    deg = np.diff(A.indptr) - 1
    assert col.max() <= deg.max()                                         # at most max degree + 1 colours
    for i in range(A.shape[0]):                                           # greedy: no smaller colour was free
        lo = C.col[(C.row == i) & coupled & (C.col < i)]
        lower = set(col[lo].tolist())
        assert all(c in lower for c in range(col[i]))


def test_forward_colour_sweep_is_sequential_gauss_seidel():
    """A forward sweep equals Gauss-Seidel in colour-major row order, computed
    here by a sparse triangular solve: u' = u + (D + L)^-1 (b - A u) with L the
    strictly lower part of the symmetrically permuted matrix."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    A = _sgs_problem()
    n = A.shape[0]
    col = oracle.matrix_colouring(A)
    S = oracle.SymmetricGaussSeidel(A, col)
    rng = np.random.default_rng(4)
    b, u = rng.normal(size=n), rng.normal(size=n)
    fwd = u.copy()
    for c in range(len(S.rows)):
        S._colour(c, b, fwd)
    perm = np.argsort(col, kind="stable")
    Ap = A[perm][:, perm]
    DL = sp.tril(Ap, format="csr")
    r = (b - A @ u)[perm]
    want = u.copy()
    want[perm] += spla.spsolve_triangular(DL, r, lower=True)
    assert np.allclose(fwd, want, atol=1e-12 * np.abs(want).max())
    # the backward sweep is the transposed (upper) solve in the same order
    full = S.apply(b, u)
    DU = sp.triu(Ap, format="csr")
    r2 = (b - A @ want)[perm]
    want2 = want.copy()
    want2[perm] += spla.spsolve_triangular(DU, r2, lower=False)
    assert np.allclose(full, want2, atol=1e-12 * np.abs(want2).max())


def test_sgs_smoother_is_symmetric_and_convergent():
    A = _sgs_problem()
    n = A.shape[0]
    S = oracle.SymmetricGaussSeidel(A, oracle.matrix_colouring(A))
    M = np.stack([S.apply(e, np.zeros(n)) for e in np.eye(n)], axis=1)   # u = M b from u = 0
    assert np.allclose(M, M.T, atol=1e-12 * np.abs(M).max())
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
    E = np.eye(n) - M @ A.toarray()
    assert np.max(np.abs(np.linalg.eigvals(E))) < 1.0
