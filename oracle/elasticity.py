"""Oracle: linear elasticity (paper Sec. 6.2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

-div sigma(u) = f with sigma(u) = 2 mu eps(u) + lambda tr(eps(u)) I,
eps(u) = (grad u + grad u^T) / 2, mu = E / (2 (1 + nu)),
lambda = E nu / ((1 + nu)(1 - 2 nu)); the paper takes E = 6.9e10, nu = 0.33.
Vector Lagrange elements: every scalar DOF s of the DofMap carries dim
components, numbered s * dim + c.  The bilinear form
a(u, v) = int 2 mu eps(u):eps(v) + lambda div u div v gives, for
u = phi_j e_q and v = phi_i e_p,
    K[(i,p),(j,q)] = int mu (grad phi_i . grad phi_j) delta_pq
                         + mu d_q phi_i d_p phi_j + lambda d_p phi_i d_q phi_j.
The integrals int d_k phi_i d_l phi_j come from the same exact reference
tensors as the Poisson stiffness (fem.reference_tensors) and the gradients of
the barycentric coordinates.  Dirichlet DOFs (all components of a Dirichlet
scalar DOF) are eliminated as for Poisson.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import DofMap, reference_tensors, simplex_geometry

YOUNG = 6.9e10
POISSON_RATIO = 0.33


def lame(young: float = YOUNG, nu: float = POISSON_RATIO):
    return young / (2.0 * (1.0 + nu)), young * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


def element_matrices(coords: np.ndarray, cells: np.ndarray, degree: int, mu: float, lam: float):
    """Ke[c, i * dim + p, j * dim + q] for every cell."""
    dim = coords.shape[1]
    Kref, Mref = reference_tensors(dim, degree)
    vol, grad, _ = simplex_geometry(coords, cells)
    nl = Kref.shape[2]
    # T[c, i, j, k, l] = int d_k phi_i d_l phi_j
    T = vol[:, None, None, None, None] * np.einsum("abij,cak,cbl->cijkl", Kref, grad, grad)
    lap = np.einsum("cijkk->cij", T)
    K = np.zeros((cells.shape[0], nl, dim, nl, dim))
    for p in range(dim):
        for q in range(dim):
            K[:, :, p, :, q] = mu * T[:, :, :, q, p] + lam * T[:, :, :, p, q]
        K[:, :, p, :, p] += mu * lap
    Me = vol[:, None, None] * Mref[None]
    return K.reshape(cells.shape[0], nl * dim, nl * dim), Me


def vector_ids(scalar_ids: np.ndarray, dim: int) -> np.ndarray:
    """All components of the given scalar DOFs, in the order s * dim + c."""
    s = np.asarray(scalar_ids, dtype=np.int64)
    return (s[:, None] * dim + np.arange(dim)[None, :]).ravel()


def assemble_full(mesh: dict, degree: int, young: float = YOUNG, nu: float = POISSON_RATIO):
    """Stiffness K and the vector mass matrix M (x) I over all vector DOFs."""
    dm = DofMap(mesh, degree)
    dim = dm.dim
    mu, lam = lame(young, nu)
    Ke, Me = element_matrices(dm.coords, dm.cells, degree, mu, lam)
    vd = np.stack([vector_ids(cd, dim) for cd in dm.cell_dofs])   # nc, nl * dim
    m = vd.shape[1]
    rows = np.repeat(vd, m, axis=1).ravel()
    cols = np.tile(vd, (1, m)).ravel()
    n = dm.n_dofs * dim
    K = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(n, n)).tocsr()
    K.sum_duplicates()
    nl = dm.cell_dofs.shape[1]
    rs = np.repeat(dm.cell_dofs, nl, axis=1).ravel()
    cs = np.tile(dm.cell_dofs, (1, nl)).ravel()
    Ms = sp.coo_matrix((Me.ravel(), (rs, cs)), shape=(dm.n_dofs, dm.n_dofs)).tocsr()
    Ms.sum_duplicates()
    M = sp.kron(Ms, sp.identity(dim), format="csr")
    return dm, K, M


def assemble(mesh: dict, degree: int, young: float = YOUNG, nu: float = POISSON_RATIO):
    """Reduced system over the free vector DOFs (Dirichlet components eliminated)."""
    dm, K, _ = assemble_full(mesh, degree, young, nu)
    free = vector_ids(dm.free, dm.dim)
    A = K[free][:, free].tocsr()
    A.sort_indices()
    return dm, A
