"""Oracle: non-nested interpolation prolongation and Galerkin coarse operators.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 2: [P_l]_ij = phi_j^(l+1)(x_i), where x_i is the node of fine DOF i and
phi_j^(l+1) the coarse basis function; R_l = P_l^T; A_(l+1) = P_l^T A_l P_l.

Point location (the paper is silent on ties): the coarse cell of a node is the
lowest-id cell whose smallest barycentric coordinate at the node is >= -1e-12;
if there is none, the cell with the largest smallest barycentric coordinate
(lowest id on ties), provided that value is >= -1e-8; otherwise the node is
outside the coarse mesh and location fails.  Basis values are continuous
across cells, so only the reported cell ids depend on the tie rule.

Rows of P are the free fine DOFs, columns the free coarse DOFs (coarse
Dirichlet columns are dropped: the coarse space carries the same homogeneous
boundary condition).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

from .fem import DofMap, local_basis, poly_eval

INSIDE_TOL = 1e-12
OUTSIDE_TOL = 1e-8


class LocateError(RuntimeError):
    pass


def barycentric(coords: np.ndarray, cells: np.ndarray, cell_ids: np.ndarray,
                pts: np.ndarray) -> np.ndarray:
    """Barycentric coordinates of pts[k] in cell cell_ids[k]."""
    x = coords[cells[cell_ids]]                         # k, d+1, d
    J = np.transpose(x[:, 1:, :] - x[:, :1, :], (0, 2, 1))
    lam = np.linalg.solve(J, (pts - x[:, 0, :])[..., None])[..., 0]
    return np.concatenate([1.0 - lam.sum(axis=1, keepdims=True), lam], axis=1)


def locate(points: np.ndarray, coords: np.ndarray, cells: np.ndarray,
           chunk: int = 200_000) -> np.ndarray:
    """Coarse cell id for every point (rule in the module docstring)."""
    coords = np.asarray(coords, dtype=np.float64)
    cells = np.asarray(cells, dtype=np.int64)
    cent = coords[cells].mean(axis=1)
    reach = np.max(np.linalg.norm(coords[cells] - cent[:, None, :], axis=2))
    tree = cKDTree(cent)
    out = np.empty(points.shape[0], dtype=np.int64)
    for s in range(0, points.shape[0], chunk):
        pts = points[s:s + chunk]
        cand = tree.query_ball_point(pts, r=reach * 1.01 + 1e-9)
        counts = np.array([len(c) for c in cand])
        pid = np.repeat(np.arange(pts.shape[0]), counts)
        cid = np.concatenate([np.asarray(c, dtype=np.int64) for c in cand]) if counts.sum() else np.zeros(0, np.int64)
        lam = barycentric(coords, cells, cid, pts[pid])
        mn = lam.min(axis=1)
        # group the candidates by point, cell ids ascending
        order = np.lexsort((cid, pid))
        pid, cid, mn = pid[order], cid[order], mn[order]
        starts = np.zeros(pts.shape[0] + 1, dtype=np.int64)
        np.cumsum(np.bincount(pid, minlength=pts.shape[0]), out=starts[1:])
        for k in range(pts.shape[0]):
            c = cid[starts[k]:starts[k + 1]]
            m = mn[starts[k]:starts[k + 1]]
            inside = np.flatnonzero(m >= -INSIDE_TOL)
            if inside.size:
                out[s + k] = c[inside].min()
                continue
            if m.size == 0 or m.max() < -OUTSIDE_TOL:
                raise LocateError(f"point {s + k} at {pts[k]} lies outside the coarse mesh")
            best = np.flatnonzero(m == m.max())
            out[s + k] = c[best].min()
    return out


def prolongation(fine: DofMap, coarse: DofMap):
    """P (free fine x free coarse, CSR) and the located coarse cell per free fine DOF."""
    pts = fine.nodes[fine.free]
    cell = locate(pts, coarse.coords, coarse.cells)
    lam = barycentric(coarse.coords, coarse.cells, cell, pts)
    basis, _ = local_basis(coarse.dim, coarse.degree)
    vals = np.stack([poly_eval(p, lam) for p in basis], axis=1)     # nf, nloc
    cols = coarse.free_index[coarse.cell_dofs[cell]]                # nf, nloc
    rows = np.repeat(np.arange(pts.shape[0]), vals.shape[1])
    keep = cols.ravel() >= 0
    P = sp.coo_matrix((vals.ravel()[keep], (rows[keep], cols.ravel()[keep])),
                      shape=(fine.n_free, coarse.n_free)).tocsr()
    P.sum_duplicates()
    P.sort_indices()
    return P, cell


def galerkin(A: sp.csr_matrix, P: sp.csr_matrix) -> sp.csr_matrix:
    """A_c = P^T A P."""
    Ac = (P.T @ (A @ P)).tocsr()
    Ac.sum_duplicates()
    Ac.sort_indices()
    return Ac
