"""Oracle: Lagrange P1/P2/P3 discretisation of the Poisson problem.

TEST INFRASTRUCTURE ONLY.  This module is part of the plain, slow, FP64
reference ("oracle") used by the tests and by the CPU baseline of the benchmark.
The product path never imports it.

What it computes (paper Sec. 2, eq. (system_finest); Sec. 6.1 Poisson problem):
the stiffness matrix K_ij = int grad(phi_i) . grad(phi_j) and the consistent mass
matrix M_ij = int phi_i phi_j of continuous Lagrange elements of degree p on a
simplicial mesh, and the reduced system A u = b obtained by eliminating the
(homogeneous) Dirichlet degrees of freedom.  The load is b = M f_hat where
f_hat interpolates f at the degree-of-freedom nodes.

Integration is exact: every basis function is a polynomial in the barycentric
coordinates lambda_0..lambda_d of the cell, and on a simplex T

    int_T lambda^alpha dx = |T| d! alpha! / (|alpha| + d)!

so the reference tensors below are exact rationals evaluated in FP64.

Degree-of-freedom numbering (the paper is silent; this is the reading used by
the whole project): vertex DOFs first (DOF id = vertex id); then edges, sorted
by their (low vertex, high vertex) pair, with one DOF per edge for P2 and two for
P3 (first the node nearer the low vertex); then, for P3 triangles, one interior
DOF per cell in cell order.  A non-vertex DOF is Dirichlet iff it lies on a
boundary facet (a facet of exactly one cell) whose vertices are all Dirichlet.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import product
from math import factorial

import numpy as np
import scipy.sparse as sp

LOCAL_EDGES = {2: [(0, 1), (0, 2), (1, 2)],
               3: [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]}


# ----------------------------------------------------------------------------
# polynomials in barycentric coordinates: dict {exponent tuple: Fraction}
# ----------------------------------------------------------------------------

def _poly_mul(p, q):
    out = {}
    for ea, ca in p.items():
        for eb, cb in q.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, 0) + ca * cb
    return {e: c for e, c in out.items() if c != 0}


def _poly_add(p, q, s=1):
    out = dict(p)
    for e, c in q.items():
        out[e] = out.get(e, 0) + s * c
    return {e: c for e, c in out.items() if c != 0}


def _poly_scale(p, s):
    return {e: c * s for e, c in p.items()}


def _lam(a, n):
    e = [0] * n
    e[a] = 1
    return {tuple(e): Fraction(1)}


def _const(c, n):
    return {tuple([0] * n): Fraction(c)}


def _poly_diff(p, a):
    out = {}
    for e, c in p.items():
        if e[a] > 0:
            f = list(e)
            f[a] -= 1
            out[tuple(f)] = out.get(tuple(f), 0) + c * e[a]
    return out


def _poly_integral(p, dim):
    """(1/|T|) int_T p dx, exact."""
    total = Fraction(0)
    for e, c in p.items():
        num = factorial(dim)
        for k in e:
            num *= factorial(k)
        total += c * Fraction(num, factorial(sum(e) + dim))
    return total


def poly_eval(p, lam):
    """Evaluate polynomial p at barycentric points lam[..., d+1] (FP64)."""
    out = np.zeros(lam.shape[:-1])
    for e, c in p.items():
        term = np.full(lam.shape[:-1], float(c))
        for a, k in enumerate(e):
            if k:
                term = term * lam[..., a] ** k
        out += term
    return out


def local_basis(dim: int, degree: int):
    """Lagrange basis of degree p on a d-simplex in local DOF order.

    Local order: vertices 0..d; then the local edges (a, b) of LOCAL_EDGES with
    one DOF (P2) or two DOFs (P3: nearer a, then nearer b); then the P3
    triangle interior DOF.  Returns (list of polynomials, list of barycentric
    node coordinates as Fractions).
    """
    n = dim + 1
    L = [_lam(a, n) for a in range(n)]
    basis, nodes = [], []

    def unit(a):
        return [Fraction(int(i == a)) for i in range(n)]

    if degree == 1:
        for a in range(n):
            basis.append(L[a])
            nodes.append(unit(a))
    elif degree == 2:
        for a in range(n):  # lambda_a (2 lambda_a - 1)
            basis.append(_poly_mul(L[a], _poly_add(_poly_scale(L[a], 2), _const(-1, n))))
            nodes.append(unit(a))
        for a, b in LOCAL_EDGES[dim]:  # 4 lambda_a lambda_b
            basis.append(_poly_scale(_poly_mul(L[a], L[b]), 4))
            nodes.append([(Fraction(1, 2) if i in (a, b) else Fraction(0)) for i in range(n)])
    elif degree == 3:
        if dim != 2:
            raise ValueError("P3 is provided on triangles only")
        for a in range(n):  # 1/2 lambda_a (3 lambda_a - 1)(3 lambda_a - 2)
            t1 = _poly_add(_poly_scale(L[a], 3), _const(-1, n))
            t2 = _poly_add(_poly_scale(L[a], 3), _const(-2, n))
            basis.append(_poly_scale(_poly_mul(_poly_mul(L[a], t1), t2), Fraction(1, 2)))
            nodes.append(unit(a))
        for a, b in LOCAL_EDGES[dim]:
            lab = _poly_mul(L[a], L[b])
            for near, far in ((a, b), (b, a)):  # 9/2 lambda_a lambda_b (3 lambda_near - 1)
                t = _poly_add(_poly_scale(L[near], 3), _const(-1, n))
                basis.append(_poly_scale(_poly_mul(lab, t), Fraction(9, 2)))
                nodes.append([(Fraction(2, 3) if i == near else Fraction(1, 3) if i == far
                               else Fraction(0)) for i in range(n)])
        basis.append(_poly_scale(_poly_mul(_poly_mul(L[0], L[1]), L[2]), 27))
        nodes.append([Fraction(1, 3)] * 3)
    else:
        raise ValueError("degree must be 1, 2 or 3")
    return basis, nodes


_REF_CACHE = {}


def reference_tensors(dim: int, degree: int):
    """Kref[a, b, i, j] = (1/|T|) int d(phi_i)/d(lambda_a) d(phi_j)/d(lambda_b),
    Mref[i, j] = (1/|T|) int phi_i phi_j; exact rationals returned as FP64."""
    key = (dim, degree)
    if key in _REF_CACHE:
        return _REF_CACHE[key]
    basis, _ = local_basis(dim, degree)
    n = dim + 1
    nl = len(basis)
    dphi = [[_poly_diff(p, a) for a in range(n)] for p in basis]
    Kref = np.zeros((n, n, nl, nl))
    for a, b, i, j in product(range(n), range(n), range(nl), range(nl)):
        Kref[a, b, i, j] = float(_poly_integral(_poly_mul(dphi[i][a], dphi[j][b]), dim))
    Mref = np.zeros((nl, nl))
    for i, j in product(range(nl), range(nl)):
        Mref[i, j] = float(_poly_integral(_poly_mul(basis[i], basis[j]), dim))
    _REF_CACHE[key] = (Kref, Mref)
    return Kref, Mref


# ----------------------------------------------------------------------------
# geometry of simplices
# ----------------------------------------------------------------------------

def simplex_geometry(coords: np.ndarray, cells: np.ndarray):
    """Volumes |T| and the gradients of the barycentric coordinates.

    Returns vol[nc], grad[nc, d+1, d] with grad[c, a] = grad(lambda_a) on cell c.
    """
    x = coords[cells]                       # nc, d+1, d
    d = coords.shape[1]
    J = np.transpose(x[:, 1:, :] - x[:, :1, :], (0, 2, 1))   # columns x_a - x_0
    det = np.linalg.det(J)
    vol = np.abs(det) / factorial(d)
    Jinv = np.linalg.inv(J)                 # rows: grad lambda_1..d
    grad = np.empty((cells.shape[0], d + 1, d))
    grad[:, 1:, :] = Jinv
    grad[:, 0, :] = -Jinv.sum(axis=1)
    return vol, grad, det


# ----------------------------------------------------------------------------
# degree-of-freedom map
# ----------------------------------------------------------------------------

def _facets(cells: np.ndarray):
    """Sorted vertex tuples of every cell facet, and whether it is a boundary
    facet (shared by exactly one cell)."""
    n = cells.shape[1]
    f = np.concatenate([np.delete(cells, k, axis=1) for k in range(n)], axis=0)
    f = np.sort(f, axis=1)
    uniq, counts = np.unique(f, axis=0, return_counts=True)
    return uniq, counts == 1


class DofMap:
    """Cell-to-DOF map, DOF node coordinates and Dirichlet flags of one mesh."""

    def __init__(self, mesh: dict, degree: int):
        coords = np.asarray(mesh["coords"], dtype=np.float64)
        cells = np.asarray(mesh["cells"], dtype=np.int64)
        dirv = np.asarray(mesh["dirichlet_vertex"]).astype(bool)
        dim = coords.shape[1]
        nv, nc = coords.shape[0], cells.shape[0]
        self.dim, self.degree = dim, degree
        self.coords, self.cells = coords, cells
        le = LOCAL_EDGES[dim]
        if degree == 1:
            self.cell_dofs = cells.copy()
            self.nodes = coords.copy()
            self.dirichlet = dirv.copy()
            self.n_edges = 0
        else:
            ends = np.stack([np.sort(cells[:, [a, b]], axis=1) for a, b in le], axis=1)
            edges, inv = np.unique(ends.reshape(-1, 2), axis=0, return_inverse=True)
            inv = inv.reshape(nc, len(le))
            ne = edges.shape[0]
            self.n_edges = ne
            # Dirichlet edges: edges of boundary facets whose vertices are all Dirichlet
            facets, is_bdry = _facets(cells)
            bf = facets[is_bdry]
            bf = bf[np.all(dirv[bf], axis=1)]
            dir_edge = np.zeros(ne, dtype=bool)
            if bf.shape[0]:
                if dim == 2:
                    fe = bf
                else:
                    fe = np.concatenate([bf[:, [0, 1]], bf[:, [0, 2]], bf[:, [1, 2]]], axis=0)
                key = fe[:, 0] * nv + fe[:, 1]
                ekey = edges[:, 0] * nv + edges[:, 1]
                pos = np.searchsorted(ekey, key)
                assert np.all(ekey[pos] == key)
                dir_edge[pos] = True
            if degree == 2:
                self.cell_dofs = np.concatenate([cells, nv + inv], axis=1)
                mid = 0.5 * (coords[edges[:, 0]] + coords[edges[:, 1]])
                self.nodes = np.concatenate([coords, mid], axis=0)
                self.dirichlet = np.concatenate([dirv, dir_edge])
            else:  # degree 3, triangles
                cols = [cells]
                for k, (a, b) in enumerate(le):
                    ga, gb = cells[:, a], cells[:, b]
                    first = nv + 2 * inv[:, k] + (ga > gb)   # node nearer local a
                    second = nv + 2 * inv[:, k] + (ga < gb)  # node nearer local b
                    cols.append(np.stack([first, second], axis=1))
                cols.append((nv + 2 * ne + np.arange(nc))[:, None])
                self.cell_dofs = np.concatenate(cols, axis=1)
                lo, hi = coords[edges[:, 0]], coords[edges[:, 1]]
                enodes = np.empty((2 * ne, dim))
                enodes[0::2] = (2.0 * lo + hi) / 3.0
                enodes[1::2] = (lo + 2.0 * hi) / 3.0
                cent = coords[cells].mean(axis=1)
                self.nodes = np.concatenate([coords, enodes, cent], axis=0)
                self.dirichlet = np.concatenate([dirv, np.repeat(dir_edge, 2),
                                                 np.zeros(nc, dtype=bool)])
        self.n_dofs = self.nodes.shape[0]
        self.free = np.flatnonzero(~self.dirichlet)
        self.free_index = np.full(self.n_dofs, -1, dtype=np.int64)
        self.free_index[self.free] = np.arange(self.free.size)
        self.n_free = self.free.size


# ----------------------------------------------------------------------------
# assembly
# ----------------------------------------------------------------------------

def element_matrices(coords: np.ndarray, cells: np.ndarray, degree: int):
    """Element stiffness K_T[i, j] = |T| sum_ab (grad l_a . grad l_b) Kref[a,b,i,j]
    and element mass M_T = |T| Mref for every cell."""
    dim = coords.shape[1]
    Kref, Mref = reference_tensors(dim, degree)
    vol, grad, _ = simplex_geometry(coords, cells)
    G = np.einsum("cad,cbd->cab", grad, grad)
    Ke = vol[:, None, None] * np.einsum("cab,abij->cij", G, Kref)
    Me = vol[:, None, None] * Mref[None]
    return Ke, Me


def assemble_full(mesh: dict, degree: int):
    """Global stiffness K and mass M over all DOFs (no boundary conditions)."""
    dm = DofMap(mesh, degree)
    Ke, Me = element_matrices(dm.coords, dm.cells, degree)
    nl = dm.cell_dofs.shape[1]
    rows = np.repeat(dm.cell_dofs, nl, axis=1).ravel()
    cols = np.tile(dm.cell_dofs, (1, nl)).ravel()
    K = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(dm.n_dofs, dm.n_dofs)).tocsr()
    M = sp.coo_matrix((Me.ravel(), (rows, cols)), shape=(dm.n_dofs, dm.n_dofs)).tocsr()
    K.sum_duplicates()
    M.sum_duplicates()
    return dm, K, M


def assemble(mesh: dict, degree: int):
    """Reduced system: A = K[free, free] (Dirichlet DOFs eliminated, g = 0) and
    the restriction Mf = M[free, :] that maps nodal data f_hat to b = M f_hat."""
    dm, K, M = assemble_full(mesh, degree)
    A = K[dm.free][:, dm.free].tocsr()
    A.sort_indices()
    Mf = M[dm.free].tocsr()
    return dm, A, Mf
