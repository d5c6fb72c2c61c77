"""Oracle: non-nested Galerkin multigrid V-cycle and MG-preconditioned CG.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Setup (Sec. 2, Sec. 4.4, Sec. 5): for each level l (0 = finest) the DOF map of
its mesh, the cell quality and local-correction patches of its mesh, the
operator (assembled on level 0, A_(l+1) = P_l^T A_l P_l below), D_l = diag(A_l),
the Chebyshev interval from the (adjusted) largest eigenvalue, and on the
coarsest level a Cholesky factorisation (direct solver).

V-cycle (Algorithm "alg:mg", correction scheme): pre-smooth nu times, restrict
the residual b_c = P^T (b - A u), solve the coarse problem for a correction
starting from zero, add P u_c, post-smooth nu times.  The printed algorithm
initialises the coarse unknown with P^T u; since the coarse right-hand side is a
residual, the coarse unknown is a correction, and the reading used is u_c = 0.
One "smoother application" is one combined S_c -> S_g -> S_c sandwich; S_g is a
Chebyshev polynomial of degree cheb_degree.

PCG (Sec. 6.2: one V-cycle per CG iteration) with x_0 = 0 and the stopping rule
||b - A x||_2 <= rtol ||b||_2 on the recursively updated residual (Sec. 6 intro);
the iteration count is the number of products with A.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .fem import DofMap, assemble
from .patches import MERGE, colour, combine, components, inherit, patches
from .quality import radius_ratio
from . import elasticity
from .smoothers import LocalCorrection, SymmetricGaussSeidel, lanczos_lmax, matrix_colouring, sandwich
from .transfer import galerkin, prolongation


@dataclass
class Options:
    degree: int = 1
    nu: int = 2
    cheb_degree: int = 2
    cheb_lo_frac: float = 0.1
    local_correction: bool = True
    adjusted_eig: bool = True
    patch_policy: int = MERGE
    eig_tol: float = 1e-8
    eig_maxit: int = 200
    global_smoother: str = "chebyshev"   # or "sgs" (multicolour symmetric Gauss-Seidel)
    problem: str = "poisson"             # or "elasticity" (Sec. 6.2)
    young: float = 6.9e10
    poisson_ratio: float = 0.33
    inherit_levels: int = 0              # coarse levels with patches inherited through P (0: the paper's)


@dataclass
class Level:
    dofmap: DofMap
    A: sp.csr_matrix
    dinv: np.ndarray
    gamma: np.ndarray
    patch_cells: list
    patch_dofs: list
    colours: np.ndarray
    lam: float = 0.0
    lam_adj: float = 0.0
    lo: float = 0.0
    hi: float = 0.0
    local: LocalCorrection | None = None
    sgs: SymmetricGaussSeidel | None = None   # global smoother when opts.global_smoother == "sgs"
    P: sp.csr_matrix | None = None            # to the next coarser level
    locate_cell: np.ndarray | None = None     # coarse cell of each free DOF node
    chol: tuple | None = None                 # coarsest only
    Mf: sp.csr_matrix | None = None           # level 0 only: b = Mf f_hat
    extra: dict = field(default_factory=dict)


class Hierarchy:
    """prolongations (optional): P_l for l = 0 .. L-2 as sparse matrices over
    the free DOFs in canonical order, used instead of point location (for
    checks at sizes where the oracle's point location is too slow; the given
    P is itself compared with the oracle's definition on sampled rows).
    intervals (optional): (lo, hi) of the Chebyshev smoother per level, used
    instead of the Lanczos estimate (likewise for large sizes)."""

    def __init__(self, meshes: list, tau: float = 0.1, layers: int = 1,
                 opts: Options | None = None, prolongations: list | None = None,
                 intervals: list | None = None):
        self.opts = opts = opts or Options()
        self.levels: list[Level] = []
        nlev = len(meshes)
        dms = [DofMap(m, opts.degree) for m in meshes]
        A = None
        elastic = opts.problem == "elasticity"
        ncomp = meshes[0]["coords"].shape[1] if elastic else 1
        for l, (mesh, dm) in enumerate(zip(meshes, dms)):
            Mf = None
            if l == 0:
                if elastic:
                    _, A = elasticity.assemble(mesh, opts.degree, opts.young, opts.poisson_ratio)
                else:
                    _, A, Mf = assemble(mesh, opts.degree)
            gamma = radius_ratio(mesh["coords"], mesh["cells"])
            pc, pd = patches(dm.cells, dm.coords.shape[0], gamma, tau, layers,
                             opts.patch_policy, dm.cell_dofs, dm.free_index)
            if elastic:  # every component of the patch's scalar DOFs
                pd = [elasticity.vector_ids(B, ncomp) for B in pd]
            if opts.local_correction and opts.inherit_levels > 0:
                if l == 0:   # seeds: the free DOFs of each degraded cell
                    seeds = []
                    for K in np.flatnonzero(gamma < tau):
                        f = dm.free_index[dm.cell_dofs[K]]
                        f = np.unique(f[f >= 0])
                        seeds.append(elasticity.vector_ids(f, ncomp) if elastic else f)
                elif l <= opts.inherit_levels:
                    seeds = inherit(self.levels[l - 1].P, seeds)
                    pd = combine(pd, components(seeds), opts.patch_policy)
                    pc = [np.zeros(0, dtype=np.int64)] * len(pd)
            cols = colour(pd)
            lev = Level(dofmap=dm, A=A, dinv=1.0 / A.diagonal(), gamma=gamma,
                        patch_cells=pc, patch_dofs=pd, colours=cols, Mf=Mf)
            if l < nlev - 1:
                if prolongations is not None:
                    lev.P = sp.csr_matrix(prolongations[l])
                else:
                    lev.P, lev.locate_cell = prolongation(dm, dms[l + 1])
                    if elastic:  # each component interpolated on its own: P (x) I
                        lev.P = sp.kron(lev.P, sp.identity(ncomp), format="csr")
                A = galerkin(A, lev.P)
            self.levels.append(lev)
        for l, lev in enumerate(self.levels):
            if l == nlev - 1:
                lev.chol = sla.cho_factor(lev.A.toarray(), lower=True)
                continue
            use_local = opts.local_correction and len(lev.patch_dofs) > 0
            if use_local:
                lev.local = LocalCorrection(lev.A, lev.patch_dofs, lev.colours)
            if intervals is not None:
                lev.lo, lev.hi = intervals[l]
            else:
                lev.lam, _ = lanczos_lmax(lev.A, None, opts.eig_tol, opts.eig_maxit)
                if use_local:
                    g = np.ones(lev.A.shape[0], dtype=bool)
                    for B in lev.patch_dofs:
                        g[B] = False
                    lev.lam_adj, _ = lanczos_lmax(lev.A, g, opts.eig_tol, opts.eig_maxit)
                else:
                    lev.lam_adj = lev.lam
                lev.hi = lev.lam_adj if (use_local and opts.adjusted_eig) else lev.lam
                lev.lo = opts.cheb_lo_frac * lev.hi
            if opts.global_smoother == "sgs":
                lev.sgs = SymmetricGaussSeidel(lev.A, matrix_colouring(lev.A))

    def replace_coarse_operators(self, operators: list) -> None:
        """Uses the given A_l (l = 1 .. L-1, sparse, canonical free-DOF order)
        instead of the Galerkin products, with their diagonals, patch
        factorisations and the coarsest Cholesky rebuilt; the Chebyshev
        intervals are kept.  For checks that separate the cycle's arithmetic
        from the rounding of the coarse operators (which are compared with the
        Galerkin products themselves)."""
        for l, A in enumerate(operators, start=1):
            lev = self.levels[l]
            lev.A = sp.csr_matrix(A)
            lev.dinv = 1.0 / lev.A.diagonal()
            if lev.local is not None:
                lev.local = LocalCorrection(lev.A, lev.patch_dofs, lev.colours)
            if l == len(self.levels) - 1:
                lev.chol = sla.cho_factor(lev.A.toarray(), lower=True)

    # -- the method --------------------------------------------------------
    def smooth(self, l: int, b: np.ndarray, u: np.ndarray, nu: int) -> np.ndarray:
        lev = self.levels[l]
        for _ in range(nu):
            u = sandwich(lev.A, lev.dinv, b, u, lev.local, self.opts.cheb_degree,
                         lev.lo, lev.hi, lev.sgs)
        return u

    def vcycle(self, b: np.ndarray, u: np.ndarray | None = None, l: int = 0) -> np.ndarray:
        lev = self.levels[l]
        if u is None:
            u = np.zeros_like(b)
        if l == len(self.levels) - 1:
            return u + sla.cho_solve(lev.chol, b - lev.A @ u)
        u = self.smooth(l, b, u, self.opts.nu)
        bc = lev.P.T @ (b - lev.A @ u)
        uc = self.vcycle(bc, None, l + 1)
        u = u + lev.P @ uc
        return self.smooth(l, b, u, self.opts.nu)

    def pcg(self, b: np.ndarray, rtol: float, maxit: int, x0: np.ndarray | None = None):
        """Returns (x, iterations, converged, history of ||r||/||b||)."""
        A = self.levels[0].A
        x = np.zeros_like(b) if x0 is None else x0.copy()
        r = b - A @ x
        bnorm = float(np.linalg.norm(b))
        hist = [float(np.linalg.norm(r)) / bnorm if bnorm > 0 else 0.0]
        if bnorm == 0.0:
            return np.zeros_like(b), 0, True, hist
        if hist[0] <= rtol:
            return x, 0, True, hist
        z = self.vcycle(r)
        p = z.copy()
        rho = float(r @ z)
        it = 0
        while it < maxit:
            q = A @ p
            it += 1
            alpha = rho / float(p @ q)
            x = x + alpha * p
            r = r - alpha * q
            rel = float(np.linalg.norm(r)) / bnorm
            hist.append(rel)
            if rel <= rtol:
                return x, it, True, hist
            z = self.vcycle(r)
            rho_new = float(r @ z)
            p = z + (rho_new / rho) * p
            rho = rho_new
        return x, it, False, hist

    def mg_solve(self, b: np.ndarray, rtol: float, maxit: int, x0: np.ndarray | None = None):
        """Multigrid as a stationary solver (Sec. 2, Algorithm alg:mg applied
        repeatedly; the paper's Poisson experiments of Sec. 6.1): one V-cycle
        per iteration from the current iterate, stopping when
        ||b - A x|| <= rtol ||b|| or after maxit cycles.
        Returns (x, cycles, converged, history of ||r||/||b||)."""
        A = self.levels[0].A
        x = np.zeros_like(b) if x0 is None else x0.copy()
        bnorm = float(np.linalg.norm(b))
        if bnorm == 0.0:
            return np.zeros_like(b), 0, True, [0.0]
        hist = [float(np.linalg.norm(b - A @ x)) / bnorm]
        it = 0
        while hist[-1] > rtol and it < maxit:
            x = self.vcycle(b, x)
            it += 1
            hist.append(float(np.linalg.norm(b - A @ x)) / bnorm)
        return x, it, hist[-1] <= rtol, hist

    def rhs_from_nodal(self, f_nodal: np.ndarray) -> np.ndarray:
        if self.levels[0].Mf is None:
            raise ValueError("b = M f_hat is defined for the Poisson problem only")
        return self.levels[0].Mf @ f_nodal
