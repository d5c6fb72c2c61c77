"""Oracle: the global-local combined smoother and its eigenvalue estimate.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Global smoother S_g (Sec. 3.2, Sec. 5, Sec. 6.1.2): Jacobi-preconditioned
  Chebyshev iteration of degree k on D^-1 A over the interval
  [lo, hi] = [frac * lmax, lmax] (frac = 1/10 in the paper).  The recurrence is
  the classical Chebyshev acceleration (Saad, Iterative Methods for Sparse Linear
  Systems, 2nd ed., Algorithm 12.1) applied to the Jacobi-preconditioned
  residual, with theta = (hi+lo)/2, delta = (hi-lo)/2, sigma = theta/delta:
      r = D^-1 (b - A x),  d = r / theta,  x = x + d,  rho = 1/sigma
      repeat k-1 times:
          r = D^-1 (b - A x),  rho' = 1/(2 sigma - rho),
          d = rho' rho d + (2 rho'/delta) r,  x = x + d,  rho = rho'
  so that the error is multiplied by T_k((theta - t)/delta) / T_k(theta/delta)
  on every eigenvector of D^-1 A with eigenvalue t.
* Largest eigenvalue (Sec. 3.2, Sec. 6 intro): the paper uses a Krylov-Schur
  solver with tolerance 1e-8.  Here: Lanczos with full reorthogonalisation on
  D^-1/2 A D^-1/2 (same spectrum as D^-1 A), stopping when the Ritz residual
  |beta_(m+1) s_m| <= tol * theta_max or after maxit steps.  The start vector is
  a fixed pseudo-random vector: SplitMix64 (Steele, Lea, Flood, "Fast splittable
  pseudorandom number generators", OOPSLA 2014) of the row index, top 53 bits
  mapped to [-1, 1).
* Adjusted eigenvalue (Sec. 5): the same estimate for the principal submatrix
  A_gg on the DOFs outside every B_d.
* Local residual correction S_c (Sec. 4.1, eqs. (local_system), (local_residual),
  (local), (local_update)): e_d = (I_d^T A I_d)^-1 I_d^T r and
  u += sum_d I_d e_d, with one residual r for all patches of a colour.  Patches
  of one colour share no DOF; colours are visited in ascending order for the
  first application of the sandwich and descending for the second, which keeps
  the combined smoother symmetric.  With one colour (disjoint subdomains, as in
  the paper) this is exactly the paper's S_c.
* Combined smoother (Sec. 4.2): u <- S_c, then S_g, then S_c.
* Symmetric Gauss-Seidel as S_g (the global smoother of most of the paper's
  Poisson experiments, Sec. 3.2 and Sec. 6.1; one forward and one backward
  sweep per application).  Here the multicolour form: the rows are coloured
  greedily in row order (each row takes the smallest colour not used by a
  lower-numbered neighbour in the matrix graph, |a_ij| > 1e-12 sqrt(a_ii a_jj));
  a forward sweep updates the
  colours in ascending order, all rows of a colour at once from the current
  iterate, u_i += (b_i - (A u)_i) / a_ii, the backward sweep in descending
  order.  Rows of one colour are not coupled, so a forward sweep is exactly
  sequential Gauss-Seidel in colour-major row order (lexicographic SGS in the
  original numbering visits the rows in another order, so iteration counts
  differ from the paper's).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

_MASK64 = (1 << 64) - 1


def splitmix64(index: np.ndarray) -> np.ndarray:
    """SplitMix64 output for state = index (one step from seed `index`)."""
    z = (index.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15))
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def start_vector(n: int) -> np.ndarray:
    bits = splitmix64(np.arange(n, dtype=np.uint64)) >> np.uint64(11)
    return bits.astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0


def tridiag_max(alpha, beta):
    """Largest eigenvalue of the symmetric tridiagonal matrix and the last
    component of its unit eigenvector."""
    w, v = sla.eigh_tridiagonal(np.asarray(alpha), np.asarray(beta))
    return w[-1], v[-1, -1]


def lanczos_lmax(A: sp.csr_matrix, mask: np.ndarray | None = None, tol: float = 1e-8,
                 maxit: int = 200):
    """Largest eigenvalue of D^-1 A (or of D_gg^-1 A_gg on mask == True).

    Returns (estimate, number of Lanczos steps)."""
    n = A.shape[0]
    dg = A.diagonal()
    s = 1.0 / np.sqrt(dg)
    m = np.ones(n) if mask is None else mask.astype(np.float64)
    if m.sum() == 0:
        return 0.0, 0

    def H(x):
        return m * (s * (A @ (s * (m * x))))

    q = m * start_vector(n)
    q = q / np.linalg.norm(q)
    Q = [q]
    alpha, beta = [], []
    theta = 0.0
    for j in range(maxit):
        w = H(Q[j])
        a = float(Q[j] @ w)
        w = w - a * Q[j]
        if j > 0:
            w = w - beta[-1] * Q[j - 1]
        Qm = np.array(Q)
        w = w - Qm.T @ (Qm @ w)           # full reorthogonalisation (one CGS pass)
        b = float(np.linalg.norm(w))
        alpha.append(a)
        theta, slast = tridiag_max(alpha, beta)
        if b * abs(slast) <= tol * theta or b == 0.0:
            return theta, j + 1
        beta.append(b)
        Q.append(w / b)
    return theta, maxit


def chebyshev(A, dinv, b, x, k, lo, hi):
    """k steps of Jacobi-preconditioned Chebyshev on [lo, hi]; returns new x."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = dinv * (b - A @ x)
    d = r / theta
    x = x + d
    for _ in range(1, k):
        r = dinv * (b - A @ x)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * r
        x = x + d
        rho = rho_new
    return x


class LocalCorrection:
    """S_c for one level: patch DOF sets, colours and Cholesky factors."""

    def __init__(self, A: sp.csr_matrix, patch_dofs: list, colours: np.ndarray):
        self.dofs = patch_dofs
        self.colours = np.asarray(colours, dtype=np.int64)
        self.factors = []
        for B in patch_dofs:
            Ad = A[B][:, B].toarray()          # A^[d] = I_d^T A I_d
            self.factors.append(sla.cho_factor(Ad, lower=True))
        self.n_colours = int(self.colours.max()) + 1 if len(patch_dofs) else 0

    def apply(self, A, b, u, descending=False):
        order = range(self.n_colours - 1, -1, -1) if descending else range(self.n_colours)
        u = u.copy()
        for c in order:
            members = np.flatnonzero(self.colours == c)
            r = b - A @ u
            corr = [sla.cho_solve(self.factors[d], r[self.dofs[d]]) for d in members]
            for d, e in zip(members, corr):
                u[self.dofs[d]] += e
        return u


COUPLING_EPS = 1e-12


def matrix_colouring(A: sp.csr_matrix) -> np.ndarray:
    """Greedy colouring of the matrix graph in row order: row i takes the
    smallest colour not used by any neighbour j < i.  Rows i and j are
    neighbours if |a_ij| > 1e-12 sqrt(a_ii a_jj): a Galerkin product can hold
    entries that cancel to zero or to rounding noise, which are not couplings
    (and whose presence depends on the summation order)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    d = np.sqrt(np.abs(A.diagonal()))
    col = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        nbr = A.indices[A.indptr[i]:A.indptr[i + 1]]
        val = A.data[A.indptr[i]:A.indptr[i + 1]]
        keep = (nbr < i) & (np.abs(val) > COUPLING_EPS * d[i] * d[nbr])
        used = set(col[nbr[keep]].tolist())
        c = 0
        while c in used:
            c += 1
        col[i] = c
    return col


class SymmetricGaussSeidel:
    """Multicolour symmetric Gauss-Seidel sweep (one forward, one backward)."""

    def __init__(self, A: sp.csr_matrix, colours: np.ndarray):
        A = sp.csr_matrix(A)
        self.colours = colours
        self.rows = [np.flatnonzero(colours == c) for c in range(int(colours.max()) + 1)]
        self.blocks = [A[r] for r in self.rows]
        self.dinv = 1.0 / A.diagonal()

    def _colour(self, c, b, u):
        r = self.rows[c]
        u[r] += self.dinv[r] * (b[r] - self.blocks[c] @ u)

    def apply(self, b, u):
        u = u.copy()
        for c in range(len(self.rows)):
            self._colour(c, b, u)
        for c in reversed(range(len(self.rows))):
            self._colour(c, b, u)
        return u


def sandwich(A, dinv, b, u, local: LocalCorrection | None, k, lo, hi, sgs: SymmetricGaussSeidel | None = None):
    """One application of the combined smoother S_c -> S_g -> S_c; S_g is the
    Chebyshev-Jacobi polynomial, or the symmetric Gauss-Seidel sweep if given."""
    if local is not None and local.n_colours:
        u = local.apply(A, b, u, descending=False)
    u = sgs.apply(b, u) if sgs is not None else chebyshev(A, dinv, b, u, k, lo, hi)
    if local is not None and local.n_colours:
        u = local.apply(A, b, u, descending=True)
    return u
