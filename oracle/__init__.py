"""Plain FP64 CPU oracle of the global-local multigrid method.

TEST INFRASTRUCTURE ONLY.  The oracle is a slow, obviously correct CPU
implementation of what the GPU library computes, written from the paper
(Chen & Wells, "Multigrid on unstructured meshes with regions of low quality
cells", arXiv 2402.12947).  It is used only by the tests, by the package's
smoke check and by the CPU-baseline leg of the benchmark; the product path
(the HIP library and its Python binding) neither imports nor calls it, and it
shares no code with that path.  Both sides only share the seeded input
generators in `meshgen`, which hold none of the method's arithmetic.

Modules and the parts of the paper they follow:
  fem         P1/P2/P3 Poisson stiffness and mass, DOF map (Sec. 2, Sec. 6.1)
  quality     normalised radius ratio (Sec. 3, eq. radius_ratio)
  patches     low-quality regions, patch DOF sets, colouring (Sec. 4.1, 4.4)
  transfer    point location, interpolation prolongation, Galerkin RAP (Sec. 2)
  smoothers   Chebyshev-Jacobi S_g, Lanczos lambda_max, adjusted lambda_max,
              local correction S_c, combined smoother (Sec. 3.2, 4.1, 4.2, 5)
  multigrid   hierarchy, V-cycle (Algorithm alg:mg), MG-preconditioned CG (Sec. 6.2)

Parity status: every function is pinned by a `-m "not gpu"` test against a
closed form, a textbook identity, brute force or the paper's own statements,
except where a test file says "parity unpinned".
"""
from .fem import DofMap, assemble, assemble_full, element_matrices, local_basis, reference_tensors
from .multigrid import Hierarchy, Options
from .patches import MERGE, OVERLAP, colour, patches
from .quality import radius_ratio
from .smoothers import (LocalCorrection, SymmetricGaussSeidel, chebyshev, lanczos_lmax, matrix_colouring, sandwich,
                        splitmix64, start_vector)
from .transfer import LocateError, barycentric, galerkin, locate, prolongation
from . import elasticity

__all__ = [
    "DofMap", "assemble", "assemble_full", "element_matrices", "local_basis",
    "reference_tensors", "Hierarchy", "Options", "MERGE", "OVERLAP", "colour",
    "patches", "radius_ratio", "LocalCorrection", "chebyshev", "lanczos_lmax",
    "sandwich", "splitmix64", "start_vector", "LocateError", "barycentric",
    "galerkin", "locate", "prolongation", "SymmetricGaussSeidel", "matrix_colouring", "elasticity",
]
