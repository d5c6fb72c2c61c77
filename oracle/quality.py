"""Oracle: cell quality and low-quality regions.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Normalised radius ratio (Sec. 3, eq. (radius_ratio)).  The paper defines it as
the inradius over the circumradius, normalised so that the ideal (equilateral)
simplex scores 1 and degenerate ones tend to 0.  The printed normalising
constant ("the geometric dimension" in the denominator) cannot give that range,
since the optimal ratio R_I/R_C is 1/d; the reading used here is
gamma = d * R_I / R_C, which has the stated range and reproduces the paper's
example of a triangle with a 1 degree minimum angle having gamma of order 1e-3.

R_I = d |T| / sum_F |F| (volume over total facet measure), and R_C is the
distance from a vertex to the circumcentre, which solves
2 (x_a - x_0) . c = |x_a|^2 - |x_0|^2, a = 1..d.

Low-quality regions (Sec. 4.4, eq. (identify)): Omega_b = {K : gamma(K) < tau}
(strict), grown by vertex layers; see patches().
"""
from __future__ import annotations

from math import factorial

import numpy as np


def radius_ratio(coords: np.ndarray, cells: np.ndarray) -> np.ndarray:
    coords = np.asarray(coords, dtype=np.float64)
    cells = np.asarray(cells, dtype=np.int64)
    d = coords.shape[1]
    x = coords[cells]                                  # nc, d+1, d
    E = x[:, 1:, :] - x[:, :1, :]                      # rows x_a - x_0
    vol = np.abs(np.linalg.det(E)) / factorial(d)
    # facet measures
    total = np.zeros(cells.shape[0])
    for k in range(d + 1):
        f = np.delete(x, k, axis=1)                    # nc, d, d
        if d == 2:
            total += np.linalg.norm(f[:, 1] - f[:, 0], axis=1)
        else:
            total += 0.5 * np.linalg.norm(np.cross(f[:, 1] - f[:, 0], f[:, 2] - f[:, 0]), axis=1)
    r_in = d * vol / total
    rhs = 0.5 * (np.sum(x[:, 1:, :] ** 2, axis=2) - np.sum(x[:, :1, :] ** 2, axis=2))
    centre = np.linalg.solve(E, rhs[..., None])[..., 0]
    r_circ = np.linalg.norm(centre - x[:, 0, :], axis=1)
    return d * r_in / r_circ
