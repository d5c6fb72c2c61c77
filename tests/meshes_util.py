"""Small hand-built meshes used by the CPU tests (no solver arithmetic here)."""
import numpy as np

import meshgen


def tiny_square(n=4, seed=0, jitter=0.2, dirichlet=("x0", "x1", "y0", "y1"), diagonal="random",
                n_single=0, single_depth=1e-3):
    return meshgen.square_mesh(n, seed, jitter=jitter, diagonal=diagonal,
                               n_single=n_single, single_depth=single_depth,
                               dirichlet=dirichlet)


def tiny_cube(n=2, seed=0, jitter=0.15, dirichlet=("x0", "x1")):
    return meshgen.cube_mesh(n, seed, jitter=jitter, dirichlet=dirichlet)


def red_refine(mesh):
    """Uniform (red) refinement of a triangulation: every triangle is split into
    four by its edge midpoints.  The refined mesh is nested in the input."""
    coords = mesh["coords"]
    cells = mesh["cells"].astype(np.int64)
    nv = coords.shape[0]
    pairs = np.concatenate([cells[:, [0, 1]], cells[:, [1, 2]], cells[:, [0, 2]]], axis=0)
    pairs = np.sort(pairs, axis=1)
    edges, inv = np.unique(pairs, axis=0, return_inverse=True)
    nc = cells.shape[0]
    m01, m12, m02 = inv[:nc] + nv, inv[nc:2 * nc] + nv, inv[2 * nc:] + nv
    mid = 0.5 * (coords[edges[:, 0]] + coords[edges[:, 1]])
    new_coords = np.concatenate([coords, mid], axis=0)
    a, b, c = cells[:, 0], cells[:, 1], cells[:, 2]
    new_cells = np.concatenate([
        np.stack([a, m01, m02], 1), np.stack([m01, b, m12], 1),
        np.stack([m02, m12, c], 1), np.stack([m01, m12, m02], 1)], axis=0)
    dv = mesh["dirichlet_vertex"].astype(bool)
    # a midpoint is Dirichlet iff it is on a boundary edge with both ends Dirichlet
    cnt = np.bincount(inv, minlength=edges.shape[0])
    dmid = (cnt == 1) & dv[edges[:, 0]] & dv[edges[:, 1]]
    return {"dim": 2, "coords": new_coords, "cells": new_cells.astype(np.int32),
            "dirichlet_vertex": np.concatenate([dv, dmid]).astype(np.uint8)}
