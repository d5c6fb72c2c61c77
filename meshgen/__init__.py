"""Seeded synthetic simplicial meshes and right-hand sides.

This module is shared input infrastructure: it builds mesh hierarchies of the
shape the paper's Poisson experiments use (unit square triangulations and unit
cube tetrahedralisations with a few controllably degraded cells, Sec. 6 and the
vertex-displacement idea of Sec. 6 intro) and random right-hand sides.  It holds
none of the solver's arithmetic: no cell-quality measure, no basis functions, no
degree-of-freedom numbering.  Degraded cells are produced purely geometrically,
by moving a vertex to a small distance from the line/plane through the opposite
facet of one incident cell, or (for the patch stress workload) by flattening
thin slabs of the cube grid; the only geometric test used is the sign of the
simplex orientation (so no cell inverts).

A mesh is a dict::

    {"dim": d, "coords": float64[nv, d], "cells": int32[nc, d+1],
     "dirichlet_vertex": uint8[nv]}

Cells are positively oriented.  Levels of a hierarchy are independent meshes of
the same domain (non-nested), finest first.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "square_mesh", "cube_mesh", "hierarchy", "random_rhs", "CONFIGS",
    "orientation", "instance_batch", "stress_cube_mesh", "lattice_mesh",
]


def orientation(coords: np.ndarray, cells: np.ndarray) -> np.ndarray:
    """d! times the signed volume of every cell (positive = counter-clockwise)."""
    x = coords[cells]
    e = x[:, 1:, :] - x[:, :1, :]
    return np.linalg.det(e)


# ----------------------------------------------------------------------------
# structured seeds
# ----------------------------------------------------------------------------

def _square_grid(n: int, rng: np.random.Generator, jitter: float,
                 diagonal: str):
    """(n+1)^2 vertices on [0,1]^2, each quad split by one diagonal."""
    h = 1.0 / n
    ix, iy = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    ix = ix.ravel()
    iy = iy.ravel()
    coords = np.stack([ix * h, iy * h], axis=1).astype(np.float64)
    interior = (ix > 0) & (ix < n) & (iy > 0) & (iy < n)
    if jitter > 0:
        disp = rng.uniform(-jitter * h, jitter * h, size=(int(interior.sum()), 2))
        coords[interior] += disp
    qi, qj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    qi = qi.ravel()
    qj = qj.ravel()
    v00 = qi + (n + 1) * qj
    v10 = v00 + 1
    v01 = v00 + (n + 1)
    v11 = v01 + 1
    if diagonal == "random":
        flip = rng.integers(0, 2, size=qi.size).astype(bool)
    elif diagonal == "right":
        flip = np.zeros(qi.size, dtype=bool)
    else:
        flip = np.ones(qi.size, dtype=bool)
    # diagonal v00-v11 (flip False) or v10-v01 (flip True)
    t1 = np.where(flip[:, None], np.stack([v00, v10, v01], 1), np.stack([v00, v10, v11], 1))
    t2 = np.where(flip[:, None], np.stack([v10, v11, v01], 1), np.stack([v00, v11, v01], 1))
    cells = np.empty((2 * qi.size, 3), dtype=np.int64)
    cells[0::2] = t1
    cells[1::2] = t2
    return coords, cells.astype(np.int32), interior


# Kuhn subdivision of the unit cube into 6 tetrahedra sharing the main
# diagonal: one tet per permutation of the axes.
_KUHN_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def _cube_grid(n: int, rng: np.random.Generator, jitter: float):
    h = 1.0 / n
    m = n + 1
    ii, jj, kk = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    # vertex id = i + m*j + m*m*k
    ii = ii.transpose(2, 1, 0).ravel()
    jj = jj.transpose(2, 1, 0).ravel()
    kk = kk.transpose(2, 1, 0).ravel()
    coords = np.stack([ii * h, jj * h, kk * h], axis=1).astype(np.float64)
    interior = (ii > 0) & (ii < n) & (jj > 0) & (jj < n) & (kk > 0) & (kk < n)
    if jitter > 0:
        disp = rng.uniform(-jitter * h, jitter * h, size=(int(interior.sum()), 3))
        coords[interior] += disp
    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    base = ci + m * cj + m * m * ck
    step = np.array([1, m, m * m])
    cells = np.empty((6 * base.size, 4), dtype=np.int64)
    for t, perm in enumerate(_KUHN_PERMS):
        v0 = base
        v1 = v0 + step[perm[0]]
        v2 = v1 + step[perm[1]]
        v3 = v2 + step[perm[2]]
        tet = np.stack([v0, v1, v2, v3], axis=1)
        cells[t::6] = tet
    cells = cells.astype(np.int32)
    vol = orientation(coords, cells)
    neg = vol < 0
    cells[neg, 2], cells[neg, 3] = cells[neg, 3].copy(), cells[neg, 2].copy()
    return coords, cells, interior


# ----------------------------------------------------------------------------
# controlled degradation by vertex displacement
# ----------------------------------------------------------------------------

def _vertex_cells(nv: int, cells: np.ndarray):
    """CSR list of the cells incident to every vertex."""
    flat = cells.ravel()
    order = np.argsort(flat, kind="stable")
    counts = np.bincount(flat, minlength=nv)
    ptr = np.zeros(nv + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    cell_of = order // cells.shape[1]
    return ptr, cell_of


def _displace_towards_facet(coords, cells, v, cell, depth, rng):
    """New position of vertex v: at distance depth*|facet| from the affine hull
    of the facet of `cell` opposite v, over a point inside that facet."""
    d = coords.shape[1]
    others = [w for w in cells[cell] if w != v]
    p = coords[others]
    if d == 2:
        a, b = p
        ab = b - a
        # foot of the perpendicular from v, kept in the middle fifth of the edge
        t = float(np.clip(np.dot(coords[v] - a, ab) / np.dot(ab, ab), 0.4, 0.6))
        foot = a + t * ab
        nrm = np.array([-ab[1], ab[0]])
        length = np.linalg.norm(ab)
    else:
        a, b, c = p
        w = rng.dirichlet([4.0, 4.0, 4.0])
        foot = w[0] * a + w[1] * b + w[2] * c
        nrm = np.cross(b - a, c - a)
        length = np.sqrt(np.linalg.norm(b - a) * np.linalg.norm(c - a))
    nrm = nrm / np.linalg.norm(nrm)
    side = np.sign(np.dot(coords[v] - foot, nrm))
    if side == 0:
        side = 1.0
    return foot + side * depth * length * nrm


def _grid_neighbours(centre, n, interior, radius):
    """Vertex ids of the structured (n+1)^d grid within `radius` grid steps
    of the grid point nearest to `centre` (ids follow i + (n+1)*j [+ ...])."""
    d = centre.shape[0]
    m = n + 1
    g = np.clip(np.rint(centre * n).astype(np.int64), 0, n)
    axes = [np.arange(max(0, g[a] - radius), min(n, g[a] + radius) + 1) for a in range(d)]
    mesh = np.meshgrid(*axes, indexing="ij")
    ids = np.zeros(mesh[0].size, dtype=np.int64)
    stride = 1
    for a in range(d):
        ids += mesh[a].ravel() * stride
        stride *= m
    ids = np.sort(ids)
    return ids[interior[ids]]


def _degrade(coords, cells, interior, centres, per_cluster, depth_range, rng,
             log_depth=True, n=None):
    """Insert clusters of degraded cells.

    For each cluster centre, the `k` interior vertices closest to it are each
    pulled to a small distance from the facet opposite them in one incident
    cell (chosen at random).  A move is kept only if every incident cell keeps
    a positive orientation.  No two displaced vertices share a cell, so every
    degraded cell has one displaced vertex and its neighbours across the
    other facets stay of normal size.  Returns the list of moved vertex ids.
    """
    nv = coords.shape[0]
    ptr, cell_of = _vertex_cells(nv, cells)
    moved = []
    used = np.zeros(nv, dtype=bool)
    for centre, k in zip(centres, per_cluster):
        ids = _grid_neighbours(centre, n, interior, 3)
        dist = np.linalg.norm(coords[ids] - centre, axis=1)
        cand = ids[np.lexsort((ids, dist))][: 4 * k + 8]
        done = 0
        for v in cand:
            if done >= k:
                break
            if used[v]:
                continue
            inc = cell_of[ptr[v]:ptr[v + 1]]
            for _attempt in range(4):
                cell = inc[rng.integers(0, inc.size)]
                if log_depth:
                    depth = float(np.exp(rng.uniform(np.log(depth_range[0]),
                                                     np.log(depth_range[1]))))
                else:
                    depth = float(rng.uniform(*depth_range))
                old = coords[v].copy()
                coords[v] = _displace_towards_facet(coords, cells, v, cell, depth, rng)
                if np.all(orientation(coords, cells[inc]) > 0):
                    # no two displaced vertices share a cell
                    used[np.unique(cells[inc])] = True
                    moved.append(int(v))
                    done += 1
                    break
                coords[v] = old
    return moved


# ----------------------------------------------------------------------------
# public mesh builders
# ----------------------------------------------------------------------------

def _dirichlet_2d(coords, where):
    x, y = coords[:, 0], coords[:, 1]
    on = np.zeros(coords.shape[0], dtype=bool)
    eps = 1e-14
    if "x0" in where:
        on |= x < eps
    if "x1" in where:
        on |= x > 1 - eps
    if "y0" in where:
        on |= y < eps
    if "y1" in where:
        on |= y > 1 - eps
    return on.astype(np.uint8)


def _dirichlet_3d(coords, where):
    on = np.zeros(coords.shape[0], dtype=bool)
    eps = 1e-14
    for axis, name in enumerate("xyz"):
        if name + "0" in where:
            on |= coords[:, axis] < eps
        if name + "1" in where:
            on |= coords[:, axis] > 1 - eps
    return on.astype(np.uint8)


def square_mesh(n: int, seed: int, jitter: float = 0.2, diagonal: str = "random",
                clusters: int = 0, cluster_size=(1, 8), depth=(3.5e-3, 3.5e-2),
                n_single: int = 0, single_depth: float = 1e-3,
                dirichlet=("x0", "x1", "y0", "y1")) -> dict:
    """Triangulation of [0,1]^2 from an (n+1)x(n+1) vertex grid.

    jitter: interior vertices move uniformly in +-jitter*h per coordinate.
    clusters: number of degraded-cell clusters at uniform interior positions,
        each with a uniform {cluster_size} number of displaced vertices; the
        displacement depth (fraction of the opposite edge length) is
        log-uniform in `depth`.
    n_single: isolated displaced vertices at depth `single_depth` * h.
    """
    rng = np.random.default_rng(seed)
    coords, cells, interior = _square_grid(n, rng, jitter, diagonal)
    moved = []
    if clusters > 0:
        centres = rng.uniform(0.05, 0.95, size=(clusters, 2))
        sizes = rng.integers(cluster_size[0], cluster_size[1] + 1, size=clusters)
        moved += _degrade(coords, cells, interior, centres, sizes, depth, rng, n=n)
    if n_single > 0:
        centres = rng.uniform(0.1, 0.9, size=(n_single, 2))
        moved += _degrade(coords, cells, interior, centres, [1] * n_single,
                          (single_depth, single_depth), rng, log_depth=False, n=n)
    assert np.all(orientation(coords, cells) > 0)
    return {"dim": 2, "coords": coords, "cells": np.ascontiguousarray(cells),
            "dirichlet_vertex": _dirichlet_2d(coords, dirichlet),
            "moved_vertices": np.array(moved, dtype=np.int64)}


def cube_mesh(n: int, seed: int, jitter: float = 0.15, slivers: int = 0,
              depth=(1e-4, 3e-3), dirichlet=("x0", "x1")) -> dict:
    """Kuhn tetrahedralisation (6 tets per cube) of an (n+1)^3 vertex grid.

    slivers: number of interior vertices (at uniform random positions) pulled
    to a log-uniform depth (fraction of the facet size) from the plane of the
    opposite face of one incident tetrahedron.
    """
    rng = np.random.default_rng(seed)
    coords, cells, interior = _cube_grid(n, rng, jitter)
    moved = []
    if slivers > 0:
        centres = rng.uniform(0.05, 0.95, size=(slivers, 3))
        moved = _degrade(coords, cells, interior, centres, [1] * slivers, depth, rng, n=n)
    assert np.all(orientation(coords, cells) > 0)
    return {"dim": 3, "coords": coords, "cells": np.ascontiguousarray(cells),
            "dirichlet_vertex": _dirichlet_3d(coords, dirichlet),
            "moved_vertices": np.array(moved, dtype=np.int64)}


def stress_cube_mesh(n: int, seed: int, jitter: float = 0.15, flat: float = 0.01, width=(2, 11),
                     dirichlet=("x0", "x1")) -> dict:
    """Kuhn cube grid with many separate flat regions (the patch stress case).

    The z levels are grouped in slabs of three (a fixed level, then two
    levels that are pressed towards their mid-plane to `flat` times their
    distance from it).  Inside a slab, the y direction is cut into strips and
    every strip is cut along x, with log-uniform box widths in `width`
    (interior grid columns between fixed lines).  The vertices of a box
    interior are pressed; vertices on the fixed levels and lines keep their
    place, so each box yields one connected region of flattened cells, and
    the regions of different boxes share no vertex.  All vertices of one grid
    column within a slab share their x, y position (the jitter of the slab's
    fixed level), which keeps every cell positively oriented.
    """
    rng = np.random.default_rng(seed)
    coords, cells, _interior = _cube_grid(n, rng, jitter)
    m = n + 1
    c3 = coords.reshape(m, m, m, 3)          # [k, j, i, :]
    lo, hi = np.log(width[0]), np.log(width[1] + 1)

    def cuts():
        c = [0]
        while c[-1] < n:
            w = int(np.exp(rng.uniform(lo, hi)))
            c.append(min(n, c[-1] + w + 1))
        return np.array(c)

    def interior_mask(c):
        mask = np.ones(m, dtype=bool)
        mask[c] = False
        return mask

    for k0 in range(0, n, 3):
        k1 = min(k0 + 3, n)                  # levels k0+1, k0+2 (< n) are pressed
        c3[k0 + 1:k1 + 1, :, :, :2] = c3[k0, :, :, :2]
        if k0 + 1 >= n:
            continue
        levels = np.arange(k0 + 1, min(k0 + 3, n))
        cy = cuts()
        ymask = interior_mask(cy)
        mid = (k0 + 1.5) / n
        for t in range(len(cy) - 1):
            j0, j1 = cy[t] + 1, cy[t + 1]
            if j1 <= j0:
                continue
            xmask = interior_mask(cuts())
            block = c3[levels[0]:levels[-1] + 1, j0:j1, :, 2]
            sel = ymask[j0:j1][:, None] & xmask[None, :]
            block[:, sel] = mid + flat * (block[:, sel] - mid)
    coords = c3.reshape(-1, 3)
    assert np.all(orientation(coords, cells) > 0)
    return {"dim": 3, "coords": coords, "cells": np.ascontiguousarray(cells),
            "dirichlet_vertex": _dirichlet_3d(coords, dirichlet)}


def lattice_mesh(n: int, seed: int, jitter: float = 0.15, slivers: int = 0, depth=(1e-4, 3e-3)) -> dict:
    """Kuhn tetrahedralisation of the truss-like lattice [0,6]^3 minus the three
    tunnels a x b^2, b x a x b, b^2 x a with a = [0, 6], b = [1, 5] (the twelve
    edges of the cube as bars of unit cross-section), on a grid of n intervals
    per side (n a multiple of 6, so the tunnel walls are grid planes).

    Vertex jitter leaves every coordinate that lies on a plane 0, 1, 5 or 6
    unchanged, so the boundary is the same for every level; degraded cells
    (`slivers`, as in cube_mesh) use vertices off those planes.  Dirichlet
    vertices: the face x = 0.
    """
    if n % 6:
        raise ValueError("lattice_mesh needs n divisible by 6")
    rng = np.random.default_rng(seed)
    coords, cells, _ = _cube_grid(n, rng, 0.0)
    coords *= 6.0
    h = 6.0 / n
    on_plane = np.zeros(coords.shape, dtype=bool)
    for v in (0.0, 1.0, 5.0, 6.0):
        on_plane |= np.abs(coords - v) < 1e-9
    disp = rng.uniform(-jitter * h, jitter * h, size=coords.shape)
    disp[on_plane] = 0.0
    coords = coords + disp
    cen = coords[cells].mean(axis=1)
    inb = (cen > 1.0) & (cen < 5.0)
    hole = (inb[:, 1] & inb[:, 2]) | (inb[:, 0] & inb[:, 2]) | (inb[:, 0] & inb[:, 1])
    cells = cells[~hole]
    used = np.unique(cells)
    remap = np.full(coords.shape[0], -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    coords = np.ascontiguousarray(coords[used])
    on_plane = on_plane[used]
    cells = remap[cells].astype(np.int32)
    if slivers > 0:
        free = ~on_plane.any(axis=1)
        # _degrade picks candidates near each centre on the structured grid; here
        # the vertex set is compacted, so candidates are the free vertices
        # nearest to each centre
        ptr, cell_of = _vertex_cells(coords.shape[0], cells)
        cand_all = np.flatnonzero(free)
        centres = coords[rng.choice(cand_all, size=min(slivers, cand_all.size), replace=False)]
        used_v = np.zeros(coords.shape[0], dtype=bool)
        for centre in centres:
            dist = np.linalg.norm(coords[cand_all] - centre, axis=1)
            for v in cand_all[np.argsort(dist, kind="stable")[:8]]:
                if used_v[v]:
                    continue
                inc = cell_of[ptr[v]:ptr[v + 1]]
                cell = inc[rng.integers(0, inc.size)]
                d = float(np.exp(rng.uniform(np.log(depth[0]), np.log(depth[1]))))
                old = coords[v].copy()
                coords[v] = _displace_towards_facet(coords, cells, v, cell, d, rng)
                if np.all(orientation(coords, cells[inc]) > 0):
                    used_v[np.unique(cells[inc])] = True
                    break
                coords[v] = old
    assert np.all(orientation(coords, cells) > 0)
    dv = (np.abs(coords[:, 0]) < 1e-12).astype(np.uint8)
    return {"dim": 3, "coords": coords, "cells": np.ascontiguousarray(cells), "dirichlet_vertex": dv}


# ----------------------------------------------------------------------------
# workload hierarchies
# ----------------------------------------------------------------------------

# Each entry: a recipe for the fine-to-coarse list of meshes.  `scale` divides
# the number of intervals per side (for reduced-size samples of a workload).
CONFIGS = {
    # 2D P1, 65x65 fine grid with 4 isolated slivers (depth 1e-3 of the edge);
    # coarse 33x33, 17x17.
    "square_p1_4k": dict(kind="square", sides=[64, 32, 16], jitter=0.2,
                         fine_single=4, single_depth=1e-3, clusters=[0, 0, 0],
                         dirichlet=("x0", "x1", "y0", "y1")),
    # 2D 1025x1025 fine grid, 256 clusters of 1-8 slivers, four coarse levels
    # obtained by halving the vertex count per side, each independently
    # jittered (the cluster counts of coarse levels apply to cases A and B).
    "square_1025": dict(kind="square", sides=[1024, 512, 256, 128, 64], jitter=0.2,
                        fine_single=0, clusters=[256, 64, 16, 4, 2],
                        dirichlet=("y0", "y1")),
    # 3D 129^3 Kuhn grid with 2000 cap/sliver tets, coarse 65^3, 33^3, 17^3, 9^3
    # (halving the intervals per side until the coarsest P2 system has a few
    # thousand unknowns).
    "cube_129": dict(kind="cube", sides=[128, 64, 32, 16, 8], jitter=0.15,
                     slivers=[2000, 250, 32, 4, 1], dirichlet=("x0", "x1")),
    # patch stress: the 129^3 cube with ~20k separate flattened regions on the
    # finest level (boxes 2-11 columns wide); coarse levels as cube_129 without
    # degraded cells.
    "cube_129_stress": dict(kind="cube_stress", sides=[128, 64, 32, 16, 8], jitter=0.15,
                            dirichlet=("x0", "x1")),
    # elasticity: the lattice [0,6]^3 minus three orthogonal tunnels, four levels
    # of 8, 4, 2 and 1 grid cells per unit (the bars are one unit thick), 400
    # degraded cells on the finest level, clamped at x = 0
    "lattice": dict(kind="lattice", sides=[48, 24, 12, 6], jitter=0.15, slivers=[400, 60, 8, 1]),
    # the same lattice at twice the resolution (16, 8, 4, 2 cells per unit)
    "lattice_96": dict(kind="lattice", sides=[96, 48, 24, 12], jitter=0.15, slivers=[400, 60, 8, 1]),
}


def hierarchy(name: str, seed: int = 0, scale: int = 1, case: str = "fine") -> list:
    """Fine-to-coarse list of meshes for a named workload.

    case "fine": degraded cells on the finest level only (the workload recipes);
    case "A": degraded cells on every level (the paper's Case A);
    case "B": finest level high quality, coarse levels degraded (Case B);
    case "ref": no degraded cells anywhere (the high-quality reference).
    scale: integer divisor of the per-side interval counts (a reduced sample).
    """
    cfg = CONFIGS[name]
    sides = [max(2, s // scale) for s in cfg["sides"]]
    out = []
    for lvl, n in enumerate(sides):
        lseed = int(seed) * 1000 + lvl
        degrade = ((case == "A") or (case == "B" and lvl > 0)
                   or (case == "fine" and lvl == 0))
        if cfg["kind"] == "square":
            nclus = (cfg["clusters"][lvl] // (scale * scale)) if degrade else 0
            if degrade and cfg["clusters"][lvl] > 0:
                nclus = max(1, nclus)
            nsingle = cfg.get("fine_single", 0) if degrade else 0
            out.append(square_mesh(n, lseed, jitter=cfg["jitter"], clusters=nclus,
                                   n_single=nsingle,
                                   single_depth=cfg.get("single_depth", 1e-3),
                                   dirichlet=cfg["dirichlet"]))
        elif cfg["kind"] == "lattice":
            m = max(6, (n // 6) * 6)
            ns = (cfg["slivers"][lvl] // (scale ** 3)) if degrade else 0
            if degrade and cfg["slivers"][lvl] > 0:
                ns = max(1, ns)
            out.append(lattice_mesh(m, lseed, jitter=cfg["jitter"], slivers=ns))
        elif cfg["kind"] == "cube_stress":
            if degrade:
                out.append(stress_cube_mesh(n, lseed, jitter=cfg["jitter"], dirichlet=cfg["dirichlet"]))
            else:
                out.append(cube_mesh(n, lseed, jitter=cfg["jitter"], dirichlet=cfg["dirichlet"]))
        else:
            ns = (cfg["slivers"][lvl] // (scale ** 3)) if degrade else 0
            if degrade and cfg["slivers"][lvl] > 0:
                ns = max(1, ns)
            out.append(cube_mesh(n, lseed, jitter=cfg["jitter"], slivers=ns,
                                 dirichlet=cfg["dirichlet"]))
    return out


def instance_batch(count: int = 32, seed: int = 0, dof_range=(5e4, 3e6), sliver_range=(10, 1000),
                   coarsest_dofs: int = 5000, scale: int = 1, sliver_cubes: int = 500, progress=None) -> list:
    """Independent unit-cube problems of uneven size for the many-instance solve.

    Per instance (seeded): degree P1 or P2, a DOF target log-uniform in
    `dof_range` (divided by scale^3), the matching Kuhn grid, a log-uniform
    number of slivers in `sliver_range`, capped at one per `sliver_cubes` grid
    cubes (about twice the sliver density of the 129^3 cube, so that the flagged
    regions of small meshes do not merge into one domain-spanning patch),
    Dirichlet on x = 0, 1, and coarse levels
    halving the intervals per side until the coarsest has <= coarsest_dofs DOFs.
    Returns a list of (meshes, degree).
    """
    rng = np.random.default_rng(77_000 + int(seed))
    out = []
    for i in range(count):
        degree = int(rng.integers(1, 3))
        target = float(np.exp(rng.uniform(np.log(dof_range[0]), np.log(dof_range[1])))) / scale ** 3
        per_side = target ** (1.0 / 3.0)
        n = max(2, int(round(per_side - 1)) if degree == 1 else int(round((per_side - 1) / 2)))
        nsl = int(np.exp(rng.uniform(np.log(sliver_range[0]), np.log(sliver_range[1]))))
        nsl = max(1, nsl // scale ** 3)
        sides = [n]
        while (degree * sides[-1] + 1) ** 3 > coarsest_dofs and sides[-1] > 2:
            sides.append(max(2, sides[-1] // 2))
        meshes = []
        for lvl, m in enumerate(sides):
            meshes.append(cube_mesh(m, seed * 100_000 + i * 100 + lvl, jitter=0.15,
                                    slivers=min(nsl, max(1, m ** 3 // sliver_cubes)) if lvl == 0 else 0,
                                    dirichlet=("x0", "x1")))
        out.append((meshes, degree))
        if progress is not None:
            progress(i, meshes, degree)
    return out


def random_rhs(n: int, seed: int) -> np.ndarray:
    """Uniform [-1, 1] vector of length n (a right-hand side or nodal data)."""
    return np.random.default_rng(10_000_019 + int(seed)).uniform(-1.0, 1.0, size=n)
