"""Oracle: local-correction subdomains, their DOF sets and colours.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows Sec. 4.1 (subdomains Omega_B^d with DOF sets B_d and inclusions I_d)
and Sec. 4.4, eq. (identify): Omega_b is the set of cells with gamma < tau, and
Omega_B adds every cell sharing a vertex with Omega_b (one layer; the number of
layers is a parameter here).  The paper asks the subdomains to have disjoint
closures; the reading used is pairwise disjointness, so under the MERGE policy
the subdomains are the connected components of Omega_B under "shares a vertex".

Canonical construction (the paper is silent on orderings):
  1. components of Omega_b under vertex sharing, found by breadth-first search
     started from the lowest unvisited flagged cell id;
  2. each component grown by `layers` vertex layers (layer k adds every cell
     sharing a vertex with the layer k-1 set);
  3. MERGE: grown sets that share a vertex are merged (union-find);
     OVERLAP: grown sets are kept as they are (they may overlap);
  4. patches ordered by their smallest cell id;
  5. B_d = the free DOFs of the patch's cells, ascending; empty patches dropped.
Colouring: greedy in patch order, each patch taking the smallest colour not used
by an earlier patch with which it shares a DOF.  MERGE always gives one colour.

Inherited patches (an option; the paper identifies every level's subdomains
from that level's own cells).  The Galerkin operator A_(l+1) = P_l^T A_l P_l
(Sec. 2) carries the stiffness of the finest level's degraded cells into the
rows of the coarse DOFs that P interpolates at those cells' nodes, whatever
the quality of the coarse mesh.  With inherit_levels = k, the seeds are the
free DOF sets of the degraded cells of level 0 (one per cell), S_(l+1) holds,
for each set of S_l, the coarse DOFs that P_l couples to it (the structural
nonzeros of its rows: the free DOFs of the coarse cell that contains each
node), and levels 1..k add the connected components of S_l under "shares a
DOF" (ordered by smallest DOF) after their own patches; MERGE joins a
component with the own patches it shares DOFs with (into the lowest-indexed
one), OVERLAP keeps them apart and colours them.
"""
from __future__ import annotations

from collections import deque

import numpy as np

MERGE = 0
OVERLAP = 1


def vertex_to_cells(nv: int, cells: np.ndarray):
    flat = cells.ravel()
    order = np.argsort(flat, kind="stable")
    ptr = np.zeros(nv + 1, dtype=np.int64)
    np.cumsum(np.bincount(flat, minlength=nv), out=ptr[1:])
    return ptr, (order // cells.shape[1]).astype(np.int64)


def patches(cells: np.ndarray, nv: int, gamma: np.ndarray, tau: float, layers: int,
            policy: int, cell_dofs: np.ndarray, free_index: np.ndarray):
    """Returns (list of patch cell arrays, list of patch DOF arrays (free ids))."""
    cells = np.asarray(cells, dtype=np.int64)
    flagged = np.flatnonzero(gamma < tau)
    if flagged.size == 0:
        return [], []
    vptr, vcells = vertex_to_cells(nv, cells)
    is_flag = np.zeros(cells.shape[0], dtype=bool)
    is_flag[flagged] = True

    def cell_neighbours(c):
        out = set()
        for v in cells[c]:
            out.update(vcells[vptr[v]:vptr[v + 1]].tolist())
        return out

    # 1. components of Omega_b
    seen = np.zeros(cells.shape[0], dtype=bool)
    comps = []
    for c0 in flagged:
        if seen[c0]:
            continue
        comp, queue = [], deque([int(c0)])
        seen[c0] = True
        while queue:
            c = queue.popleft()
            comp.append(c)
            for nb in sorted(cell_neighbours(c)):
                if is_flag[nb] and not seen[nb]:
                    seen[nb] = True
                    queue.append(nb)
        comps.append(sorted(comp))

    # 2. layer growth
    grown = []
    for comp in comps:
        cur = set(comp)
        for _ in range(layers):
            verts = np.unique(cells[sorted(cur)])
            nxt = set(cur)
            for v in verts:
                nxt.update(vcells[vptr[v]:vptr[v + 1]].tolist())
            cur = nxt
        grown.append(np.array(sorted(cur), dtype=np.int64))

    # 3. merge or keep
    if policy == MERGE:
        parent = list(range(len(grown)))

        def find(a):
            while parent[a] != a:
                parent[a] = parent[parent[a]]
                a = parent[a]
            return a

        owner = {}
        for p, cs in enumerate(grown):
            for v in np.unique(cells[cs]).tolist():
                if v in owner:
                    ra, rb = find(owner[v]), find(p)
                    if ra != rb:
                        parent[max(ra, rb)] = min(ra, rb)
                else:
                    owner[v] = p
        groups = {}
        for p in range(len(grown)):
            groups.setdefault(find(p), []).append(p)
        sets = [np.unique(np.concatenate([grown[p] for p in g])) for g in groups.values()]
    else:
        sets = grown

    # 4. order by smallest cell id; 5. DOF sets
    sets.sort(key=lambda s: int(s[0]))
    out_cells, out_dofs = [], []
    for s in sets:
        dofs = np.unique(cell_dofs[s].ravel())
        f = free_index[dofs]
        f = np.sort(f[f >= 0])
        if f.size:
            out_cells.append(s)
            out_dofs.append(f)
    return out_cells, out_dofs


def colour(patch_dofs: list) -> np.ndarray:
    """Greedy colouring of the 'shares a DOF' conflict graph in patch order."""
    col = np.full(len(patch_dofs), -1, dtype=np.int64)
    owner = {}  # dof -> list of patches that contain it
    for p, dofs in enumerate(patch_dofs):
        used = set()
        for i in dofs.tolist():
            for q in owner.get(i, ()):
                used.add(int(col[q]))
        c = 0
        while c in used:
            c += 1
        col[p] = c
        for i in dofs.tolist():
            owner.setdefault(i, []).append(p)
    return col


def inherit(P, sets: list) -> list:
    """For each fine DOF set, the coarse DOFs that P couples to it: the column
    indices of P's rows at the set (P stores every free DOF of the coarse cell
    that contains a fine node, zero values included)."""
    import scipy.sparse as sp
    P = sp.csr_matrix(P)
    out = []
    for s in sets:
        idx = [P.indices[P.indptr[i]:P.indptr[i + 1]] for i in np.asarray(s, dtype=np.int64)]
        out.append(np.unique(np.concatenate(idx)) if idx else np.zeros(0, dtype=np.int64))
    return out


def components(sets: list) -> list:
    """Connected components of a family of DOF sets under "shares a DOF", each
    the sorted union of its sets, ordered by their smallest DOF."""
    parent = list(range(len(sets)))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    owner = {}
    for k, s in enumerate(sets):
        for d in np.asarray(s).tolist():
            if d in owner:
                ra, rb = find(owner[d]), find(k)
                if ra != rb:
                    parent[max(ra, rb)] = min(ra, rb)
            else:
                owner[d] = k
    groups = {}
    for k in range(len(sets)):
        groups.setdefault(find(k), []).append(k)
    out = [np.unique(np.concatenate([np.asarray(sets[k], dtype=np.int64) for k in g])) for g in groups.values()]
    out = [c for c in out if c.size]
    out.sort(key=lambda c: int(c[0]))
    return out


def combine(own: list, inherited: list, policy: int) -> list:
    """A level's patches: its own, then the inherited components.  MERGE: an
    inherited component that shares DOFs with own patches joins them, all
    into the lowest-indexed of them (own patches are pairwise disjoint, and so
    are the components); OVERLAP: kept apart."""
    allp = [np.asarray(p, dtype=np.int64) for p in own] + [np.asarray(p, dtype=np.int64) for p in inherited]
    if policy != MERGE:
        return allp
    parent = list(range(len(allp)))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    owner = {}
    for k, p in enumerate(allp):
        for d in p.tolist():
            if d in owner:
                ra, rb = find(owner[d]), find(k)
                if ra != rb:
                    parent[max(ra, rb)] = min(ra, rb)
            else:
                owner[d] = k
    groups = {}
    for k in range(len(allp)):
        groups.setdefault(find(k), []).append(k)
    roots = sorted(groups)
    return [np.unique(np.concatenate([allp[k] for k in groups[r]])) for r in roots]
