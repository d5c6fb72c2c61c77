"""Pins of the oracle's cell quality (Sec. 3 eq. radius_ratio) and of the
local-correction regions (Sec. 4.1, Sec. 4.4 eq. identify)."""
import os

import numpy as np
import pytest

import meshgen
import oracle
from oracle.fem import DofMap
from oracle.patches import MERGE, OVERLAP, colour, patches
from tests.meshes_util import tiny_square

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "quality_examples.txt")


def _golden_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            name, dim, xs, expect, tol = [s.strip() for s in line.split("|")]
            dim = int(dim)
            x = np.array([float(v) for v in xs.split()]).reshape(dim + 1, dim)
            rows.append((name, x, float(expect), float(tol)))
    return rows


@pytest.mark.parametrize("name,x,expect,tol", _golden_rows())
def test_quality_golden(name, x, expect, tol):
    g = oracle.radius_ratio(x, np.arange(x.shape[0])[None, :])[0]
    assert abs(g - expect) <= tol * expect, name


def test_quality_triangle_half_angle_identity():
    """gamma = 2 r/R = 8 prod sin(angle/2) for every triangle."""
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, size=(200, 3, 2))
    g = oracle.radius_ratio(x.reshape(-1, 2), np.arange(600).reshape(200, 3))
    for k in range(200):
        p = x[k]
        ang = []
        for i in range(3):
            u, v = p[(i + 1) % 3] - p[i], p[(i + 2) % 3] - p[i]
            ang.append(np.arccos(np.clip(u @ v / np.linalg.norm(u) / np.linalg.norm(v), -1, 1)))
        expect = 8 * np.prod(np.sin(np.array(ang) / 2))
        assert abs(g[k] - expect) <= 1e-9 * max(expect, 1e-3)


def test_quality_range_and_invariance():
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, size=(50, 4, 3))
    cells = np.arange(200).reshape(50, 4)
    g = oracle.radius_ratio(x.reshape(-1, 3), cells)
    assert np.all((g > 0) & (g <= 1 + 1e-12))
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    y = 3.7 * x.reshape(-1, 3) @ Q.T + 0.5
    assert np.allclose(oracle.radius_ratio(y, cells), g, rtol=1e-10)


def test_quality_degenerates_with_displacement():
    """A vertex pulled towards the opposite edge drives gamma to 0."""
    a, b = np.array([0.0, 0.0]), np.array([1.0, 0.0])
    prev = 1.0
    for depth in (0.5, 0.1, 1e-2, 1e-3, 1e-4):
        g = oracle.radius_ratio(np.array([a, b, [0.5, depth]]), np.array([[0, 1, 2]]))[0]
        assert g < prev
        prev = g
    assert prev < 1e-6


def _regions_by_hand(mesh, gamma, tau, layers):
    """Omega_B by definition: flagged cells plus `layers` rounds of adding every
    cell that shares a vertex with the current set (set algebra, no BFS)."""
    cells = mesh["cells"]
    cur = gamma < tau
    for _ in range(layers):
        verts = np.zeros(mesh["coords"].shape[0], dtype=bool)
        verts[cells[cur].ravel()] = True
        cur = cur | np.any(verts[cells], axis=1)
    return cur


def _components(cells, member):
    """Connected components of the member cells under vertex sharing (dense
    adjacency, brute force)."""
    ids = np.flatnonzero(member)
    sets = [set(cells[c].tolist()) for c in ids]
    n = len(ids)
    adj = np.array([[bool(sets[i] & sets[j]) for j in range(n)] for i in range(n)])
    label = -np.ones(n, dtype=int)
    k = 0
    for i in range(n):
        if label[i] >= 0:
            continue
        stack = [i]
        label[i] = k
        while stack:
            a = stack.pop()
            for b in np.flatnonzero(adj[a]):
                if label[b] < 0:
                    label[b] = k
                    stack.append(b)
        k += 1
    return [np.sort(ids[label == j]) for j in range(k)]


@pytest.mark.parametrize("layers", [1, 2])
def test_merge_patches_are_components_of_region(layers):
    mesh = meshgen.square_mesh(12, 5, n_single=3, single_depth=1e-3)
    dm = DofMap(mesh, 2)
    gamma = oracle.radius_ratio(mesh["coords"], mesh["cells"])
    pc, pd = patches(dm.cells, dm.coords.shape[0], gamma, 0.1, layers, MERGE,
                     dm.cell_dofs, dm.free_index)
    region = _regions_by_hand(mesh, gamma, 0.1, layers)
    comps = _components(mesh["cells"], region)
    comps.sort(key=lambda s: s[0])
    assert len(pc) == len(comps)
    for got, want in zip(pc, comps):
        assert np.array_equal(got, want)
    # DOF sets: free DOFs of the patch cells, ascending, disjoint across patches
    seen = set()
    for cs, B in zip(pc, pd):
        want = np.unique(dm.free_index[np.unique(dm.cell_dofs[cs])])
        want = want[want >= 0]
        assert np.array_equal(B, want)
        assert not (seen & set(B.tolist()))
        seen |= set(B.tolist())
    assert np.all(colour(pd) == 0)


def test_paper_region_definition_one_layer():
    """tau = 0.1 and one vertex layer reproduce eq. identify literally."""
    mesh = meshgen.square_mesh(10, 9, n_single=2, single_depth=1e-3)
    dm = DofMap(mesh, 1)
    gamma = oracle.radius_ratio(mesh["coords"], mesh["cells"])
    pc, _ = patches(dm.cells, dm.coords.shape[0], gamma, 0.1, 1, MERGE, dm.cell_dofs, dm.free_index)
    flagged = gamma < 0.1
    verts = np.unique(mesh["cells"][flagged])
    shares = np.any(np.isin(mesh["cells"], verts), axis=1)
    expect = np.flatnonzero(flagged | shares)
    got = np.sort(np.concatenate(pc))
    assert np.array_equal(got, expect)


def test_threshold_is_strict():
    mesh = tiny_square(3, seed=0)
    dm = DofMap(mesh, 1)
    gamma = np.full(mesh["cells"].shape[0], 0.5)
    gamma[4] = 0.1
    pc, _ = patches(dm.cells, dm.coords.shape[0], gamma, 0.1, 1, MERGE, dm.cell_dofs, dm.free_index)
    assert pc == []
    gamma[4] = np.nextafter(0.1, 0)
    pc, _ = patches(dm.cells, dm.coords.shape[0], gamma, 0.1, 1, MERGE, dm.cell_dofs, dm.free_index)
    assert len(pc) == 1


def test_overlap_patches_and_colouring():
    """Two flagged cells two cells apart: grown patches overlap under OVERLAP
    and must get different colours; under MERGE they form one patch."""
    mesh = tiny_square(6, seed=2, jitter=0.0, diagonal="right", dirichlet=())
    dm = DofMap(mesh, 1)
    gamma = np.ones(mesh["cells"].shape[0])
    # cells of quads (1,2) and (3,2): separated by one quad, so they do not
    # share a vertex, but their one-layer extensions do
    q = lambda i, j: 2 * (i + 6 * j)
    gamma[q(1, 2)] = 0.01
    gamma[q(3, 2)] = 0.01
    pc, pd = patches(dm.cells, dm.coords.shape[0], gamma, 0.1, 1, OVERLAP, dm.cell_dofs, dm.free_index)
    assert len(pc) == 2
    assert set(pd[0].tolist()) & set(pd[1].tolist())
    col = colour(pd)
    assert list(col) == [0, 1]
    pcm, _ = patches(dm.cells, dm.coords.shape[0], gamma, 0.1, 1, MERGE, dm.cell_dofs, dm.free_index)
    assert len(pcm) == 1


def test_colouring_is_proper_and_greedy():
    rng = np.random.default_rng(4)
    pd = [np.unique(rng.integers(0, 60, size=rng.integers(3, 9))) for _ in range(25)]
    col = colour(pd)
    for i in range(25):
        for j in range(i):
            if set(pd[i].tolist()) & set(pd[j].tolist()):
                assert col[i] != col[j]
        # greedy: every smaller colour is blocked by an earlier conflicting patch
        for c in range(col[i]):
            assert any(col[j] == c and set(pd[i].tolist()) & set(pd[j].tolist()) for j in range(i))


def test_inherited_seeds_follow_the_located_cells():
    """The coarse DOFs inherited from a fine DOF set are the free DOFs of the
    coarse cells that contain its nodes (the structure of P)."""
    from oracle.fem import DofMap
    from oracle.patches import inherit
    from oracle.transfer import prolongation
    meshes = meshgen.hierarchy("cube_129", seed=0, scale=16)
    fine, coarse = DofMap(meshes[0], 2), DofMap(meshes[1], 2)
    P, cell = prolongation(fine, coarse)
    rng = np.random.default_rng(0)
    sets = [np.sort(rng.choice(fine.n_free, 12, replace=False)) for _ in range(5)]
    for s, got in zip(sets, inherit(P, sets)):
        want = coarse.free_index[coarse.cell_dofs[cell[s]]].ravel()
        assert np.array_equal(got, np.unique(want[want >= 0]))


def test_components_and_combine():
    from oracle.patches import MERGE, OVERLAP, combine, components
    sets = [np.array([5, 6]), np.array([1, 2]), np.array([6, 9]), np.array([]), np.array([2, 3])]
    comps = components(sets)
    assert [c.tolist() for c in comps] == [[1, 2, 3], [5, 6, 9]]
    own = [np.array([7, 8]), np.array([3, 4])]
    merged = combine(own, comps, MERGE)
    assert [m.tolist() for m in merged] == [[7, 8], [1, 2, 3, 4], [5, 6, 9]]
    kept = combine(own, comps, OVERLAP)
    assert [m.tolist() for m in kept] == [[7, 8], [3, 4], [1, 2, 3], [5, 6, 9]]


def test_inherited_patches_restore_the_reference_eigenvalue():
    """With degraded cells on the finest level only, the Galerkin operator of
    level 1 inherits their stiffness: lambda_max(D^-1 A_1) roughly doubles
    against the high-quality reference mesh, and the paper's adjusted
    eigenvalue cannot see it (level 1 has no patches of its own).  The
    patches inherited through P bring the adjusted eigenvalue of level 1 back
    to the reference level's lambda_max."""
    from oracle.multigrid import Hierarchy, Options
    ref = Hierarchy(meshgen.hierarchy("cube_129", seed=0, scale=8, case="ref"), tau=0.1, layers=1,
                    opts=Options(degree=2))
    meshes = meshgen.hierarchy("cube_129", seed=0, scale=8)
    paper = Hierarchy(meshes, tau=0.1, layers=1, opts=Options(degree=2))
    inh = Hierarchy(meshes, tau=0.1, layers=1, opts=Options(degree=2, inherit_levels=1))
    lam_ref = ref.levels[1].lam
    assert len(paper.levels[1].patch_dofs) == 0 and paper.levels[1].hi > 1.5 * lam_ref
    assert len(inh.levels[1].patch_dofs) > 0
    assert abs(inh.levels[1].hi - lam_ref) < 0.01 * lam_ref
    # level 2 keeps the paper's patches (none)
    assert len(inh.levels[2].patch_dofs) == 0
