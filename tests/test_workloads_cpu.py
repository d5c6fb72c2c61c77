"""Shape of the synthetic workloads (CPU): the patch stress mesh keeps every
cell positively oriented, its flagged regions are separate (one patch per
pressed box under either policy, so OVERLAP needs a single colour), and the
patch sizes span the intended range; the many-instance batch stays within its
DOF range and has no domain-spanning patch."""
import numpy as np

import meshgen
import oracle
from oracle.fem import DofMap
from oracle.patches import MERGE, OVERLAP, colour, patches


def test_stress_mesh_regions_are_separate_and_sized():
    m = meshgen.stress_cube_mesh(32, 3)
    assert np.all(meshgen.orientation(m["coords"], m["cells"]) > 0)
    gamma = oracle.radius_ratio(m["coords"], m["cells"])
    flagged = gamma < 0.1
    assert 0.1 < flagged.mean() < 0.4
    dm = DofMap(m, 2)
    _, po = patches(dm.cells, dm.coords.shape[0], gamma, 0.1, 0, OVERLAP, dm.cell_dofs, dm.free_index)
    _, pm = patches(dm.cells, dm.coords.shape[0], gamma, 0.1, 0, MERGE, dm.cell_dofs, dm.free_index)
    assert len(po) == len(pm) > 150
    assert all(np.array_equal(a, b) for a, b in zip(po, pm))
    assert colour(po).max() == 0
    sizes = np.array([len(p) for p in po])
    assert sizes.min() < 60 and 1000 < sizes.max() <= 2048
    assert 0.25 < sizes.sum() / dm.n_free < 0.5


def test_stress_hierarchy_coarse_levels_are_clean():
    meshes = meshgen.hierarchy("cube_129_stress", seed=0, scale=8)
    assert [m["cells"].shape[0] for m in meshes] == [6 * 16 ** 3, 6 * 8 ** 3, 6 * 4 ** 3, 6 * 2 ** 3, 6 * 2 ** 3]
    for m in meshes[1:]:
        assert oracle.radius_ratio(m["coords"], m["cells"]).min() > 0.1


def test_instance_batch_sizes():
    inst = meshgen.instance_batch(6, seed=1, dof_range=(2e3, 3e4), coarsest_dofs=800)
    for meshes, degree in inst:
        m = meshes[0]
        n = DofMap(m, degree).n_free
        assert 1e3 < n < 5e4
        gamma = oracle.radius_ratio(m["coords"], m["cells"])
        dm = DofMap(m, degree)
        _, pd = patches(dm.cells, dm.coords.shape[0], gamma, 0.1, 1, MERGE, dm.cell_dofs, dm.free_index)
        assert max((len(p) for p in pd), default=0) < 0.5 * n
