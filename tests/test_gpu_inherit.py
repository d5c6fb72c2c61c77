"""Patches inherited through the interpolation (patch_inherit_levels).

With degraded cells on the finest level only, the Galerkin operators of the
coarse levels carry those cells' stiffness (through P) while the coarse meshes
have no degraded cells of their own, so the paper's construction gives them
no patches.  The option adds, on levels 1..k, the connected components of the
coarse DOF sets that P couples to each degraded cell's DOFs.  Checked against
the oracle, which builds the same sets from its own interpolation: patch
membership and colours bit-exact on every level, the adjusted eigenvalue
1e-7, one V-cycle 1e-10, PCG iterations +-1 and the solution 1e-8 (FP64) /
1e-6 (mixed); and the purpose: level 1's Chebyshev bound back at the
reference mesh's lambda_max.
"""
import functools

import numpy as np
import pytest

import meshgen
import oracle
from tests.parity_util import build_pair, from_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    # name: (workload, scale, degree, layers, policy, inherit levels)
    "cube_p2_1": ("cube_129", 8, 2, 1, "merge", 1),
    "cube_p2_2": ("cube_129", 8, 2, 1, "merge", 2),
    "square_p2_1": ("square_1025", 16, 2, 1, "merge", 1),
    "square_p2_overlap_1": ("square_1025", 16, 2, 1, "overlap", 1),
}


@functools.lru_cache(maxsize=None)
def pair(name, precision="fp64"):
    wl, scale, degree, layers, policy, k = CASES[name]
    meshes = meshgen.hierarchy(wl, seed=0, scale=scale)
    print(f"[inherit {name} {precision}]", flush=True)
    return build_pair(meshes, degree, layers=layers, policy=policy, precision=precision, inherit=k,
                      build_oracle=precision == "fp64")


@pytest.mark.parametrize("name", list(CASES))
def test_inherited_patches(name):
    gpu, ora = pair(name)
    k = CASES[name][5]
    for l, lev in enumerate(ora.levels[:-1]):
        info = gpu.level_info(l)
        ptr, dofs = gpu.get_array(l, "patch_ptr"), gpu.get_array(l, "patch_dofs")
        assert len(ptr) - 1 == len(lev.patch_dofs), (l, len(ptr) - 1, len(lev.patch_dofs))
        for d, B in enumerate(lev.patch_dofs):
            assert np.array_equal(dofs[ptr[d]:ptr[d + 1]], B)
        assert np.array_equal(gpu.get_array(l, "patch_colour"), lev.colours)
        if 1 <= l <= k:
            assert info["patches_inherited"] > 0
        assert info["cheb_hi"] == pytest.approx(lev.hi, rel=1e-7)
    n = ora.levels[0].A.shape[0]
    b, u0 = meshgen.random_rhs(n, 61), meshgen.random_rhs(n, 62)
    u = to_dev(u0)
    gpu.vcycle(to_dev(b), u)
    assert rel_err(from_dev(u), ora.vcycle(b, u0.copy())) < 1e-10
    x_o, it_o, conv_o, _ = ora.pcg(b, 1e-10, 300)
    u = to_dev(np.zeros(n))
    st = gpu.pcg(to_dev(b), u, 1e-10, 300)
    assert conv_o and st["converged"] and abs(st["iterations"] - it_o) <= 1
    assert rel_err(from_dev(u), x_o) < 1e-8


@pytest.mark.parametrize("name", ["cube_p2_1", "square_p2_overlap_1"])
def test_inherited_patches_mixed(name):
    _, ora = pair(name)
    gmix, _ = pair(name, "mixed")
    n = ora.levels[0].A.shape[0]
    b = meshgen.random_rhs(n, 63)
    x_ref = ora.pcg(b, 1e-12, 300)[0]
    _, it_o, _, _ = ora.pcg(b, 1e-8, 300)
    u = to_dev(np.zeros(n))
    st = gmix.pcg(to_dev(b), u, 1e-8, 300)
    assert st["converged"] and abs(st["iterations"] - it_o) <= 1
    assert rel_err(from_dev(u), x_ref) < 1e-6


def test_level1_bound_back_at_the_reference():
    from paper_2402_12947_amd import Solver
    gpu, _ = pair("cube_p2_1")
    ref = Solver(meshgen.hierarchy("cube_129", seed=0, scale=8, case="ref"), degree=2)
    plain = Solver(meshgen.hierarchy("cube_129", seed=0, scale=8), degree=2)
    lam_ref = ref.level_info(1)["lambda_max"]
    assert plain.level_info(1)["cheb_hi"] > 1.5 * lam_ref
    assert abs(gpu.level_info(1)["cheb_hi"] - lam_ref) < 0.01 * lam_ref
    ref.close()
    plain.close()


def test_inheritance_too_large_is_refused():
    """On the patch stress mesh (about 40 % of the fine DOFs in patches) the
    inherited components cover most of level 1: set-up stops with MG_ERR_LIMIT
    and names the inheritance, before any dense allocation."""
    from paper_2402_12947_amd import MG_ERR_LIMIT, setup_status
    meshes = meshgen.hierarchy("cube_129_stress", seed=0, scale=2)
    code, msg = setup_status(meshes, degree=2, layers=0, policy="overlap", patch_inherit_levels=1)
    print(f"[inherit stress] {code} {msg}", flush=True)
    assert code == MG_ERR_LIMIT and "patch_inherit_levels" in msg
