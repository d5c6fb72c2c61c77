"""GPU parity for local-correction patches too large for the one-workgroup
factorisation: dense sliver clusters on small P2 cubes merge (MERGE policy)
into patches of thousands of DOFs, which are factored by the blocked
multi-workgroup Cholesky and applied with the patch residual in LDS (up to
64 KiB) or read from global memory (beyond).  Bars as in the other parity
tests: patch membership bit-exact, one smoother application and one V-cycle
within 1e-10 (FP64), PCG iterations +-1 and the solution within 1e-8 of the
oracle's at the same tolerance (FP64) or 1e-6 of the converged one (mixed)."""
import functools

import numpy as np
import pytest

import meshgen
from tests.parity_util import build_pair, from_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu

# side of the fine cube, slivers on it; the largest patch has 5768 DOFs (small
# and blocked factorisation, LDS-staged apply) and 9301 DOFs (FP64 apply from
# global memory)
CASES = {"mixed_sizes": (12, 40, 11), "one_domain": (12, 80, 123)}


def meshes_of(side, slivers, seed):
    return [meshgen.cube_mesh(side, seed, jitter=0.15, slivers=slivers, dirichlet=("x0", "x1")),
            meshgen.cube_mesh(side // 2, seed + 1, jitter=0.15, slivers=0, dirichlet=("x0", "x1")),
            meshgen.cube_mesh(side // 4, seed + 2, jitter=0.15, slivers=0, dirichlet=("x0", "x1"))]


@functools.lru_cache(maxsize=None)
def pair(name, precision="fp64"):
    meshes = meshes_of(*CASES[name])
    print(f"[large patches {name} {precision}]", flush=True)
    return build_pair(meshes, 2, precision=precision, build_oracle=precision == "fp64")


@pytest.mark.parametrize("name", list(CASES))
def test_patches_and_smoother(name):
    gpu, ora = pair(name)
    lev = ora.levels[0]
    ptr, dofs = gpu.get_array(0, "patch_ptr"), gpu.get_array(0, "patch_dofs")
    assert len(ptr) - 1 == len(lev.patch_dofs)
    for d, B in enumerate(lev.patch_dofs):
        assert np.array_equal(dofs[ptr[d]:ptr[d + 1]], B)
    assert max(len(B) for B in lev.patch_dofs) > 4000
    n = lev.A.shape[0]
    b, u0 = meshgen.random_rhs(n, 1), meshgen.random_rhs(n, 2)
    want = ora.smooth(0, b, u0.copy(), 1)
    u = to_dev(u0)
    gpu.smooth(0, to_dev(b), u, 1)
    assert rel_err(from_dev(u), want) < 1e-10
    want = ora.vcycle(b)
    got = to_dev(np.zeros(n))
    gpu.vcycle(to_dev(b), got)
    assert rel_err(from_dev(got), want) < 1e-10


@pytest.mark.parametrize("name", list(CASES))
def test_pcg_fp64(name):
    gpu, ora = pair(name)
    n = ora.levels[0].A.shape[0]
    b = meshgen.random_rhs(n, 3)
    rtol = 1e-10
    x_o, it_o, conv_o, _ = ora.pcg(b, rtol, 200)
    u = to_dev(np.zeros(n))
    st = gpu.pcg(to_dev(b), u, rtol, 200)
    assert conv_o and st["converged"] and abs(st["iterations"] - it_o) <= 1
    assert rel_err(from_dev(u), x_o) < 1e-8
    assert st["true_rel_residual"] < 10 * rtol


@pytest.mark.parametrize("name", list(CASES))
def test_pcg_mixed(name):
    ora = pair(name)[1]
    gpu = pair(name, "mixed")[0]
    n = ora.levels[0].A.shape[0]
    b = meshgen.random_rhs(n, 4)
    x_ref, _, _, _ = ora.pcg(b, 1e-12, 200)
    _, it_o, _, _ = ora.pcg(b, 1e-8, 200)
    u = to_dev(np.zeros(n))
    st = gpu.pcg(to_dev(b), u, 1e-8, 200)
    assert st["converged"] and abs(st["iterations"] - it_o) <= 1
    assert rel_err(from_dev(u), x_ref) < 1e-6
