"""One step of iterative refinement of the patch solves (patch_refine).

Each local correction solves A^[d] e = r with the stored inverse X; with
refinement it forms e1 = X r, the FP64 residual r2 = r - A^[d] e1 of the patch
system (the patch rows of A restricted to the patch's own columns) and
returns e1 + X r2.  The explicit inverse's rounding error, of order
eps kappa(A^[d]) relative, becomes of order (eps kappa)^2, which brings the
GPU's patch solves onto the oracle's Cholesky solves on ill-conditioned
patches.  Checked on the FP64 path (one smoother application and one V-cycle
within 1e-10 of the oracle, PCG iterations +-1 and the solution within 1e-8),
on the mixed path with FP32-factored patches (PCG +-1, 1e-6 of the converged
solution) and in block solves (equal to the single-vector solves to rounding).
The elasticity lattice, whose patch matrices reach kappa = 1.6e5, is checked
at the plain 1e-10 bar in test_gpu_elasticity.
"""
import functools

import numpy as np
import pytest

import meshgen
from tests.parity_util import build_pair, from_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    # name: (workload, scale, degree, layers, policy)
    "square_p2": ("square_1025", 16, 2, 1, "merge"),
    "cube_stress_p2": ("cube_129_stress", 8, 2, 0, "overlap"),
    "square_p2_overlap": ("square_1025", 16, 2, 1, "overlap"),
}


@functools.lru_cache(maxsize=None)
def pair(name, precision="fp64"):
    wl, scale, degree, layers, policy = CASES[name]
    meshes = meshgen.hierarchy(wl, seed=0, scale=scale)
    print(f"[refine {name} {precision}]", flush=True)
    return build_pair(meshes, degree, layers=layers, policy=policy, precision=precision, patch_refine=True,
                      build_oracle=precision == "fp64")


@pytest.mark.parametrize("name", list(CASES))
def test_refined_fp64(name):
    gpu, ora = pair(name)
    n = ora.levels[0].A.shape[0]
    b, u0 = meshgen.random_rhs(n, 41), meshgen.random_rhs(n, 42)
    u = to_dev(u0)
    gpu.smooth(0, to_dev(b), u, 1)
    assert rel_err(from_dev(u), ora.smooth(0, b, u0.copy(), 1)) < 1e-10
    u = to_dev(u0)
    gpu.vcycle(to_dev(b), u)
    assert rel_err(from_dev(u), ora.vcycle(b, u0.copy())) < 1e-10
    x_o, it_o, conv_o, _ = ora.pcg(b, 1e-10, 300)
    u = to_dev(np.zeros(n))
    st = gpu.pcg(to_dev(b), u, 1e-10, 300)
    assert conv_o and st["converged"] and abs(st["iterations"] - it_o) <= 1
    assert rel_err(from_dev(u), x_o) < 1e-8


@pytest.mark.parametrize("name", list(CASES))
def test_refined_mixed(name):
    _, ora = pair(name)
    gmix, _ = pair(name, "mixed")
    n = ora.levels[0].A.shape[0]
    b = meshgen.random_rhs(n, 43)
    x_ref = ora.pcg(b, 1e-12, 300)[0]
    _, it_o, _, _ = ora.pcg(b, 1e-8, 300)
    u = to_dev(np.zeros(n))
    st = gmix.pcg(to_dev(b), u, 1e-8, 300)
    assert st["converged"] and abs(st["iterations"] - it_o) <= 1
    assert rel_err(from_dev(u), x_ref) < 1e-6


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_refined_block_solves(precision):
    gpu = pair("cube_stress_p2", precision)[0]
    n = gpu.n_free(0)
    bs = [to_dev(meshgen.random_rhs(n, 50 + r)) for r in range(3)]
    us = [to_dev(np.zeros(n)) for _ in range(3)]
    res = gpu.pcg_multi(bs, us, 1e-8, 300)
    tol = 1e-10 if precision == "fp64" else 1e-6
    for r in range(3):
        u = to_dev(np.zeros(n))
        st = gpu.pcg(bs[r], u, 1e-8, 300)
        assert abs(res["stats"][r]["iterations"] - st["iterations"]) <= 1
        assert rel_err(from_dev(us[r]), from_dev(u)) < tol
