"""FP32 matrix-core factorisation of the patch systems (the mixed-precision
cycle's default): symmetric diagonal equilibration, Cholesky, inverse and
W^T W products on v_mfma_f32_16x16x4 with FP32 accumulate; patches whose
scaled pivots fall below 2^-12 keep the FP64 factorisation.

Checked against the FP64-factored mixed cycle and the oracle: the number of
patches taken in FP32, one smoother application within 1e-3 of the one with
FP64-factored patches (both store the inverse in FP32; the FP32 factorisation
adds an error of order eps_32 / (smallest scaled pivot)), the mixed PCG
iteration count within one of the oracle's and the solution within 1e-6 of
the oracle's converged solution.
"""
import functools

import numpy as np
import pytest

import meshgen
import oracle
from tests.parity_util import from_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    # name: (workload, scale, degree, layers, policy)
    "cube_stress_p2": ("cube_129_stress", 8, 2, 0, "overlap"),
    "square_p2": ("square_1025", 8, 2, 1, "merge"),
    "cube_p2": ("cube_129", 8, 2, 1, "merge"),
}


@functools.lru_cache(maxsize=None)
def _oracle(name):
    wl, scale, degree, layers, policy = CASES[name]
    meshes = meshgen.hierarchy(wl, seed=0, scale=scale)
    ora = oracle.Hierarchy(meshes, tau=0.1, layers=layers,
                           opts=oracle.Options(degree=degree,
                                               patch_policy=oracle.OVERLAP if policy == "overlap" else oracle.MERGE))
    return meshes, ora


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_patch_factorisation(name):
    from paper_2402_12947_amd import Solver
    wl, scale, degree, layers, policy = CASES[name]
    meshes, ora = _oracle(name)
    print(f"[patch f32 {name}]", flush=True)
    kw = dict(degree=degree, tau=0.1, layers=layers, policy=policy, precision="mixed")
    g32 = Solver(meshes, patch_factor_f32=True, **kw)
    g64 = Solver(meshes, patch_factor_f32=False, **kw)
    i32, i64 = g32.level_info(0), g64.level_info(0)
    print(f"[patch f32 {name}] patches {i32['n_patches']} (max {i32['max_patch']} DOFs), "
          f"factored in FP32: {i32['patches_f32']}", flush=True)
    assert i64["patches_f32"] == 0
    assert 0 < i32["patches_f32"] <= i32["n_patches"]
    n = ora.levels[0].A.shape[0]
    b, u0 = meshgen.random_rhs(n, 31), meshgen.random_rhs(n, 32)
    out = []
    for g in (g32, g64):
        u = to_dev(u0)
        g.smooth(0, to_dev(b), u, 1)
        out.append(from_dev(u))
    d = rel_err(out[0], out[1])
    print(f"[patch f32 {name}] one smoother application: FP32- vs FP64-factored {d:.2e}", flush=True)
    assert d < 1e-3
    x_ref = ora.pcg(b, 1e-12, 300)[0]
    _, it_o, _, _ = ora.pcg(b, 1e-8, 300)
    for g in (g32, g64):
        u = to_dev(np.zeros(n))
        st = g.pcg(to_dev(b), u, 1e-8, 300)
        assert st["converged"] and abs(st["iterations"] - it_o) <= 1, (st["iterations"], it_o)
        assert rel_err(from_dev(u), x_ref) < 1e-6
        g.close()
