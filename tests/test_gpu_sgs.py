"""GPU parity of symmetric Gauss-Seidel as the global smoother (the paper's
SGS experiments, Sec. 3.2 and Sec. 6.1, in multicolour form): the greedy
colouring of every level bit-exact against the oracle's, one sandwich and one
V-cycle within 1e-10 (FP64), PCG iterations and stationary cycles within one,
mixed precision within 1e-6 of the converged FP64 solution."""
import functools

import numpy as np
import pytest

import meshgen
from tests.parity_util import build_pair, from_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    # name: (workload, scale, degree, layers)
    "square_p1_4k": ("square_p1_4k", 1, 1, 2),
    "square_p2": ("square_1025", 16, 2, 1),
    "cube_p1": ("cube_129", 8, 1, 1),
}


@functools.lru_cache(maxsize=None)
def pair(name, precision="fp64"):
    wl, scale, degree, layers = CASES[name]
    meshes = meshgen.hierarchy(wl, seed=0, scale=scale)
    print(f"[sgs {name} {precision}]", flush=True)
    return build_pair(meshes, degree, layers=layers, precision=precision, smoother="sgs",
                      build_oracle=precision == "fp64")


@pytest.mark.parametrize("name", list(CASES))
def test_colouring_bit_exact(name):
    gpu, ora = pair(name)
    for l, lev in enumerate(ora.levels[:-1]):
        assert np.array_equal(gpu.get_array(l, "sgs_colour"), lev.sgs.colours)


@pytest.mark.parametrize("name", list(CASES))
def test_smoother_vcycle(name):
    gpu, ora = pair(name)
    n = ora.levels[0].A.shape[0]
    b, u0 = meshgen.random_rhs(n, 1), meshgen.random_rhs(n, 2)
    u = to_dev(u0)
    gpu.smooth(0, to_dev(b), u, 1)
    assert rel_err(from_dev(u), ora.smooth(0, b, u0.copy(), 1)) < 1e-10
    u = to_dev(u0)
    gpu.vcycle(to_dev(b), u)
    assert rel_err(from_dev(u), ora.vcycle(b, u0.copy())) < 1e-10


@pytest.mark.parametrize("name", list(CASES))
def test_pcg_and_stationary(name):
    gpu, ora = pair(name)
    n = ora.levels[0].A.shape[0]
    b = meshgen.random_rhs(n, 5)
    x_o, it_o, conv_o, _ = ora.pcg(b, 1e-10, 200)
    u = to_dev(np.zeros(n))
    st = gpu.pcg(to_dev(b), u, 1e-10, 200)
    assert conv_o and st["converged"] and abs(st["iterations"] - it_o) <= 1
    assert rel_err(from_dev(u), x_o) < 1e-8
    _, c_o, cc_o, _ = ora.mg_solve(b, 1e-8, 300)
    st = gpu.mg_solve(to_dev(b), to_dev(np.zeros(n)), 1e-8, 300)
    assert cc_o and st["converged"] and abs(st["iterations"] - c_o) <= 1


@pytest.mark.parametrize("name", ["square_p2", "cube_p1"])
def test_mixed_precision(name):
    _, ora = pair(name)
    gmix, _ = pair(name, "mixed")
    n = ora.levels[0].A.shape[0]
    b = meshgen.random_rhs(n, 6)
    x_ref, _, _, _ = ora.pcg(b, 1e-12, 300)
    _, it_o, _, _ = ora.pcg(b, 1e-8, 300)
    u = to_dev(np.zeros(n))
    st = gmix.pcg(to_dev(b), u, 1e-8, 300)
    assert st["converged"] and abs(st["iterations"] - it_o) <= 1
    assert rel_err(from_dev(u), x_ref) < 1e-6
