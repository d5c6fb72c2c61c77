"""Every column form of the sparse layouts against the oracle.

The SELL layouts store a slice's column indices in the narrowest form that
fits: 16-bit in two windows of 32768 columns, in eight windows of 8192 or in
sixteen of 4096 (decoded with a cross-lane read of the window table), else
32-bit.  The small parity cases fit the two-window form everywhere, so the
option sell_colform forces the wider forms (every slice of these sizes fits
each of them) on every sparse product of the cycle: level operators, transfers,
patch rows and the split first step.  Bars as in test_gpu_parity: one V-cycle
1e-10, PCG iterations +-1 with the solution within 1e-8 (FP64) / 1e-6 of the
oracle's solution (mixed).
"""
import functools

import numpy as np
import pytest

import meshgen
import oracle
from tests.parity_util import from_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    # name: (workload, scale, degree, layers)
    "square_p2": ("square_1025", 16, 2, 1),
    "cube_p2": ("cube_129", 16, 2, 1),
}
FORMS = {1: "sell_slices_multiwindow", 2: "sell_slices_16window", 3: "sell_slices_32bit"}


@functools.lru_cache(maxsize=None)
def _oracle(name):
    wl, scale, degree, layers = CASES[name]
    meshes = meshgen.hierarchy(wl, seed=0, scale=scale)
    return meshes, oracle.Hierarchy(meshes, tau=0.1, layers=layers, opts=oracle.Options(degree=degree))


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("name", list(CASES))
def test_forced_column_form(name, form):
    from paper_2402_12947_amd import Solver
    wl, scale, degree, layers = CASES[name]
    meshes, ora = _oracle(name)
    print(f"[colform {name} form={form}]", flush=True)
    gpu = Solver(meshes, degree=degree, layers=layers, sell_colform=form)
    for l in range(gpu.n_levels):
        info = gpu.level_info(l)
        assert info["sell_slices"] > 0
        assert info[FORMS[form]] == info["sell_slices"], (l, info[FORMS[form]], info["sell_slices"])
        if form == 3:
            assert info["sell_nnz16"] == 0
    n = ora.levels[0].A.shape[0]
    b, u0 = meshgen.random_rhs(n, 21), meshgen.random_rhs(n, 22)
    u = to_dev(u0)
    gpu.vcycle(to_dev(b), u)
    assert rel_err(from_dev(u), ora.vcycle(b, u0.copy())) < 1e-10
    x_o, it_o, _, _ = ora.pcg(b, 1e-10, 300)
    u = to_dev(np.zeros(n))
    st = gpu.pcg(to_dev(b), u, 1e-10, 300)
    assert st["converged"] and abs(st["iterations"] - it_o) <= 1
    assert rel_err(from_dev(u), x_o) < 1e-8
    gpu.close()
    # the FP32 copies of the same layouts
    mix = Solver(meshes, degree=degree, layers=layers, precision="mixed", sell_colform=form)
    assert mix.level_info(0)[FORMS[form]] == mix.level_info(0)["sell_slices"]
    x_ref = ora.pcg(b, 1e-12, 300)[0]
    _, it8, _, _ = ora.pcg(b, 1e-8, 300)
    u = to_dev(np.zeros(n))
    st = mix.pcg(to_dev(b), u, 1e-8, 300)
    assert st["converged"] and abs(st["iterations"] - it8) <= 1
    assert rel_err(from_dev(u), x_ref) < 1e-6
    mix.close()
