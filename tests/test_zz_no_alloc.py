"""The allocation-free V-cycle (mg_vcycle_noalloc) against mg_vcycle.

mg_vcycle_noalloc keeps its level-0 staging vectors in the library's static
device array and runs the same kernels on the same data as mg_vcycle, so the
two must agree bitwise (a stricter bar than the 1e-10 FP64 parity of the
cycle).  Two calls in a row on different contexts, the second with a smaller
level 0, then the larger one again (the array keeps the previous call's
contents, which must not matter); FP64 and mixed precision, eager and graph
contexts; the size limit; and one comparison with the oracle's cycle.
"""
import numpy as np
import pytest

import meshgen
import oracle
from tests.parity_util import from_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu

MAX_UNKNOWNS = 1048576  # MG_NOALLOC_MAX_UNKNOWNS


def _same_cycle(solver, seed):
    n = solver.n_free(0)
    b = to_dev(meshgen.random_rhs(n, seed))
    u0 = meshgen.random_rhs(n, seed + 1)
    u_ref, u_na = to_dev(u0), to_dev(u0)
    solver.vcycle(b, u_ref)
    solver.vcycle_noalloc(b, u_na)
    x_ref, x_na = from_dev(u_ref), from_dev(u_na)
    print(f"[noalloc] n={n} seed={seed} max|diff|={np.max(np.abs(x_na - x_ref)):.3e}", flush=True)
    assert np.array_equal(x_na, x_ref)
    return b, u0, x_na


@pytest.mark.parametrize("precision,graph", [("fp64", False), ("mixed", True)])
def test_noalloc_vcycle_equals_vcycle(precision, graph):
    from paper_2402_12947_amd import Solver
    big = Solver(meshgen.hierarchy("square_1025", seed=0, scale=16), degree=2, precision=precision,
                 use_graph=graph)
    small = Solver(meshgen.hierarchy("square_p1_4k", seed=0), degree=1, layers=2, precision=precision,
                   use_graph=graph)
    assert big.n_free(0) > small.n_free(0)
    _same_cycle(big, 11)
    _same_cycle(small, 13)   # second call, smaller input
    _same_cycle(big, 15)     # larger again over the smaller call's leftovers
    big.close()
    small.close()


def test_noalloc_vcycle_matches_oracle():
    from paper_2402_12947_amd import Solver
    meshes = meshgen.hierarchy("square_p1_4k", seed=0)
    gpu = Solver(meshes, degree=1, layers=2)
    ora = oracle.Hierarchy(meshes, tau=0.1, layers=2, opts=oracle.Options(degree=1))
    b, u0, x = _same_cycle(gpu, 17)
    assert rel_err(x, ora.vcycle(from_dev(b), u0.copy())) < 1e-10
    gpu.close()


def test_noalloc_vcycle_size_limit():
    from paper_2402_12947_amd import MG_ERR_LIMIT, MgError, Solver
    s = Solver(meshgen.hierarchy("square_1025", seed=0, scale=2), degree=3)
    n = s.n_free(0)
    assert n > MAX_UNKNOWNS
    b, u = to_dev(np.ones(n)), to_dev(np.zeros(n))
    with pytest.raises(MgError) as e:
        s.vcycle_noalloc(b, u)
    assert e.value.code == MG_ERR_LIMIT
    assert float(u.abs().max()) == 0.0   # rejected before any device work
    s.close()
