"""Edge cases of the CG driver (single vector, blocks, many instances), with
host launches and with the captured CG iteration: a right-hand side holding a
NaN ends in MG_ERR_BREAKDOWN (so does the stationary solver) and leaves the
context usable; in a batch the broken instance fails alone; maxit = 0
returns the start after 0 iterations with MG_NOT_CONVERGED; b = 0 returns
u = 0 after 0 iterations."""
import functools

import numpy as np
import pytest

import meshgen
from tests.parity_util import from_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _solver(graph, k=0):
    from paper_2402_12947_amd import Solver
    print(f"[cg edges] square_p1_4k graph={graph} #{k}", flush=True)
    return Solver(meshgen.hierarchy("square_p1_4k"), degree=1, layers=2, use_graph=graph)


def _nan_rhs(n, seed):
    b = meshgen.random_rhs(n, seed)
    b[n // 3] = np.nan
    return b


@pytest.mark.parametrize("graph", [False, True])
def test_nan_rhs_breaks_down_and_context_recovers(graph):
    from paper_2402_12947_amd import MG_ERR_BREAKDOWN, MgError
    s = _solver(graph)
    n = s.n_free(0)
    with pytest.raises(MgError) as e:
        s.pcg(to_dev(_nan_rhs(n, 1)), to_dev(np.zeros(n)), 1e-10, 100)
    assert e.value.code == MG_ERR_BREAKDOWN and "breakdown" in str(e.value)
    with pytest.raises(MgError) as e:
        s.pcg_multi([to_dev(meshgen.random_rhs(n, 2)), to_dev(_nan_rhs(n, 3))],
                    [to_dev(np.zeros(n)), to_dev(np.zeros(n))], 1e-10, 100)
    assert e.value.code == MG_ERR_BREAKDOWN
    with pytest.raises(MgError) as e:
        s.mg_solve(to_dev(_nan_rhs(n, 11)), to_dev(np.zeros(n)), 1e-8, 20)
    assert e.value.code == MG_ERR_BREAKDOWN
    # a valid solve afterwards: the same as on a fresh context
    b = to_dev(meshgen.random_rhs(n, 4))
    u = to_dev(np.zeros(n))
    st = s.pcg(b, u, 1e-10, 100)
    fresh = _solver(graph, 1)
    v = to_dev(np.zeros(n))
    st2 = fresh.pcg(b, v, 1e-10, 100)
    assert st["converged"] and st["iterations"] == st2["iterations"]
    assert np.array_equal(from_dev(u), from_dev(v))


@pytest.mark.parametrize("graph", [False, True])
def test_maxit_zero_and_zero_rhs(graph):
    from paper_2402_12947_amd import MG_NOT_CONVERGED, MG_OK
    s = _solver(graph)
    n = s.n_free(0)
    b = to_dev(meshgen.random_rhs(n, 5))
    u = to_dev(meshgen.random_rhs(n, 6))
    st = s.pcg(b, u, 1e-10, 0)
    assert st["status"] == MG_NOT_CONVERGED and st["iterations"] == 0 and not st["converged"]
    assert np.all(from_dev(u) == 0.0)  # cold start: u = 0 whatever it held
    res = s.pcg_multi([b, to_dev(np.zeros(n))], [to_dev(np.ones(n)), to_dev(np.ones(n))], 1e-10, 100)
    assert res["status"] == MG_OK
    assert res["stats"][1]["iterations"] == 0 and res["stats"][1]["converged"]
    zero = to_dev(np.ones(n))
    st = s.pcg(to_dev(np.zeros(n)), zero, 1e-10, 100)
    assert st["status"] == MG_OK and st["iterations"] == 0 and np.all(from_dev(zero) == 0.0)


def test_batch_breakdown_fails_alone():
    from paper_2402_12947_amd import MG_ERR_BREAKDOWN, MgError, pcg_solve_batch
    a, c = _solver(True), _solver(False)
    n = a.n_free(0)
    ba = [to_dev(meshgen.random_rhs(n, 7)), to_dev(meshgen.random_rhs(n, 8))]
    bc = [to_dev(meshgen.random_rhs(n, 9)), to_dev(_nan_rhs(n, 10))]
    ua = [to_dev(np.zeros(n)) for _ in range(2)]
    uc = [to_dev(np.zeros(n)) for _ in range(2)]
    with pytest.raises(MgError) as e:
        pcg_solve_batch([a, c], [ba, bc], [ua, uc], 1e-10, 100)
    assert e.value.code == MG_ERR_BREAKDOWN
    own = [to_dev(np.zeros(n)) for _ in range(2)]
    a.pcg_multi(ba, own, 1e-10, 100)
    for r in range(2):
        assert np.array_equal(from_dev(ua[r]), from_dev(own[r]))
        assert rel_err(from_dev(ua[r]), from_dev(own[r])) == 0.0
