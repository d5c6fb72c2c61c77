"""Block solve of several right-hand sides (mg_pcg_solve_multi): the columns
run in blocks of 4 (a remainder of 3 padded with a zero column, 2 as a block
of two, 1 as a single-vector solve) with interleaved vectors.  Each column
must reproduce the single-vector mg_pcg_solve of the same context: the method
and the per-column scalars are the same, only the summation order of the FP64
row products differs in blocks of 4, so the bars are FP64 solutions within
1e-10 of the single solves and iterations within one (mixed: 1e-6, within
one); against the oracle the single-solve bars (iterations within one,
solution 1e-8).  A zero right-hand side gives u = 0 after 0 iterations;
graph replays of the block cycle reproduce the eager block cycle exactly."""
import functools

import numpy as np
import pytest

import meshgen
import oracle
from tests.parity_util import build_pair, from_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    # name: (workload, scale, degree, layers[, patch policy])
    "cube_p1": ("cube_129", 8, 1, 1),
    "square_p2": ("square_1025", 16, 2, 1),
    "cube_stress_p2": ("cube_129_stress", 8, 2, 0, "overlap"),
}


@functools.lru_cache(maxsize=None)
def solver(name, precision="fp64", use_graph=False, smoother="chebyshev"):
    wl, scale, degree, layers = CASES[name][:4]
    policy = CASES[name][4] if len(CASES[name]) > 4 else "merge"
    meshes = meshgen.hierarchy(wl, seed=0, scale=scale)
    print(f"[block {name} {precision} graph={use_graph} {smoother}]", flush=True)
    return build_pair(meshes, degree, layers=layers, precision=precision, policy=policy, use_graph=use_graph,
                      smoother=smoother, build_oracle=False)[0]


def _rhs(n, count, seed, zero=()):
    return [to_dev(np.zeros(n) if r in zero else meshgen.random_rhs(n, seed + r)) for r in range(count)]


def _check_against_single(gpu, bs, us, res, rtol, bar, zero=()):
    n = gpu.n_free(0)
    for r, b in enumerate(bs):
        st = res["stats"][r]
        if r in zero:
            assert st["converged"] and st["iterations"] == 0
            assert not np.any(from_dev(us[r]))
            continue
        u1 = to_dev(np.zeros(n))
        s1 = gpu.pcg(b, u1, rtol, 300)
        assert st["converged"] and s1["converged"], r
        assert abs(st["iterations"] - s1["iterations"]) <= 1, (r, st["iterations"], s1["iterations"])
        assert rel_err(from_dev(us[r]), from_dev(u1)) < bar, r
        assert st["true_rel_residual"] < 10 * rtol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_block_matches_single_solves(name, precision):
    gpu = solver(name, precision)
    n = gpu.n_free(0)
    # 7 columns: a block of 4 (one of them zero), a block of 2, one single
    zero = (2,)
    bs = _rhs(n, 7, 300, zero)
    us = [to_dev(np.zeros(n)) for _ in bs]
    rtol = 1e-10 if precision == "fp64" else 1e-8
    res = gpu.pcg_multi(bs, us, rtol, 300)
    assert res["status"] == 0
    _check_against_single(gpu, bs, us, res, rtol, 1e-10 if precision == "fp64" else 1e-6, zero)


def test_block_of_three_is_padded():
    gpu = solver("cube_p1")
    n = gpu.n_free(0)
    bs = _rhs(n, 3, 400)
    us = [to_dev(np.zeros(n)) for _ in bs]
    res = gpu.pcg_multi(bs, us, 1e-10, 300)
    assert res["status"] == 0 and len(res["stats"]) == 3
    _check_against_single(gpu, bs, us, res, 1e-10, 1e-10)


def test_block_against_oracle():
    wl, scale, degree, layers = CASES["square_p2"]
    meshes = meshgen.hierarchy(wl, seed=0, scale=scale)
    gpu = solver("square_p2")
    H = oracle.Hierarchy(meshes, tau=0.1, layers=layers, opts=oracle.Options(degree=degree))
    n = gpu.n_free(0)
    bs = _rhs(n, 4, 500)
    us = [to_dev(np.zeros(n)) for _ in bs]
    res = gpu.pcg_multi(bs, us, 1e-10, 200)
    for r in (0, 3):
        x_o, it_o, conv_o, _ = H.pcg(from_dev(bs[r]), 1e-10, 200)
        assert conv_o and res["stats"][r]["converged"]
        assert abs(res["stats"][r]["iterations"] - it_o) <= 1
        assert rel_err(from_dev(us[r]), x_o) < 1e-8


def test_block_graph_replay_matches_eager():
    eager = solver("cube_p1", "mixed")
    graph = solver("cube_p1", "mixed", use_graph=True)
    n = eager.n_free(0)
    for rep in range(3):
        bs = _rhs(n, 4 if rep != 1 else 2, 600 + 10 * rep)
        ue = [to_dev(np.zeros(n)) for _ in bs]
        ug = [to_dev(np.zeros(n)) for _ in bs]
        re = eager.pcg_multi(bs, ue, 1e-8, 300)
        rg = graph.pcg_multi(bs, ug, 1e-8, 300)
        for r in range(len(bs)):
            assert re["stats"][r]["iterations"] == rg["stats"][r]["iterations"]
            assert np.array_equal(from_dev(ue[r]), from_dev(ug[r]))


def test_block_with_gauss_seidel():
    gpu = solver("square_p2", smoother="sgs")
    n = gpu.n_free(0)
    bs = _rhs(n, 4, 700)
    us = [to_dev(np.zeros(n)) for _ in bs]
    res = gpu.pcg_multi(bs, us, 1e-10, 300)
    assert res["status"] == 0
    _check_against_single(gpu, bs, us, res, 1e-10, 1e-10)


def test_block_elasticity():
    from paper_2402_12947_amd import Solver
    meshes = meshgen.hierarchy("lattice", seed=0, scale=2)
    gpu = Solver(meshes, degree=1, tau=0.1, layers=1, problem="elasticity")
    n = gpu.n_free(0)
    bs = _rhs(n, 2, 800)
    us = [to_dev(np.zeros(n)) for _ in bs]
    res = gpu.pcg_multi(bs, us, 1e-10, 300)
    assert res["status"] == 0
    _check_against_single(gpu, bs, us, res, 1e-10, 1e-10)
    gpu.close()


def test_block_argument_errors():
    from paper_2402_12947_amd import MG_ERR_ARG, MgError
    gpu = solver("cube_p1")
    n = gpu.n_free(0)
    bs = _rhs(n, 2, 900)
    assert gpu.pcg_multi([], [])["status"] == 0
    with pytest.raises(MgError) as e:
        gpu.pcg_multi(bs, [bs[1], to_dev(np.zeros(n))])
    assert e.value.code == MG_ERR_ARG
    u = to_dev(np.zeros(n))
    with pytest.raises(MgError) as e:
        gpu.pcg_multi(bs, [u, u])
    assert e.value.code == MG_ERR_ARG
