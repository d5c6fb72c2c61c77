"""Many-instance solve (mg_pcg_solve_batch): independent problems of uneven
size solved together from one host thread, mixed precision with each CG
iteration replayed from a captured graph.  Each system must equal the same
context's own solve exactly (same kernels, same order), and agree with the
oracle's FP64 solution to 1e-6 with iterations +-1.  Also: right-hand side
counts that cut into a block of four and a single vector, graph and eager
contexts in one batch, and an instance whose arguments are wrong failing alone
while the others are solved."""
import numpy as np
import pytest

import meshgen
import oracle
from tests.parity_util import from_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu


def test_batch_equals_single_solves_and_oracle():
    from paper_2402_12947_amd import Solver, pcg_solve_batch
    inst = meshgen.instance_batch(3, seed=5, dof_range=(2e3, 2e4), sliver_range=(3, 20), coarsest_dofs=600)
    solvers = [Solver(m, degree=d, precision="mixed", use_graph=True) for m, d in inst]
    nrhs = 2
    bs = [[to_dev(meshgen.random_rhs(s.n_free(0), 10 * i + r)) for r in range(nrhs)] for i, s in enumerate(solvers)]
    us = [[to_dev(np.zeros(s.n_free(0))) for _ in range(nrhs)] for s in solvers]
    res = pcg_solve_batch(solvers, bs, us, 1e-8, 300)
    assert res["status"] == 0 and all(x["converged"] for x in res["stats"])
    for i, s in enumerate(solvers):
        for r in range(nrhs):
            u1 = to_dev(np.zeros(s.n_free(0)))
            st = s.pcg(bs[i][r], u1, 1e-8, 300)
            assert st["iterations"] == res["stats"][i * nrhs + r]["iterations"]
            assert np.array_equal(from_dev(u1), from_dev(us[i][r]))
    meshes, degree = inst[0]
    H = oracle.Hierarchy(meshes, tau=0.1, layers=1, opts=oracle.Options(degree=degree))
    b = from_dev(bs[0][0])
    x_ref, _, _, _ = H.pcg(b, 1e-12, 300)
    _, it_o, _, _ = H.pcg(b, 1e-8, 300)
    assert abs(res["stats"][0]["iterations"] - it_o) <= 1
    assert rel_err(from_dev(us[0][0]), x_ref) < 1e-6
    for s in solvers:
        s.close()


def test_batch_rejects_repeated_context():
    from paper_2402_12947_amd import MG_ERR_ARG, MgError, Solver, pcg_solve_batch
    s = Solver(meshgen.hierarchy("square_p1_4k"), degree=1)
    b = to_dev(meshgen.random_rhs(s.n_free(0), 0))
    with pytest.raises(MgError) as e:
        pcg_solve_batch([s, s], [[b], [b]], [[to_dev(np.zeros(s.n_free(0)))], [to_dev(np.zeros(s.n_free(0)))]])
    assert e.value.code == MG_ERR_ARG
    s.close()


def _instances(count, seed):
    return meshgen.instance_batch(count, seed=seed, dof_range=(2e3, 2e4), sliver_range=(3, 20), coarsest_dofs=600)


def test_batch_mixed_runs_equal_own_solves():
    from paper_2402_12947_amd import Solver, pcg_solve_batch
    inst = _instances(3, 7)
    kinds = [("mixed", True), ("fp64", False), ("mixed", False)]
    solvers = [Solver(m, degree=d, precision=p, use_graph=g) for (m, d), (p, g) in zip(inst, kinds)]
    for nrhs in (5, 3, 1):
        print(f"[batch nrhs={nrhs}]", flush=True)
        bs = [[to_dev(meshgen.random_rhs(s.n_free(0), 100 * i + r)) for r in range(nrhs)]
              for i, s in enumerate(solvers)]
        us = [[to_dev(np.zeros(s.n_free(0))) for _ in range(nrhs)] for s in solvers]
        res = pcg_solve_batch(solvers, bs, us, 1e-8, 300)
        assert res["status"] == 0
        for i, s in enumerate(solvers):
            own = [to_dev(np.zeros(s.n_free(0))) for _ in range(nrhs)]
            ro = s.pcg_multi(bs[i], own, 1e-8, 300)
            for r in range(nrhs):
                got = res["stats"][i * nrhs + r]
                assert got["converged"] and got["iterations"] == ro["stats"][r]["iterations"]
                assert got["true_rel_residual"] == ro["stats"][r]["true_rel_residual"]
                assert np.array_equal(from_dev(us[i][r]), from_dev(own[r]))
    for s in solvers:
        s.close()


def test_batch_failing_instance_leaves_the_others():
    from paper_2402_12947_amd import MG_ERR_ARG, MgError, Solver, pcg_solve_batch
    inst = _instances(2, 9)
    solvers = [Solver(m, degree=d, precision="mixed", use_graph=True) for m, d in inst]
    n0, n1 = solvers[0].n_free(0), solvers[1].n_free(0)
    b0 = [to_dev(meshgen.random_rhs(n0, 1)), to_dev(meshgen.random_rhs(n0, 2))]
    b1 = [to_dev(meshgen.random_rhs(n1, 3)), to_dev(meshgen.random_rhs(n1, 4))]
    u0 = [to_dev(np.zeros(n0)) for _ in range(2)]
    u1 = [b1[0], to_dev(np.zeros(n1))]  # instance 1: a solution aliases a right-hand side
    with pytest.raises(MgError) as e:
        pcg_solve_batch(solvers, [b0, b1], [u0, u1], 1e-8, 300)
    assert e.value.code == MG_ERR_ARG
    own = [to_dev(np.zeros(n0)) for _ in range(2)]
    solvers[0].pcg_multi(b0, own, 1e-8, 300)
    for r in range(2):
        assert np.array_equal(from_dev(u0[r]), from_dev(own[r]))
    for s in solvers:
        s.close()
