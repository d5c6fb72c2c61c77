"""Many-instance solve (mg_pcg_solve_batch): independent problems of uneven
size solved together, mixed precision with graph-captured V-cycles.  Each
system must equal the same context's single solve exactly (same kernels, same
order), and agree with the oracle's FP64 solution to 1e-6 with iterations +-1."""
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
