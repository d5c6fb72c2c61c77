"""The many-instance solve at full size: 32 unit cubes of 50k-3M DOFs (P1 and
P2, 18.1M DOFs in total), 4 right-hand sides each, mixed precision with
captured CG iterations, all solved together by mg_pcg_solve_batch.

Checks: every system converged with a true residual near the tolerance and
6-8 iterations; every instance's solutions bitwise equal to the same
context's own block solve of its 4 right-hand sides (the batch changes only
the order in which the host drives the contexts); and the smallest instance
against the oracle (iterations +-1 of the oracle's FP64 PCG, solution within
1e-6 of the oracle's converged solution).
"""
import numpy as np
import pytest

import meshgen
import oracle
from tests.parity_util import from_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu


def test_full_size_batch():
    from paper_2402_12947_amd import Solver, pcg_solve_batch
    print("[batch full] generating 32 instances", flush=True)
    inst = meshgen.instance_batch(32, seed=0)
    solvers = []
    for i, (m, d) in enumerate(inst):
        solvers.append(Solver(m, degree=d, precision="mixed", use_graph=True))
    ns = [s.n_free(0) for s in solvers]
    print(f"[batch full] {sum(ns)} DOFs set up", flush=True)
    assert len(ns) == 32 and 1.7e7 < sum(ns) < 2.0e7
    nrhs = 4
    bs = [[to_dev(meshgen.random_rhs(n, 100 * i + r)) for r in range(nrhs)] for i, n in enumerate(ns)]
    us = [[to_dev(np.zeros(n)) for _ in range(nrhs)] for n in ns]
    res = pcg_solve_batch(solvers, bs, us, 1e-8, 300)
    assert res["status"] == 0
    its = [x["iterations"] for x in res["stats"]]
    print(f"[batch full] iterations {min(its)}..{max(its)}, {res['wall_ms']:.1f} ms", flush=True)
    assert all(x["converged"] for x in res["stats"]) and 5 <= min(its) and max(its) <= 9
    assert max(x["true_rel_residual"] for x in res["stats"]) < 2e-8
    for i, s in enumerate(solvers):
        own = [to_dev(np.zeros(ns[i])) for _ in range(nrhs)]
        ro = s.pcg_multi(bs[i], own, 1e-8, 300)
        for r in range(nrhs):
            assert res["stats"][i * nrhs + r]["iterations"] == ro["stats"][r]["iterations"]
            assert np.array_equal(from_dev(us[i][r]), from_dev(own[r])), (i, r)
    k = int(np.argmin(ns))
    print(f"[batch full] oracle on instance {k} ({ns[k]} DOFs, P{inst[k][1]})", flush=True)
    H = oracle.Hierarchy(inst[k][0], tau=0.1, layers=1, opts=oracle.Options(degree=inst[k][1]))
    for r in range(2):
        b = from_dev(bs[k][r])
        x_ref = H.pcg(b, 1e-12, 300)[0]
        _, it_o, conv_o, _ = H.pcg(b, 1e-8, 300)
        assert conv_o and abs(res["stats"][k * nrhs + r]["iterations"] - it_o) <= 1
        assert rel_err(from_dev(us[k][r]), x_ref) < 1e-6
    for s in solvers:
        s.close()
