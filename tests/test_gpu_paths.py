"""GPU parity of the paths that the default cases do not reach.

* The plain global smoother (no local correction, unadjusted lambda_max:
  paper Sec. 3.2 and Sec. 5, the "plain" arm of the Sec. 6 comparisons).  Its
  V-cycle starts every level with a first Chebyshev step that reads no u.
* The coloured local correction: OVERLAP patches whose grown sets share DOFs
  need several colours; the first S_c of a sandwich visits them ascending, the
  second descending (Sec. 4.1, eq. local_update and Algorithm alg:local,
  applied additively within a colour).
* The load b = M f_hat (Sec. 2, eq. system_finest; the nodal interpolant of f
  times the consistent mass matrix).
* Warm starts of CG and of the stationary multigrid solver.

Bars as in test_gpu_parity: bit-exact indexing, 1e-10 for one smoother
application and one V-cycle, PCG iterations +-1 with the solution within 1e-8,
mixed precision within 1e-6 of the FP64 oracle solution; b = M f_hat 1e-12.
"""
import functools

import numpy as np
import pytest

import meshgen
import oracle
from tests.parity_util import build_pair, from_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu

PLAIN = {
    "square_p1_4k": ("square_p1_4k", 1, 1, 2),
    "square_p2": ("square_1025", 16, 2, 1),
    "cube_p2": ("cube_129", 16, 2, 1),
}

# OVERLAP hierarchies whose patches need several colours (counts from the
# oracle's greedy colouring: 4, 2 and 7)
COLOURED = {
    "square_p2_overlap": ("square_1025", 16, 2, 1),
    "cube_p1_overlap": ("cube_129", 4, 1, 1),
    # the patch stress recipe grown by one layer: 54 patches of 226-2795 DOFs
    # (the largest beyond the one-workgroup factorisation)
    "cube_stress_overlap": ("cube_129_stress", 8, 2, 1),
}


@functools.lru_cache(maxsize=None)
def plain_pair(name):
    wl, scale, degree, layers = PLAIN[name]
    meshes = meshgen.hierarchy(wl, seed=0, scale=scale)
    print(f"[plain {name}] levels={[m['cells'].shape[0] for m in meshes]}", flush=True)
    return build_pair(meshes, degree, layers=layers, local=False, adjusted=False)


@functools.lru_cache(maxsize=None)
def coloured_pair(name, precision="fp64"):
    wl, scale, degree, layers = COLOURED[name]
    meshes = meshgen.hierarchy(wl, seed=0, scale=scale)
    print(f"[overlap {name} {precision}] levels={[m['cells'].shape[0] for m in meshes]}", flush=True)
    return build_pair(meshes, degree, layers=layers, policy="overlap", precision=precision,
                      build_oracle=precision == "fp64")


def _smooth_and_cycle(gpu, ora, seed):
    n = ora.levels[0].A.shape[0]
    b, u0 = meshgen.random_rhs(n, seed), meshgen.random_rhs(n, seed + 1)
    u = to_dev(u0)
    gpu.smooth(0, to_dev(b), u, 1)
    assert rel_err(from_dev(u), ora.smooth(0, b, u0.copy(), 1)) < 1e-10
    u = to_dev(u0)
    gpu.vcycle(to_dev(b), u)
    assert rel_err(from_dev(u), ora.vcycle(b, u0.copy())) < 1e-10
    # the cycle from zero (the preconditioner's form: every level starts at 0)
    u = to_dev(np.zeros(n))
    gpu.vcycle(to_dev(b), u)
    assert rel_err(from_dev(u), ora.vcycle(b, None)) < 1e-10


def _pcg(gpu, ora, seed, rtol=1e-10):
    n = ora.levels[0].A.shape[0]
    b = meshgen.random_rhs(n, seed)
    x_o, it_o, conv_o, _ = ora.pcg(b, rtol, 300)
    u = to_dev(np.zeros(n))
    st = gpu.pcg(to_dev(b), u, rtol, 300)
    assert conv_o and st["converged"]
    assert abs(st["iterations"] - it_o) <= 1, (st["iterations"], it_o)
    assert rel_err(from_dev(u), x_o) < 1e-8


@pytest.mark.parametrize("name", list(PLAIN))
def test_plain_smoother_arm(name):
    gpu, ora = plain_pair(name)
    for l in range(len(ora.levels) - 1):
        info = gpu.level_info(l)
        assert info["cheb_hi"] == pytest.approx(ora.levels[l].lam, rel=1e-7)
    _smooth_and_cycle(gpu, ora, 21)
    _pcg(gpu, ora, 23)


@pytest.mark.parametrize("name", list(COLOURED))
def test_coloured_local_correction(name):
    gpu, ora = coloured_pair(name)
    lev = ora.levels[0]
    info = gpu.level_info(0)
    assert info["n_colours"] >= 2 and info["n_colours"] == int(lev.colours.max()) + 1
    ptr, dofs = gpu.get_array(0, "patch_ptr"), gpu.get_array(0, "patch_dofs")
    assert len(ptr) - 1 == len(lev.patch_dofs)
    for d, B in enumerate(lev.patch_dofs):
        assert np.array_equal(dofs[ptr[d]:ptr[d + 1]], B)
    assert np.array_equal(gpu.get_array(0, "patch_colour"), lev.colours)
    _smooth_and_cycle(gpu, ora, 31)
    _pcg(gpu, ora, 33)


@pytest.mark.parametrize("name", list(COLOURED))
def test_coloured_local_correction_mixed(name):
    _, ora = coloured_pair(name)
    gmix, _ = coloured_pair(name, "mixed")
    n = ora.levels[0].A.shape[0]
    b = meshgen.random_rhs(n, 35)
    x_ref, _, _, _ = ora.pcg(b, 1e-12, 300)
    _, it_o, _, _ = ora.pcg(b, 1e-8, 300)
    u = to_dev(np.zeros(n))
    st = gmix.pcg(to_dev(b), u, 1e-8, 300)
    assert st["converged"] and abs(st["iterations"] - it_o) <= 1
    assert rel_err(from_dev(u), x_ref) < 1e-6


@pytest.mark.parametrize("wl,scale,degree", [("square_1025", 16, 1), ("square_1025", 16, 2), ("square_1025", 16, 3),
                                             ("cube_129", 16, 1), ("cube_129", 16, 2)])
def test_rhs_from_nodal(wl, scale, degree):
    from paper_2402_12947_amd import Solver
    meshes = meshgen.hierarchy(wl, seed=0, scale=scale)
    gpu = Solver(meshes, degree=degree)
    dm, _, Mf = oracle.assemble(meshes[0], degree)
    f = meshgen.random_rhs(dm.nodes.shape[0], 41)
    want = Mf @ f
    b = to_dev(np.zeros(Mf.shape[0]))
    gpu.rhs_from_nodal(to_dev(f), b)
    assert rel_err(from_dev(b), want) < 1e-12
    # smooth nodal data (the paper's cube load) as well
    x = dm.nodes
    fs = 10.0 * np.exp(-((x - 0.5) ** 2).sum(axis=1) / 0.02)
    gpu.rhs_from_nodal(to_dev(fs), b)
    assert rel_err(from_dev(b), Mf @ fs) < 1e-12
    gpu.close()


@functools.lru_cache(maxsize=None)
def warm_pair():
    meshes = meshgen.hierarchy("square_1025", seed=0, scale=16)
    gpu, ora = build_pair(meshes, 2, layers=1, use_initial_guess=True)
    return meshes, gpu, ora


def test_warm_start_pcg():
    meshes, gpu, ora = warm_pair()
    n = ora.levels[0].A.shape[0]
    b, x0 = meshgen.random_rhs(n, 51), meshgen.random_rhs(n, 52)
    x_o, it_o, conv_o, hist_o = ora.pcg(b, 1e-10, 200, x0=x0)
    u = to_dev(x0)
    st = gpu.pcg(to_dev(b), u, 1e-10, 200)
    assert conv_o and st["converged"] and abs(st["iterations"] - it_o) <= 1
    assert st["history"][0] == pytest.approx(hist_o[0], rel=1e-12)
    assert rel_err(from_dev(u), x_o) < 1e-8
    # a start that already meets the tolerance: no iteration, u unchanged
    x1 = from_dev(u).copy()
    st = gpu.pcg(to_dev(b), u, 1e-6, 200)
    assert st["iterations"] == 0 and st["converged"] and np.array_equal(from_dev(u), x1)
    # b = 0 gives u = 0 whatever the start
    z = to_dev(x0)
    st = gpu.pcg(to_dev(np.zeros(n)), z, 1e-8, 10)
    assert st["iterations"] == 0 and float(z.abs().max()) == 0.0


def test_warm_start_stationary():
    meshes, gpu, ora = warm_pair()
    n = ora.levels[0].A.shape[0]
    b, x0 = meshgen.random_rhs(n, 53), meshgen.random_rhs(n, 54)
    x_o, _, _, hist_o = ora.mg_solve(b, 1e-300, 12, x0=x0)
    u = to_dev(x0)
    st = gpu.mg_solve(to_dev(b), u, 1e-300, 12)
    assert st["iterations"] == 12
    assert rel_err(from_dev(u), x_o) < 1e-9
    assert np.allclose(st["history"], hist_o, rtol=1e-6, atol=1e-12)
    _, it_o, conv_o, _ = ora.mg_solve(b, 1e-8, 200, x0=x0)
    st = gpu.mg_solve(to_dev(b), to_dev(x0), 1e-8, 200)
    assert conv_o and st["converged"] and abs(st["iterations"] - it_o) <= 1


def test_warm_start_block_solves():
    """Block solves from given starts equal the single-vector warm solves."""
    meshes, gpu, ora = warm_pair()
    n = ora.levels[0].A.shape[0]
    for nrhs in (2, 3, 4):
        bs = [to_dev(meshgen.random_rhs(n, 60 + r)) for r in range(nrhs)]
        x0 = [meshgen.random_rhs(n, 70 + r) for r in range(nrhs)]
        us = [to_dev(x) for x in x0]
        res = gpu.pcg_multi(bs, us, 1e-10, 200)
        for r in range(nrhs):
            x_o, it_o, _, _ = ora.pcg(from_dev(bs[r]), 1e-10, 200, x0=x0[r])
            st = res["stats"][r]
            assert st["converged"] and abs(st["iterations"] - it_o) <= 1
            assert rel_err(from_dev(us[r]), x_o) < 1e-8
