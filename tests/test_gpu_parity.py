"""GPU parity: the HIP library (through its C ABI) against the oracle, stage by
stage, on seeded synthetic hierarchies shaped like the paper's workloads.

Bars: bit-exact for indexing (flags, DOF maps, patch membership, colours,
point location); FP64 values within 1e-12 relative for assembled, transfer and
Galerkin operators; lambda_max within 1e-7; one smoother application and one
V-cycle within 1e-10 relative (patch solves amplify rounding by the patch
condition number, so this is the FP64 bar); PCG iterations within +-1 and the
solution within 1e-8; mixed precision within 1e-6 of the FP64 oracle solution
with iterations within +-1.
"""
import functools

import numpy as np
import pytest

import meshgen
from tests.parity_util import build_pair, from_dev, rel_err, sparse_close, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    # name: (workload, scale, degree, layers[, patch policy])
    "square_p1_4k": ("square_p1_4k", 1, 1, 2),
    "square_p2": ("square_1025", 16, 2, 1),
    "square_p3": ("square_1025", 32, 3, 1),
    "cube_p1": ("cube_129", 8, 1, 1),
    "cube_p2": ("cube_129", 16, 2, 1),
    # patch stress at 1/8 size: 54 separate flattened regions, patches of
    # 27-1587 DOFs (one to fifty 32x32 tiles per side in the batched factorisation)
    "cube_stress_p2": ("cube_129_stress", 8, 2, 0, "overlap"),
    # 1/8 of the 1025^2 P3 square: most level-0 slices need the eight-window
    # form of the 16-bit column indices
    "square_p3_s8": ("square_1025", 8, 3, 1),
}


@functools.lru_cache(maxsize=None)
def pair(name, precision="fp64"):
    wl, scale, degree, layers = CASES[name][:4]
    policy = CASES[name][4] if len(CASES[name]) > 4 else "merge"
    meshes = meshgen.hierarchy(wl, seed=0, scale=scale)
    print(f"[case {name} {precision}] levels={[m['cells'].shape[0] for m in meshes]}", flush=True)
    gpu, ora = build_pair(meshes, degree, layers=layers, precision=precision, policy=policy)
    return meshes, gpu, ora


@pytest.mark.parametrize("name", list(CASES))
def test_indexing_bit_exact(name):
    meshes, gpu, ora = pair(name)
    for l, lev in enumerate(ora.levels):
        g = gpu.get_array(l, "quality")
        assert rel_err(g, lev.gamma) < 1e-9
        assert np.array_equal(gpu.get_array(l, "flags").astype(bool), lev.gamma < 0.1)
        assert np.array_equal(gpu.get_array(l, "cell_dofs"), lev.dofmap.cell_dofs)
        assert np.array_equal(gpu.get_array(l, "free_dofs"), lev.dofmap.free)
        assert np.max(np.abs(gpu.get_array(l, "dof_nodes") - lev.dofmap.nodes)) < 1e-15
        if l < len(ora.levels) - 1:
            assert np.array_equal(gpu.get_array(l, "locate"), lev.locate_cell)
            ptr = gpu.get_array(l, "patch_ptr")
            dofs = gpu.get_array(l, "patch_dofs")
            assert len(ptr) - 1 == len(lev.patch_dofs)
            for d, B in enumerate(lev.patch_dofs):
                assert np.array_equal(dofs[ptr[d]:ptr[d + 1]], B)
            assert np.array_equal(gpu.get_array(l, "patch_colour"), lev.colours)


@pytest.mark.parametrize("name", list(CASES))
def test_operators(name):
    meshes, gpu, ora = pair(name)
    for l, lev in enumerate(ora.levels):
        A = gpu.matrix(l)
        tol = 1e-12 if l == 0 else 1e-11
        assert sparse_close(A, lev.A, tol), f"A_{l}"
        if l < len(ora.levels) - 1:
            assert sparse_close(gpu.prolongation(l), lev.P, 1e-12), f"P_{l}"


@pytest.mark.parametrize("name", list(CASES))
def test_eigenvalues(name):
    meshes, gpu, ora = pair(name)
    for l, lev in enumerate(ora.levels[:-1]):
        info = gpu.level_info(l)
        assert abs(info["lambda_max"] - lev.lam) <= 1e-7 * lev.lam
        assert abs(info["lambda_adj"] - lev.lam_adj) <= 1e-7 * lev.lam_adj
        assert abs(info["cheb_hi"] - lev.hi) <= 1e-7 * lev.hi


@pytest.mark.parametrize("name", list(CASES))
def test_smoother_and_vcycle(name):
    meshes, gpu, ora = pair(name)
    n = ora.levels[0].A.shape[0]
    b = meshgen.random_rhs(n, 1)
    u0 = meshgen.random_rhs(n, 2)
    u = to_dev(u0)
    gpu.smooth(0, to_dev(b), u, 1)
    want = ora.smooth(0, b, u0.copy(), 1)
    assert rel_err(from_dev(u), want) < 1e-10
    u = to_dev(u0)
    gpu.vcycle(to_dev(b), u)
    want = ora.vcycle(b, u0.copy())
    assert rel_err(from_dev(u), want) < 1e-10
    # coarse level smoother
    if len(ora.levels) > 2:
        n1 = ora.levels[1].A.shape[0]
        b1, v1 = meshgen.random_rhs(n1, 3), meshgen.random_rhs(n1, 4)
        v = to_dev(v1)
        gpu.smooth(1, to_dev(b1), v, 2)
        assert rel_err(from_dev(v), ora.smooth(1, b1, v1.copy(), 2)) < 1e-10


@pytest.mark.parametrize("name", list(CASES))
def test_pcg_fp64(name):
    meshes, gpu, ora = pair(name)
    n = ora.levels[0].A.shape[0]
    b = meshgen.random_rhs(n, 5)
    rtol = 1e-10
    x_o, it_o, conv_o, _ = ora.pcg(b, rtol, 200)
    u = to_dev(np.zeros(n))
    st = gpu.pcg(to_dev(b), u, rtol, 200)
    assert conv_o and st["converged"]
    assert abs(st["iterations"] - it_o) <= 1
    assert rel_err(from_dev(u), x_o) < 1e-8
    assert st["true_rel_residual"] < 10 * rtol


@pytest.mark.parametrize("name", ["square_p1_4k", "square_p2", "cube_p2", "cube_stress_p2"])
def test_pcg_mixed_precision(name):
    meshes, gpu, ora = pair(name)
    _, gmix, _ = pair(name, "mixed")
    n = ora.levels[0].A.shape[0]
    b = meshgen.random_rhs(n, 6)
    rtol = 1e-8
    x_ref, _, _, _ = ora.pcg(b, 1e-12, 300)
    _, it_o, _, _ = ora.pcg(b, rtol, 300)
    u = to_dev(np.zeros(n))
    st = gmix.pcg(to_dev(b), u, rtol, 300)
    assert st["converged"]
    assert abs(st["iterations"] - it_o) <= 1
    assert rel_err(from_dev(u), x_ref) < 1e-6


def test_graph_replay_matches_eager():
    meshes, gpu, ora = pair("square_p2")
    wl, scale, degree, layers = CASES["square_p2"][:4]
    gg = build_pair(meshes, degree, layers=layers, use_graph=True, build_oracle=False)[0]
    n = ora.levels[0].A.shape[0]
    for rep in range(3):
        b = meshgen.random_rhs(n, 10 + rep)
        u1, u2 = to_dev(np.zeros(n)), to_dev(np.zeros(n))
        s1 = gpu.pcg(to_dev(b), u1, 1e-10, 200)
        s2 = gg.pcg(to_dev(b), u2, 1e-10, 200)
        assert s1["iterations"] == s2["iterations"]
        assert rel_err(from_dev(u2), from_dev(u1)) < 1e-13
    gg.close()


def test_error_paths_on_gpu():
    from paper_2402_12947_amd import MG_ERR_ARG, MG_ERR_LOCATE, MG_NOT_CONVERGED, MgError, setup_status
    fine = meshgen.square_mesh(8, 0)
    coarse = meshgen.square_mesh(4, 1)
    shrunk = dict(coarse)
    shrunk["coords"] = coarse["coords"] * 0.5
    assert setup_status([fine, shrunk])[0] == MG_ERR_LOCATE
    meshes, gpu, ora = pair("square_p1_4k")
    n = ora.levels[0].A.shape[0]
    b = to_dev(meshgen.random_rhs(n, 0))
    st = gpu.pcg(b, to_dev(np.zeros(n)), 1e-12, 1)
    assert st["status"] == MG_NOT_CONVERGED and st["iterations"] == 1
    with pytest.raises(MgError) as e:
        gpu.pcg(b, b, 1e-8, 10)
    assert e.value.code == MG_ERR_ARG
    with pytest.raises(MgError):
        gpu.smooth(len(ora.levels) - 1, b, to_dev(np.zeros(n)), 1)
    z = to_dev(np.zeros(n))
    st = gpu.pcg(to_dev(np.zeros(n)), z, 1e-8, 10)
    assert st["converged"] and st["iterations"] == 0 and float(z.abs().max()) == 0.0


@pytest.mark.parametrize("k", [1, 3])
def test_chebyshev_degree(k):
    """Chebyshev polynomials of degree 1 and 3 (first, middle and last steps)."""
    meshes = meshgen.hierarchy("square_p1_4k", seed=0)
    gpu, ora = build_pair(meshes, 1, layers=2, k=k)
    n = ora.levels[0].A.shape[0]
    b, u0 = meshgen.random_rhs(n, 7), meshgen.random_rhs(n, 8)
    u = to_dev(u0)
    gpu.smooth(0, to_dev(b), u, 1)
    assert rel_err(from_dev(u), ora.smooth(0, b, u0.copy(), 1)) < 1e-10
    u = to_dev(u0)
    gpu.vcycle(to_dev(b), u)
    assert rel_err(from_dev(u), ora.vcycle(b, u0.copy())) < 1e-10
    gpu.close()


@pytest.mark.parametrize("name", ["square_p1_4k", "square_p2", "cube_p2"])
def test_stationary_multigrid(name):
    """mg_vcycle_solve: twelve V-cycles from zero equal the oracle's iterate, and
    the number of cycles to rtol 1e-8 matches within one."""
    meshes, gpu, ora = pair(name)
    n = ora.levels[0].A.shape[0]
    b = meshgen.random_rhs(n, 9)
    x_o, it_o, _, hist_o = ora.mg_solve(b, 1e-300, 12)
    u = to_dev(np.zeros(n))
    st = gpu.mg_solve(to_dev(b), u, 1e-300, 12)
    assert st["iterations"] == 12 and not st["converged"]
    assert rel_err(from_dev(u), x_o) < 1e-9
    assert np.allclose(st["history"], hist_o, rtol=1e-6, atol=1e-12)
    _, it_o, conv_o, _ = ora.mg_solve(b, 1e-8, 200)
    st = gpu.mg_solve(to_dev(b), to_dev(np.zeros(n)), 1e-8, 200)
    assert conv_o and st["converged"] and abs(st["iterations"] - it_o) <= 1
