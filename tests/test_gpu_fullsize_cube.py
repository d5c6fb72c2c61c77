"""GPU parity on the 3D P2 cube at the largest size the oracle assembles in
seconds: the cube_129 recipe at half the intervals per side (65^3 vertices,
2.11M DOFs, five levels; the full-size benchmark has 16.8M).

At this size nearly every level-0 slice stores its columns in eight 16-bit
windows, a form the small 3D cases never reach (a row's columns span the
vertex block and the edge block of the numbering; the sixteen-window form
appears at full size, checked at the end).
Checks: the forms are reached on levels 0 and 1; flags and patches exact; the
assembled operator at 1e-12; point location and prolongation rows sampled;
one combined smoother application on level 0 and whole V-cycles at 1e-10, and
the PCG iteration count +-1 with the solution within 1e-8, against an oracle
hierarchy that takes the GPU's Chebyshev intervals (its Lanczos is too slow at
this size; the eigenvalues are pinned by the small-case tests) and the GPU's
prolongations (its point location is too slow; P is compared row by row on a
sample here), with its own assembly, Galerkin products, patch factorisations
and coarsest Cholesky; the true residuals of the FP64 and mixed solutions
under the oracle's operator, and mixed within 1e-6 of FP64.
"""
import numpy as np
import pytest

import meshgen
import oracle
from oracle.fem import DofMap
from oracle.patches import MERGE, colour, patches
from oracle.transfer import barycentric, locate
from tests.parity_util import from_dev, rel_err, sparse_close, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cube():
    from paper_2402_12947_amd import Solver
    meshes = meshgen.hierarchy("cube_129", seed=0, scale=2)
    print("[fullsize cube] building GPU hierarchy (FP64)", flush=True)
    gpu = Solver(meshes, degree=2, tau=0.1, layers=1)
    nl = gpu.n_levels
    Ps = [gpu.prolongation(l) for l in range(nl - 1)]
    iv = [(gpu.level_info(l)["cheb_lo"], gpu.level_info(l)["cheb_hi"]) for l in range(nl - 1)]
    print("[fullsize cube] oracle hierarchy (assembly, Galerkin products, patches)", flush=True)
    ora = oracle.Hierarchy(meshes, tau=0.1, layers=1, opts=oracle.Options(degree=2), prolongations=Ps,
                           intervals=iv)
    print("[fullsize cube] ready", flush=True)
    yield meshes, gpu, ora
    gpu.close()


def test_column_forms_reached(cube):
    """At this size nearly every level-0 slice takes the eight-window form (the
    sixteen-window and 32-bit forms appear at full size: test_full_size_forms)."""
    meshes, gpu, ora = cube
    for l in (0, 1):
        info = gpu.level_info(l)
        print(f"[fullsize cube] level {l}: slices {info['sell_slices']} multiwindow "
              f"{info['sell_slices_multiwindow']} (16 windows {info['sell_slices_16window']}) "
              f"32-bit {info['sell_slices_32bit']}", flush=True)
        assert info["sell_slices_multiwindow"] > 0
    assert gpu.level_info(0)["sell_slices_multiwindow"] > 0.9 * gpu.level_info(0)["sell_slices"]


def test_flags_patches_operator(cube):
    meshes, gpu, ora = cube
    lev = ora.levels[0]
    assert np.array_equal(gpu.get_array(0, "flags").astype(bool), lev.gamma < 0.1)
    ptr, dofs = gpu.get_array(0, "patch_ptr"), gpu.get_array(0, "patch_dofs")
    assert len(ptr) - 1 == len(lev.patch_dofs) and len(lev.patch_dofs) > 100
    for d, B in enumerate(lev.patch_dofs):
        assert np.array_equal(dofs[ptr[d]:ptr[d + 1]], B)
    assert sparse_close(gpu.matrix(0), lev.A, 1e-12)
    for l in range(1, gpu.n_levels):
        assert sparse_close(gpu.matrix(l), ora.levels[l].A, 1e-11)


def test_transfer_sampled(cube):
    meshes, gpu, ora = cube
    dm, dmc = ora.levels[0].dofmap, DofMap(meshes[1], 2)
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(dm.n_free, 20000, replace=False))
    pts = dm.nodes[dm.free[rows]]
    cell = locate(pts, dmc.coords, dmc.cells)
    assert np.array_equal(gpu.get_array(0, "locate")[rows], cell)
    lam = barycentric(dmc.coords, dmc.cells, cell, pts)
    basis, _ = oracle.local_basis(3, 2)
    vals = np.stack([oracle.fem.poly_eval(p, lam) for p in basis], axis=1)
    cols = dmc.free_index[dmc.cell_dofs[cell]]
    vals[cols < 0] = 0.0
    gcols, gvals = gpu.get_array(0, "p_cols")[rows], gpu.get_array(0, "p_vals")[rows]
    assert np.array_equal(gcols, cols)
    assert np.max(np.abs(gvals - vals)) < 1e-12


def test_smoother_and_vcycle(cube):
    meshes, gpu, ora = cube
    n = ora.levels[0].A.shape[0]
    b, u0 = meshgen.random_rhs(n, 4), meshgen.random_rhs(n, 5)
    u = to_dev(u0)
    gpu.smooth(0, to_dev(b), u, 1)
    assert rel_err(from_dev(u), ora.smooth(0, b, u0.copy(), 1)) < 1e-10
    u = to_dev(u0)
    gpu.vcycle(to_dev(b), u)
    assert rel_err(from_dev(u), ora.vcycle(b, u0.copy())) < 1e-10
    u = to_dev(np.zeros(n))
    gpu.vcycle(to_dev(b), u)
    assert rel_err(from_dev(u), ora.vcycle(b, None)) < 1e-10


def test_pcg_and_mixed(cube):
    from paper_2402_12947_amd import Solver
    meshes, gpu, ora = cube
    A = ora.levels[0].A
    n = A.shape[0]
    b = meshgen.random_rhs(n, 6)
    print("[fullsize cube] oracle PCG", flush=True)
    x_o, it_o, conv_o, _ = ora.pcg(b, 1e-8, 100)
    u = to_dev(np.zeros(n))
    st = gpu.pcg(to_dev(b), u, 1e-8, 100)
    assert conv_o and st["converged"] and abs(st["iterations"] - it_o) <= 1, (st["iterations"], it_o)
    x64 = from_dev(u)
    assert rel_err(x64, x_o) < 1e-8
    assert np.linalg.norm(b - A @ x64) <= 1.05e-8 * np.linalg.norm(b)
    print("[fullsize cube] mixed-precision hierarchy", flush=True)
    mix = Solver(meshes, degree=2, tau=0.1, layers=1, precision="mixed")
    u = to_dev(np.zeros(n))
    st = mix.pcg(to_dev(b), u, 1e-8, 100)
    mix.close()
    xm = from_dev(u)
    assert st["converged"] and abs(st["iterations"] - it_o) <= 1
    assert np.linalg.norm(b - A @ xm) <= 1.05e-8 * np.linalg.norm(b)
    assert np.linalg.norm(xm - x64) <= 1e-6 * np.linalg.norm(x64)


def test_full_size_forms():
    """The benchmark's size (16.8M DOFs): levels 0 and 1 hold slices in the
    eight- and sixteen-window forms (every slice of this workload fits 16
    bits), and the cycle with these forms is bitwise the cycle with every
    slice at 32 bits (whose decode is compared with the oracle in
    test_gpu_colforms), for one smoother application, one V-cycle and a
    whole solve.  Both hierarchies fix the same layouts (sorting window,
    gathers in flight, padding skip, lanes per row, and the local
    correction's chunk, size class and lanes per patch row, which the
    autotuner would otherwise choose by timing, each setting an order of
    summation) so that only the column forms differ."""
    from paper_2402_12947_amd import Solver
    meshes = meshgen.hierarchy("cube_129", seed=0)
    fixed = dict(degree=2, tau=0.1, layers=1, sell_sigma=128, sell_unroll=8, sell_mask=1, sell_rpl=1,
                 patch_chunk=16, patch_small_bound=-1, patch_rows_rpl=1)
    print("[full-size cube] natural column forms", flush=True)
    nat = Solver(meshes, **fixed)
    for l in (0, 1):
        info = nat.level_info(l)
        print(f"[full-size cube] level {l}: slices {info['sell_slices']} multiwindow "
              f"{info['sell_slices_multiwindow']} (16 windows {info['sell_slices_16window']}) "
              f"32-bit {info['sell_slices_32bit']}", flush=True)
        assert info["sell_slices_multiwindow"] > 0
    assert sum(nat.level_info(l)["sell_slices_16window"] for l in (0, 1)) > 0
    n = nat.n_free(0)
    b, u0 = to_dev(meshgen.random_rhs(n, 9)), meshgen.random_rhs(n, 10)
    out = []
    for s in (nat, None):
        if s is None:
            print("[full-size cube] every slice at 32 bits", flush=True)
            nat.close()
            s = Solver(meshes, sell_colform=3, **fixed)
            assert s.level_info(0)["sell_slices_32bit"] == s.level_info(0)["sell_slices"]
        u = to_dev(u0)
        s.smooth(0, b, u, 1)
        v = to_dev(u0)
        s.vcycle(b, v)
        w = to_dev(np.zeros(n))
        st = s.pcg(b, w, 1e-8, 100)
        out.append((from_dev(u), from_dev(v), from_dev(w), st["iterations"]))
        s.close()
    for a, c in zip(out[0][:3], out[1][:3]):
        assert np.array_equal(a, c)
    assert out[0][3] == out[1][3]
