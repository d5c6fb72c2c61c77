"""The patch paths the autotuner chooses between, each against the oracle.

Local correction: the one-workgroup kernel in its size classes (patches of up
to 128, 256 or 384 DOFs per workgroup; one launch per colour, two for a
colour whose patches couple) or the three-launch path (patch-row residual,
packed-inverse row items, gather); the packed row items hold 8, 16 or 32 tiles
(`patch_chunk`), which also applies to the coarsest level's inverse; the
patch-row residual runs with 1, 2, 4 or 8 lanes per row (`patch_rows_rpl`).
Every forced combination: one V-cycle within 1e-10 of the oracle; the size
classes bitwise equal to each other and to the three-launch path while a tile
row fits one chunk.  The automatic choice is reported in the level info.
"""
import functools

import numpy as np
import pytest

import meshgen
import oracle
from tests.parity_util import from_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    # name: (workload, scale, degree, layers, policy)
    "square_p2_s8": ("square_1025", 8, 2, 1, "merge"),      # 61 patches of up to ~300 DOFs
    "square_p2_overlap": ("square_1025", 16, 2, 1, "overlap"),
    "cube_stress_p2": ("cube_129_stress", 8, 2, 0, "overlap"),  # up to 855 DOFs: three-launch only
}


@functools.lru_cache(maxsize=None)
def _case(name):
    wl, scale, degree, layers, policy = CASES[name]
    meshes = meshgen.hierarchy(wl, seed=0, scale=scale)
    ora = oracle.Hierarchy(meshes, tau=0.1, layers=layers,
                           opts=oracle.Options(degree=degree,
                                               patch_policy=oracle.OVERLAP if policy == "overlap" else oracle.MERGE))
    n = ora.levels[0].A.shape[0]
    b, u0 = meshgen.random_rhs(n, 71), meshgen.random_rhs(n, 72)
    return meshes, ora, b, u0, ora.vcycle(b, u0.copy())


def _cycle(name, **kw):
    from paper_2402_12947_amd import Solver
    wl, scale, degree, layers, policy = CASES[name]
    meshes, ora, b, u0, want = _case(name)
    s = Solver(meshes, degree=degree, layers=layers, policy=policy, **kw)
    info = s.level_info(0)
    u = to_dev(u0)
    s.vcycle(to_dev(b), u)
    s.close()
    x = from_dev(u)
    assert rel_err(x, want) < 1e-10, (kw, rel_err(x, want))
    return x, info


@pytest.mark.parametrize("name", list(CASES))
def test_patch_paths(name):
    maxn = _cycle(name, patch_small_bound=-1)[1]["max_patch"]
    print(f"[patch bins {name}] max patch {maxn} DOFs", flush=True)
    for chunk in (8, 16, 32):
        ref, info = _cycle(name, patch_small_bound=-1, patch_chunk=chunk)
        assert info["patch_small_bound"] == 0 and info["patch_chunk"] == chunk
        for bound in (128, 256, 384):
            x, info = _cycle(name, patch_small_bound=bound, patch_chunk=chunk)
            if bound < maxn:   # the class cannot take the level's patches
                assert info["patch_small_bound"] == 0
                continue
            assert info["patch_small_bound"] == bound
            if bound // 32 <= chunk:
                assert np.array_equal(x, ref), (chunk, bound)
    # the autotuner's choice is one of the candidates
    _, info = _cycle(name)
    assert info["patch_chunk"] in (8, 16, 32) and info["patch_small_bound"] in (0, 128, 256, 384)
    if maxn > 384:
        assert info["patch_small_bound"] == 0


@functools.lru_cache(maxsize=None)
def _square4():
    meshes = meshgen.hierarchy("square_1025", seed=0, scale=4)
    full = oracle.Hierarchy(meshes, tau=0.1, layers=1, opts=oracle.Options(degree=2))
    n = full.levels[0].A.shape[0]
    b, u0 = meshgen.random_rhs(n, 73), meshgen.random_rhs(n, 74)
    return meshes, b, u0, full.vcycle(b, u0.copy())


@pytest.mark.parametrize("chunk", [8, 16, 32])
def test_coarsest_chunk(chunk):
    """The coarsest inverse (1023 unknowns, 32 tile rows) in row items of 8, 16
    or 32 tiles, through whole V-cycles against the oracle."""
    from paper_2402_12947_amd import Solver
    meshes, b, u0, want = _square4()
    s = Solver(meshes, degree=2, patch_chunk=chunk)
    last = s.n_levels - 1
    assert s.level_info(last)["patch_chunk"] == chunk and s.level_info(last)["n_free"] > 32 * 16
    u = to_dev(u0)
    s.vcycle(to_dev(b), u)
    assert rel_err(from_dev(u), want) < 1e-10
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_patch_row_lanes(name):
    """The patch-row residual with 1, 2, 4 or 8 lanes per row, on the
    three-launch path and (where the patches fit) with the one-workgroup
    kernel taking the residual from it; block solves with 8 lanes equal the
    single-vector solves."""
    maxn = _cycle(name, patch_small_bound=-1)[1]["max_patch"]
    for rpl in (1, 2, 4, 8):
        _, info = _cycle(name, patch_small_bound=-1, patch_rows_rpl=rpl)
        assert info["patch_rows_rpl"] == rpl
        if maxn <= 384:
            _, info = _cycle(name, patch_small_bound=384, patch_rows_rpl=rpl)
            assert info["patch_rows_rpl"] == rpl and info["patch_small_bound"] == 384
    from paper_2402_12947_amd import Solver
    wl, scale, degree, layers, policy = CASES[name]
    meshes, ora, b, u0, want = _case(name)
    s = Solver(meshes, degree=degree, layers=layers, policy=policy, patch_rows_rpl=8)
    n = s.n_free(0)
    bs = [to_dev(meshgen.random_rhs(n, 80 + r)) for r in range(2)]
    us = [to_dev(np.zeros(n)) for _ in bs]
    res = s.pcg_multi(bs, us, 1e-10, 300)
    for r in range(2):
        u = to_dev(np.zeros(n))
        st = s.pcg(bs[r], u, 1e-10, 300)
        assert abs(res["stats"][r]["iterations"] - st["iterations"]) <= 1
        assert rel_err(from_dev(us[r]), from_dev(u)) < 1e-10
    s.close()
