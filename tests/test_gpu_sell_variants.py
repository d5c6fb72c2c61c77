"""The sparse-product variants: bitwise equal where the summation order is the
same, every one at the oracle's bar.

Every SELL row product sums entry j of a lane's share of its row into
accumulator j mod U and adds the accumulators pairwise, whether it skips the
padding of the shorter rows of a slice (sell_mask = 1) or reads every stored
entry (sell_mask = 0), so that choice of the autotuner cannot change a result.
With several lanes per row (sell_rpl: 2 to 32; 16 and 32 for the long rows of
the Galerkin levels, the transfers keeping at most 8) the row is split over
the lanes, which changes the rounding of the row products only.  Checked on whole solves
(every level operator, transfer, patch-row and split first-step product of
the cycle) with the variant fixed by the options.
"""
import functools

import numpy as np
import pytest

import meshgen
import oracle
from tests.parity_util import from_dev, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    # name: (workload, scale, degree, layers)
    "square_p2": ("square_1025", 16, 2, 1),
    "cube_p2": ("cube_129", 16, 2, 1),
}


@functools.lru_cache(maxsize=None)
def _case(name):
    wl, scale, degree, layers = CASES[name]
    meshes = meshgen.hierarchy(wl, seed=0, scale=scale)
    ora = oracle.Hierarchy(meshes, tau=0.1, layers=layers, opts=oracle.Options(degree=degree))
    return meshes, ora


def _solve(meshes, degree, layers, precision, unroll, mask, b, rtol, rpl=1):
    import torch
    from paper_2402_12947_amd import Solver
    s = Solver(meshes, degree=degree, layers=layers, precision=precision, sell_sigma=128,
               sell_unroll=unroll, sell_mask=mask, sell_rpl=rpl)
    info = [s.level_info(l) for l in range(s.n_levels - 1)]
    assert all(lv["sell_unroll"] == unroll and lv["sell_mask"] == mask and lv["sell_rpl"] == rpl for lv in info)
    u = torch.zeros_like(b)
    st = s.pcg(b, u, rtol, 300)
    s.close()
    return from_dev(u), st["iterations"], info


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_masked_and_full_products_agree_bitwise(name, precision):
    wl, scale, degree, layers = CASES[name]
    meshes, ora = _case(name)
    print(f"[case {name} {precision}] levels={[m['cells'].shape[0] for m in meshes]}", flush=True)
    n = ora.levels[0].A.shape[0]
    rhs = meshgen.random_rhs(n, 7)
    # FP64: the oracle's iterate at the same tolerance; mixed: its solution
    rtol = 1e-10 if precision == "fp64" else 1e-8
    x_o, it_o, _, _ = ora.pcg(rhs, rtol, 300)
    x_ref = x_o if precision == "fp64" else ora.pcg(rhs, 1e-12, 300)[0]
    tol = 1e-8 if precision == "fp64" else 1e-6
    b = to_dev(rhs)
    for unroll, rpl in ((4, 1), (8, 1), (4, 2), (8, 4), (4, 8), (8, 16), (4, 32)):
        u0, it0, info = _solve(meshes, degree, layers, precision, unroll, 0, b, rtol, rpl)
        u1, it1, _ = _solve(meshes, degree, layers, precision, unroll, 1, b, rtol, rpl)
        # the layouts pad, so the masked variant really skips entries
        assert info[0]["sell_stored"] > info[0]["nnz"]
        assert it0 == it1 and np.array_equal(u0, u1), (unroll, rpl, it0, it1)
        assert abs(it0 - it_o) <= 1
        assert np.max(np.abs(u0 - x_ref)) <= tol * np.max(np.abs(x_ref))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("scale,one_launch", [(16, True), (4, False)])
def test_fused_patch_correction_agrees_bitwise(precision, scale, one_launch):
    """Small patches: one launch per colour when no patch row reads another
    patch's DOF (1/16 of the 1025^2 P2 square: one patch), else the residual
    launch and one launch for the packed-inverse product and update (1/4 size:
    16 patches, two of them coupled through A); both bitwise equal to the
    three-launch local correction, for one smoother application and a whole
    solve."""
    import torch
    from paper_2402_12947_amd import Solver
    meshes = meshgen.hierarchy("square_1025", seed=0, scale=scale)
    print(f"[case square_1025/{scale} P2 {precision}]", flush=True)
    out = {}
    for fused in (True, False):
        s = Solver(meshes, degree=2, layers=1, precision=precision, sell_sigma=128, sell_unroll=8,
                   sell_mask=0, sell_rpl=1, patch_fused=fused, patch_chunk=16,
                   patch_small_bound=256 if fused else -1)
        info = s.level_info(0)
        assert info["max_patch"] <= 256
        assert info["patch_fused_colours"] == (int(one_launch) if fused else 0)
        n = s.n_free(0)
        b = to_dev(meshgen.random_rhs(n, 11))
        u_s = to_dev(np.zeros(n))
        s.smooth(0, b, u_s, 2)
        u = torch.zeros_like(b)
        st = s.pcg(b, u, 1e-8, 300)
        out[fused] = (from_dev(u_s), from_dev(u), st["iterations"])
        s.close()
    assert np.array_equal(out[True][0], out[False][0])
    assert np.array_equal(out[True][1], out[False][1]) and out[True][2] == out[False][2]


def test_per_level_layout_is_repeated():
    """sell_layout fixes each level operator's layout: a hierarchy built with
    the layouts another run's autotuner chose reports the same choices and
    gives the same cycle to rounding (the transfer products are still chosen
    by timing, and their gathers in flight set the order of a few sums)."""
    from paper_2402_12947_amd import Solver
    meshes = meshgen.hierarchy("square_1025", seed=0, scale=4)
    print("[case square_1025/4 P2 layouts]", flush=True)
    a = Solver(meshes, degree=2, layers=1)
    keys = ("sell_sigma", "sell_unroll", "sell_mask", "sell_rpl")
    la = [[a.level_info(l)[k] for k in keys] for l in range(a.n_levels - 1)]
    n = a.n_free(0)
    b = to_dev(meshgen.random_rhs(n, 5))
    ua = to_dev(np.zeros(n))
    a.vcycle(b, ua)
    a.close()
    fixed = Solver(meshes, degree=2, layers=1, sell_layout=la)
    assert [[fixed.level_info(l)[k] for k in keys] for l in range(fixed.n_levels - 1)] == la
    ub = to_dev(np.zeros(n))
    fixed.vcycle(b, ub)
    fixed.close()
    x, y = from_dev(ua), from_dev(ub)
    assert np.max(np.abs(x - y)) <= 1e-12 * np.max(np.abs(x))
    # an explicit layout on level 0 only; the other levels stay autotuned
    other = Solver(meshes, degree=2, layers=1, sell_layout=[[128, 4, 1, 2]])
    assert [other.level_info(0)[k] for k in keys] == [128, 4, 1, 2]
    other.close()
