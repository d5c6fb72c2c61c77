"""The C ABI without a GPU: the library loads, exports every entry point that
include/mgpcg.h declares, and rejects malformed input in host validation
before any device work (so these error paths are testable on the CPU)."""
import os
import re

import numpy as np
import pytest

import meshgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgpcg.h")
LIB = os.path.join(ROOT, "paper_2402_12947_amd", "libmgpcg.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libmgpcg.so not built")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    import ctypes
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert "mg_setup" in names and "mg_pcg_solve" in names and "mg_vcycle" in names and "mg_smooth" in names
    for name in names:
        assert hasattr(lib, name), name


def test_default_options_are_the_papers():
    from paper_2402_12947_amd.binding import MgOptions, lib
    import ctypes
    o = MgOptions()
    lib().mg_default_options(ctypes.byref(o))
    assert (o.degree, o.nu, o.cheb_degree, o.local_correction, o.adjusted_eig) == (1, 2, 2, 1, 1)
    assert o.cheb_lo_frac == 0.1 and o.eig_tol == 1e-8 and o.eig_maxit == 200
    assert (o.sell_sigma, o.sell_unroll, o.sell_mask, o.sell_rpl, o.patch_fused) == (0, 0, -1, 0, 1)
    assert o.use_initial_guess == 0


def test_setup_rejects_bad_input_on_host():
    from paper_2402_12947_amd import MG_ERR_ARG, MG_ERR_MESH, setup_status
    mesh = meshgen.square_mesh(4, 0)
    bad = dict(mesh)
    bad["cells"] = mesh["cells"].copy()
    bad["cells"][3, 1] = 10_000
    assert setup_status([bad])[0] == MG_ERR_MESH
    neg = dict(mesh)
    neg["cells"] = mesh["cells"].copy()
    neg["cells"][0, 0] = -1
    assert setup_status([neg])[0] == MG_ERR_MESH
    nan = dict(mesh)
    nan["coords"] = mesh["coords"].copy()
    nan["coords"][5, 0] = np.nan
    assert setup_status([nan])[0] == MG_ERR_MESH
    assert setup_status([meshgen.cube_mesh(2, 0)], degree=3)[0] == MG_ERR_ARG
    assert setup_status([mesh], degree=4)[0] == MG_ERR_ARG
    assert setup_status([mesh, meshgen.cube_mesh(2, 0)])[0] == MG_ERR_ARG
    assert setup_status([mesh], problem="elasticity", poisson_ratio=0.5)[0] == MG_ERR_ARG
    assert setup_status([mesh], problem="elasticity", young=-1.0)[0] == MG_ERR_ARG
    assert setup_status([mesh], sell_sigma=100)[0] == MG_ERR_ARG
    assert setup_status([mesh], nu=-1)[0] == MG_ERR_ARG
    assert setup_status([mesh], sell_unroll=16)[0] == MG_ERR_ARG
    assert setup_status([mesh], sell_mask=2)[0] == MG_ERR_ARG
    assert setup_status([mesh], sell_rpl=3)[0] == MG_ERR_ARG
    assert setup_status([mesh], sell_colform=4)[0] == MG_ERR_ARG
    assert setup_status([mesh], patch_rows_rpl=3)[0] == MG_ERR_ARG
    assert setup_status([mesh], patch_rows_rpl=4, patch_refine=True)[0] == MG_ERR_ARG
    # per-level layouts follow the same rules as the global layout options
    assert setup_status([mesh], sell_layout=[[100, 0, -1, 0]])[0] == MG_ERR_ARG
    assert setup_status([mesh], sell_layout=[[0, 16, -1, 0]])[0] == MG_ERR_ARG
    assert setup_status([mesh], sell_layout=[[0, 0, 2, 0]])[0] == MG_ERR_ARG
    assert setup_status([mesh], sell_layout=[[0, 0, -1, 0], [1, 8, 1, 3]])[0] == MG_ERR_ARG


def test_binding_requires_built_library(tmp_path):
    from paper_2402_12947_amd.binding import load_library
    with pytest.raises(ImportError):
        load_library(str(tmp_path / "missing.so"))


def test_solve_entry_points_reject_null_context_on_host():
    import ctypes
    from paper_2402_12947_amd import MG_ERR_ARG
    from paper_2402_12947_amd.binding import MgSolveStats, lib
    st = (MgSolveStats * 2)()
    ptrs = (ctypes.c_void_p * 2)(None, None)
    assert lib().mg_pcg_solve(None, None, None, 1e-8, 10, st) == MG_ERR_ARG
    assert lib().mg_pcg_solve_multi(None, 2, ptrs, ptrs, 1e-8, 10, st) == MG_ERR_ARG
    assert lib().mg_pcg_solve_batch(None, 1, 1, ptrs, ptrs, 1e-8, 10, st, None) == MG_ERR_ARG


def test_stream_probe_rejects_bad_arguments_on_host():
    import ctypes
    from paper_2402_12947_amd import MG_ERR_ARG
    from paper_2402_12947_amd.binding import lib
    g = ctypes.c_double()
    assert lib().mg_stream_probe(3, 1 << 30, 1, ctypes.byref(g)) == MG_ERR_ARG
    assert lib().mg_stream_probe(0, 1 << 10, 1, ctypes.byref(g)) == MG_ERR_ARG
    assert lib().mg_stream_probe(0, 1 << 30, 0, ctypes.byref(g)) == MG_ERR_ARG
    assert lib().mg_stream_probe(0, 1 << 30, 1, None) == MG_ERR_ARG


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of mg_options and mg_level_info have the C layout
    (sizes and the offsets of their last fields), compiled from the header."""
    import ctypes
    import shutil
    import subprocess
    from paper_2402_12947_amd.binding import MgLevelInfo, MgOptions, MgSolveStats
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "mgpcg.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(mg_options), sizeof(mg_level_info),'
                   ' sizeof(mg_solve_stats), offsetof(mg_options, patch_rows_rpl),'
                   ' offsetof(mg_level_info, patch_rows_rpl), offsetof(mg_solve_stats, history));return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    want = [ctypes.sizeof(MgOptions), ctypes.sizeof(MgLevelInfo), ctypes.sizeof(MgSolveStats),
            MgOptions.patch_rows_rpl.offset, MgLevelInfo.patch_rows_rpl.offset, MgSolveStats.history.offset]
    assert got == want
