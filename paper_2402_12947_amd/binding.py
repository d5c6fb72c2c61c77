"""ctypes binding of libmgpcg.so (include/mgpcg.h): argument marshalling only.

Every numerical step runs in the HIP library; there is no Python or CPU
fallback.  Importing this module raises if the library has not been built.
Device vectors are torch CUDA (HIP) float64 tensors; meshes are NumPy arrays.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgpcg.so")

MG_OK, MG_NOT_CONVERGED = 0, 1
MG_ERR_ARG, MG_ERR_MESH, MG_ERR_LOCATE, MG_ERR_NOT_SPD = -1, -2, -3, -4
MG_ERR_BREAKDOWN, MG_ERR_HIP, MG_ERR_OOM, MG_ERR_LIMIT = -5, -6, -7, -8
MG_FP64, MG_MIXED = 0, 1
MG_PATCH_MERGE, MG_PATCH_OVERLAP = 0, 1
MAX_HISTORY = 1024

ARR = {"quality": 1, "flags": 2, "patch_ptr": 3, "patch_dofs": 4, "patch_colour": 5, "locate": 6,
       "free_dofs": 7, "dof_nodes": 8, "a_rowptr": 9, "a_cols": 10, "a_vals": 11, "p_cols": 12,
       "p_vals": 13, "cell_dofs": 14, "p_width": 15, "sgs_colour": 16}


class MgMesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_vertices", C.c_int64), ("coords", C.POINTER(C.c_double)),
                ("n_cells", C.c_int64), ("cells", C.POINTER(C.c_int32)),
                ("dirichlet_vertex", C.POINTER(C.c_uint8))]


class MgOptions(C.Structure):
    _fields_ = [("degree", C.c_int32), ("precision", C.c_int32), ("nu", C.c_int32),
                ("cheb_degree", C.c_int32), ("cheb_lo_frac", C.c_double),
                ("local_correction", C.c_int32), ("adjusted_eig", C.c_int32),
                ("patch_policy", C.c_int32), ("eig_tol", C.c_double), ("eig_maxit", C.c_int32),
                ("use_graph", C.c_int32), ("sell_sigma", C.c_int32), ("stream", C.c_void_p),
                ("global_smoother", C.c_int32), ("problem", C.c_int32), ("young", C.c_double),
                ("poisson_ratio", C.c_double), ("sell_unroll", C.c_int32), ("sell_mask", C.c_int32),
                ("sell_rpl", C.c_int32), ("patch_fused", C.c_int32), ("use_initial_guess", C.c_int32),
                ("sell_colform", C.c_int32), ("patch_factor_f32", C.c_int32), ("patch_refine", C.c_int32),
                ("patch_inherit_levels", C.c_int32), ("patch_chunk", C.c_int32),
                ("patch_small_bound", C.c_int32), ("coarse_solver", C.c_int32), ("coarse_nd_leaf", C.c_int32),
                ("sell_layout_levels", C.c_int32),
                ("sell_layout", C.POINTER(C.c_int32)), ("patch_rows_rpl", C.c_int32)]


class MgSolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("rel_residual", C.c_double),
                ("true_rel_residual", C.c_double), ("solve_ms", C.c_double), ("n_history", C.c_int32),
                ("history", C.c_double * MAX_HISTORY)]


class MgLevelInfo(C.Structure):
    _fields_ = [("n_vertices", C.c_int64), ("n_cells", C.c_int64), ("n_dofs", C.c_int64),
                ("n_free", C.c_int64), ("nnz", C.c_int64), ("n_flagged", C.c_int64),
                ("n_patches", C.c_int32), ("n_colours", C.c_int32), ("max_patch", C.c_int32),
                ("sum_patch_dofs", C.c_int64), ("gamma_min", C.c_double), ("lambda_max", C.c_double),
                ("lambda_adj", C.c_double), ("cheb_lo", C.c_double), ("cheb_hi", C.c_double),
                ("lanczos_steps", C.c_int32), ("lanczos_steps_adj", C.c_int32), ("sell_sigma", C.c_int32),
                ("sell_stored", C.c_int64), ("is_coarsest", C.c_int32), ("setup_ms", C.c_double),
                ("sell_nnz16", C.c_int64), ("n_components", C.c_int32),
                ("sell_unroll", C.c_int32), ("sell_mask", C.c_int32), ("sell_rpl", C.c_int32),
                ("patch_fused_colours", C.c_int32), ("sell_slices", C.c_int64),
                ("sell_slices_multiwindow", C.c_int64), ("sell_slices_32bit", C.c_int64),
                ("sell_slices_16window", C.c_int64), ("patches_f32", C.c_int32),
                ("patches_inherited", C.c_int32), ("patch_small_bound", C.c_int32),
                ("patch_chunk", C.c_int32), ("coarse_nd_supernodes", C.c_int32),
                ("coarse_solve_bytes", C.c_double), ("patch_rows_rpl", C.c_int32)]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                          "(there is no CPU fallback)")
    # torch ships its own HIP runtime with the same soname as the system one;
    # loading torch first makes this library bind to that single runtime, so
    # torch tensors and the library share one device context.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P = C.c_void_p
    sig = {
        "mg_default_options": (None, [C.POINTER(MgOptions)]),
        "mg_setup": (C.c_int, [C.POINTER(MgMesh), C.c_int32, C.c_double, C.c_int32, C.POINTER(MgOptions),
                               C.POINTER(P)]),
        "mg_smooth": (C.c_int, [P, C.c_int32, P, P, C.c_int32]),
        "mg_vcycle": (C.c_int, [P, P, P]),
        "mg_vcycle_noalloc": (C.c_int, [P, P, P]),
        "mg_pcg_solve": (C.c_int, [P, P, P, C.c_double, C.c_int32, C.POINTER(MgSolveStats)]),
        "mg_vcycle_solve": (C.c_int, [P, P, P, C.c_double, C.c_int32, C.POINTER(MgSolveStats)]),
        "mg_pcg_solve_multi": (C.c_int, [P, C.c_int32, C.POINTER(P), C.POINTER(P), C.c_double, C.c_int32,
                                         C.POINTER(MgSolveStats)]),
        "mg_rhs_from_nodal": (C.c_int, [P, P, P]),
        "mg_pcg_solve_batch": (C.c_int, [C.POINTER(P), C.c_int32, C.c_int32, C.POINTER(P), C.POINTER(P),
                                         C.c_double, C.c_int32, C.POINTER(MgSolveStats), C.POINTER(C.c_double)]),
        "mg_get_level_info": (C.c_int, [P, C.c_int32, C.POINTER(MgLevelInfo)]),
        "mg_get_array": (C.c_int, [P, C.c_int32, C.c_int32, P]),
        "mg_enable_kernel_timing": (C.c_int, [P, C.c_int32]),
        "mg_kernel_time": (C.c_int, [P, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
        "mg_level_kernel_time": (C.c_int, [P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
        "mg_cheb_algorithmic_bytes": (C.c_int, [P, C.POINTER(C.c_double)]),
        "mg_stream_probe": (C.c_int, [C.c_int32, C.c_int64, C.c_int32, C.POINTER(C.c_double)]),
        "mg_last_error": (C.c_char_p, [P]),
        "mg_global_error": (C.c_char_p, []),
        "mg_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


class MgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _mesh_struct(m: dict, keep: list) -> MgMesh:
    coords = np.ascontiguousarray(m["coords"], dtype=np.float64)
    cells = np.ascontiguousarray(m["cells"], dtype=np.int32)
    dirv = np.ascontiguousarray(m["dirichlet_vertex"], dtype=np.uint8)
    keep += [coords, cells, dirv]
    return MgMesh(int(m["dim"]), coords.shape[0], coords.ctypes.data_as(C.POINTER(C.c_double)),
                  cells.shape[0], cells.ctypes.data_as(C.POINTER(C.c_int32)),
                  dirv.ctypes.data_as(C.POINTER(C.c_uint8)))


def _ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return t.data_ptr()


def _sync():
    import torch
    torch.cuda.synchronize()


class Solver:
    """One multigrid hierarchy (mg_setup) and its solve-phase entry points."""

    def __init__(self, meshes: list, degree: int = 1, tau: float = 0.1, layers: int = 1,
                 precision: str = "fp64", nu: int = 2, cheb_degree: int = 2, cheb_lo_frac: float = 0.1,
                 local_correction: bool = True, adjusted_eig: bool = True, policy: str = "merge",
                 eig_tol: float = 1e-8, eig_maxit: int = 200, use_graph: bool = False, sell_sigma: int = 0,
                 global_smoother: str = "chebyshev", problem: str = "poisson", young: float = 6.9e10,
                 poisson_ratio: float = 0.33, sell_unroll: int = 0, sell_mask: int = -1, sell_rpl: int = 0,
                 patch_fused: bool = True, use_initial_guess: bool = False, sell_layout=None,
                 sell_colform: int = 0, patch_factor_f32: bool = True, patch_refine: bool = False,
                 patch_inherit_levels: int = 0, patch_chunk: int = 0, patch_small_bound: int = 0,
                 coarse_solver: int = 0, coarse_nd_leaf: int = 1024, patch_rows_rpl: int = 0):
        L = lib()
        opt = MgOptions()
        L.mg_default_options(C.byref(opt))
        opt.degree = degree
        opt.precision = MG_MIXED if precision == "mixed" else MG_FP64
        opt.nu = nu
        opt.cheb_degree = cheb_degree
        opt.cheb_lo_frac = cheb_lo_frac
        opt.local_correction = int(bool(local_correction))
        opt.adjusted_eig = int(bool(adjusted_eig))
        opt.patch_policy = MG_PATCH_OVERLAP if policy == "overlap" else MG_PATCH_MERGE
        opt.eig_tol = eig_tol
        opt.eig_maxit = eig_maxit
        opt.use_graph = int(bool(use_graph))
        opt.sell_sigma = sell_sigma
        if global_smoother not in ("chebyshev", "sgs"):
            raise ValueError("global_smoother must be 'chebyshev' or 'sgs'")
        opt.global_smoother = 1 if global_smoother == "sgs" else 0
        if problem not in ("poisson", "elasticity"):
            raise ValueError("problem must be 'poisson' or 'elasticity'")
        opt.problem = 1 if problem == "elasticity" else 0
        opt.young = young
        opt.poisson_ratio = poisson_ratio
        opt.sell_unroll = sell_unroll
        opt.sell_mask = sell_mask
        opt.sell_rpl = sell_rpl
        opt.patch_fused = int(bool(patch_fused))
        opt.use_initial_guess = int(bool(use_initial_guess))
        opt.sell_colform = sell_colform
        opt.patch_factor_f32 = int(bool(patch_factor_f32))
        opt.patch_refine = int(bool(patch_refine))
        opt.patch_inherit_levels = patch_inherit_levels
        opt.patch_chunk = patch_chunk
        opt.patch_small_bound = patch_small_bound
        opt.coarse_solver = coarse_solver
        opt.coarse_nd_leaf = coarse_nd_leaf
        opt.patch_rows_rpl = patch_rows_rpl
        keep: list = []
        if sell_layout:  # [(sigma, unroll, mask, rpl) per level]
            lay = np.ascontiguousarray(np.asarray(sell_layout, dtype=np.int32).reshape(-1, 4))
            keep.append(lay)
            opt.sell_layout_levels = lay.shape[0]
            opt.sell_layout = lay.ctypes.data_as(C.POINTER(C.c_int32))
        arr = (MgMesh * len(meshes))(*[_mesh_struct(m, keep) for m in meshes])
        h = C.c_void_p()
        st = L.mg_setup(arr, len(meshes), tau, layers, C.byref(opt), C.byref(h))
        if st != MG_OK:
            raise MgError(st, L.mg_global_error().decode())
        self._h = h
        self.n_levels = len(meshes)
        self.dim = int(meshes[0]["dim"])
        self.degree = degree

    # -- bookkeeping -------------------------------------------------------
    def _check(self, st: int, allow=(MG_OK,)) -> int:
        if st not in allow:
            raise MgError(st, lib().mg_last_error(self._h).decode())
        return st

    def close(self):
        if getattr(self, "_h", None):
            lib().mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_info(self, level: int = 0) -> dict:
        info = MgLevelInfo()
        self._check(lib().mg_get_level_info(self._h, level, C.byref(info)))
        return {name: getattr(info, name) for name, _ in MgLevelInfo._fields_}

    def n_free(self, level: int = 0) -> int:
        return self.level_info(level)["n_free"]

    def get_array(self, level: int, what: str) -> np.ndarray:
        info = self.level_info(level)
        nloc = {(2, 1): 3, (2, 2): 6, (2, 3): 10, (3, 1): 4, (3, 2): 10}[(self.dim, self.degree)]
        pw = np.zeros(1, dtype=np.int32)
        if what in ("p_cols", "p_vals"):
            self._check(lib().mg_get_array(self._h, level, ARR["p_width"], pw.ctypes.data))
        n, nf = info["n_cells"], info["n_free"]
        nodes = nf // max(1, info["n_components"])   # free DOF nodes
        spec = {
            "quality": (np.float64, n), "flags": (np.uint8, n),
            "patch_ptr": (np.int32, info["n_patches"] + 1), "patch_dofs": (np.int32, info["sum_patch_dofs"]),
            "patch_colour": (np.int32, info["n_patches"]), "locate": (np.int32, nodes),
            "sgs_colour": (np.int32, nf),
            "free_dofs": (np.int32, nodes), "dof_nodes": (np.float64, info["n_dofs"] * self.dim),
            "a_rowptr": (np.int64, nf + 1), "a_cols": (np.int32, info["nnz"]), "a_vals": (np.float64, info["nnz"]),
            "p_cols": (np.int32, nf * int(pw[0])), "p_vals": (np.float64, nf * int(pw[0])),
            "cell_dofs": (np.int32, n * nloc),
        }[what]
        out = np.zeros(max(1, spec[1]), dtype=spec[0])
        self._check(lib().mg_get_array(self._h, level, ARR[what], out.ctypes.data))
        out = out[:spec[1]]
        if what == "dof_nodes":
            out = out.reshape(-1, self.dim)
        elif what == "cell_dofs":
            out = out.reshape(n, nloc)
        elif what in ("p_cols", "p_vals"):
            out = out.reshape(nf, int(pw[0]))
        return out

    def matrix(self, level: int = 0):
        """A_level as a SciPy CSR matrix (copied to the host)."""
        import scipy.sparse as sp
        nf = self.n_free(level)
        return sp.csr_matrix((self.get_array(level, "a_vals"), self.get_array(level, "a_cols"),
                              self.get_array(level, "a_rowptr")), shape=(nf, nf))

    def prolongation(self, level: int = 0):
        import scipy.sparse as sp
        cols, vals = self.get_array(level, "p_cols"), self.get_array(level, "p_vals")
        rows = np.repeat(np.arange(cols.shape[0]), cols.shape[1])
        keep = cols.ravel() >= 0
        return sp.csr_matrix((vals.ravel()[keep], (rows[keep], cols.ravel()[keep])),
                             shape=(cols.shape[0], self.n_free(level + 1)))

    # -- the method ----------------------------------------------------------
    def smooth(self, level: int, b, u, nu: int = 1):
        _sync()
        self._check(lib().mg_smooth(self._h, level, _ptr(b), _ptr(u), nu))

    def vcycle(self, b, u):
        _sync()
        self._check(lib().mg_vcycle(self._h, _ptr(b), _ptr(u)))

    def vcycle_noalloc(self, b, u):
        """mg_vcycle_noalloc: the cycle with its staging vectors in the
        library's static device array; it returns without synchronising, so
        the device is synchronised here before u is handed back."""
        _sync()
        self._check(lib().mg_vcycle_noalloc(self._h, _ptr(b), _ptr(u)))
        _sync()

    def pcg(self, b, u, rtol: float = 1e-8, maxit: int = 500) -> dict:
        _sync()
        st = MgSolveStats()
        code = self._check(lib().mg_pcg_solve(self._h, _ptr(b), _ptr(u), rtol, maxit, C.byref(st)),
                           allow=(MG_OK, MG_NOT_CONVERGED))
        return {"status": code, "iterations": st.iterations, "converged": bool(st.converged),
                "rel_residual": st.rel_residual, "true_rel_residual": st.true_rel_residual,
                "solve_ms": st.solve_ms, "history": list(st.history[:st.n_history])}

    def pcg_multi(self, bs: list, us: list, rtol: float = 1e-8, maxit: int = 500) -> dict:
        """mg_pcg_solve_multi: the right-hand sides bs[r] (device float64
        tensors) solved together in blocks; us[r] receive the solutions.
        Returns the status and one statistics record per right-hand side."""
        if len(bs) != len(us):
            raise ValueError("bs and us must have the same length")
        n = len(bs)
        _sync()
        pb = (C.c_void_p * max(1, n))(*[_ptr(t) for t in bs])
        pu = (C.c_void_p * max(1, n))(*[_ptr(t) for t in us])
        st = (MgSolveStats * max(1, n))()
        code = self._check(lib().mg_pcg_solve_multi(self._h, n, pb, pu, rtol, maxit, st),
                           allow=(MG_OK, MG_NOT_CONVERGED))
        stats = [{"iterations": x.iterations, "converged": bool(x.converged), "rel_residual": x.rel_residual,
                  "true_rel_residual": x.true_rel_residual, "solve_ms": x.solve_ms,
                  "history": list(x.history[:x.n_history])} for x in st[:n]]
        return {"status": code, "stats": stats}

    def mg_solve(self, b, u, rtol: float = 1e-8, maxit: int = 100) -> dict:
        """Multigrid as a stationary solver: V-cycles from u = 0 until the
        relative residual is at most rtol (mg_vcycle_solve)."""
        _sync()
        st = MgSolveStats()
        code = self._check(lib().mg_vcycle_solve(self._h, _ptr(b), _ptr(u), rtol, maxit, C.byref(st)),
                           allow=(MG_OK, MG_NOT_CONVERGED))
        return {"status": code, "iterations": st.iterations, "converged": bool(st.converged),
                "rel_residual": st.rel_residual, "solve_ms": st.solve_ms,
                "history": list(st.history[:st.n_history])}

    def rhs_from_nodal(self, f, b):
        _sync()
        self._check(lib().mg_rhs_from_nodal(self._h, _ptr(f), _ptr(b)))

    def enable_kernel_timing(self, on: bool = True):
        self._check(lib().mg_enable_kernel_timing(self._h, int(on)))

    def kernel_time(self, level: int = 0):
        """(launches, summed ms) of the timed kernels of `level` since timing
        was enabled: full Chebyshev steps, or the coarsest solves on the
        coarsest level."""
        n = C.c_int64()
        t = C.c_double()
        self._check(lib().mg_level_kernel_time(self._h, level, C.byref(n), C.byref(t)))
        return n.value, t.value

    def cheb_bytes(self) -> float:
        b = C.c_double()
        self._check(lib().mg_cheb_algorithmic_bytes(self._h, C.byref(b)))
        return b.value


def pcg_solve_batch(solvers: list, bs: list, us: list, rtol: float = 1e-8, maxit: int = 500) -> dict:
    """mg_pcg_solve_batch: bs[i][r], us[i][r] are instance i's right-hand sides
    and solutions (device float64 tensors).  Returns status, wall time and the
    per-system statistics."""
    n_inst = len(solvers)
    nrhs = len(bs[0]) if n_inst else 0
    if any(len(x) != nrhs for x in bs) or any(len(x) != nrhs for x in us) or len(bs) != n_inst:
        raise ValueError("bs and us must be n_inst x nrhs")
    _sync()
    hs = (C.c_void_p * n_inst)(*[s._h.value for s in solvers])
    pb = (C.c_void_p * (n_inst * nrhs))(*[_ptr(t) for row in bs for t in row])
    pu = (C.c_void_p * (n_inst * nrhs))(*[_ptr(t) for row in us for t in row])
    st = (MgSolveStats * max(1, n_inst * nrhs))()
    wall = C.c_double()
    code = lib().mg_pcg_solve_batch(hs, n_inst, nrhs, pb, pu, rtol, maxit, st, C.byref(wall))
    if code < 0:
        msg = lib().mg_global_error().decode()
        for s in solvers:
            m = lib().mg_last_error(s._h).decode()
            if m:
                msg = m
                break
        raise MgError(code, msg)
    stats = [{"iterations": x.iterations, "converged": bool(x.converged), "true_rel_residual": x.true_rel_residual,
              "solve_ms": x.solve_ms} for x in st[:n_inst * nrhs]]
    return {"status": code, "wall_ms": wall.value, "stats": stats}


def setup_status(meshes: list, **kw) -> tuple:
    """mg_setup's status code and message without raising (for error-path tests)."""
    try:
        s = Solver(meshes, **kw)
        s.close()
        return MG_OK, ""
    except MgError as e:
        return e.code, str(e)


def stream_probe(kind: str, nbytes: int = 2 << 30, reps: int = 10) -> float:
    """mg_stream_probe: GB/s of a plain stream ("read", "copy", or "mix7:1" =
    seven read streams and one write stream) over nbytes of device memory."""
    k = {"read": 0, "copy": 1, "mix7:1": 2}[kind]
    gbs = C.c_double()
    code = lib().mg_stream_probe(k, int(nbytes), int(reps), C.byref(gbs))
    if code != MG_OK:
        raise MgError(code, "mg_stream_probe failed")
    return gbs.value
