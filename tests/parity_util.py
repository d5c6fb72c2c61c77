"""Helpers of the GPU parity tests: build the oracle and the HIP hierarchy on
the same seeded meshes and compare them stage by stage."""
import numpy as np

import meshgen
import oracle


def build_pair(meshes, degree, tau=0.1, layers=1, precision="fp64", local=True, adjusted=True,
               policy="merge", use_graph=False, nu=2, k=2, eig_maxit=200, build_oracle=True,
               smoother="chebyshev", inherit=0, **gpu_kw):
    from paper_2402_12947_amd import Solver
    gpu = Solver(meshes, degree=degree, tau=tau, layers=layers, precision=precision,
                 local_correction=local, adjusted_eig=adjusted, policy=policy, use_graph=use_graph,
                 nu=nu, cheb_degree=k, eig_maxit=eig_maxit, global_smoother=smoother,
                 patch_inherit_levels=inherit, **gpu_kw)
    ora = None
    if build_oracle:
        ora = oracle.Hierarchy(meshes, tau=tau, layers=layers,
                               opts=oracle.Options(degree=degree, nu=nu, cheb_degree=k, local_correction=local,
                                                   adjusted_eig=adjusted,
                                                   patch_policy=oracle.OVERLAP if policy == "overlap"
                                                   else oracle.MERGE, eig_maxit=eig_maxit,
                                                   global_smoother=smoother, inherit_levels=inherit))
    return gpu, ora


def sparse_close(A, B, rtol):
    D = (A - B).tocoo()
    scale = max(abs(A).max(), abs(B).max())
    return (abs(D.data).max() if D.nnz else 0.0) <= rtol * scale


def rel_err(x, y):
    return float(np.max(np.abs(x - y)) / max(np.max(np.abs(y)), 1e-300))


def to_dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def from_dev(t):
    return t.detach().cpu().numpy()
