"""Helpers shared by the GPU parity tests (binding + oracle side by side)."""
import numpy as np
import scipy.sparse as sp


def gpu_solver(mesh, nu=None, rhs=None, load_points=3):
    import torch

    from paper_1901_02330_amd.vem import Solver

    s = Solver()
    s.set_mesh(mesh)
    s.discretize("lo", load_points=load_points)
    if nu is not None:
        s.set_coefficient(torch.as_tensor(nu, dtype=torch.float64))
    if rhs is not None:
        s.set_rhs_functions(rhs.f, rhs.pD)
    return s


def to_scipy(rp, col, val, shape):
    return sp.csr_matrix((val.cpu().numpy(), col.cpu().numpy(), rp.cpu().numpy()), shape=shape)


def assert_same_csr(G, O, rtol=1e-13):
    """Same sparsity pattern (columns sorted in both) and values within rtol of max |O|."""
    O = O.tocsr().copy()
    O.sort_indices()
    O.eliminate_zeros()
    G = G.tocsr()
    scale = abs(O).max()
    D = (G - O).tocsr()
    assert abs(D).max() <= rtol * scale, f"max value diff {abs(D).max()} vs scale {scale}"
    # pattern: every stored GPU entry is where the oracle has one, or numerically zero there
    Gp = G.copy()
    Gp.data[:] = 1.0
    Op = O.copy()
    Op.data[:] = 1.0
    extra = (Gp - Gp.multiply(Op)).tocsr()
    extra.eliminate_zeros()
    if extra.nnz:
        vals = G.multiply(extra).data
        assert vals.size == 0 or np.abs(vals).max() <= rtol * scale


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))
