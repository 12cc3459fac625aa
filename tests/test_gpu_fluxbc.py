"""GPU parity with the paper's own boundary data (Section 3, eq. mod_prob_eq): the normal flux given on
the whole boundary, the pressure with zero mean.  Against `oracle.fluxbc`:
  * K, S, A_gamma (prescribed DOFs as identity rows and columns, B without their columns) and the
    right-hand side (known fluxes moved to the right, pressure part projected off the constant
    pressure), element by element;
  * solves with both preconditioners against the oracle's direct solve with the zero-mean
    multiplier; the GPU pressure has zero mean;
  * the patch test (linear pressure, lowest order; P_{k+1} pressure, the paper's k = 1, 2).
Tolerances as in the other parity tests: 1e-13 for the lowest order, 1e-11 for order k (local Gram
systems with condition numbers up to about 1e5 on these meshes); solves at tol 1e-13 within 1e-10."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.fluxbc import flux_system, solve_flux
from paper_1901_02330_amd.inputs import LinearSolution, SineSolution, cube_mesh, lognormal_field, voronoi_mesh
from tests.gpu_helpers import assert_same_csr, to_scipy
from tests.test_oracle_paperk import _Poly

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "cube534_lo": (lambda: cube_mesh(5, 3, 4), "lo", 0),
    "voronoi60_lo": (lambda: voronoi_mesh(60, seed=7), "lo", 0),
    "cube322_k1": (lambda: cube_mesh(3, 2, 2), "paper", 1),
    "cube322_k2": (lambda: cube_mesh(3, 2, 2), "paper", 2),
    "voronoi20_k2": (lambda: voronoi_mesh(20, seed=8), "paper", 2),
}


def _gpu(mesh, family, k, nu, sol):
    import torch

    from paper_1901_02330_amd.vem import Solver

    s = Solver()
    s.set_mesh(mesh)
    s.discretize(family, k=k, load_points=3)
    s.set_boundary("flux")
    if nu is not None:
        s.set_coefficient(torch.as_tensor(nu, dtype=torch.float64))

    def u(X):  # the test solutions' flux fields are NumPy code
        return torch.as_tensor(sol.u(X.cpu().numpy()), dtype=torch.float64, device=X.device)

    s.set_rhs_functions(sol.f, u)
    return s


def _blocks(d):
    """S and A_gamma of the oracle's flux system."""
    Nu = d["Nu"]
    K = d["K_t"]
    M = K[:Nu, :Nu]
    B = K[Nu:, :Nu]
    S = (B @ sp.diags(1.0 / M.diagonal()) @ B.T).tocsr()
    return M, B, S


@pytest.mark.parametrize("case", list(CASES))
def test_flux_matrices_and_rhs(case):
    _say("flux matrices", case)
    mk, fam, k = CASES[case]
    m = mk()
    nc = len(m["cell_ptr"]) - 1
    nu = 1.0 / lognormal_field(nc, 1.0, 2)
    s = _gpu(m, fam, k, nu, SineSolution())
    d = flux_system(m, nu=nu, rhs=SineSolution(), family=fam, k=k)
    rtol = 1e-13 if fam == "lo" else 1e-11
    N = d["Nu"] + d["Np"]
    assert_same_csr(to_scipy(*s.export_csr("K"), (N, N)), d["K_t"], rtol)
    M, B, S = _blocks(d)
    assert_same_csr(to_scipy(*s.export_csr("schur"), (d["Np"], d["Np"])), S, rtol)
    gam = s.sizes()["gamma"]
    A = (M + B.T @ B / gam).tocsr()
    assert_same_csr(to_scipy(*s.export_csr("reg"), (d["Nu"], d["Nu"])), A, rtol)
    b = s.rhs().cpu().numpy()
    assert np.abs(b - d["b_t"]).max() <= rtol * np.abs(d["b_t"]).max()
    assert s.sizes()["n"] + 1 == d["n_paper"]


@pytest.mark.parametrize("precond", ["schur", "reg"])
@pytest.mark.parametrize("case", ["cube534_lo", "voronoi60_lo", "cube322_k2"])
def test_flux_solve_matches_oracle(case, precond):
    _say("flux solve", case, precond)
    mk, fam, k = CASES[case]
    m = mk()
    nc = len(m["cell_ptr"]) - 1
    nu = 1.0 / lognormal_field(nc, 1.0, 4)
    s = _gpu(m, fam, k, nu, SineSolution())
    u, p, info = s.solve(precond=precond, tol=1e-13, maxit=3000, inner_tol=1e-10)
    _say(info)
    d = flux_system(m, nu=nu, rhs=SineSolution(), family=fam, k=k)
    uo, po, lam = solve_flux(d)
    u, p = u.cpu().numpy(), p.cpu().numpy()
    eu = np.linalg.norm(u - uo) / np.linalg.norm(uo)
    ep = np.linalg.norm(p - po) / np.linalg.norm(po)
    _say("rel err u", eu, "p", ep, "mean", d["w"] @ p, "multiplier", lam)
    assert info["converged"]
    assert eu < 1e-10 and ep < 1e-10
    assert abs(d["w"] @ p) <= 1e-12 * np.abs(d["w"]).sum() * np.abs(po).max()


@pytest.mark.parametrize("case", ["cube534_lo", "voronoi60_lo", "cube322_k1", "cube322_k2"])
def test_flux_patch_test_on_gpu(case):
    from oracle.assemble import interpolate_lo
    from oracle.paperk import interpolate_paper

    _say("flux patch", case)
    mk, fam, k = CASES[case]
    m = mk()
    sol = LinearSolution(0.4, (1.0, -0.5, 2.0)) if fam == "lo" else _Poly(k)
    s = _gpu(m, fam, k, None, sol)
    u, p, info = s.solve(precond="reg", tol=1e-13, maxit=3000, inner_tol=1e-10)
    d = flux_system(m, rhs=sol, family=fam, k=k)
    if fam == "lo":
        ue, pe = interpolate_lo(m, d["fgeo"], d["cgeo"], sol)
    else:
        ue, pe = interpolate_paper(m, d, sol)
    pe = pe - d["n_p"] * (d["w"] @ pe) / (d["w"] @ d["n_p"])
    assert np.abs(u.cpu().numpy() - ue).max() < 1e-9 * max(1.0, np.abs(ue).max())
    assert np.abs(p.cpu().numpy() - pe).max() < 1e-9 * max(1.0, np.abs(pe).max())


def test_adjoint_rejected_with_flux_data():
    """The adjoint entry points take pressure data only: with flux data K is singular and its
    prescribed rows fix the boundary DOFs, so vem_solve_rhs and vem_coefficient_gradient return
    VEM_EINVAL, and the autograd path raises before solving."""
    import torch

    from paper_1901_02330_amd.adjoint import solve_logk
    from paper_1901_02330_amd.vem import VemError

    _say("flux adjoint rejected")
    m = cube_mesh(3)
    s = _gpu(m, "lo", 0, None, SineSolution())
    sz = s.sizes()
    u, p, info = s.solve(precond="schur", tol=1e-10)
    assert info["converged"]
    with pytest.raises(VemError) as e:
        s.solve(rhs=torch.ones(sz["n"], dtype=torch.float64, device=u.device))
    assert e.value.code == -1 and "pressure boundary data" in str(e.value)
    with pytest.raises(VemError) as e:
        s.coefficient_gradient(u, u)
    assert e.value.code == -1
    with pytest.raises(ValueError):
        solve_logk(s, torch.zeros(sz["n_cells"], dtype=torch.float64, device=u.device), tol=1e-10)
