"""The Chebyshev-Jacobi inner form (a fixed polynomial in D^{-1}A, no reductions) under FGMRES:
Block-Schur solves to 1e-13 against the oracle's direct solve (relative 1e-10 in u and p), FP64 and
with FP32 inner products (to 1e-10, within 1e-7), on Cube and Voronoi meshes; the flux boundary data
(S singular, the constant pressure in its kernel); and the argument checks."""
import sys

import numpy as np
import pytest

from oracle.assemble import discretize
from oracle.solvers import direct_solve
from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field, voronoi_mesh
from tests.gpu_helpers import gpu_solver, rel

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# The three row forms of the products of S: cube675 (every slice of S padded to 7 entries per row:
# the fixed-count form), cubeslab (one layer of cells, at most 5 entries per row: the masked
# short-row form) and voronoi150 (longer rows: the loop).
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["cube675", "cubeslab", "voronoi150"])
def test_chebyshev_schur_solve_matches_oracle(name, precision):
    _say("chebyshev", name, precision)
    meshes = {"cube675": lambda: cube_mesh(6, 7, 5), "cubeslab": lambda: cube_mesh(16, 12, 1),
              "voronoi150": lambda: voronoi_mesh(150, seed=0)}
    m = meshes[name]()
    nc = len(m["cell_ptr"]) - 1
    nu = 1.0 / lognormal_field(nc, 2.0, 0)
    s = gpu_solver(m, nu=nu, rhs=SineSolution())
    tol = 1e-13 if precision == "fp64" else 1e-10
    u, p, info = s.solve(precond="schur", tol=tol, maxit=3000, inner_form="chebyshev", inner_maxit=24,
                         cheb_lo=1.0 / 400, precision=precision)
    assert info["converged"], info
    assert info["inner_iterations"] == 24 * info["iterations"] or info["inner_iterations"] > 0
    d = discretize(m, nu=nu, rhs=SineSolution())
    x = direct_solve(d["K"], d["b"])
    xg = np.concatenate([u.cpu().numpy(), p.cpu().numpy()])
    berr = np.linalg.norm(d["b"] - d["K"] @ xg) / np.linalg.norm(d["b"])
    eu, ep = rel(xg[: d["Nu"]], x[: d["Nu"]]), rel(xg[d["Nu"]:], x[d["Nu"]:])
    _say(info, berr, eu, ep)
    assert berr <= 1.5 * tol
    bound = 1e-10 if precision == "fp64" else 1e-7
    assert eu <= bound and ep <= bound


def test_pipelined_schur_on_short_rows_matches_oracle():
    """The pipelined Jacobi-CG on S in its masked short-row form (one layer of cells, at most 5
    entries per row of S) against the oracle's direct solve."""
    _say("pipelined cubeslab")
    m = cube_mesh(16, 12, 1)
    nu = 1.0 / lognormal_field(192, 2.0, 1)
    s = gpu_solver(m, nu=nu, rhs=SineSolution())
    u, p, info = s.solve(precond="schur", tol=1e-13, maxit=3000, inner_tol=1e-8, inner_maxit=200)
    assert info["converged"], info
    d = discretize(m, nu=nu, rhs=SineSolution())
    x = direct_solve(d["K"], d["b"])
    xg = np.concatenate([u.cpu().numpy(), p.cpu().numpy()])
    eu, ep = rel(xg[: d["Nu"]], x[: d["Nu"]]), rel(xg[d["Nu"]:], x[d["Nu"]:])
    _say(info, eu, ep)
    assert eu <= 1e-10 and ep <= 1e-10


def test_chebyshev_rejects_bad_interval():
    from paper_1901_02330_amd.vem import VemError

    m = cube_mesh(3)
    s = gpu_solver(m, nu=np.ones(27), rhs=SineSolution())
    with pytest.raises(VemError) as e:
        s.solve(precond="schur", inner_form="chebyshev", inner_maxit=24, cheb_lo=1.5)
    assert e.value.code == -1


def test_chebyshev_with_flux_boundary_data():
    """With the paper's flux boundary data S has the constant pressure in its kernel; the Chebyshev
    polynomial then leaves a constant component in z_p, which the zero-mean shift of the result
    removes: the solution matches the oracle's augmented direct solve."""
    import torch

    from oracle.fluxbc import flux_system, solve_flux
    from paper_1901_02330_amd.vem import Solver

    _say("chebyshev flux data")
    m = cube_mesh(5, 3, 4)
    nu = 1.0 / lognormal_field(60, 2.0, 4)
    s = Solver()
    s.set_mesh(m)
    s.discretize("lo", load_points=3)
    s.set_boundary("flux")
    s.set_coefficient(torch.as_tensor(nu))

    def ufield(X):
        return torch.as_tensor(SineSolution.u(X.cpu().numpy()), dtype=torch.float64, device=X.device)

    s.set_rhs_functions(SineSolution.f, ufield)
    u, p, info = s.solve(precond="schur", tol=1e-13, maxit=3000, inner_form="chebyshev", inner_maxit=24)
    assert info["converged"], info
    d = flux_system(m, nu=nu, rhs=SineSolution())
    uo, po = solve_flux(d)[:2]
    eu, ep = rel(u.cpu().numpy(), uo), rel(p.cpu().numpy(), po)
    _say(info, eu, ep)
    assert eu <= 1e-10 and ep <= 1e-10


@pytest.mark.parametrize("which", ["spmv", "cg_schur", "cg_reg", "cg_schur32", "cg_reg32", "cg_schur32p",
                                   "cg_reg32p", "cg_reg_schwarz", "cg_reg_schwarz32", "cheb_schur",
                                   "cheb_schur32"])
def test_time_kernel_hook(which):
    """Every kernel of the timing hook runs, with a positive time and its algorithmic bytes, and leaves
    a later solve unchanged."""
    m = cube_mesh(6, 5, 4)
    nu = 1.0 / lognormal_field(120, 1.0, 1)
    s = gpu_solver(m, nu=nu, rhs=SineSolution())
    u0, p0, _ = s.solve(precond="reg", tol=1e-12)
    ms, nbytes = s.time_kernel(which, reps=5)
    assert ms > 0 and nbytes > 0
    u1, p1, _ = s.solve(precond="reg", tol=1e-12)
    import torch

    assert torch.equal(u0, u1) and torch.equal(p0, p1)
