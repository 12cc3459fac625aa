"""GPU adjoint gradient dJ/d(log K) (hand-written adjoint behind torch.autograd) against the
oracle's adjoint and against central finite differences."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("family", ["lo", "paper"])
def test_adjoint_gradient_matches_oracle(family):
    import torch

    from oracle.adjoint import misfit_gradient
    from oracle.assemble import discretize
    from paper_1901_02330_amd.adjoint import solve_logk
    from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, voronoi_mesh
    from paper_1901_02330_amd.vem import Solver

    _say("adjoint vs oracle", family)
    m = cube_mesh(4, 3, 5) if family == "lo" else voronoi_mesh(12, seed=4)
    nc = len(m["cell_ptr"]) - 1
    rng = np.random.default_rng(0)
    theta = rng.standard_normal(nc)
    kw = {"family": "paper", "k": 2} if family == "paper" else {}
    d = discretize(m, nu=np.exp(-theta), rhs=SineSolution(), **kw)
    p_obs = 0.01 * rng.standard_normal(d["Np"])
    J_or, g_or, _, _ = misfit_gradient(m, d, p_obs)
    s = Solver()
    s.set_mesh(m)
    s.discretize(*(("paper", 2) if family == "paper" else ("lo", 0)))
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    logk = torch.tensor(theta, dtype=torch.float64, device="cuda", requires_grad=True)
    u, p = solve_logk(s, logk, precond="reg" if family == "paper" else "schur", tol=1e-13, inner_tol=1e-10,
                      maxit=4000)
    J = 0.5 * torch.sum((p - torch.as_tensor(p_obs, device="cuda")) ** 2)
    J.backward()
    g = logk.grad.cpu().numpy()
    _say("J", float(J), J_or, "max rel grad diff", np.abs(g - g_or).max() / np.abs(g_or).max())
    assert float(J) == pytest.approx(J_or, rel=1e-9)
    assert np.abs(g - g_or).max() <= 1e-8 * np.abs(g_or).max()


def test_adjoint_vs_finite_differences_cube48():
    """Cube 48^3, lowest order, log K ~ N(0, 1) (seed 0), p_obs from a second field (seed 1),
    J = 1/2 ||p - p_obs||^2; central differences with step 1e-6 on 20 cells (seed 2)."""
    import time

    import torch

    from paper_1901_02330_amd.adjoint import solve_logk
    from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field
    from paper_1901_02330_amd.vem import Solver

    n = 48
    m = cube_mesh(n)
    nc = n**3
    theta = np.log(lognormal_field(nc, 1.0, 0))
    theta_obs = np.log(lognormal_field(nc, 1.0, 1))
    s = Solver()
    s.set_mesh(m)
    s.discretize("lo")
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    kw = dict(precond="schur", tol=1e-13, inner_tol=1e-8, maxit=5000)
    s.set_coefficient(torch.as_tensor(np.exp(-theta_obs)))
    _, p_obs, _ = s.solve(**kw)
    logk = torch.tensor(theta, dtype=torch.float64, device="cuda", requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, p = solve_logk(s, logk, **kw)
    J = 0.5 * torch.sum((p - p_obs) ** 2)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g = logk.grad.cpu().numpy()
    _say(f"forward {t1 - t0:.3f}s backward {t2 - t1:.3f}s ratio {(t2 - t1) / (t1 - t0):.2f}")
    cells = np.random.default_rng(2).choice(nc, 20, replace=False)
    h = 1e-6
    fd = []
    for P in cells:
        Js = []
        for sg in (1.0, -1.0):
            th = theta.copy()
            th[P] += sg * h
            s.set_coefficient(torch.as_tensor(np.exp(-th)))
            _, pp, info = s.solve(**kw)
            assert info["converged"]
            Js.append(0.5 * float(torch.sum((pp - p_obs) ** 2)))
        fd.append((Js[0] - Js[1]) / (2 * h))
    fd = np.array(fd)
    err = np.abs(fd - g[cells]) / np.abs(g[cells]).max()
    _say("adjoint", g[cells][:5], "fd", fd[:5], "max rel err", err.max())
    assert err.max() <= 1e-4
    assert (t2 - t1) <= 2.5 * (t1 - t0)
