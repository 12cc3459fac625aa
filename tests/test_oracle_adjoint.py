"""Pin of the oracle's adjoint gradient against central finite differences of the misfit."""
import numpy as np
import pytest

from oracle.adjoint import misfit_gradient
from oracle.assemble import discretize
from oracle.solvers import direct_solve
from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, voronoi_mesh


@pytest.mark.parametrize("family", ["lo", "paper"])
def test_adjoint_matches_central_differences(family):
    m = cube_mesh(3) if family == "lo" else voronoi_mesh(10, seed=2)
    nc = len(m["cell_ptr"]) - 1
    rng = np.random.default_rng(0)
    theta = rng.standard_normal(nc)
    kw = {"family": family, "k": 2} if family == "paper" else {}
    d = discretize(m, nu=np.exp(-theta), rhs=SineSolution(), **kw)
    p_obs = rng.standard_normal(d["Np"]) * 0.01
    J, g, x, lam = misfit_gradient(m, d, p_obs)
    step = 1e-6
    for P in rng.choice(nc, size=min(6, nc), replace=False):
        Js = []
        for sgn in (1, -1):
            th = theta.copy()
            th[P] += sgn * step
            dd = discretize(m, nu=np.exp(-th), rhs=SineSolution(), local=d["local"], geo=(d["fgeo"], d["cgeo"]), **kw)
            xx = direct_solve(dd["K"], dd["b"])
            Js.append(0.5 * np.sum((xx[dd["Nu"]:] - p_obs) ** 2))
        fd = (Js[0] - Js[1]) / (2 * step)
        assert fd == pytest.approx(g[P], rel=1e-6, abs=1e-9 * abs(g).max())
