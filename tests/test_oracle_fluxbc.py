"""Pins of the flux-boundary-data oracle (the paper's model problem, Section 3 eq. mod_prob_eq):
  * patch test: with u_N from a solution whose flux lies in the discrete space, the discrete flux is
    the interpolant and the discrete pressure is the interpolant shifted to zero mean (lowest order
    with a linear pressure; the paper's k = 1, 2 with pressures in P_{k+1}), on Cube and Voronoi meshes;
  * the zero-mean constraint holds, and its multiplier is zero (the right-hand side is consistent);
  * the unknown count plus the multiplier equals the DOF count the paper prints (Table 4, 512 cells);
  * the discrete constant pressure n_p is in the kernel of B^T on the free flux DOFs."""
import json
import os

import numpy as np
import pytest

from oracle.assemble import interpolate_lo
from oracle.fluxbc import flux_system, solve_flux
from oracle.paperk import interpolate_paper
from paper_1901_02330_amd.inputs import LinearSolution, cube_mesh, lognormal_field, voronoi_mesh
from tests.test_oracle_paperk import _Poly


def _mesh(name):
    return cube_mesh(4, 3, 3) if name == "cube" else voronoi_mesh(30, seed=5)


def _zero_mean(p, d):
    return p - d["n_p"] * (d["w"] @ p) / (d["w"] @ d["n_p"])


@pytest.mark.parametrize("name", ["cube", "voronoi"])
def test_lowest_order_patch(name):
    m = _mesh(name)
    sol = LinearSolution(0.4, (1.0, -0.5, 2.0))
    d = flux_system(m, rhs=sol)
    u, p, lam = solve_flux(d)
    ue, pe = interpolate_lo(m, d["fgeo"], d["cgeo"], sol)
    assert np.abs(u - ue).max() < 1e-12 * np.abs(ue).max()
    assert np.abs(p - _zero_mean(pe, d)).max() < 1e-12 * np.abs(pe).max()
    assert abs(d["w"] @ p) < 1e-12 * np.abs(d["w"]).sum() * np.abs(pe).max()
    assert abs(lam) < 1e-12


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("name", ["cube", "voronoi"])
def test_paper_element_patch(name, k):
    m = cube_mesh(3, 2, 2) if name == "cube" else voronoi_mesh(12, seed=3)
    sol = _Poly(k)
    d = flux_system(m, rhs=sol, family="paper", k=k)
    u, p, lam = solve_flux(d)
    ue, pe = interpolate_paper(m, d, sol)
    assert np.abs(u - ue).max() < 1e-10
    assert np.abs(p - _zero_mean(pe, d)).max() < 1e-10
    assert abs(lam) < 1e-10


def test_constant_pressure_is_in_the_kernel():
    m = voronoi_mesh(25, seed=2)
    nc = len(m["cell_ptr"]) - 1
    for fam, k in (("lo", 0), ("paper", 2)):
        d = flux_system(m, nu=1.0 / lognormal_field(nc, 1.0, 0), rhs=_Poly(2), family=fam, k=k)
        free = np.ones(d["Nu"], dtype=bool)
        free[d["bdofs"]] = False
        r = d["B"].T @ d["n_p"]
        assert np.abs(r[free]).max() < 1e-13 * np.abs(d["B"]).max()
        assert np.abs(d["n_p"] @ d["b_t"][d["Nu"]:]) < 1e-12 * np.abs(d["b_t"]).max()


def test_unknowns_plus_multiplier_equal_the_papers_count():
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_dof_counts.json")))
    row = next(r for r in golden["cube"] if r["cells"] == 512)
    d = flux_system(cube_mesh(8), rhs=_Poly(2), family="paper", k=row["k"])
    assert d["n_paper"] == row["dofs"]
