"""Pins of the assembled system and the solvers: patch test, mass conservation,
convergence, direct vs iterative, ideal block-preconditioner spectrum."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.assemble import discretize, interpolate_lo
from oracle.solvers import block_reg, block_schur, direct_solve, fgmres
from paper_1901_02330_amd.inputs import (LinearSolution, SineSolution, cube_mesh, lognormal_field,
                                         voronoi_mesh)


@pytest.mark.parametrize("mesh", ["cube", "cube345", "voronoi"])
def test_patch_linear_pressure_exact(mesh):
    m = {"cube": lambda: cube_mesh(4), "cube345": lambda: cube_mesh(3, 4, 5),
         "voronoi": lambda: voronoi_mesh(30, seed=2)}[mesh]()
    sol = LinearSolution(0.3, (1.0, -2.0, 0.5))
    d = discretize(m, rhs=sol)
    x = direct_solve(d["K"], d["b"])
    ue, pe = interpolate_lo(m, d["fgeo"], d["cgeo"], sol)
    assert np.abs(x[: d["Nu"]] - ue).max() < 1e-12
    assert np.abs(x[d["Nu"]:] - pe).max() < 1e-12


def test_symmetry_and_mass_conservation():
    m = voronoi_mesh(30, seed=5)
    nu = 1.0 / lognormal_field(30, 1.0, 0)
    d = discretize(m, nu=nu, rhs=SineSolution())
    K = d["K"]
    assert abs(K - K.T).max() < 1e-15
    x = direct_solve(K, d["b"])
    # B_div u = F per cell
    r = d["Bdiv"] @ x[: d["Nu"]] - d["F"]
    assert np.abs(r).max() < 1e-12 * np.abs(d["F"]).max()


def test_dense_lu_equals_sparse_and_fgmres():
    m = cube_mesh(3)
    d = discretize(m, nu=1.0 / lognormal_field(27, 2.0, 0), rhs=SineSolution())
    K = d["K"].toarray()
    xd = np.linalg.solve(K, d["b"])
    xs = direct_solve(d["K"], d["b"])
    assert np.linalg.norm(xd - xs) <= 1e-12 * np.linalg.norm(xd)
    assert np.linalg.svd(K, compute_uv=False).min() > 0  # unique discrete solution
    for prec in (block_schur(d["M"], d["B"]), block_reg(d["M"], d["B"], d["cgeo"]["h"] ** 2),
                 block_schur(d["M"], d["B"], inner="pcg", tol=1e-8)):
        x, info = fgmres(d["K"], d["b"], prec, m=30, tol=1e-13)
        assert info["converged"]
        assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


def test_ideal_block_diagonal_three_iterations():
    # with the exact M^{-1} and the exact Schur complement B M^{-1} B^T the
    # block-diagonal preconditioned saddle matrix has three eigenvalues,
    # 1 and (1 +- sqrt 5)/2, so (F)GMRES ends in at most three iterations
    m = cube_mesh(3)
    d = discretize(m, nu=1.0 / lognormal_field(27, 1.0, 1), rhs=SineSolution())
    M = d["M"].toarray()
    B = d["B"].toarray()
    S = B @ np.linalg.solve(M, B.T)
    Nu = d["Nu"]
    prec = lambda r: np.concatenate([np.linalg.solve(M, r[:Nu]), np.linalg.solve(S, r[Nu:])])  # noqa: E731
    x, info = fgmres(d["K"], d["b"], prec, m=30, tol=1e-10)
    assert info["iterations"] <= 3
    P = np.block([[np.linalg.inv(M), np.zeros((Nu, S.shape[0]))], [np.zeros((S.shape[0], Nu)), np.linalg.inv(S)]])
    ev = np.linalg.eigvals(P @ d["K"].toarray())
    targets = np.array([1.0, (1 + 5**0.5) / 2, (1 - 5**0.5) / 2])
    assert np.abs(ev[:, None] - targets[None]).min(1).max() < 1e-8


def test_convergence_rates_sine():
    errs, hs = [], []
    for n in (4, 8, 16):
        m = cube_mesh(n)
        d = discretize(m, rhs=SineSolution())
        x = direct_solve(d["K"], d["b"])
        ue, pe = interpolate_lo(m, d["fgeo"], d["cgeo"], SineSolution())
        vol = d["cgeo"]["volume"]
        ep = np.sqrt((vol * (x[d["Nu"]:] - pe) ** 2).sum()) / np.sqrt((vol * pe**2).sum())
        eu = np.linalg.norm(x[: d["Nu"]] - ue) / np.linalg.norm(ue)
        errs.append((ep, eu))
        hs.append(d["cgeo"]["h"])
    rates = np.log(np.array(errs[:-1]) / np.array(errs[1:])) / np.log(np.array(hs[:-1]) / np.array(hs[1:]))[:, None]
    assert rates.min() >= 0.8  # lowest order: O(h) at least


def test_block_preconditioners_mass_matrix_scaling():
    # Block-Schur's S is B diag(M)^-1 B^T: on cubes a 7-point operator whose
    # off-diagonals are -(4h/3)/(nu_L + nu_R) (diag(M) interior = 3/4 h^3 (nu_L + nu_R))
    n = 4
    m = cube_mesh(n)
    nu = 1.0 / lognormal_field(n**3, 1.0, 4)
    d = discretize(m, nu=nu)
    S = block_schur(d["M"], d["B"]).S.tocoo()
    h = 1.0 / n
    off = S.row != S.col
    expect = -(4 * h / 3) / (nu[S.row[off]] + nu[S.col[off]])
    assert np.allclose(S.data[off], expect, rtol=1e-12)
    assert sp.csr_matrix(S).nnz == n**3 + 2 * 3 * n * n * (n - 1)
