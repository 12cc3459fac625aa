"""Pins of the oracle's order-k element (Sections 2 and 4): dimension counts against the paper's
tables, the polynomial decomposition identities, projector and consistency checks, the patch test
and convergence rates."""
import json
import os

import numpy as np
import pytest

from oracle.geometry import cell_geometry, face_geometry
from oracle.paperk import (counts, cross_set, decompose, dim_Gplus, discretize_paper, exps3,
                           interpolate_paper, local_element, paper_dofs)
from oracle.solvers import direct_solve
from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, voronoi_mesh
from tests.meshes import single_prism, single_tet

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_dof_counts.json")


def test_dof_counts_reproduce_the_papers_tables():
    g = json.load(open(GOLDEN))
    for row in g["cube"]:
        n = round(row["cells"] ** (1 / 3))
        assert n**3 == row["cells"]
        assert paper_dofs(3 * n * n * (n + 1), row["cells"], row["k"]) == row["dofs"], row
    # Octa/CVT: the face count is not printed; it must come out integral and agree between
    # the tables that list the same mesh at two orders
    for fam in ("octa", "cvt"):
        nf = {}
        for row in g[fam]:
            nfd, ng, nc, npd = counts(row["k"])
            rest = row["dofs"] - 1 - (ng + nc + npd) * row["cells"]
            assert rest % nfd == 0, row
            nf.setdefault(row["cells"], set()).add(rest // nfd)
        assert all(len(v) == 1 for v in nf.values())
        assert any(True for c, v in nf.items())


def test_cross_set_dimension_and_rank():
    # dim G+_k = (2k^3 + 9k^2 + 7k)/6: 0, 3, 11, 26, 50 (eq. dimGperp, Prop. dimMAndG)
    assert [dim_Gplus(k) for k in range(5)] == [0, 3, 11, 26, 50]
    rng = np.random.default_rng(0)
    X = rng.standard_normal((400, 3))
    for k in range(1, 5):
        S = cross_set(k)
        assert len(S) == dim_Gplus(k)
        cols = []
        for d, mu in S:
            m = X[:, 0] ** mu[0] * X[:, 1] ** mu[1] * X[:, 2] ** mu[2]
            e = np.zeros_like(X)
            e[:, d] = m
            cols.append(np.cross(X, e).ravel())
        # m_I x m over the set is linearly independent: the image spans G+_k
        assert np.linalg.matrix_rank(np.array(cols).T, tol=1e-9) == dim_Gplus(k)


def test_decomposition_identities():
    # e_c m_alpha = g grad m_beta + sum coef m_I x (e_d m_mu)  (Props. xDec, yDec, zDec,
    # inTermsOfGPerpBasis), checked pointwise, h_P = 0.37
    rng = np.random.default_rng(1)
    X = rng.standard_normal((50, 3))
    h = 0.37
    mono = lambda a, Y: Y[:, 0] ** a[0] * Y[:, 1] ** a[1] * Y[:, 2] ** a[2]  # noqa: E731
    for k in (1, 2, 3):
        keep = set(cross_set(k))
        for c in range(3):
            for al in exps3(k):
                g, beta, terms = decompose(c, al, h)
                grad = np.zeros_like(X)
                for i in range(3):
                    if beta[i] > 0:
                        b = list(beta)
                        b[i] -= 1
                        grad[:, i] = beta[i] / h * mono(b, X)
                rhs = g * grad
                for coef, d, mu in terms:
                    assert (d, mu) in keep
                    e = np.zeros_like(X)
                    e[:, d] = mono(mu, X)
                    rhs = rhs + coef * np.cross(X, e)
                lhs = np.zeros_like(X)
                lhs[:, c] = mono(al, X)
                assert np.allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("cell", ["tet", "prism", "voronoi"])
def test_local_projector_and_forms(k, cell):
    rng = np.random.default_rng(k)
    m = {"tet": lambda: single_tet(rng.random((4, 3))), "prism": lambda: single_prism(0.6),
         "voronoi": lambda: voronoi_mesh(6, seed=k)}[cell]()
    fg, cg = face_geometry(m), cell_geometry(m)
    loc = local_element(m, fg, cg, 0, k)
    n3 = loc["D"].shape[1]
    # projector reproduces [P_k]^3, up to the conditioning of the monomial Gram matrix
    tol = max(1e-12, 10 * np.finfo(float).eps * np.linalg.cond(loc["G"]))
    assert np.abs(loc["PiStar"] @ loc["D"] - np.eye(n3)).max() < tol
    M1 = loc["M1"]
    assert np.abs(M1 - M1.T).max() <= 1e-12 * np.abs(M1).max()
    assert np.linalg.eigvalsh(M1).min() > 0
    # consistency: d(p)^T M_P d(q) = int p . q on [P_k]^3 (G = I (x) H_k)
    assert np.abs(loc["D"].T @ M1 @ loc["D"] - loc["G"]).max() <= max(1e-11, tol) * np.abs(loc["G"]).max()
    nfd, ng, nc, npd = counts(k)
    assert M1.shape[0] == len(loc["faces"]) * nfd + ng + nc


class _Poly:
    """p in P_{k+1}, u = -grad p, f = div u: the discrete solution is exact (patch test)."""

    def __init__(self, k):
        self.k = k

    def p(self, X):
        x, y, z = X[..., 0], X[..., 1], X[..., 2]
        v = 0.5 + x - 2 * y + 0.3 * z + x * y - 0.5 * z * z
        if self.k >= 2:
            v = v + x * y * z + 0.25 * y**3
        if self.k >= 3:
            v = v + 0.2 * x * x * y * y - 0.1 * x * z**3
        return v

    pD = p

    def u(self, X):
        x, y, z = X[..., 0], X[..., 1], X[..., 2]
        g = np.stack([1 + y + 0 * x, -2 + x, 0.3 - z], -1)
        if self.k >= 2:
            g = g + np.stack([y * z, x * z + 0.75 * y**2, x * y], -1)
        if self.k >= 3:
            g = g + np.stack([0.4 * x * y * y - 0.1 * z**3, 0.4 * x * x * y, -0.3 * x * z * z], -1)
        return -g

    def f(self, X):
        y = X[..., 1]
        v = 1.0 + 0 * y
        if self.k >= 2:
            v = v - 1.5 * y
        if self.k >= 3:
            x, z = X[..., 0], X[..., 2]
            v = v - 0.4 * y * y - 0.4 * x * x + 0.6 * x * z
        return v


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("mesh", ["cube", "voronoi"])
def test_patch_test(k, mesh):
    m = cube_mesh(2, 3, 2) if mesh == "cube" else voronoi_mesh(12, seed=3)
    sol = _Poly(k)
    # boundary data p_D in P_{k+1} against face monomials of degree k: the load rule must be exact
    # to degree 2k + 1, i.e. k + 1 points per direction; k + 2 leaves one to spare
    d = discretize_paper(m, rhs=sol, k=k, nq_load=max(3, k + 2))
    x = direct_solve(d["K"], d["b"])
    ue, pe = interpolate_paper(m, d, sol)
    assert np.abs(x[: d["Nu"]] - ue).max() < 1e-10
    assert np.abs(x[d["Nu"]:] - pe).max() < 1e-11


def test_convergence_rates():
    from oracle.paperk import _cell_quadrature, exps3 as e3, mono3

    for k, ns in ((1, (2, 4, 8)), (2, (2, 4))):
        errs, hs = [], []
        for n in ns:
            m = cube_mesh(n)
            d = discretize_paper(m, rhs=SineSolution(), k=k)
            x = direct_solve(d["K"], d["b"])
            cg, nfd, nint, npd = d["cgeo"], d["nfd"], d["nint"], d["npd"]
            nf = len(m["face_ptr"]) - 1
            Mk, Mk1 = e3(k), e3(k - 1)
            eu = nu_ = eq = nq_ = 0.0
            for P, loc in enumerate(d["local"]):
                X, W = _cell_quadrature(m, cg, P, k + 3)
                F = len(loc["faces"])
                gid = np.concatenate([np.repeat(loc["faces"] * nfd, nfd) + np.tile(np.arange(nfd), F),
                                      nf * nfd + P * nint + np.arange(nint)])
                sg = np.concatenate([np.repeat(loc["sign"], nfd), np.ones(nint)])
                c = loc["PiStar"] @ (x[gid] * sg)
                mk = mono3(X, cg["centroid"][P], cg["diam"][P], Mk)
                Pu = np.stack([mk @ c[i * len(Mk):(i + 1) * len(Mk)] for i in range(3)], -1)
                U = SineSolution.u(X)
                eu += (W * ((U - Pu) ** 2).sum(1)).sum()
                nu_ += (W * (U**2).sum(1)).sum()
                coef = loc["vol"] * np.linalg.solve(loc["Hk1"], x[d["Nu"] + P * npd:d["Nu"] + (P + 1) * npd])
                ph = mono3(X, cg["centroid"][P], cg["diam"][P], Mk1) @ coef
                eq += (W * (SineSolution.p(X) - ph) ** 2).sum()
                nq_ += (W * SineSolution.p(X) ** 2).sum()
            errs.append((np.sqrt(eu / nu_), np.sqrt(eq / nq_)))
            hs.append(cg["h"])
        E, H = np.array(errs), np.array(hs)
        rates = np.log(E[:-1] / E[1:]) / np.log(H[:-1] / H[1:])[:, None]
        assert rates[-1].min() >= k - 0.2, (k, rates)
