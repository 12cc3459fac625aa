"""GPU parity: every step of the HIP path against the FP64 oracle on the same seeded inputs."""
import sys

import numpy as np
import pytest

from oracle.assemble import discretize, interpolate_lo
from oracle.solvers import block_reg, block_schur, direct_solve
from paper_1901_02330_amd.inputs import (LinearSolution, SineSolution, cube_mesh, lognormal_field,
                                         voronoi_mesh)
from tests.gpu_helpers import assert_same_csr, gpu_solver, rel, to_scipy
from tests.meshes import single_prism, single_tet

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


TET = [[0.1, 0.0, 0.0], [1.0, 0.2, 0.0], [0.0, 1.0, 0.1], [0.2, 0.1, 0.9]]

MESHES = {
    "cube8": lambda: cube_mesh(8),
    "cube534": lambda: cube_mesh(5, 3, 4),
    "voronoi80": lambda: voronoi_mesh(80, seed=4),
    # degenerate sizes: one cell, every face on the boundary
    "tet1": lambda: single_tet(TET),
    "prism1": lambda: single_prism(0.7),
}


@pytest.mark.parametrize("name", list(MESHES))
def test_geometry(name):
    _say("geometry", name)
    m = MESHES[name]()
    s = gpu_solver(m)
    g = {k: v.cpu().numpy() for k, v in s.geometry().items()}
    d = discretize(m)
    fg, cg = d["fgeo"], d["cgeo"]
    assert np.allclose(g["area"], fg["area"], rtol=1e-13, atol=0)
    assert np.allclose(g["normal"], fg["normal"], rtol=0, atol=1e-14)
    assert np.allclose(g["fcentroid"], fg["centroid"], rtol=0, atol=1e-14)
    assert np.allclose(g["volume"], cg["volume"], rtol=1e-13, atol=0)
    assert np.allclose(g["centroid"], cg["centroid"], rtol=0, atol=1e-14)
    assert np.allclose(g["diam"], cg["diam"], rtol=1e-14, atol=0)
    sz = s.sizes()
    assert sz["h"] == pytest.approx(cg["h"], rel=1e-14)


@pytest.mark.parametrize("name", list(MESHES))
def test_matrices_and_rhs(name):
    _say("matrices", name)
    m = MESHES[name]()
    nc = len(m["cell_ptr"]) - 1
    nu = 1.0 / lognormal_field(nc, 2.0, 0)
    sol = LinearSolution(0.25, (0.5, -1.0, 2.0))
    s = gpu_solver(m, nu=nu, rhs=sol)
    d = discretize(m, nu=nu, rhs=sol)
    N = d["Nu"] + d["Np"]
    G = to_scipy(*s.export_csr("K"), (N, N))
    assert_same_csr(G, d["K"])
    Sg = to_scipy(*s.export_csr("schur"), (d["Np"], d["Np"]))
    assert_same_csr(Sg, block_schur(d["M"], d["B"]).S)
    gam = s.sizes()["gamma"]
    Ag = to_scipy(*s.export_csr("reg"), (d["Nu"], d["Nu"]))
    assert_same_csr(Ag, block_reg(d["M"], d["B"], gam, inner="pcg").A)
    b = s.rhs().cpu().numpy()
    assert np.abs(b - d["b"]).max() <= 1e-13 * np.abs(d["b"]).max()
    # sine load (non-polynomial f): same rule on both sides
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    d2 = discretize(m, nu=nu, rhs=SineSolution(), local=d["local"], geo=(d["fgeo"], d["cgeo"]))
    b = s.rhs().cpu().numpy()
    assert np.abs(b - d2["b"]).max() <= 1e-13 * np.abs(d2["b"]).max()


def test_spmv():
    import torch

    _say("spmv")
    m = voronoi_mesh(120, seed=9)
    nc = len(m["cell_ptr"]) - 1
    nu = 1.0 / lognormal_field(nc, 1.0, 3)
    s = gpu_solver(m, nu=nu)
    d = discretize(m, nu=nu)
    x = np.random.default_rng(0).standard_normal(d["Nu"] + d["Np"])
    y = s.apply(torch.as_tensor(x)).cpu().numpy()
    yo = d["K"] @ x
    assert np.abs(y - yo).max() <= 1e-13 * np.abs(yo).max()


def test_spmv_on_a_side_stream():
    """A Solver bound to a side stream, called while another stream is current: the product is read on
    the caller's stream right away, with no synchronisation by the caller (the binding orders the two
    streams both ways)."""
    import torch

    from paper_1901_02330_amd.vem import Solver

    _say("spmv side stream")
    m = cube_mesh(12)
    nu = 1.0 / lognormal_field(12**3, 1.0, 4)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        s = Solver()
    s.set_mesh(m)
    s.discretize("lo")
    s.set_coefficient(torch.as_tensor(nu))
    d = discretize(m, nu=nu)
    x = np.random.default_rng(1).standard_normal(d["Nu"] + d["Np"])
    for _ in range(3):
        xt = torch.as_tensor(x, device="cuda") * 2.0  # produced on the current stream
        y = (s.apply(xt) * 0.5).cpu().numpy()  # consumed on the current stream
        yo = d["K"] @ x
        assert np.abs(y - yo).max() <= 1e-13 * np.abs(yo).max()


@pytest.mark.parametrize("precond", ["schur", "reg"])
@pytest.mark.parametrize("case", ["cube8_K1", "cube675_lognormal", "voronoi150_lognormal", "tet1"])
def test_solve_matches_oracle(case, precond):
    _say("solve", case, precond)
    if case == "cube8_K1":
        m, nu = cube_mesh(8), None
    elif case == "tet1":
        m, nu = single_tet(TET), None
    elif case == "cube675_lognormal":
        m = cube_mesh(6, 7, 5)
        nu = 1.0 / lognormal_field(210, 2.0, 0)
    else:
        m = voronoi_mesh(150, seed=11)
        nu = 1.0 / lognormal_field(150, 1.0, 5)
    s = gpu_solver(m, nu=nu, rhs=SineSolution())
    u, p, info = s.solve(precond=precond, tol=1e-13, maxit=3000, inner_tol=1e-10)
    assert info["converged"], info
    d = discretize(m, nu=nu, rhs=SineSolution())
    x = direct_solve(d["K"], d["b"])
    uo, po = x[: d["Nu"]], x[d["Nu"]:]
    u, p = u.cpu().numpy(), p.cpu().numpy()
    _say(info, rel(u, uo), rel(p, po))
    assert rel(u, uo) <= 1e-10
    assert rel(p, po) <= 1e-10
    # mass conservation B_div u = F per cell
    r = d["Bdiv"] @ u - d["F"]
    assert np.abs(r).max() <= 1e-10 * np.abs(d["F"]).max()


@pytest.mark.parametrize("precond", ["schur", "reg"])
def test_solve_classical_inner_form(precond):
    """The classical (two-kernel) FP64 inner CG: full solves against the oracle's direct solve, and
    the same outer iteration count as the pipelined form within a few iterations."""
    _say("solve classical inner", precond)
    m = cube_mesh(6, 7, 5)
    nu = 1.0 / lognormal_field(210, 2.0, 0)
    s = gpu_solver(m, nu=nu, rhs=SineSolution())
    kw = dict(precond=precond, tol=1e-13, maxit=3000, inner_tol=1e-10)
    u, p, info = s.solve(inner_form="classical", **kw)
    _, _, info_p = s.solve(**kw)
    assert info["converged"], info
    d = discretize(m, nu=nu, rhs=SineSolution())
    x = direct_solve(d["K"], d["b"])
    u, p = u.cpu().numpy(), p.cpu().numpy()
    _say(info, info_p["iterations"], rel(u, x[: d["Nu"]]), rel(p, x[d["Nu"]:]))
    assert rel(u, x[: d["Nu"]]) <= 1e-10
    assert rel(p, x[d["Nu"]:]) <= 1e-10
    assert abs(info["iterations"] - info_p["iterations"]) <= 3


def test_patch_test_exact_on_gpu():
    _say("patch")
    m = voronoi_mesh(60, seed=8)
    sol = LinearSolution(0.1, (2.0, 1.0, -1.0))
    s = gpu_solver(m, rhs=sol)
    u, p, info = s.solve(precond="schur", tol=1e-14, maxit=500, inner_tol=1e-12)
    d = discretize(m)
    ue, pe = interpolate_lo(m, d["fgeo"], d["cgeo"], sol)
    assert np.abs(u.cpu().numpy() - ue).max() < 1e-11
    assert np.abs(p.cpu().numpy() - pe).max() < 1e-11


def test_deterministic_bits():
    import torch

    _say("determinism")
    m = cube_mesh(7)
    nu = 1.0 / lognormal_field(343, 2.0, 1)
    s = gpu_solver(m, nu=nu, rhs=SineSolution())
    u1, p1, _ = s.solve(precond="schur", tol=1e-10)
    u2, p2, _ = s.solve(precond="schur", tol=1e-10)
    assert torch.equal(u1, u2) and torch.equal(p1, p2)


def test_error_paths():
    import torch

    from paper_1901_02330_amd.vem import Solver, VemError

    _say("errors")
    m = cube_mesh(3)
    bad = dict(m)
    bad["cell_face"] = m["cell_face"].copy()
    bad["cell_face"][5] = 10**6  # out of range face id: caught by the validation kernel
    s = Solver()
    with pytest.raises(VemError) as e:
        s.set_mesh(bad)
    assert e.value.code == -2
    # offset arrays are checked on the device before anything is indexed through them
    for key, i, msg in (("face_ptr", 7, "face_ptr not monotone"), ("cell_ptr", 4, "cell_ptr not monotone"),
                        ("cell_ptr", 0, "start at 0")):
        bad = dict(m)
        bad[key] = m[key].copy()
        bad[key][i] = bad[key][i - 1] - 1 if i > 0 else 1
        with pytest.raises(VemError) as e:
            s.set_mesh(bad)
        assert e.value.code == -2 and msg in str(e.value), (key, i, str(e.value))
    # an empty mesh is rejected before anything runs on the device
    empty = {k: m[k][:0] for k in ("xyz", "face_vtx", "cell_face", "cell_face_sign")}
    empty["face_ptr"] = m["face_ptr"][:1]
    empty["cell_ptr"] = m["cell_ptr"][:1]
    with pytest.raises(VemError) as e:
        s.set_mesh(empty)
    assert e.value.code == -1
    # solving before a discretisation is a call-order error
    with pytest.raises(VemError) as e:
        Solver().solve()
    assert e.value.code == -1
    s = gpu_solver(m, rhs=SineSolution())
    u, p, info = s.solve(tol=1e-14, maxit=1)
    assert not info["converged"] and info["iterations"] == 1
    qc, qf = s.quadrature()
    f = torch.full((qc.shape[0],), float("nan"), dtype=torch.float64, device=qc.device)
    s.set_rhs(f)
    with pytest.raises(VemError) as e:
        s.solve()
    assert e.value.code == -6
    # a coefficient that is not positive and finite is rejected on the device, and the previous
    # coefficient stays in place (host and device arrays)
    nu = 1.0 / lognormal_field(27, 1.0, 4)
    s = gpu_solver(m, nu=nu, rhs=SineSolution())
    u0, p0, _ = s.solve(tol=1e-12)
    for v, dev in ((0.0, "cpu"), (-1.0, "cuda"), (float("nan"), "cpu"), (float("inf"), "cuda")):
        nu_bad = nu.copy()
        nu_bad[13] = v
        with pytest.raises(VemError) as e:
            s.set_coefficient(torch.as_tensor(nu_bad, device=dev))
        assert e.value.code == -1 and "positive and finite" in str(e.value), str(e.value)
    u1, p1, _ = s.solve(tol=1e-12)
    assert torch.equal(u0, u1) and torch.equal(p0, p1)


@pytest.mark.parametrize("precond", ["schur", "reg"])
def test_mixed_precision_inner_solves(precond):
    """FP32 inner CG under FP64 FGMRES: the FP64 outer residual test still reaches the tolerance,
    and the solution agrees with the oracle's FP64 direct solve to the tolerance times the
    conditioning of this small system."""
    _say("mixed", precond)
    m = cube_mesh(6, 7, 5)
    nu = 1.0 / lognormal_field(210, 2.0, 0)
    s = gpu_solver(m, nu=nu, rhs=SineSolution())
    u, p, info = s.solve(precond=precond, tol=1e-10, maxit=3000, inner_tol=1e-3, precision="mixed")
    assert info["converged"], info
    d = discretize(m, nu=nu, rhs=SineSolution())
    xg = np.concatenate([u.cpu().numpy(), p.cpu().numpy()])
    berr = np.linalg.norm(d["b"] - d["K"] @ xg) / np.linalg.norm(d["b"])
    assert berr <= 1.01e-10
    x = direct_solve(d["K"], d["b"])
    _say(info, berr, rel(xg[: d["Nu"]], x[: d["Nu"]]), rel(xg[d["Nu"]:], x[d["Nu"]:]))
    assert rel(xg[: d["Nu"]], x[: d["Nu"]]) <= 1e-7
    assert rel(xg[d["Nu"]:], x[d["Nu"]:]) <= 1e-7


@pytest.mark.parametrize("precond,cap,inner_tol", [("schur", 24, 1e-12), ("reg", 64, 1e-1)])
def test_mixed_precision_capped_inner_solves(precond, cap, inner_tol):
    """Capped FP32 inner solves take the pipelined iteration (FP32 vectors and column-scaled
    values, FP64 dot products); the FP64 outer solve still meets its tolerance and matches the
    oracle's direct solve to the tolerance times the conditioning."""
    _say("mixed capped", precond, cap)
    m = cube_mesh(6, 7, 5)
    nu = 1.0 / lognormal_field(210, 2.0, 0)
    s = gpu_solver(m, nu=nu, rhs=SineSolution())
    # the Jacobi inner preconditioner (the FP32 pipelined iteration is its form)
    kw = dict(precond=precond, tol=1e-10, maxit=3000, inner_tol=inner_tol, inner_maxit=cap, reg_inner="jacobi")
    u, p, info = s.solve(precision="mixed", **kw)
    _, _, info64 = s.solve(**kw)
    assert info["converged"], info
    assert info["inner_iterations"] <= cap * (info["iterations"] + 1)
    d = discretize(m, nu=nu, rhs=SineSolution())
    xg = np.concatenate([u.cpu().numpy(), p.cpu().numpy()])
    berr = np.linalg.norm(d["b"] - d["K"] @ xg) / np.linalg.norm(d["b"])
    assert berr <= 1.01e-10
    x = direct_solve(d["K"], d["b"])
    _say(info, info64["iterations"], berr, rel(xg[: d["Nu"]], x[: d["Nu"]]), rel(xg[d["Nu"]:], x[d["Nu"]:]))
    assert rel(xg[: d["Nu"]], x[: d["Nu"]]) <= 1e-7
    assert rel(xg[d["Nu"]:], x[d["Nu"]:]) <= 1e-7
    # FP32 inner solves should cost few extra outer iterations
    assert info["iterations"] <= 1.5 * info64["iterations"] + 5


@pytest.mark.parametrize("cap", [5000, 20])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replays_match_eager(precision, cap):
    """Inner-CG iterations replayed from a captured HIP graph give the same bits as direct launches,
    over several solves with eager work and synchronisations in between; with a large inner cap
    (host polls the inner state) and with a small one (every iteration enqueued without polling)."""
    import torch

    _say("graphs", precision, cap)
    m = cube_mesh(9, 8, 7)
    nu = 1.0 / lognormal_field(9 * 8 * 7, 2.0, 3)
    s = gpu_solver(m, nu=nu, rhs=SineSolution())
    for precond in ("schur", "reg"):
        kw = dict(precond=precond, tol=1e-10, inner_tol=1e-4, inner_maxit=cap, precision=precision,
                  reg_inner="jacobi")  # graphs replay the Jacobi inner iterations
        ue, pe, ie = s.solve(graphs=False, **kw)
        for rep in range(3):
            y = s.apply(torch.cat([ue, pe]))  # eager work between replays
            torch.cuda.synchronize()
            ug, pg, ig = s.solve(graphs=True, **kw)
            assert ig["iterations"] == ie["iterations"]
            assert ig["inner_iterations"] == ie["inner_iterations"]
            assert torch.equal(ug, ue) and torch.equal(pg, pe), (precond, rep)
            assert torch.isfinite(y).all()


def test_values_follow_coefficient_and_gamma():
    """The coefficient-dependent values are built lazily, per preconditioner: after a Block-Schur
    solve, a new coefficient and a Block-Reg solve (which builds K and A_gamma only), S must still
    come out for the new coefficient, and a Block-Reg solve with another gamma must rebuild
    A_gamma for that gamma.  Every matrix against the oracle, then a solve."""
    import scipy.sparse as sp

    _say("lazy values")
    m = cube_mesh(5, 4, 3)
    nc = 60
    nu1, nu2 = 1.0 / lognormal_field(nc, 1.0, 1), 1.0 / lognormal_field(nc, 1.0, 2)
    s = gpu_solver(m, nu=nu1, rhs=SineSolution())
    s.solve(precond="schur", tol=1e-10)
    import torch

    s.set_coefficient(torch.as_tensor(nu2, dtype=torch.float64))
    s.solve(precond="reg", tol=1e-10, inner_tol=1e-2)
    d = discretize(m, nu=nu2, rhs=SineSolution())
    M, B = d["M"].tocsr(), d["B"].tocsr()
    Nu, Np = M.shape[0], B.shape[0]
    assert_same_csr(to_scipy(*s.export_csr("K"), (Nu + Np, Nu + Np)), d["K"].tocsr())
    S = (B @ sp.diags(1.0 / M.diagonal()) @ B.T).tocsr()
    assert_same_csr(to_scipy(*s.export_csr("schur"), (Np, Np)), S)
    g0 = s.sizes()["gamma"]
    assert_same_csr(to_scipy(*s.export_csr("reg"), (Nu, Nu)), (M + B.T @ B / g0).tocsr())
    g2 = 3.0 * g0
    s.solve(precond="reg", tol=1e-10, inner_tol=1e-2, gamma=g2)
    assert_same_csr(to_scipy(*s.export_csr("reg"), (Nu, Nu)), (M + B.T @ B / g2).tocsr())
    u, p, info = s.solve(precond="schur", tol=1e-13, maxit=2000, inner_tol=1e-12)
    x = direct_solve(d["K"], d["b"])
    uo, po = x[:Nu], x[Nu:]
    assert info["converged"]
    assert rel(u.cpu().numpy(), uo) < 1e-10 and rel(p.cpu().numpy(), po) < 1e-10
