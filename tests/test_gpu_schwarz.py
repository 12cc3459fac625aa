"""Block-Reg with the edge-patch Schwarz preconditioner on its inner CG (the default inner form).

* The library's face system (A_gamma, with the cell interiors condensed at order k) and its Schwarz
  operator P = sum_e R_e^T F_e^{-1} R_e, against a NumPy construction from the oracle's matrices:
  the edges taken from the mesh's face loops, the patches as the DOFs of the faces around each edge,
  dense inverses.  Lowest order and the paper's k = 1, 2; Cube and Voronoi; pressure and flux data.
* Solves to 1e-13 against the oracle's direct solve (relative 1e-10 in u and p), FP64 and with FP32
  inner iterations (within the tolerance times the conditioning).
* The preconditioner's purpose: far fewer inner iterations than the Jacobi-CG on the same solve.
* At order k the face system and P are stored as dense face-to-face blocks (k = 1, 2, 3: 3, 6, 10
  DOFs per face); the operator and solve tests above run through that storage, and the timing hook
  counts its bytes (one index per block).
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.assemble import discretize
from oracle.solvers import direct_solve
from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field, voronoi_mesh
from tests.gpu_helpers import assert_same_csr, rel, to_scipy

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def edge_face_lists(mesh):
    """Faces around each mesh edge (edges = distinct vertex pairs of the face loops)."""
    fp, fv = mesh["face_ptr"], mesh["face_vtx"]
    E = {}
    for f in range(len(fp) - 1):
        loop = [int(v) for v in fv[fp[f]:fp[f + 1]]]
        for a, b in zip(loop, loop[1:] + loop[:1]):
            E.setdefault((min(a, b), max(a, b)), []).append(f)
    return [sorted(v) for v in E.values()]


def condensed_face_system(mesh, A, nfd, nint):
    """F = A_ff - A_fi A_ii^{-1} A_if (interiors condensed cell by cell; F = A without interiors), and
    the largest condition number of the A_ii blocks (0 without interiors)."""
    nf = len(mesh["face_ptr"]) - 1
    nc = len(mesh["cell_ptr"]) - 1
    nF = nf * nfd
    A = A.tocsr()
    if not nint:
        return A, 0.0
    Aii = A[nF:, nF:].tocsr()
    blocks = [Aii[c * nint:(c + 1) * nint, c * nint:(c + 1) * nint].toarray() for c in range(nc)]
    inv = sp.block_diag([np.linalg.inv(b) for b in blocks], format="csr")
    F = (A[:nF, :nF] - A[:nF, nF:] @ inv @ A[nF:, :nF]).tocsr()
    return F, max(np.linalg.cond(b) for b in blocks)


def schwarz_operator(mesh, F, nfd):
    """P = sum_e R_e^T F_e^{-1} R_e over the mesh edges, and the largest condition number of the
    patch matrices F_e."""
    F = F.tocsr()
    nF = F.shape[0]
    rows, cols, vals, kappa = [], [], [], 0.0
    for faces in edge_face_lists(mesh):
        dofs = np.concatenate([np.arange(f * nfd, (f + 1) * nfd) for f in faces])
        Fe = F[dofs][:, dofs].toarray()
        kappa = max(kappa, np.linalg.cond(Fe))
        rows.append(np.repeat(dofs, len(dofs)))
        cols.append(np.tile(dofs, len(dofs)))
        vals.append(np.linalg.inv(Fe).ravel())
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nF, nF))
    P.sum_duplicates()
    return P, kappa


def schwarz_reference(mesh, A, nfd, nint):
    """Face system F (interiors condensed cell by cell) and P = sum_e R_e^T F_e^{-1} R_e."""
    F, _ = condensed_face_system(mesh, A, nfd, nint)
    P, _ = schwarz_operator(mesh, F, nfd)
    return F, P


CASES = {
    "cube534_lo": (lambda: cube_mesh(5, 3, 4), "lo", 0),
    "voronoi60_lo": (lambda: voronoi_mesh(60, seed=7), "lo", 0),
    "cube322_k1": (lambda: cube_mesh(3, 2, 2), "paper", 1),
    "cube322_k2": (lambda: cube_mesh(3, 2, 2), "paper", 2),
    "voronoi25_k2": (lambda: voronoi_mesh(25, seed=3), "paper", 2),
    # order 3 on Voronoi cells: too many face DOFs per cell for the LDS-staged condensation, so the
    # face system comes from the per-entry gather instead
    "voronoi25_k3": (lambda: voronoi_mesh(25, seed=3), "paper", 3),
}


def _solver(mesh, family, k, nu, flux=False):
    import torch

    from paper_1901_02330_amd.vem import Solver

    s = Solver()
    s.set_mesh(mesh)
    s.discretize(family, k=k, load_points=3)
    if flux:
        s.set_boundary("flux")
    s.set_coefficient(torch.as_tensor(nu, dtype=torch.float64))
    return s


def _oracle(mesh, family, k, nu):
    return discretize(mesh, nu=nu, rhs=SineSolution(), family=family, k=k)


@pytest.mark.parametrize("flux", [False, True])
@pytest.mark.parametrize("name", list(CASES))
def test_schwarz_operators_match_reference(name, flux):
    _say("schwarz operators", name, flux)
    make, family, k = CASES[name]
    m = make()
    nc = len(m["cell_ptr"]) - 1
    nu = 1.0 / lognormal_field(nc, 1.5, 11)
    s = _solver(m, family, k, nu, flux)
    sz = s.sizes()
    d = _oracle(m, family, k, nu)
    nfd, nint = (d["nfd"], d["nint"]) if family == "paper" else (1, 0)
    nF = sz["n_face_dofs"]
    assert nF == (len(m["face_ptr"]) - 1) * nfd
    A = (d["M"] + d["B"].T @ d["B"] / sz["gamma"]).tocsr()
    if flux:
        # prescribed boundary-face DOFs: identity rows and columns of A_gamma
        cnt = np.bincount(m["cell_face"].astype(np.int64), minlength=len(m["face_ptr"]) - 1)
        fixed = np.zeros(A.shape[0], dtype=bool)
        fixed[:nF] = np.repeat(cnt == 1, nfd)
        keep = sp.diags((~fixed).astype(np.float64))
        A = (keep @ A @ keep + sp.diags(fixed.astype(np.float64))).tocsr()
    # F against the oracle's matrices condensed in NumPy; P against the edge-patch construction from
    # the library's own F.  Each within the larger of a fixed bound and 10 eps times the condition
    # number of the inverted blocks (A_ii for F, F_e for P): the first-order error of the inversions.
    eps = np.finfo(np.float64).eps
    base = 1e-12 if family == "lo" else 1e-10
    F, kappa_ii = condensed_face_system(m, A, nfd, nint)
    Fg = to_scipy(*s.export_csr("reg_face"), (nF, nF))
    assert_same_csr(Fg, F, max(base, 10 * eps * kappa_ii))
    P, kappa_e = schwarz_operator(m, Fg, nfd)
    Pg = to_scipy(*s.export_csr("reg_schwarz"), (nF, nF))
    assert_same_csr(Pg, P, max(base, 10 * eps * kappa_e))
    # P is symmetric and positive definite (a sum of SPD patch inverses covering every face DOF)
    assert abs(Pg - Pg.T).max() <= max(1e-12, 10 * eps * kappa_e) * abs(Pg).max()
    assert np.linalg.eigvalsh(Pg.toarray()).min() > 0


SOLVE_CASES = {
    "cube675_lo": (lambda: cube_mesh(6, 7, 5), "lo", 0, 2.0),
    "voronoi150_lo": (lambda: voronoi_mesh(150, seed=0), "lo", 0, 1.0),
    "cube432_k1": (lambda: cube_mesh(4, 3, 2), "paper", 1, 1.5),
    "cube322_k2": (lambda: cube_mesh(3, 2, 2), "paper", 2, 1.0),
    "voronoi25_k2": (lambda: voronoi_mesh(25, seed=3), "paper", 2, 1.0),
    "cube322_k3": (lambda: cube_mesh(3, 2, 2), "paper", 3, 1.0),
    "voronoi25_k3": (lambda: voronoi_mesh(25, seed=3), "paper", 3, 1.0),
    # cells of up to 20 faces: W of the largest cell exceeds the staged kernels' LDS
    "voronoi60_k3": (lambda: voronoi_mesh(60, seed=7), "paper", 3, 1.0),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(SOLVE_CASES))
def test_schwarz_solve_matches_oracle(name, precision):
    _say("schwarz solve", name, precision)
    make, family, k, sigma = SOLVE_CASES[name]
    m = make()
    nc = len(m["cell_ptr"]) - 1
    nu = 1.0 / lognormal_field(nc, sigma, 7)
    s = _solver(m, family, k, nu)
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    tol = 1e-13 if precision == "fp64" else 1e-10
    u, p, info = s.solve(precond="reg", tol=tol, maxit=2000, inner_tol=1e-2, precision=precision)
    assert info["converged"], info
    d = _oracle(m, family, k, nu)
    u, p = u.cpu().numpy(), p.cpu().numpy()
    xg = np.concatenate([u, p])
    berr = np.linalg.norm(d["b"] - d["K"] @ xg) / np.linalg.norm(d["b"])
    x = direct_solve(d["K"], d["b"])
    eu, ep = rel(u, x[: d["Nu"]]), rel(p, x[d["Nu"]:])
    # b - K x = (b - b_g) + (b_g - K_g x) + (K_g - K) x with the library's own matrix and right-hand
    # side K_g, b_g: the solve bounds the middle term by its tolerance, the rest is what separates the
    # two discretisations (rounding, larger for the ill-conditioned order-k local problems)
    N = d["Nu"] + d["Np"]
    Kg = to_scipy(*s.export_csr("K"), (N, N))
    bg = s.rhs().cpu().numpy()
    nb = np.linalg.norm(d["b"])
    bound = (np.linalg.norm(d["b"] - bg) + 1.01 * tol * np.linalg.norm(bg)
             + np.linalg.norm((Kg - d["K"]) @ xg)) / nb
    _say(info, "backward error", berr, "bound", bound, "err u", eu, "err p", ep)
    assert berr <= bound
    bound = 1e-10 if precision == "fp64" and k < 3 else 1e-7
    assert eu <= bound and ep <= bound


def test_schwarz_flux_boundary_solve():
    """The paper's boundary data (flux given, zero-mean pressure) with the Schwarz inner solve,
    against the oracle's augmented direct solve."""
    import torch

    from oracle.fluxbc import flux_system, solve_flux

    _say("schwarz flux data")
    m = cube_mesh(5, 3, 4)
    nu = 1.0 / lognormal_field(60, 2.0, 4)
    s = _solver(m, "lo", 0, nu, flux=True)

    def ufield(X):
        return torch.as_tensor(SineSolution.u(X.cpu().numpy()), dtype=torch.float64, device=X.device)

    s.set_rhs_functions(SineSolution.f, ufield)
    u, p, info = s.solve(precond="reg", tol=1e-13, maxit=2000, inner_tol=1e-2)
    assert info["converged"], info
    d = flux_system(m, nu=nu, rhs=SineSolution())
    uo, po = solve_flux(d)[:2]
    eu, ep = rel(u.cpu().numpy(), uo), rel(p.cpu().numpy(), po)
    _say(info, eu, ep)
    assert eu <= 1e-10 and ep <= 1e-10


def test_schwarz_needs_far_fewer_inner_iterations_than_jacobi():
    _say("schwarz vs jacobi")
    m = cube_mesh(12)
    nu = 1.0 / lognormal_field(12 ** 3, 2.0, 0)
    s = _solver(m, "lo", 0, nu)
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    kw = dict(precond="reg", tol=1e-8, maxit=3000, inner_tol=1e-1)
    _, _, ij = s.solve(reg_inner="jacobi", **kw)
    _, _, isz = s.solve(reg_inner="schwarz", **kw)
    _say("jacobi", ij, "schwarz", isz)
    assert ij["converged"] and isz["converged"]
    assert isz["inner_iterations"] * 3 < ij["inner_iterations"]


def test_voronoi_checkerboard_order2_converges_with_fp32_inner_solves():
    """The mixed-precision workload's recipe at 2,000 cells: Random Voronoi mesh, the paper's k = 2,
    checkerboard K in {1e-3, 1e3} on 4x4x4 blocks, Block-Reg with FP32 inner Schwarz-CG under FP64
    FGMRES to 1e-8.  The backward error of the result in the library's exported K (FP64) meets the
    tolerance, and the FP64-inner solve agrees with it to the tolerance times this system's
    conditioning (bounded here by 1e-5)."""
    import torch

    from paper_1901_02330_amd.inputs import checkerboard_field

    _say("voronoi checkerboard k=2, 2000 cells")
    m = voronoi_mesh(2000, seed=0)
    nu = 1.0 / checkerboard_field(m["seeds"])
    s = _solver(m, "paper", 2, nu)
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    kw = dict(precond="reg", tol=1e-8, maxit=1500, inner_tol=1e-2)
    u, p, info = s.solve(precision="mixed", **kw)
    _say("mixed", info)
    assert info["converged"], info
    N = s.sizes()["n"]
    K = to_scipy(*s.export_csr("K"), (N, N))
    b = s.rhs().cpu().numpy()
    x = np.concatenate([u.cpu().numpy(), p.cpu().numpy()])
    berr = np.linalg.norm(b - K @ x) / np.linalg.norm(b)
    u64, p64, i64 = s.solve(**kw)
    assert i64["converged"], i64
    x64 = np.concatenate([u64.cpu().numpy(), p64.cpu().numpy()])
    diff = np.linalg.norm(x - x64) / np.linalg.norm(x64)
    _say("fp64", i64, "backward error", berr, "mixed vs fp64", diff)
    assert berr <= 1.01e-8
    assert diff <= 1e-5


@pytest.mark.parametrize("k", [1, 2, 3])
def test_face_block_iteration_bytes_and_solve_unchanged(k):
    """The timing hook's Schwarz-CG iteration at order k runs on the face blocks, and its algorithmic
    bytes are the blocks' own: 8 (FP64) or 4 (FP32) bytes per entry of F and P, one 4-byte column per
    nfd x nfd block, two block offsets per face, and 13 vector accesses per face DOF.  A solve after
    the timing loops gives the same bits as before them."""
    _say("face blocks", k)
    m = cube_mesh(4, 3, 3)
    nc = 36
    nu = 1.0 / lognormal_field(nc, 1.0, 2)
    s = _solver(m, "paper", k, nu)
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    kw = dict(precond="reg", tol=1e-12, maxit=500, inner_tol=1e-2)
    u0, p0, i0 = s.solve(**kw)
    assert i0["converged"], i0
    u1, p1, i1 = s.solve(precision="mixed", **dict(kw, tol=1e-9))
    assert i1["converged"], i1
    sz = s.sizes()
    nF, nf = sz["n_face_dofs"], sz["n_faces"]
    nfd = nF // nf
    assert nfd == (k + 1) * (k + 2) // 2
    nnzF = int(s.export_csr("reg_face")[0][-1])
    nnzP = int(s.export_csr("reg_schwarz")[0][-1])
    assert nnzF % (nfd * nfd) == 0 and nnzP % (nfd * nfd) == 0
    nblk = (nnzF + nnzP) // (nfd * nfd)
    for which, vb in (("cg_reg_schwarz", 8), ("cg_reg_schwarz32", 4)):
        ms, nbytes = s.time_kernel(which, reps=5)
        assert ms > 0
        assert nbytes == vb * (nnzF + nnzP) + 4 * nblk + 16 * (nf + 1) + vb * 13 * nF, (which, nbytes)
    u2, p2, i2 = s.solve(**kw)
    assert i2["iterations"] == i0["iterations"]
    import torch

    assert torch.equal(u0, u2) and torch.equal(p0, p2)
