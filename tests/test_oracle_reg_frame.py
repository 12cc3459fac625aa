"""Pins of the oracle's regularised block A_gamma = M + B^T B / gamma (Section 5, eq. block_diag)
and of its face frame (reading R9), each against something other than the oracle's own formula.

* A closed form on cubes: per cell nu h^3 (I - N N^T / 4) (the lowest-order M_P derived by hand,
  eigenvalues nu h^3 {1/2, 1}) plus gamma^{-1} h^4 sigma sigma^T (B_div,P = h^2 [1 .. 1] in outward
  orientation), assembled here from the cube's topology and vertex coordinates alone.
* On the kernel of B the regularisation vanishes: A_gamma v = M v.
* The spectrum of the Block-Reg preconditioned saddle matrix with an exact A_gamma solve:
  diag(A_gamma, gamma I)^{-1} [M B^T; B 0] has the eigenvalue 1 with multiplicity N_u (every
  u with p = B u / gamma) and -s / (s + gamma) for each eigenvalue s of B M^{-1} B^T.
* The face frame of a hand-built face: e1 along its longest loop edge (first on ties), e2 = n x e1.
"""
import numpy as np
import pytest

from oracle.assemble import discretize
from oracle.geometry import face_geometry
from oracle.paperk import discretize_paper
from oracle.solvers import block_reg
from paper_1901_02330_amd.inputs import cube_mesh, lognormal_field, voronoi_mesh


def _cube_reg_closed_form(mesh, n, nu, gamma):
    """A_gamma on an n^3 cube from the topology: no oracle code involved."""
    xyz = mesh["xyz"]
    fp, fv = mesh["face_ptr"], mesh["face_vtx"]
    cp, cf, cs = mesh["cell_ptr"], mesh["cell_face"], mesh["cell_face_sign"]
    nf = len(fp) - 1
    h = 1.0 / n
    A = np.zeros((nf, nf))
    for P in range(len(cp) - 1):
        faces = cf[cp[P]:cp[P + 1]]
        sg = cs[cp[P]:cp[P + 1]].astype(np.float64)
        # outward normal of each local face: the axis on which all its vertices agree, signed by
        # which side of the cell's centre the face lies on
        centre = xyz[np.unique(np.concatenate([fv[fp[f]:fp[f + 1]] for f in faces]))].mean(0)
        N = np.zeros((len(faces), 3))
        for i, f in enumerate(faces):
            V = xyz[fv[fp[f]:fp[f + 1]]]
            ax = int(np.argmin(np.ptp(V, axis=0)))
            N[i, ax] = np.sign(V[0, ax] - centre[ax])
        MP = nu[P] * h**3 * (np.eye(len(faces)) - 0.25 * N @ N.T)
        GP = (h**4 / gamma) * np.ones((len(faces), len(faces)))
        A[np.ix_(faces, faces)] += sg[:, None] * (MP + GP) * sg[None, :]
    return A


@pytest.mark.parametrize("n", [2, 3])
def test_reg_block_closed_form_on_cubes(n):
    m = cube_mesh(n)
    nu = 1.0 / lognormal_field(n**3, 1.5, 3)
    d = discretize(m, nu=nu)
    gamma = 0.37 * d["cgeo"]["h"] ** 2
    A = block_reg(d["M"], d["B"], gamma).A.toarray()
    Ae = _cube_reg_closed_form(m, n, nu, gamma)
    assert np.abs(A - Ae).max() <= 1e-13 * np.abs(Ae).max()


@pytest.mark.parametrize("case", ["lo-voronoi", "k2-cube"])
def test_reg_block_equals_mass_on_kernel_of_B(case):
    if case == "lo-voronoi":
        m = voronoi_mesh(20, seed=7)
        d = discretize(m, nu=1.0 / lognormal_field(20, 1.0, 2))
    else:
        m = cube_mesh(2, 2, 1)
        d = discretize_paper(m, nu=1.0 / lognormal_field(4, 1.0, 2), k=2)
    M, B = d["M"].toarray(), d["B"].toarray()
    gamma = d["cgeo"]["h"] ** 2
    A = block_reg(d["M"], d["B"], gamma).A.toarray()
    # an orthonormal basis of ker B from the SVD, and random fields in it
    _, sv, Vt = np.linalg.svd(B)
    rank = int((sv > 1e-12 * sv[0]).sum())
    Z = Vt[rank:].T
    assert Z.shape[1] == B.shape[1] - B.shape[0]  # B has full row rank (pressure data)
    v = Z @ np.random.default_rng(0).standard_normal((Z.shape[1], 4))
    assert np.abs(A @ v - M @ v).max() <= 1e-12 * np.abs(M @ v).max()
    # and it does not vanish off the kernel: on B^T q the difference is B^T B B^T q / gamma
    w = B.T @ np.random.default_rng(1).standard_normal(B.shape[0])
    assert np.linalg.norm(A @ w - M @ w) > 1e-3 * np.linalg.norm(M @ w)


@pytest.mark.parametrize("mesh", ["cube", "voronoi"])
def test_block_reg_preconditioned_spectrum(mesh):
    m = cube_mesh(3) if mesh == "cube" else voronoi_mesh(15, seed=4)
    nc = len(m["cell_ptr"]) - 1
    d = discretize(m, nu=1.0 / lognormal_field(nc, 1.0, 5))
    Nu, Np = d["Nu"], d["Np"]
    gamma = d["cgeo"]["h"] ** 2
    pre = block_reg(d["M"], d["B"], gamma)
    K = d["K"].toarray()
    PK = np.column_stack([pre(K[:, j]) for j in range(Nu + Np)])
    ev = np.linalg.eigvals(PK)
    M, B = d["M"].toarray(), d["B"].toarray()
    s = np.linalg.eigvalsh(B @ np.linalg.solve(M, B.T))
    expect = np.sort(np.concatenate([np.ones(Nu), -s / (s + gamma)]))
    assert np.abs(ev.imag).max() < 1e-8
    assert np.abs(np.sort(ev.real) - expect).max() < 1e-8


def _one_face_mesh(loop_xyz):
    n = len(loop_xyz)
    return {"xyz": np.asarray(loop_xyz, dtype=np.float64), "face_ptr": np.array([0, n], dtype=np.int32),
            "face_vtx": np.arange(n, dtype=np.int32)}


def test_face_frame_longest_edge():
    # a planar pentagon, tilted out of the coordinate planes; its longest loop edge is v2 -> v3
    R = np.linalg.qr(np.random.default_rng(3).standard_normal((3, 3)))[0]
    R *= np.sign(np.linalg.det(R))
    P2 = np.array([[0.0, 0.0], [1.0, -0.2], [1.6, 0.5], [0.4, 2.1], [-0.3, 0.9]])
    loop = np.column_stack([P2, np.zeros(5)]) @ R.T + np.array([0.2, -0.1, 0.4])
    fg = face_geometry(_one_face_mesh(loop))
    L = np.linalg.norm(np.roll(loop, -1, 0) - loop, axis=1)
    assert int(np.argmax(L)) == 2 and L[2] > 1.01 * np.sort(L)[-2]
    e1 = (loop[3] - loop[2]) / L[2]
    n = R[:, 2]  # counter-clockwise loop in the rotated xy plane: normal = rotated +z
    assert np.allclose(fg["normal"][0], n, atol=1e-14)
    assert np.allclose(fg["e1"][0], e1, atol=1e-14)
    assert np.allclose(fg["e2"][0], np.cross(n, e1), atol=1e-14)
    assert abs(fg["e1"][0] @ fg["normal"][0]) < 1e-14


def test_face_frame_ties_take_the_first_edge():
    # a square: four equal edges, so e1 follows the first edge of the loop, v0 -> v1
    sq = np.array([[0, 0, 0], [0, 1, 0], [0, 1, 1], [0, 0, 1]], dtype=np.float64)  # normal +x
    fg = face_geometry(_one_face_mesh(sq))
    assert np.allclose(fg["normal"][0], [1, 0, 0], atol=1e-15)
    assert np.allclose(fg["e1"][0], [0, 1, 0], atol=1e-15)
    assert np.allclose(fg["e2"][0], [0, 0, 1], atol=1e-15)
    # starting the same loop one vertex later moves e1 to the new first edge
    fg = face_geometry(_one_face_mesh(np.roll(sq, -1, 0)))
    assert np.allclose(fg["e1"][0], [0, 0, 1], atol=1e-15)
