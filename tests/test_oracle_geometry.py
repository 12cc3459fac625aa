"""Pins of the oracle's geometry: closed forms on cubes, simplices and prisms; divergence-theorem identities."""
import numpy as np
import pytest

from oracle.geometry import cell_geometry, face_geometry
from oracle.quadrature import map_tris
from oracle.geometry import face_triangles
from paper_1901_02330_amd.inputs import cube_mesh, voronoi_mesh
from tests.meshes import single_prism, single_tet


@pytest.mark.parametrize("dims", [(4, 4, 4), (3, 5, 2)])
def test_cube_closed_forms(dims):
    nx, ny, nz = dims
    m = cube_mesh(nx, ny, nz)
    fg, cg = face_geometry(m), cell_geometry(m)
    nfx, nfy = (nx + 1) * ny * nz, nx * (ny + 1) * nz
    assert np.allclose(fg["area"][:nfx], 1 / (ny * nz), rtol=1e-14)
    assert np.allclose(fg["area"][nfx:nfx + nfy], 1 / (nx * nz), rtol=1e-14)
    assert np.allclose(fg["area"][nfx + nfy:], 1 / (nx * ny), rtol=1e-14)
    assert np.allclose(fg["normal"][:nfx], [1, 0, 0], atol=1e-15)
    assert np.allclose(fg["normal"][nfx:nfx + nfy], [0, 1, 0], atol=1e-15)
    assert np.allclose(fg["normal"][nfx + nfy:], [0, 0, 1], atol=1e-15)
    assert np.allclose(cg["volume"], 1 / (nx * ny * nz), rtol=1e-13)
    assert np.allclose(cg["centroid"], m["seeds"], atol=1e-15)
    d = np.sqrt(1 / nx**2 + 1 / ny**2 + 1 / nz**2)
    assert np.allclose(cg["diam"], d, rtol=1e-14)
    assert cg["h"] == pytest.approx(d, rel=1e-14)


def test_tet_and_prism():
    rng = np.random.default_rng(0)
    P = rng.random((4, 3))
    m = single_tet(P)
    cg = cell_geometry(m)
    vol = abs(np.linalg.det(np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]]))) / 6
    assert cg["volume"][0] == pytest.approx(vol, rel=1e-13)
    assert np.allclose(cg["centroid"][0], P.mean(0), rtol=1e-13)
    dmax = max(np.linalg.norm(P[i] - P[j]) for i in range(4) for j in range(4))
    assert cg["diam"][0] == pytest.approx(dmax, rel=1e-15)
    m = single_prism(0.7)
    fg, cg = face_geometry(m), cell_geometry(m)
    assert cg["volume"][0] == pytest.approx(0.5 * 0.7, rel=1e-14)
    assert np.allclose(cg["centroid"][0], [1 / 3, 1 / 3, 0.35], rtol=1e-14)
    assert np.allclose(fg["normal"][0], [0, 0, -1]) and np.allclose(fg["normal"][1], [0, 0, 1])
    assert fg["area"][3] == pytest.approx(np.sqrt(2) * 0.7, rel=1e-14)
    assert np.allclose(fg["centroid"][3], [0.5, 0.5, 0.35], rtol=1e-14)


@pytest.fixture(scope="module")
def vmesh():
    return voronoi_mesh(40, seed=1)


def test_voronoi_divergence_identities(vmesh):
    m = vmesh
    fg, cg = face_geometry(m), cell_geometry(m)
    assert cg["volume"].sum() == pytest.approx(1.0, rel=1e-13)
    cp, cf, cs = m["cell_ptr"], m["cell_face"].astype(int), m["cell_face_sign"].astype(float)
    # face second moments int_f x_c^2 (degree 2, exact with the 2-point triangle rule)
    tf, a, b, c = face_triangles(m)
    X, W = map_tris(m["xyz"][a], m["xyz"][b], m["xyz"][c], 2)
    x2 = np.zeros((len(fg["area"]), 3))
    np.add.at(x2, tf, np.einsum("tm,tmc->tc", W, X**2))
    for P in range(len(cp) - 1):
        sl = slice(cp[P], cp[P + 1])
        f, s = cf[sl], cs[sl]
        nout = s[:, None] * fg["normal"][f]
        A = fg["area"][f]
        # closed surface
        assert np.abs((A[:, None] * nout).sum(0)).max() < 1e-14
        # sum |f| n (x_f - x_P)^T = |P| I
        G = (A[:, None, None] * nout[:, :, None] * (fg["centroid"][f] - cg["centroid"][P])[:, None, :]).sum(0)
        assert np.allclose(G, cg["volume"][P] * np.eye(3), atol=1e-15)
        # |P| x_P = 1/2 sum_f sigma n_f int_f x^2 (divergence theorem)
        mom = 0.5 * (nout * x2[f]).sum(0)
        assert np.allclose(mom, cg["volume"][P] * cg["centroid"][P], atol=1e-15)
