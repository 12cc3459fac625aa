"""Pins of the oracle's lowest-order local matrices (Section 4.1 projector, Section 4.3 forms)."""
import numpy as np
import pytest

from oracle.geometry import cell_geometry, face_geometry
from oracle.lo import lo_local
from paper_1901_02330_amd.inputs import cube_mesh, voronoi_mesh
from tests.meshes import single_prism, single_tet


def local_of(m):
    fg, cg = face_geometry(m), cell_geometry(m)
    return fg, cg, lo_local(m, fg, cg)


def test_cube_closed_form():
    # derived by hand: on a cube of side h, Pi* = N^T / 2 and
    # M_P = h^3 (I - N N^T / 4) with N the outward normals (eigenvalues h^3 {1/2, 1})
    for n in (2, 5):
        m = cube_mesh(n)
        fg, cg, loc = local_of(m)
        grp = loc[6]
        h = 1.0 / n
        N = grp["D"]
        ref = h**3 * (np.eye(6)[None] - 0.25 * N @ np.transpose(N, (0, 2, 1)))
        assert np.abs(grp["M1"] - ref).max() < 1e-15 * h**3 * 10
        # hand-written explicit form: diagonal 3/4 h^3, opposite faces +1/4 h^3, rest 0
        E = np.zeros((6, 6))
        for i in range(6):
            E[i, i] = 0.75
            E[i, i ^ 1] = 0.25
        assert np.allclose(grp["M1"][0], h**3 * E, atol=1e-17)
        ev = np.linalg.eigvalsh(grp["M1"][0]) / h**3
        assert np.allclose(sorted(ev), [0.5] * 3 + [1.0] * 3)
        assert np.allclose(grp["Bdiv"], h**2)


@pytest.mark.parametrize("which", ["tet", "prism", "voronoi"])
def test_projector_consistency_and_spd(which):
    rng = np.random.default_rng(7)
    m = {"tet": lambda: single_tet(rng.random((4, 3))), "prism": lambda: single_prism(0.4),
         "voronoi": lambda: voronoi_mesh(25, seed=3)}[which]()
    fg, cg, loc = local_of(m)
    for F, grp in loc.items():
        D, Pi, M1 = grp["D"], grp["PiStar"], grp["M1"]
        vol = cg["volume"][grp["cells"]]
        # Pi* D = I: the projector reproduces constant vector fields
        assert np.allclose(Pi @ D, np.eye(3)[None], atol=1e-12)
        # consistency: d(c)^T M_P d(c') = int_P c . c' for constants (nu = 1)
        C = rng.standard_normal((3, 2))
        dc = D @ C  # (g, F, 2)
        lhs = np.transpose(dc, (0, 2, 1)) @ M1 @ dc
        assert np.allclose(lhs, vol[:, None, None] * (C.T @ C)[None], rtol=1e-12, atol=1e-16)
        # symmetric positive definite
        assert np.allclose(M1, np.transpose(M1, (0, 2, 1)), atol=1e-17)
        assert np.linalg.eigvalsh(M1).min() > 0
        # div of a constant field is zero: B_div,P d(c) = 0; B_div,P = |f_i|
        assert np.abs(np.einsum("gf,gfk->gk", grp["Bdiv"], dc)).max() < 1e-14
        assert np.allclose(grp["Bdiv"], fg["area"][grp["faces"]], rtol=1e-13)
