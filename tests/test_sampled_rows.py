"""The sampled-row oracle used by the full-size GPU parity tests reproduces the full oracle's rows.

Pinned against the full oracle itself on meshes small enough to discretise whole: every sampled row of
K and every sampled entry of b is identical (same arithmetic, same order, on a sub-mesh whose faces and
cells carry the same loops, orientations and signs)."""
import numpy as np
import pytest

from oracle.assemble import discretize
from oracle.paperk import counts
from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field, voronoi_mesh
from tests.gpu_helpers import oracle_sampled_rows


@pytest.mark.parametrize("name,family,k", [("cube", "lo", 0), ("voronoi", "lo", 0), ("voronoi", "paper", 2),
                                           ("cube", "paper", 2)])
def test_sampled_rows_equal_full_oracle(name, family, k):
    m = cube_mesh(4, 3, 3) if name == "cube" else voronoi_mesh(30, seed=3)
    nc, nf = len(m["cell_ptr"]) - 1, len(m["face_ptr"]) - 1
    nu = 1.0 / lognormal_field(nc, 1.0, 1)
    full = discretize(m, nu=nu, rhs=SineSolution(), family=family, k=k)
    K = full["K"].tocsr()
    rng = np.random.default_rng(0)
    faces = np.sort(rng.choice(nf, 6, replace=False))
    cells = np.sort(rng.choice(nc, 4, replace=False))
    rows, bv, _, _ = oracle_sampled_rows(m, nu, faces, cells, SineSolution(), family=family, k=k)
    nfd, ng, ncx, npd = counts(k) if family == "paper" else (1, 0, 0, 1)
    assert len(rows) == len(faces) * nfd + len(cells) * (ng + ncx + npd)
    for r, (c, v) in rows.items():
        sl = slice(K.indptr[r], K.indptr[r + 1])
        assert dict(zip(c.tolist(), v.tolist())) == dict(zip(K.indices[sl].tolist(), K.data[sl].tolist()))
    for r, v in bv.items():
        assert v == full["b"][r]
