"""Pins of the oracle's conical-product quadrature against closed-form simplex moments."""
from math import factorial

import numpy as np
import pytest

from oracle.quadrature import map_tets, map_tris, tet_rule, tri_rule


def tet_moment(a, b, c):
    # Dirichlet integral over the reference tetrahedron
    return factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)


def tri_moment(a, b):
    return factorial(a) * factorial(b) / factorial(a + b + 2)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_tet_rule_exact_to_degree_2n_minus_1(n):
    X, W = tet_rule(n)
    assert W.sum() == pytest.approx(1 / 6, rel=1e-14)
    deg = 2 * n - 1
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            for c in range(deg + 1 - a - b):
                q = (W * X[:, 0] ** a * X[:, 1] ** b * X[:, 2] ** c).sum()
                assert q == pytest.approx(tet_moment(a, b, c), rel=1e-12, abs=1e-16)
    # and not exact one degree higher (the rule really has n points per direction)
    q = (W * X[:, 0] ** (2 * n)).sum()
    assert abs(q - tet_moment(2 * n, 0, 0)) > 1e-8 * tet_moment(2 * n, 0, 0)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_tri_rule_exact_to_degree_2n_minus_1(n):
    X, W = tri_rule(n)
    assert W.sum() == pytest.approx(0.5, rel=1e-14)
    deg = 2 * n - 1
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            q = (W * X[:, 0] ** a * X[:, 1] ** b).sum()
            assert q == pytest.approx(tri_moment(a, b), rel=1e-12, abs=1e-16)


def test_mapped_simplices_measure():
    rng = np.random.default_rng(3)
    P = rng.random((5, 4, 3))
    X, W = map_tets(P[:, 0], P[:, 1], P[:, 2], P[:, 3], 2)
    vol = np.array([np.linalg.det(np.stack([p[1] - p[0], p[2] - p[0], p[3] - p[0]])) / 6 for p in P])
    assert np.allclose(W.sum(1), vol, rtol=1e-13)
    # centroid reproduced (degree 1)
    cen = (W[..., None] * X).sum(1) / W.sum(1)[:, None]
    assert np.allclose(cen, P.mean(1), rtol=1e-12)
    X, W = map_tris(P[:, 0], P[:, 1], P[:, 2], 3)
    area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    assert np.allclose(W.sum(1), area, rtol=1e-13)
