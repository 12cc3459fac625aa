"""Conical-product (Stroud) quadrature on triangles and tetrahedra.

The paper leaves the quadrature open (Remark in Section 4.3: the load and
divergence terms depend only on the integration rule).  Reading used here:
cells are split into tetrahedra and faces into triangles; each simplex gets
the collapsed Gauss-Jacobi product rule with n points per direction, exact
for polynomials of total degree 2n - 1.

Reference tetrahedron {xi, eta, zeta >= 0, xi + eta + zeta <= 1}:
    xi = a,  eta = b (1 - a),  zeta = c (1 - a)(1 - b),
    Jacobian (1 - a)^2 (1 - b): a takes the Gauss-Jacobi rule of weight
    (1 - a)^2 on [0, 1], b the one of weight (1 - b), c plain Gauss-Legendre.
Reference triangle {xi, eta >= 0, xi + eta <= 1}: xi = a, eta = b (1 - a),
    a with weight (1 - a), b Gauss-Legendre.
"""

from __future__ import annotations

from functools import lru_cache

import numpy as np
from scipy.special import roots_jacobi


@lru_cache(maxsize=None)
def gauss_jacobi01(n: int, alpha: int):
    """Nodes/weights for int_0^1 (1 - t)^alpha g(t) dt, n points (exact to degree 2n - 1)."""
    x, w = roots_jacobi(n, alpha, 0.0)
    t = 0.5 * (1.0 + x)
    return t, w * 0.5 ** (alpha + 1)


@lru_cache(maxsize=None)
def tet_rule(n: int):
    """Barycentric-free reference rule: points (m, 3) in the reference tet, weights summing to 1/6."""
    a, wa = gauss_jacobi01(n, 2)
    b, wb = gauss_jacobi01(n, 1)
    c, wc = gauss_jacobi01(n, 0)
    A, B, C = np.meshgrid(a, b, c, indexing="ij")
    W = (wa[:, None, None] * wb[None, :, None] * wc[None, None, :]).ravel()
    xi = A.ravel()
    eta = (B * (1 - A)).ravel()
    zeta = (C * (1 - A) * (1 - B)).ravel()
    return np.stack([xi, eta, zeta], 1), W


@lru_cache(maxsize=None)
def tri_rule(n: int):
    """Reference triangle rule: points (m, 2), weights summing to 1/2."""
    a, wa = gauss_jacobi01(n, 1)
    b, wb = gauss_jacobi01(n, 0)
    A, B = np.meshgrid(a, b, indexing="ij")
    W = (wa[:, None] * wb[None, :]).ravel()
    return np.stack([A.ravel(), (B * (1 - A)).ravel()], 1), W


def map_tets(p0, p1, p2, p3, n: int, sign=None):
    """Physical points/weights for a batch of tetrahedra (T, 3) each.

    Weights carry the signed Jacobian sign * det[p1-p0, p2-p0, p3-p0], so a
    positively oriented tetrahedron gets positive weights summing to its
    volume.  Returns X (T, m, 3), W (T, m).
    """
    ref, w = tet_rule(n)
    e1, e2, e3 = p1 - p0, p2 - p0, p3 - p0
    det = np.einsum("ti,ti->t", e1, np.cross(e2, e3))
    if sign is not None:
        det = det * sign
    X = (
        p0[:, None, :]
        + ref[None, :, 0:1] * e1[:, None, :]
        + ref[None, :, 1:2] * e2[:, None, :]
        + ref[None, :, 2:3] * e3[:, None, :]
    )
    return X, det[:, None] * w[None, :]


def map_tris(p0, p1, p2, n: int):
    """Physical points/weights for triangles (T, 3): weights sum to the area."""
    ref, w = tri_rule(n)
    e1, e2 = p1 - p0, p2 - p0
    area2 = np.linalg.norm(np.cross(e1, e2), axis=1)
    X = p0[:, None, :] + ref[None, :, 0:1] * e1[:, None, :] + ref[None, :, 1:2] * e2[:, None, :]
    return X, area2[:, None] * w[None, :]
