"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module holds no arithmetic of the method itself: it only builds mesh
topology and vertex coordinates, draws per-cell coefficient fields from a
seed, and states the analytic data (right-hand side, boundary pressure and
exact solutions) as plain functions.  Everything that the mixed virtual
element method computes (geometry, projectors, local forms, assembly,
solvers) lives elsewhere, twice: once in the HIP library and once in the
oracle, with no code shared between the two.

Mesh format (a polyhedral mesh of the unit cube, Section 4.4 of the paper
uses Cube and Voronoi-type meshes of [0,1]^3):

    xyz            float64 [nv, 3]   vertex coordinates
    face_ptr       int32   [nf + 1]  CSR offsets into face_vtx
    face_vtx       int32   [sum]     vertex loop of each planar face, ordered
                                     counter-clockwise about the face's global
                                     normal n_f (right-hand rule)
    cell_ptr       int32   [nc + 1]  CSR offsets into cell_face
    cell_face      int32   [sum]     faces bounding each cell
    cell_face_sign int8    [sum]     +1 if n_f points out of the cell, else -1
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "cube_mesh",
    "voronoi_mesh",
    "lognormal_field",
    "checkerboard_field",
    "SineSolution",
    "PolynomialSolution",
    "LinearSolution",
]


def _as_mesh(xyz, face_ptr, face_vtx, cell_ptr, cell_face, cell_face_sign, **extra):
    mesh = {
        "xyz": np.ascontiguousarray(xyz, dtype=np.float64),
        "face_ptr": np.ascontiguousarray(face_ptr, dtype=np.int32),
        "face_vtx": np.ascontiguousarray(face_vtx, dtype=np.int32),
        "cell_ptr": np.ascontiguousarray(cell_ptr, dtype=np.int32),
        "cell_face": np.ascontiguousarray(cell_face, dtype=np.int32),
        "cell_face_sign": np.ascontiguousarray(cell_face_sign, dtype=np.int8),
    }
    mesh.update(extra)
    return mesh


def cube_mesh(nx: int, ny: int | None = None, nz: int | None = None):
    """Structured hexahedral mesh of [0,1]^3 with nx*ny*nz cells ("Cube").

    Cell (i, j, k) has id i + nx*(j + ny*k).  Faces are numbered x-normal
    first, then y-normal, then z-normal; every global normal points along
    +axis.  Each cell lists its faces in the order -x, +x, -y, +y, -z, +z.
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    if min(nx, ny, nz) < 1:
        raise ValueError("cube_mesh needs at least one cell per direction")
    vx, vy, vz = nx + 1, ny + 1, nz + 1

    def vid(i, j, k):
        return i + vx * (j + vy * k)

    gi, gj, gk = np.meshgrid(np.arange(vx), np.arange(vy), np.arange(vz), indexing="ij")
    xyz = np.zeros((vx * vy * vz, 3))
    ids = vid(gi, gj, gk).ravel()
    xyz[ids, 0] = (gi / nx).ravel()
    xyz[ids, 1] = (gj / ny).ravel()
    xyz[ids, 2] = (gk / nz).ravel()

    # x-normal faces: index i + vx*(j + ny*k), loop (j,k)->(j+1,k)->(j+1,k+1)->(j,k+1)
    i, j, k = np.meshgrid(np.arange(vx), np.arange(ny), np.arange(nz), indexing="ij")
    fx_id = (i + vx * (j + ny * k)).ravel()
    fx = np.stack([vid(i, j, k), vid(i, j + 1, k), vid(i, j + 1, k + 1), vid(i, j, k + 1)], -1)
    fx = fx.reshape(-1, 4)
    nfx = vx * ny * nz
    # y-normal faces: index i + nx*(j + vy*k), loop (i,j,k)->(i,j,k+1)->(i+1,j,k+1)->(i+1,j,k)
    i, j, k = np.meshgrid(np.arange(nx), np.arange(vy), np.arange(nz), indexing="ij")
    fy_id = (i + nx * (j + vy * k)).ravel()
    fy = np.stack([vid(i, j, k), vid(i, j, k + 1), vid(i + 1, j, k + 1), vid(i + 1, j, k)], -1)
    fy = fy.reshape(-1, 4)
    nfy = nx * vy * nz
    # z-normal faces: index i + nx*(j + ny*k), loop (i,j)->(i+1,j)->(i+1,j+1)->(i,j+1)
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(vz), indexing="ij")
    fz_id = (i + nx * (j + ny * k)).ravel()
    fz = np.stack([vid(i, j, k), vid(i + 1, j, k), vid(i + 1, j + 1, k), vid(i, j + 1, k)], -1)
    fz = fz.reshape(-1, 4)
    nfz = nx * ny * vz

    nf = nfx + nfy + nfz
    face_vtx = np.zeros((nf, 4), dtype=np.int64)
    face_vtx[fx_id] = fx
    face_vtx[nfx + fy_id] = fy
    face_vtx[nfx + nfy + fz_id] = fz
    face_ptr = np.arange(0, 4 * nf + 1, 4)

    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cid = (i + nx * (j + ny * k)).ravel()
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    cf = np.stack(
        [
            i + vx * (j + ny * k),
            (i + 1) + vx * (j + ny * k),
            nfx + i + nx * (j + vy * k),
            nfx + i + nx * ((j + 1) + vy * k),
            nfx + nfy + i + nx * (j + ny * k),
            nfx + nfy + i + nx * (j + ny * (k + 1)),
        ],
        -1,
    )
    nc = nx * ny * nz
    cell_face = np.zeros((nc, 6), dtype=np.int64)
    cell_face[cid] = cf
    sign = np.tile(np.array([-1, 1, -1, 1, -1, 1], dtype=np.int8), (nc, 1))
    cell_ptr = np.arange(0, 6 * nc + 1, 6)
    # cell centres are known from the grid indices; used only to place
    # piecewise-constant coefficient fields, never by the method
    centres = np.zeros((nc, 3))
    centres[cid, 0] = (i + 0.5) / nx
    centres[cid, 1] = (j + 0.5) / ny
    centres[cid, 2] = (k + 0.5) / nz
    return _as_mesh(
        xyz, face_ptr, face_vtx.ravel(), cell_ptr, cell_face.ravel(), sign.ravel(),
        kind="cube", dims=(nx, ny, nz), seeds=centres,
    )


def voronoi_mesh(n_points: int, seed: int = 0, weld_tol: float = 1e-12):
    """Voronoi tessellation of n_points uniform random points in [0,1]^3 ("Random").

    The cells are clipped to the cube by reflecting the generators across the
    six faces of the cube: the bisector planes with the mirror images are the
    cube's faces, so the Voronoi cells of the original generators are exactly
    the clipped cells.  Each shared face is taken once, from the generator
    pair (lower id first), and every loop is oriented about its global normal
    (the direction from the lower-id generator to the other one, or the
    outward normal of the cube on the boundary).  Vertices closer than
    weld_tol are merged; faces that collapse below three distinct vertices
    are dropped.
    """
    from scipy.spatial import Voronoi

    rng = np.random.default_rng(seed)
    pts = rng.random((n_points, 3))
    mirrors = [pts]
    for ax in range(3):
        for side in (0.0, 1.0):
            m = pts.copy()
            m[:, ax] = 2.0 * side - m[:, ax]
            mirrors.append(m)
    allp = np.concatenate(mirrors, 0)
    vor = Voronoi(allp)

    # weld vertices by rounding to a grid of size weld_tol, keep only used ones
    used = set()
    ridges = []
    for (a, b), rv in zip(vor.ridge_points, vor.ridge_vertices):
        if a >= n_points and b >= n_points:
            continue
        if -1 in rv:
            raise RuntimeError("unbounded ridge next to an inner generator")
        ridges.append((a, b, rv))
        used.update(rv)
    used = np.array(sorted(used))
    V = vor.vertices[used]
    V = np.clip(V, 0.0, 1.0)
    key = np.round(V / weld_tol).astype(np.int64)
    _, inv = np.unique(key, axis=0, return_inverse=True)
    inv = inv.ravel()
    remap_old = {int(o): int(inv[n]) for n, o in enumerate(used)}
    nv = int(inv.max()) + 1
    xyz = np.zeros((nv, 3))
    xyz[inv] = V

    faces = []  # (loop, owner, neighbour or -1)
    for a, b, rv in ridges:
        loop = []
        for v in rv:
            w = remap_old[int(v)]
            if not loop or loop[-1] != w:
                loop.append(w)
        if len(loop) > 1 and loop[0] == loop[-1]:
            loop.pop()
        if len(set(loop)) < 3:
            continue
        if a < n_points and b < n_points:
            lo, hi = (a, b) if a < b else (b, a)
            normal = allp[hi] - allp[lo]
            owner, nb = lo, hi
        else:
            owner = a if a < n_points else b
            other = b if owner == a else a
            normal = allp[other] - allp[owner]
            nb = -1
        P = xyz[loop]
        c = P.mean(0)
        area_vec = np.zeros(3)
        for t in range(len(loop)):
            area_vec += np.cross(P[t] - c, P[(t + 1) % len(loop)] - c)
        if np.dot(area_vec, normal) < 0:
            loop = loop[::-1]
        faces.append((loop, owner, nb))

    nf = len(faces)
    face_ptr = np.zeros(nf + 1, dtype=np.int64)
    face_ptr[1:] = np.cumsum([len(f[0]) for f in faces])
    face_vtx = np.concatenate([np.array(f[0]) for f in faces])
    cell_faces = [[] for _ in range(n_points)]
    for fid, (_, owner, nb) in enumerate(faces):
        cell_faces[owner].append((fid, 1))
        if nb >= 0:
            cell_faces[nb].append((fid, -1))
    cell_ptr = np.zeros(n_points + 1, dtype=np.int64)
    cell_ptr[1:] = np.cumsum([len(c) for c in cell_faces])
    cell_face = np.array([f for c in cell_faces for f, _ in c])
    cell_sign = np.array([s for c in cell_faces for _, s in c])
    return _as_mesh(
        xyz, face_ptr, face_vtx, cell_ptr, cell_face, cell_sign, kind="voronoi", seeds=pts,
    )


def lognormal_field(n_cells: int, sigma: float, seed: int):
    """Per-cell log-normal permeability K = exp(g), g ~ N(0, sigma^2) i.i.d. in cell order."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.normal(0.0, sigma, n_cells))


def checkerboard_field(seeds, lo: float = 1e-3, hi: float = 1e3, blocks: int = 4):
    """K = lo on even blocks and hi on odd blocks of a blocks^3 pattern of [0,1]^3.

    A cell is placed by its seed point (the generator of a Voronoi cell, the
    centre of a cube cell).
    """
    b = np.minimum(np.floor(blocks * np.asarray(seeds)).astype(np.int64), blocks - 1)
    return np.where(b.sum(1) % 2 == 0, lo, hi).astype(np.float64)


def _lib(x):
    try:
        import torch

        if isinstance(x, torch.Tensor):
            return torch
    except ImportError:  # pragma: no cover
        pass
    return np


class SineSolution:
    """p = sin(pi x) sin(pi y) sin(pi z), nu = 1: u = -grad p, f = div u = 3 pi^2 p, p = 0 on the boundary."""

    @staticmethod
    def p(x):
        # sin(pi x_d) for the three coordinates in one pass over the (n, 3) points, then their product
        # in one reduction over the last axis
        L = _lib(x)
        s = math.pi * x
        L.sin(s, out=s)
        return L.prod(s, -1)

    @staticmethod
    def f(x):
        q = SineSolution.p(x)
        q *= 3.0 * math.pi**2
        return q

    @staticmethod
    def pD(x):
        return 0.0 * x[..., 0]

    @staticmethod
    def u(x):
        L = _lib(x)
        s = [L.sin(math.pi * x[..., d]) for d in range(3)]
        c = [L.cos(math.pi * x[..., d]) for d in range(3)]
        return -math.pi * L.stack([c[0] * s[1] * s[2], s[0] * c[1] * s[2], s[0] * s[1] * c[2]], -1)


class PolynomialSolution:
    """The manufactured pair of the paper's convergence test, nu = 1:
    q = x^5 + 6y^4 + 9z^3 + x y^2 z^3, v = -grad q, f = div v = -lap q, p_D = q."""

    @staticmethod
    def p(x):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        return X**5 + 6 * Y**4 + 9 * Z**3 + X * Y**2 * Z**3

    pD = p

    @staticmethod
    def f(x):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        return -(20 * X**3 + 72 * Y**2 + 54 * Z + 2 * X * Z**3 + 6 * X * Y**2 * Z)

    @staticmethod
    def u(x):
        L = _lib(x)
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        return L.stack(
            [-5 * X**4 - Y**2 * Z**3, -24 * Y**3 - 2 * X * Y * Z**3, -27 * Z**2 - 3 * X * Y**2 * Z**2], -1
        )


class LinearSolution:
    """p = a + b.x, nu = 1: u = -b (constant), f = 0, p_D = p."""

    def __init__(self, a=0.3, b=(1.0, -2.0, 0.5)):
        self.a = float(a)
        self.b = tuple(float(t) for t in b)

    def p(self, x):
        return self.a + self.b[0] * x[..., 0] + self.b[1] * x[..., 1] + self.b[2] * x[..., 2]

    pD = p

    def f(self, x):
        return 0.0 * x[..., 0]

    def u(self, x):
        L = _lib(x)
        one = 1.0 + 0.0 * x[..., 0]
        return L.stack([-self.b[0] * one, -self.b[1] * one, -self.b[2] * one], -1)
