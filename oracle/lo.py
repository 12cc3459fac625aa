"""Lowest-order mixed virtual element, computed with the paper's recipe.

Element: one normal-flux moment per face (face space P_0), divergence and
pressure in P_0, L2 projector onto constant vectors [P_0]^3.  This is the
lowest member of the face-space family of Section 4.1 (the paper's own
family starts at face space P_k, k >= 1, with divergence in P_{k-1}); the
construction below takes the paper's steps with k = 0 for the projector:

  1. DOFs (eq. facePoly):  dof_i(v) = (1/|f_i|) int_{f_i} v . n_i,  n_i the
     outward normal of P on its i-th face, so the DOF matrix of the
     constants e_c is D[i, c] = n_i[c].
  2. Divergence (Section 4.1, second computable quantity): div phi_i is the
     constant solving H_0 c = int_P div phi_i m_0, the right-hand side
     taken by integration by parts; phi_i . n_j = delta_ij on the faces and
     there are no gradient moments, so the right-hand side is |f_i|.
  3. Projector (Section 4.1, third item; Prop. xDec with alpha = 0 gives
     e_c = h_P grad m_{e_c} with no cross terms): int_P phi_i . e_c =
     h_P ( - int_P div phi_i m_{e_c} + sum_f int_f (phi_i . n_f) m_{e_c} ).
     Pi* = G^{-1} B_proj with G[c, d] = int_P e_c . e_d.
  4. Local forms (Section 4.3): a_h,P = nu int Pi v . Pi w + s_P((I-Pi)v, (I-Pi)w),
     s_P(v, w) = nu(x_P) |P| sum_i dof_i(v) dof_i(w), so
     M_P = nu [Pi*^T G Pi* + |P| (I - D Pi*)^T (I - D Pi*)].
  5. Divergence form and load with the pressure basis psi dual to the moment
     DOF (eq. presMom): psi = 1, B_div,P[i] = int_P div phi_i,
     F_P = int_P f.
Every monomial integral is taken by quadrature, as the paper does.
"""

from __future__ import annotations

import numpy as np

from .geometry import cell_tets, face_triangles
from .quadrature import map_tets, map_tris


def _cell_quad(mesh, cgeo, n):
    t_cell, P0, P1, P2, P3, s = cell_tets(mesh, cgeo)
    X, W = map_tets(P0, P1, P2, P3, n, sign=s)
    return t_cell, X, W


def cell_integral(mesh, cgeo, n, func):
    """int_P func(x) for every cell; func maps (T, m, 3) points to (T, m, ...) values."""
    t_cell, X, W = _cell_quad(mesh, cgeo, n)
    vals = func(X, t_cell)
    contrib = np.einsum("tm,tm...->t...", W, vals)
    out = np.zeros((len(cgeo["volume"]),) + contrib.shape[1:])
    np.add.at(out, t_cell, contrib)
    return out


def face_integral(mesh, n, func):
    """int_f func(x) for every face; func maps (T, m, 3) points and the triangle's face ids."""
    xyz = mesh["xyz"]
    tri_face, ia, ib, ic = face_triangles(mesh)
    X, W = map_tris(xyz[ia], xyz[ib], xyz[ic], n)
    vals = func(X, tri_face)
    contrib = np.einsum("tm,tm...->t...", W, vals)
    out = np.zeros((len(mesh["face_ptr"]) - 1,) + contrib.shape[1:])
    np.add.at(out, tri_face, contrib)
    return out


def lo_local(mesh, fgeo, cgeo, nq=2):
    """Coefficient-free local matrices (nu = 1) of every cell, grouped by face count.

    Returns {F: {"cells", "faces", "sign", "M1" (g,F,F), "Bdiv" (g,F), "PiStar" (g,3,F), "D" (g,F,3)}}.
    """
    cp = mesh["cell_ptr"].astype(np.int64)
    cf = mesh["cell_face"].astype(np.int64)
    cs = mesh["cell_face_sign"].astype(np.float64)
    xP, hP, volP = cgeo["centroid"], cgeo["diam"], cgeo["volume"]

    # int_P m_0 m_0 and int_P m_{e_c} (scaled monomials about x_P, Section 2)
    H0 = cell_integral(mesh, cgeo, nq, lambda X, c: np.ones(X.shape[:2]))
    Im = cell_integral(mesh, cgeo, nq, lambda X, c: (X - xP[c][:, None, :]) / hP[c][:, None, None])

    nfc = np.diff(cp)
    out = {}
    for F in np.unique(nfc):
        cells = np.nonzero(nfc == F)[0]
        idx = cp[cells][:, None] + np.arange(F)[None, :]
        faces, sign = cf[idx], cs[idx]
        g = len(cells)
        nout = sign[..., None] * fgeo["normal"][faces]  # (g, F, 3)
        D = nout
        # face integrals of m_0 and m_{e_c} with this cell's monomials (the
        # face is planar, the monomial linear, so a one-direction rule of
        # degree >= 1 is exact; the general triangle rule is used anyway)
        xyz = mesh["xyz"]
        fp = mesh["face_ptr"].astype(np.int64)
        fv = mesh["face_vtx"].astype(np.int64)
        If0 = np.zeros((g, F))
        Ifm = np.zeros((g, F, 3))
        for i in range(F):
            fi = faces[:, i]
            nv = fp[fi + 1] - fp[fi]
            for nvv in np.unique(nv):
                sel = np.nonzero(nv == nvv)[0]
                for a in range(1, nvv - 1):
                    v0 = xyz[fv[fp[fi[sel]]]]
                    va = xyz[fv[fp[fi[sel]] + a]]
                    vb = xyz[fv[fp[fi[sel]] + a + 1]]
                    X, W = map_tris(v0, va, vb, nq)
                    If0[sel, i] += W.sum(1)
                    mono = (X - xP[cells[sel]][:, None, :]) / hP[cells[sel]][:, None, None]
                    Ifm[sel, i] += np.einsum("tm,tmc->tc", W, mono)
        # step 2: divergence coefficients (H_0 c = rhs)
        divphi = If0 / H0[cells][:, None]  # (g, F)
        # step 3: B_proj[c, i] = h_P(-div phi_i int_P m_ec + int_{f_i} m_ec)
        Bproj = hP[cells][:, None, None] * (
            -divphi[:, None, :] * Im[cells][:, :, None] + np.transpose(Ifm, (0, 2, 1))
        )  # (g, 3, F)
        G = H0[cells][:, None, None] * np.eye(3)[None]
        PiS = np.linalg.solve(G, Bproj)
        # step 4: M_P with nu = 1
        IDP = np.eye(F)[None] - D @ PiS
        M1 = np.transpose(PiS, (0, 2, 1)) @ G @ PiS + volP[cells][:, None, None] * (
            np.transpose(IDP, (0, 2, 1)) @ IDP
        )
        # step 5: B_div,P[i] = int_P div phi_i psi_0, psi_0 = 1
        Bdiv = divphi * H0[cells][:, None]
        out[int(F)] = {"cells": cells, "faces": faces, "sign": sign, "M1": M1, "Bdiv": Bdiv,
                       "PiStar": PiS, "D": D}
    return out


def lo_loads(mesh, cgeo, f, nq_load=3):
    """F_P = int_P f psi_0 (psi_0 = 1) with the load rule of nq_load points per direction."""
    return cell_integral(mesh, cgeo, nq_load, lambda X, c: f(X))


def lo_boundary(mesh, pD, nq_load=3):
    """int_f p_D over every face (used on boundary faces only)."""
    return face_integral(mesh, nq_load, lambda X, t: pD(X))
