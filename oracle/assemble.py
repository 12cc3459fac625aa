"""Global assembly of the saddle-point system (eqs. mod_prob_eqDisc and Section 5).

Global unknowns: one flux moment per face w.r.t. the face's global normal
n_f (the cell-local DOF is sigma_{P,f} times it, sigma = +1 when n_f points
out of P), then the pressure moments cell by cell.  The assembled system is
written in symmetric form

    [ M   B^T ] [u]   [ g ]
    [ B    0  ] [p] = [ -F ],     B = -B_div,

which is the discrete problem a_h(u, v) - b_h(v, p) = -int_{dOmega} p_D v.n,
b_h(u, q) = (f, q) with the second row multiplied by -1 (the paper's block
matrix [A B^T; B -C] with C = 0).  Pressure boundary data enter naturally
through g; every boundary flux is an unknown and no mean-value constraint
is imposed.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .geometry import cell_geometry, face_geometry
from .lo import lo_boundary, lo_loads, lo_local


def boundary_faces(mesh):
    """Faces with a single adjacent cell, and that cell's sign on them."""
    nf = len(mesh["face_ptr"]) - 1
    cnt = np.bincount(mesh["cell_face"].astype(np.int64), minlength=nf)
    if np.any(cnt == 0) or np.any(cnt > 2):
        raise ValueError("every face needs one or two adjacent cells")
    sgn = np.zeros(nf)
    np.add.at(sgn, mesh["cell_face"].astype(np.int64), mesh["cell_face_sign"].astype(np.float64))
    bnd = np.nonzero(cnt == 1)[0]
    return bnd, sgn[bnd]


def discretize(mesh, nu=None, rhs=None, family="lo", k=0, nq=2, nq_load=3, local=None, geo=None):
    """Local matrices, global K and right-hand side b for the given coefficient nu = 1/K per cell.

    rhs: object with methods f(x) and pD(x) (numpy arrays of points (..., 3)).
    Returns a dict with the geometry, the local matrices, the sparse blocks
    M, B (=-B_div), K and the vectors g, F, b.
    """
    if family != "lo":
        from .paperk import discretize_paper

        return discretize_paper(mesh, nu=nu, rhs=rhs, k=k, local=local, geo=geo)
    nf = len(mesh["face_ptr"]) - 1
    nc = len(mesh["cell_ptr"]) - 1
    if geo is None:
        fgeo = face_geometry(mesh)
        cgeo = cell_geometry(mesh)
    else:
        fgeo, cgeo = geo
    if local is None:
        local = lo_local(mesh, fgeo, cgeo, nq=nq)
    nu = np.ones(nc) if nu is None else np.asarray(nu, dtype=np.float64)

    rows, cols, vals = [], [], []
    brow, bcol, bval = [], [], []
    for F, grp in local.items():
        cells, faces, sign = grp["cells"], grp["faces"], grp["sign"]
        Mg = nu[cells][:, None, None] * grp["M1"] * sign[:, :, None] * sign[:, None, :]
        rows.append(np.repeat(faces, F, axis=1).ravel())
        cols.append(np.tile(faces, (1, F)).ravel())
        vals.append(Mg.ravel())
        brow.append(np.repeat(cells, F))
        bcol.append(faces.ravel())
        bval.append((grp["Bdiv"] * sign).ravel())
    M = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nf, nf))
    Bdiv = sp.csr_matrix((np.concatenate(bval), (np.concatenate(brow), np.concatenate(bcol))), shape=(nc, nf))
    M.sum_duplicates()
    Bdiv.sum_duplicates()
    B = -Bdiv
    K = sp.bmat([[M, B.T], [B, None]], format="csr")

    g = np.zeros(nf)
    Fload = np.zeros(nc)
    if rhs is not None:
        Fload = lo_loads(mesh, cgeo, rhs.f, nq_load)
        bnd, bsgn = boundary_faces(mesh)
        ipD = lo_boundary(mesh, rhs.pD, nq_load)
        g[bnd] = -bsgn * ipD[bnd]
    b = np.concatenate([g, -Fload])
    return {
        "fgeo": fgeo, "cgeo": cgeo, "local": local, "nu": nu,
        "M": M, "Bdiv": Bdiv, "B": B, "K": K,
        "g": g, "F": Fload, "b": b, "Nu": nf, "Np": nc,
    }


def interpolate_lo(mesh, fgeo, cgeo, sol, nq=3):
    """Degrees of freedom of the exact (u, p): face flux moments w.r.t. n_f and cell averages of p."""
    from .lo import cell_integral, face_integral

    un = face_integral(mesh, nq, lambda X, t: np.einsum("tmc,tc->tm", sol.u(X), fgeo["normal"][t]))
    u_dof = un / fgeo["area"]
    p_dof = cell_integral(mesh, cgeo, nq, lambda X, c: sol.p(X)) / cgeo["volume"]
    return u_dof, p_dof
