"""Face and cell geometry of a polyhedral mesh (Section 2 of the paper).

Definitions (the paper names barycentres and diameters without fixing
them; readings used here):
  * |f|, n_f, x_f: area, unit normal and area centroid of the planar face f,
    from the triangle fan (v0, v_a, v_{a+1}) of its vertex loop;
  * h_f: face diameter, the largest distance between two of its vertices;
  * face frame: e1 along the longest edge of the loop (first one on ties),
    e2 = n_f x e1 (used by the face scaled monomials m^f_beta);
  * |P|, x_P: volume and volume centroid of the cell P, summed over the
    tetrahedra (x_ref, v0, v_a, v_{a+1}) of its faces, x_ref being the mean
    of the cell's face-vertex incidences;
  * h_P: cell diameter, the largest distance between two of its vertices;
  * h = mean of h_P over the cells (eq. meshSize).
"""

from __future__ import annotations

import numpy as np


def face_triangles(mesh):
    """Fan triangles of every face: (tri_face, a, b, c) with vertex ids, fan from the loop's first vertex."""
    fp = mesh["face_ptr"].astype(np.int64)
    fv = mesh["face_vtx"].astype(np.int64)
    nvf = np.diff(fp)
    if np.any(nvf < 3):
        raise ValueError("face with fewer than three vertices")
    ntri = nvf - 2
    tri_face = np.repeat(np.arange(len(nvf)), ntri)
    first = np.repeat(np.cumsum(ntri) - ntri, ntri)
    a = np.arange(len(tri_face)) - first + 1  # 1 .. n-2
    base = fp[tri_face]
    return tri_face, fv[base], fv[base + a], fv[base + a + 1]


def face_geometry(mesh):
    xyz = mesh["xyz"]
    fp = mesh["face_ptr"].astype(np.int64)
    fv = mesh["face_vtx"].astype(np.int64)
    nf = len(fp) - 1
    tri_face, ia, ib, ic = face_triangles(mesh)
    A, B, C = xyz[ia], xyz[ib], xyz[ic]
    cr = 0.5 * np.cross(B - A, C - A)
    avec = np.zeros((nf, 3))
    np.add.at(avec, tri_face, cr)
    area = np.linalg.norm(avec, axis=1)
    if np.any(area <= 0):
        raise ValueError("face with zero area")
    normal = avec / area[:, None]
    ta = np.einsum("ti,ti->t", cr, normal[tri_face])
    cen = np.zeros((nf, 3))
    np.add.at(cen, tri_face, ta[:, None] * (A + B + C) / 3.0)
    cen /= area[:, None]

    nvf = np.diff(fp)
    diam = np.zeros(nf)
    e1 = np.zeros((nf, 3))
    for n in np.unique(nvf):
        sel = np.nonzero(nvf == n)[0]
        idx = fp[sel][:, None] + np.arange(n)[None, :]
        P = xyz[fv[idx]]  # (g, n, 3)
        d = np.linalg.norm(P[:, :, None, :] - P[:, None, :, :], axis=-1)
        diam[sel] = d.reshape(len(sel), -1).max(1)
        E = np.roll(P, -1, axis=1) - P
        L = np.linalg.norm(E, axis=-1)
        k = np.argmax(L, axis=1)
        e1[sel] = E[np.arange(len(sel)), k] / L[np.arange(len(sel)), k][:, None]
    e2 = np.cross(normal, e1)
    return {"area": area, "normal": normal, "centroid": cen, "diam": diam, "e1": e1, "e2": e2}


def cell_incidence(mesh):
    """Per cell-face incidence arrays: (cell id, face id, sign)."""
    cp = mesh["cell_ptr"].astype(np.int64)
    nfc = np.diff(cp)
    inc_cell = np.repeat(np.arange(len(nfc)), nfc)
    return inc_cell, mesh["cell_face"].astype(np.int64), mesh["cell_face_sign"].astype(np.float64)


def cell_geometry(mesh, fgeo=None):
    xyz = mesh["xyz"]
    fp = mesh["face_ptr"].astype(np.int64)
    fv = mesh["face_vtx"].astype(np.int64)
    cp = mesh["cell_ptr"].astype(np.int64)
    nc = len(cp) - 1
    inc_cell, inc_face, inc_sign = cell_incidence(mesh)

    # reference point: mean over the cell's face-vertex incidences
    nvf = np.diff(fp)
    vsum = np.zeros((len(nvf), 3))
    np.add.at(vsum, np.repeat(np.arange(len(nvf)), nvf), xyz[fv])
    xref = np.zeros((nc, 3))
    np.add.at(xref, inc_cell, vsum[inc_face])
    cnt = np.zeros(nc)
    np.add.at(cnt, inc_cell, nvf[inc_face])
    xref /= cnt[:, None]

    tri_face, ia, ib, ic = face_triangles(mesh)
    # expand each incidence (cell, face) to the triangles of that face
    tri_ptr = np.zeros(len(nvf) + 1, dtype=np.int64)
    tri_ptr[1:] = np.cumsum(nvf - 2)
    ntri_inc = (nvf - 2)[inc_face]
    t_inc = np.repeat(np.arange(len(inc_face)), ntri_inc)
    first = np.repeat(np.cumsum(ntri_inc) - ntri_inc, ntri_inc)
    t_idx = tri_ptr[inc_face[t_inc]] + (np.arange(len(t_inc)) - first)
    t_cell = inc_cell[t_inc]
    O = xref[t_cell]
    A, B, C = xyz[ia[t_idx]], xyz[ib[t_idx]], xyz[ic[t_idx]]
    vol6 = np.einsum("ti,ti->t", A - O, np.cross(B - O, C - O)) * inc_sign[t_inc]
    vol = np.zeros(nc)
    np.add.at(vol, t_cell, vol6 / 6.0)
    if np.any(vol <= 0):
        raise ValueError("cell with non-positive volume (check orientation signs)")
    cen = np.zeros((nc, 3))
    np.add.at(cen, t_cell, (vol6 / 6.0)[:, None] * (O + A + B + C) / 4.0)
    cen /= vol[:, None]

    # diameter over the distinct vertices of each cell
    ninc_v = nvf[inc_face]
    pair_cell = np.repeat(inc_cell, ninc_v)
    starts = fp[inc_face]
    firstv = np.repeat(np.cumsum(ninc_v) - ninc_v, ninc_v)
    pair_v = fv[np.repeat(starts, ninc_v) + (np.arange(len(pair_cell)) - firstv)]
    key = np.unique(pair_cell * (len(xyz) + 1) + pair_v)
    uc = key // (len(xyz) + 1)
    uv = key % (len(xyz) + 1)
    counts = np.bincount(uc, minlength=nc)
    diam = np.zeros(nc)
    ustart = np.cumsum(counts) - counts
    for n in np.unique(counts):
        sel = np.nonzero(counts == n)[0]
        for lo in range(0, len(sel), 4096):
            s = sel[lo:lo + 4096]
            idx = ustart[s][:, None] + np.arange(n)[None, :]
            P = xyz[uv[idx]]
            d = np.linalg.norm(P[:, :, None, :] - P[:, None, :, :], axis=-1)
            diam[s] = d.reshape(len(s), -1).max(1)
    return {
        "volume": vol,
        "centroid": cen,
        "diam": diam,
        "xref": xref,
        "h": float(diam.mean()),
    }


def cell_tets(mesh, cgeo):
    """All tetrahedra (x_ref, v0, v_a, v_{a+1}) of every cell, in face-loop order.

    Returns (tet_cell, P0, P1, P2, P3, s) where s = sign of the face in the
    cell, so that s * det[P1-P0, P2-P0, P3-P0] > 0 for a convex cell.  The
    vertex order is never swapped: a quadrature rule mapped onto these
    tetrahedra takes the weight s * det * w_ref.
    """
    xyz = mesh["xyz"]
    fp = mesh["face_ptr"].astype(np.int64)
    nvf = np.diff(fp)
    inc_cell, inc_face, inc_sign = cell_incidence(mesh)
    tri_face, ia, ib, ic = face_triangles(mesh)
    tri_ptr = np.zeros(len(nvf) + 1, dtype=np.int64)
    tri_ptr[1:] = np.cumsum(nvf - 2)
    ntri_inc = (nvf - 2)[inc_face]
    t_inc = np.repeat(np.arange(len(inc_face)), ntri_inc)
    first = np.repeat(np.cumsum(ntri_inc) - ntri_inc, ntri_inc)
    t_idx = tri_ptr[inc_face[t_inc]] + (np.arange(len(t_inc)) - first)
    t_cell = inc_cell[t_inc]
    return t_cell, cgeo["xref"][t_cell], xyz[ia[t_idx]], xyz[ib[t_idx]], xyz[ic[t_idx]], inc_sign[t_inc]
