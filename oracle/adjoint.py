"""Gradient of a pressure misfit with respect to the per-cell log-permeability (oracle).

With nu_P = exp(-theta_P), theta_P = log K_P, only the flux block depends on
theta: M = sum_P nu_P R_P^T S_P M1_P S_P R_P (Section 4.3: the local form is
linear in nu, and nu is constant on each cell).  For K(theta) x = b and
J = J(x), differentiating K x = b gives dJ/dtheta_P = -lambda^T (dK/dtheta_P) x
with K^T lambda = dJ/dx; K is symmetric, and dK/dtheta_P = -nu_P (local M1_P
embedded), so

    dJ/dtheta_P = nu_P lambda_{u,P}^T M1_P u_P      (local, oriented DOFs).
"""

from __future__ import annotations

import numpy as np

from .solvers import direct_solve


def cell_dofs(mesh, d, P):
    """Global flux DOF ids and orientation signs of cell P's local DOFs (either element)."""
    cp, cf, cs = mesh["cell_ptr"], mesh["cell_face"], mesh["cell_face_sign"]
    faces = cf[cp[P]:cp[P + 1]].astype(np.int64)
    sig = cs[cp[P]:cp[P + 1]].astype(np.float64)
    nfd, nint = d.get("nfd", 1), d.get("nint", 0)
    nf = len(mesh["face_ptr"]) - 1
    F = len(faces)
    gid = np.concatenate([np.repeat(faces * nfd, nfd) + np.tile(np.arange(nfd), F),
                          nf * nfd + P * nint + np.arange(nint)])
    sg = np.concatenate([np.repeat(sig, nfd), np.ones(nint)])
    return gid, sg


def local_M1(d, P):
    loc = d["local"]
    if isinstance(loc, list):
        return loc[P]["M1"]
    for grp in loc.values():
        hit = np.nonzero(grp["cells"] == P)[0]
        if len(hit):
            return grp["M1"][hit[0]]
    raise KeyError(P)


def coefficient_gradient(mesh, d, u, lam):
    """g[P] = nu_P lambda_P^T M1_P u_P for every cell."""
    nc = len(mesh["cell_ptr"]) - 1
    g = np.zeros(nc)
    for P in range(nc):
        gid, sg = cell_dofs(mesh, d, P)
        g[P] = d["nu"][P] * (sg * lam[gid]) @ local_M1(d, P) @ (sg * u[gid])
    return g


def misfit_gradient(mesh, d, p_obs):
    """J = 1/2 ||p - p_obs||^2 over the pressure DOF vector: returns (J, dJ/dtheta, x, lambda)."""
    x = direct_solve(d["K"], d["b"])
    Nu = d["Nu"]
    r = x[Nu:] - p_obs
    lam = direct_solve(d["K"], np.concatenate([np.zeros(Nu), r]))
    return 0.5 * r @ r, coefficient_gradient(mesh, d, x[:Nu], lam[:Nu]), x, lam
