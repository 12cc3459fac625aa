"""The paper's model problem with its own boundary data (test infrastructure only: the
library must not import this module).

Section 3 (eq. mod_prob_eq) poses the mixed problem on V = {v : v.n = u_N on the
boundary} with pressures in Q = {q : int_Omega q = 0}, and the parallel tests of
Section 6 solve it with the polynomial solution of Section 5.  On top of the discrete
forms of `oracle.assemble` (lowest order) and `oracle.paperk` (order k), in this order:

  1. the DOFs of a boundary face are prescribed: the face moments of u_N = u.n_f
     (eq. facePoly, (1/|f|) int_f u_N m^f_beta, n_f the face's global normal);
  2. their rows and columns become identity rows carrying those values in b, and the
     known fluxes move to the right-hand side of the other rows,
     b_I = -(K x_B)_I and b_p = -F - (K x_B)_p;
  3. the remaining operator has the discrete constant pressure n_p (the moment DOFs of
     p = 1) in its kernel: B^T n_p = 0 on every free flux DOF, because the flux of a
     basis function out of one cell enters the neighbour.  The pressure part of b is
     projected onto the complement of n_p (this removes the quadrature-level mismatch
     between int f and the boundary flux), and of the pressures that solve the system
     the one with zero mean is taken: int_Omega p_h = sum_P |P| p_{P,0} = 0;
  4. the system with that constraint appended as a Lagrange multiplier (one more
     unknown: the "+1" of the paper's DOF counts) is solved by sparse LU.  With the
     projected right-hand side the multiplier is zero.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import boundary_faces, discretize
from .paperk import _face_quadrature, exps2, mono2


def boundary_flux_moments(mesh, fgeo, faces, u, nfd, k, nq):
    """Face moments (1/|f|) int_f (u . n_f) m^f_beta of a vector field u on the given faces."""
    out = np.zeros((len(faces), nfd))
    betas = exps2(k) if nfd > 1 else [(0, 0)]
    for i, f in enumerate(faces):
        X, W = _face_quadrature(mesh, f, nq)
        un = np.asarray(u(X)) @ fgeo["normal"][f]
        m = mono2(X, fgeo["centroid"][f], fgeo["diam"][f], fgeo["e1"][f], fgeo["e2"][f], betas)
        out[i] = (W * un) @ m / fgeo["area"][f]
    return out


def constant_pressure(d, family):
    """n_p: the pressure DOFs (moments) of p = 1, cell by cell."""
    if family == "lo":
        return np.ones(d["Np"])
    return np.concatenate([loc["Hk1"][0] / loc["vol"] for loc in d["local"]])


def mean_weights(d, family):
    """w with w . p = int_Omega p_h: |P| on the moment of the constant, 0 on the others."""
    if family == "lo":
        return d["cgeo"]["volume"].copy()
    npd = d["npd"]
    w = np.zeros(d["Np"])
    w[::npd] = [loc["vol"] for loc in d["local"]]
    return w


def flux_system(mesh, nu=None, rhs=None, family="lo", k=0, nq_load=3, local=None, geo=None):
    """The saddle system with flux boundary data (steps 1-3 above).

    rhs provides f(x) and the flux field u(x); p_D is not used.  Returns the base
    discretisation `d` extended with K_t (identity rows and columns on the prescribed
    DOFs), b_t (projected), the prescribed DOFs `bdofs` and values `uB`, `n_p`, `w` and
    `n_paper` = N + 1, the paper's DOF count."""

    class _Loads:
        f = staticmethod(rhs.f)

        @staticmethod
        def pD(x):
            return 0.0 * x[..., 0]

    d = discretize(mesh, nu=nu, rhs=_Loads(), family=family, k=k, nq_load=nq_load, local=local, geo=geo)
    nfd = 1 if family == "lo" else d["nfd"]
    Nu, Np = d["Nu"], d["Np"]
    N = Nu + Np
    bnd, _ = boundary_faces(mesh)
    bdofs = (bnd[:, None] * nfd + np.arange(nfd)[None, :]).ravel()
    uB = boundary_flux_moments(mesh, d["fgeo"], bnd, rhs.u, nfd, k, nq_load).ravel()
    xB = np.zeros(N)
    xB[bdofs] = uB
    K = d["K"].tocsr()
    b_t = d["b"] - K @ xB  # g = 0: no pressure data
    b_t[bdofs] = uB
    free = np.ones(N)
    free[bdofs] = 0.0
    Fr = sp.diags(free)
    K_t = (Fr @ K @ Fr + sp.diags(1.0 - free)).tocsr()
    K_t.eliminate_zeros()
    n_p = constant_pressure(d, family)
    bp = b_t[Nu:]
    b_t[Nu:] = bp - n_p * (n_p @ bp) / (n_p @ n_p)
    d.update(K_t=K_t, b_t=b_t, bdofs=bdofs, uB=uB, n_p=n_p, w=mean_weights(d, family), n_paper=N + 1)
    return d


def solve_flux(d):
    """Step 4: (u, p, multiplier) from the system with the zero-mean constraint appended."""
    Nu, Np = d["Nu"], d["Np"]
    N = Nu + Np
    c = np.concatenate([np.zeros(Nu), d["w"]])
    A = sp.bmat([[d["K_t"], sp.csr_matrix(c[:, None])], [sp.csr_matrix(c[None, :]), None]], format="csc")
    x = spla.spsolve(A, np.concatenate([d["b_t"], [0.0]]))
    return x[:Nu], x[Nu:N], x[N]
