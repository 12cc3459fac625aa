"""Linear solvers for the saddle-point system (Section 5 of the paper).

* direct_solve: sparse LU of the whole matrix (the role the paper gives
  to its direct solver; here only a correctness reference).
* fgmres: right-preconditioned restarted flexible GMRES with classical
  Gram-Schmidt applied twice, zero initial guess by default, stopping on the
  relative residual ||b - K x|| / ||b|| (the paper uses GMRES; restart,
  orthogonalisation and stopping rule are not stated there).
* block_schur (eq. block_schur): B_1 = diag(M); B_2^{-1} solves the
  approximate Schur complement S = B diag(M)^{-1} B^T (taken with the sign
  that makes it SPD), exactly by sparse LU or by Jacobi-preconditioned CG
  to a relative tolerance.
* block_reg (eq. block_diag): B_1^{-1} approximates (M + gamma^{-1} B^T B)^{-1}
  (exact LU, or Jacobi-preconditioned CG), B_2^{-1} = gamma^{-1} I,
  W = gamma I with gamma = h^2.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def direct_solve(K, b):
    return spla.spsolve(sp.csc_matrix(K), b)


def pcg_jacobi(A, rhs, tol=1e-6, maxit=10000, dinv=None):
    """Jacobi-preconditioned conjugate gradients from x = 0.

    Stops when r.z <= tol^2 * r0.z0 (relative preconditioned residual).
    Returns (x, iterations).
    """
    if dinv is None:
        dinv = 1.0 / A.diagonal()
    x = np.zeros_like(rhs)
    r = rhs.copy()
    z = dinv * r
    p = z.copy()
    rho = r @ z
    rho0 = rho
    it = 0
    if rho0 == 0.0:
        return x, 0
    while it < maxit and rho > tol * tol * rho0:
        q = A @ p
        alpha = rho / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = dinv * r
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
        it += 1
    return x, it


class block_schur:
    """Block-Schur preconditioner: diag(M)^{-1} on the flux block, S^{-1} on the pressure block."""

    def __init__(self, M, B, inner="exact", tol=1e-6, maxit=10000):
        self.Nu = M.shape[0]
        self.dM = M.diagonal().copy()
        self.S = (B @ sp.diags(1.0 / self.dM) @ B.T).tocsr()
        self.inner, self.tol, self.maxit = inner, tol, maxit
        self.lu = spla.splu(sp.csc_matrix(self.S)) if inner == "exact" else None
        self.inner_its = 0

    def __call__(self, r):
        zu = r[: self.Nu] / self.dM
        if self.lu is not None:
            zp = self.lu.solve(r[self.Nu:])
        else:
            zp, it = pcg_jacobi(self.S, r[self.Nu:], self.tol, self.maxit)
            self.inner_its += it
        return np.concatenate([zu, zp])


class block_reg:
    """Block-Reg preconditioner: (M + B^T B / gamma)^{-1} on the flux block, I / gamma on the pressure block."""

    def __init__(self, M, B, gamma, inner="exact", tol=1e-6, maxit=10000):
        self.Nu = M.shape[0]
        self.gamma = float(gamma)
        self.A = (M + (B.T @ B) / self.gamma).tocsr()
        self.inner, self.tol, self.maxit = inner, tol, maxit
        self.lu = spla.splu(sp.csc_matrix(self.A)) if inner == "exact" else None
        self.inner_its = 0

    def __call__(self, r):
        if self.lu is not None:
            zu = self.lu.solve(r[: self.Nu])
        else:
            zu, it = pcg_jacobi(self.A, r[: self.Nu], self.tol, self.maxit)
            self.inner_its += it
        return np.concatenate([zu, r[self.Nu:] / self.gamma])


def fgmres(K, b, prec=None, m=30, tol=1e-10, maxit=10000, x0=None):
    """Right-preconditioned restarted FGMRES(m) with CGS2.  Returns (x, info)."""
    N = len(b)
    x = np.zeros(N) if x0 is None else np.array(x0, dtype=np.float64)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros(N), {"iterations": 0, "relres": 0.0, "converged": True, "history": []}
    if prec is None:
        prec = lambda v: v  # noqa: E731
    r = b - K @ x
    beta = np.linalg.norm(r)
    its = 0
    hist = [beta / bn]
    while beta / bn > tol and its < maxit:
        V = np.zeros((m + 1, N))
        Z = np.zeros((m, N))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        gv = np.zeros(m + 1)
        gv[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(m):
            Z[j] = prec(V[j])
            w = K @ Z[j]
            for _ in range(2):
                h = V[: j + 1] @ w
                w = w - V[: j + 1].T @ h
                H[: j + 1, j] += h
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gv[j + 1] = -sn[j] * gv[j]
            gv[j] = cs[j] * gv[j]
            its += 1
            j_end = j + 1
            hist.append(abs(gv[j + 1]) / bn)
            if abs(gv[j + 1]) / bn <= tol or its >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_end, :j_end]), gv[:j_end])
        x = x + Z[:j_end].T @ y
        r = b - K @ x
        beta = np.linalg.norm(r)
    return x, {"iterations": its, "relres": beta / bn, "converged": beta / bn <= tol, "history": hist}
