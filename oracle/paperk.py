"""The paper's order-k mixed virtual element (Sections 2 and 4), k >= 1.

Local space (eq. vectSpaceDef): v.n_f in P_k(f) on every face, div v in
P_{k-1}(P), curl v in [P_{k-1}(P)]^3.  Degrees of freedom:
  * face moments (eq. facePoly): (1/|f|) int_f (v.n_f) m^f_beta, beta in M_k(f);
  * gradient moments (eq. gradMom): (h_P/|P|) int_P v.grad m_alpha,
    alpha in M_{k-1}(P) minus the constant;
  * cross moments (eq. crossMom): (1/|P|) int_P v.(m_I x m), m in the set
    M^{G,+}_{k-1}(P) = {(m,0,0): m in N_{k-1}} u {(0,m,0), (0,0,m): m in M_{k-1}},
    with N_{k-1} the monomials of degree <= k-1 without x (the constant
    included: reading R2, needed for the set to span G^+_k).
Pressure (eq. presSpace, presMom): P_{k-1}(P), DOFs (1/|P|) int_P q m_alpha.

Computation, in the order of Section 4.1 and 4.3 (everything per cell, in
the cell's outward orientation; monomial integrals by quadrature exact for
the degrees involved):
  1. D[i, j] = dof_i(m_j) for the vector monomials m_j = e_c m_alpha, alpha in M_k;
  2. v.n_f on a face from the face moments (face Gram system), div v from the
     moments by integration by parts and the cell Gram system H_{k-1};
  3. int_P phi_i . m_j through the decomposition of Props. xDec, yDec, zDec
     and inTermsOfGPerpBasis (gradient part: a gradient moment when the degree
     is at most k-1, integration by parts otherwise; cross part: cross moments);
  4. Pi* = G^{-1} B_proj, G = I_3 (x) H_k;
  5. M_P = nu [Pi*^T G Pi* + |P| (I - D Pi*)^T (I - D Pi*)] (stabilisation
     s_P = nu |P| sum of DOF products);
  6. B_div,P[g, i] = int_P div phi_i psi_g with psi dual to the pressure
     moments, loads F_P[g] = int_P f psi_g, boundary g_i = -int p_D phi_i.n.
Local DOF order: face DOFs face by face (beta graded), then gradient moments
(alpha graded), then cross moments (x part, y part, z part).
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .geometry import cell_geometry, face_geometry
from .quadrature import map_tets, map_tris


# ---------------------------------------------------------------------------------------------
# multi-indices and counts (Section 2)
def exps3(k):
    """Multi-indices alpha with |alpha| <= k, graded, then x-power descending, then y-power descending."""
    out = []
    for d in range(k + 1):
        for a1 in range(d, -1, -1):
            for a2 in range(d - a1, -1, -1):
                out.append((a1, a2, d - a1 - a2))
    return out


def exps2(k):
    out = []
    for d in range(k + 1):
        for b1 in range(d, -1, -1):
            out.append((b1, d - b1))
    return out


def dim_P3(k):
    return 0 if k < 0 else (k + 1) * (k + 2) * (k + 3) // 6


def dim_P2(k):
    return 0 if k < 0 else (k + 1) * (k + 2) // 2


def dim_Gplus(k):
    """dim G^+_k(P) = (2k^3 + 9k^2 + 7k)/6 (eq. dimGperp)."""
    return (2 * k**3 + 9 * k**2 + 7 * k) // 6


def cross_set(k):
    """M^{G,+}_{k-1}: list of (component d, alpha) in DOF order."""
    Mk1 = exps3(k - 1)
    N = [a for a in Mk1 if a[0] == 0]
    return [(0, a) for a in N] + [(1, a) for a in Mk1] + [(2, a) for a in Mk1]


def counts(k):
    nfd = dim_P2(k)
    ng = dim_P3(k - 1) - 1
    nc = len(cross_set(k))
    npd = dim_P3(k - 1)
    return nfd, ng, nc, npd


def paper_dofs(n_faces, n_cells, k):
    """Total DOF count of the paper's set-up (flux BC + one global mean constraint: the '+1')."""
    nfd, ng, nc, npd = counts(k)
    return nfd * n_faces + (ng + nc) * n_cells + npd * n_cells + 1


def mono3(X, xP, hP, alphas):
    """Scaled monomials m_alpha((x - x_P)/h_P) at points X (..., 3) -> (..., len(alphas))."""
    Y = (X - xP) / hP
    return np.stack([Y[..., 0] ** a[0] * Y[..., 1] ** a[1] * Y[..., 2] ** a[2] for a in alphas], -1)


def mono2(X, xf, hf, e1, e2, betas):
    Y = X - xf
    s = (Y @ e1) / hf
    t = (Y @ e2) / hf
    return np.stack([s ** b[0] * t ** b[1] for b in betas], -1)


def _sub(a, i, d=1):
    b = list(a)
    b[i] -= d
    return tuple(b)


def _add(a, i, d=1):
    b = list(a)
    b[i] += d
    return tuple(b)


def decompose(c, alpha, hP):
    """e_c m_alpha = g grad m_beta + sum_t coef_t m_I x (e_{d_t} m_{mu_t}) (Props. xDec, yDec, zDec),
    with x-component cross terms whose monomial contains x rewritten by Prop. inTermsOfGPerpBasis.
    Returns (g, beta, [(coef, d, mu), ...])."""
    s = sum(alpha) + 1
    beta = _add(alpha, c)
    terms = []
    a1, a2, a3 = alpha
    if c == 0:
        terms += [(-a3 / s, 1, _sub(alpha, 2)), (a2 / s, 2, _sub(alpha, 1))]
    elif c == 1:
        terms += [(a3 / s, 0, _sub(alpha, 2)), (-a1 / s, 2, _sub(alpha, 0))]
    else:
        terms += [(a1 / s, 1, _sub(alpha, 0)), (-a2 / s, 0, _sub(alpha, 1))]
    out = []
    for coef, d, mu in terms:
        if coef == 0.0:
            continue
        if d == 0 and mu[0] >= 1:
            # m_I x (m_mu,0,0) = -m_I x (0,m_{mu-e1+e2},0) - m_I x (0,0,m_{mu-e1+e3})
            out.append((-coef, 1, _add(_sub(mu, 0), 1)))
            out.append((-coef, 2, _add(_sub(mu, 0), 2)))
        else:
            out.append((coef, d, mu))
    return hP / s, beta, out


EPS = np.zeros((3, 3, 3))
EPS[0, 1, 2] = EPS[1, 2, 0] = EPS[2, 0, 1] = 1.0
EPS[0, 2, 1] = EPS[2, 1, 0] = EPS[1, 0, 2] = -1.0


# ---------------------------------------------------------------------------------------------
def _cell_quadrature(mesh, cgeo, P, n):
    xyz = mesh["xyz"]
    fp, fv = mesh["face_ptr"], mesh["face_vtx"]
    cp, cf, cs = mesh["cell_ptr"], mesh["cell_face"], mesh["cell_face_sign"]
    O, A, B, C, S = [], [], [], [], []
    for j in range(cp[P], cp[P + 1]):
        f = cf[j]
        loop = fv[fp[f]:fp[f + 1]]
        for a in range(1, len(loop) - 1):
            O.append(cgeo["xref"][P])
            A.append(xyz[loop[0]])
            B.append(xyz[loop[a]])
            C.append(xyz[loop[a + 1]])
            S.append(float(cs[j]))
    X, W = map_tets(np.array(O), np.array(A), np.array(B), np.array(C), n, sign=np.array(S))
    return X.reshape(-1, 3), W.ravel()


def _face_quadrature(mesh, f, n):
    xyz = mesh["xyz"]
    loop = mesh["face_vtx"][mesh["face_ptr"][f]:mesh["face_ptr"][f + 1]]
    A = np.array([xyz[loop[0]]] * (len(loop) - 2))
    B = np.array([xyz[loop[a]] for a in range(1, len(loop) - 1)])
    C = np.array([xyz[loop[a + 1]] for a in range(1, len(loop) - 1)])
    X, W = map_tris(A, B, C, n)
    return X.reshape(-1, 3), W.ravel()


def local_element(mesh, fgeo, cgeo, P, k, nq=None):
    """Local matrices of cell P (nu = 1): dict with D, PiStar, M1, Bdiv, Hf^-1 data, ..."""
    nq = nq if nq is not None else k + 2
    cp, cf, cs = mesh["cell_ptr"], mesh["cell_face"], mesh["cell_face_sign"]
    faces = cf[cp[P]:cp[P + 1]].astype(np.int64)
    sig = cs[cp[P]:cp[P + 1]].astype(np.float64)
    F = len(faces)
    xP, hP, vol = cgeo["centroid"][P], cgeo["diam"][P], cgeo["volume"][P]
    Mk, Mk1, Mk2 = exps3(k), exps3(k - 1), exps3(k + 1)
    idx = {a: i for i, a in enumerate(Mk2)}
    Fk = exps2(k)
    nfd, ng, nc, npd = counts(k)
    ns = len(Mk)
    grad_set = Mk1[1:]
    gidx = {a: i for i, a in enumerate(grad_set)}
    xset = cross_set(k)
    xidx = {t: i for i, t in enumerate(xset)}
    ndof = F * nfd + ng + nc
    o_g, o_c = F * nfd, F * nfd + ng

    # cell integrals of products of monomials (degree <= 2k + 1)
    Xc, Wc = _cell_quadrature(mesh, cgeo, P, nq)
    m2 = mono3(Xc, xP, hP, Mk2)  # (q, |M_{k+1}|)
    mI = mono3(Xc, xP, hP, [(1, 0, 0), (0, 1, 0), (0, 0, 1)])

    def cint(*cols):
        v = Wc.copy()
        for c in cols:
            v = v * c
        return v.sum()

    H = np.array([[cint(m2[:, idx[a]], m2[:, idx[b]]) for b in Mk] for a in Mk])
    Hk1 = H[: len(Mk1), : len(Mk1)]

    # face data: Gram H_f, T_f = |f| H_f^{-1}, FM[j] = int_f m^f_delta m_gamma (gamma in M_{k+1})
    T, FM = [], []
    for j, f in enumerate(faces):
        Xf, Wf = _face_quadrature(mesh, f, nq)
        mf = mono2(Xf, fgeo["centroid"][f], fgeo["diam"][f], fgeo["e1"][f], fgeo["e2"][f], Fk)
        Hf = (Wf[:, None, None] * mf[:, :, None] * mf[:, None, :]).sum(0)
        T.append(fgeo["area"][f] * np.linalg.inv(Hf))
        mc = mono3(Xf, xP, hP, Mk2)
        FM.append((Wf[:, None, None] * mf[:, :, None] * mc[:, None, :]).sum(0))

    # 1. DOF matrix of the vector monomials, columns j = c * ns + a
    D = np.zeros((ndof, 3 * ns))
    for c in range(3):
        for a, al in enumerate(Mk):
            col = c * ns + a
            for j, f in enumerate(faces):
                n_out = sig[j] * fgeo["normal"][f]
                D[j * nfd:(j + 1) * nfd, col] = n_out[c] * FM[j][:, idx[al]] / fgeo["area"][f]
            for g, ga in enumerate(grad_set):
                if ga[c] > 0:
                    D[o_g + g, col] = ga[c] * cint(m2[:, idx[al]], m2[:, idx[_sub(ga, c)]]) / vol
            for x, (d, mu) in enumerate(xset):
                s = sum(EPS[c, aa, d] * cint(m2[:, idx[al]], m2[:, idx[mu]], mI[:, aa]) for aa in range(3))
                D[o_c + x, col] = s / vol

    # 2. R[gamma, i] = int_P div phi_i m_gamma (integration by parts), div phi_i = H_{k-1}^{-1} R
    R = np.zeros((len(Mk1), ndof))
    for g, ga in enumerate(Mk1):
        if sum(ga) >= 1:
            R[g, o_g + gidx[ga]] -= vol / hP
        for j in range(F):
            R[g, j * nfd:(j + 1) * nfd] += T[j].T @ FM[j][:, idx[ga]]
    cdiv = np.linalg.solve(Hk1, R)

    # 3. B_proj[(c, alpha), i] = int_P phi_i . e_c m_alpha
    Bp = np.zeros((3 * ns, ndof))
    for c in range(3):
        for a, al in enumerate(Mk):
            row = c * ns + a
            gco, beta, terms = decompose(c, al, hP)
            if 1 <= sum(beta) <= k - 1:
                Bp[row, o_g + gidx[beta]] += gco * vol / hP
            else:
                # - int div phi_i m_beta + sum_f int_f (phi_i . n) m_beta
                Hb = np.array([cint(m2[:, idx[ga]], m2[:, idx[beta]]) for ga in Mk1])
                Bp[row] += gco * (-(Hb @ cdiv))
                for j in range(F):
                    Bp[row, j * nfd:(j + 1) * nfd] += gco * (T[j].T @ FM[j][:, idx[beta]])
            for coef, d, mu in terms:
                Bp[row, o_c + xidx[(d, mu)]] += coef * vol

    # 4. projector
    G = np.kron(np.eye(3), H)
    PiS = np.linalg.solve(G, Bp)
    # 5. local forms (nu = 1)
    IDP = np.eye(ndof) - D @ PiS
    M1 = PiS.T @ G @ PiS + vol * IDP.T @ IDP
    # 6. divergence form with the pressure basis dual to the moments
    Bdiv = vol * cdiv
    return {"faces": faces, "sign": sig, "D": D, "PiStar": PiS, "M1": M1, "Bdiv": Bdiv, "G": G,
            "Hk1": Hk1, "T": T, "ndof": ndof, "vol": vol}


def paper_local(mesh, fgeo, cgeo, k, nq=None):
    nc = len(mesh["cell_ptr"]) - 1
    return [local_element(mesh, fgeo, cgeo, P, k, nq) for P in range(nc)]


def paper_loads(mesh, cgeo, local, k, f, nq_load):
    """F_P[g] = int_P f psi_g = sum_a (|P| H_{k-1}^{-1})_{a g} int_P f m_a."""
    Mk1 = exps3(k - 1)
    out = []
    for P, loc in enumerate(local):
        X, W = _cell_quadrature(mesh, cgeo, P, nq_load)
        m = mono3(X, cgeo["centroid"][P], cgeo["diam"][P], Mk1)
        fm = (W * f(X))[:, None] * m
        out.append(loc["vol"] * np.linalg.solve(loc["Hk1"], fm.sum(0)))
    return np.concatenate(out)


def discretize_paper(mesh, nu=None, rhs=None, k=2, local=None, geo=None, nq=None, nq_load=3):
    """Global saddle system for the paper's order-k element (same conventions as the lowest order)."""
    from .assemble import boundary_faces

    nf = len(mesh["face_ptr"]) - 1
    nc = len(mesh["cell_ptr"]) - 1
    if geo is None:
        fgeo, cgeo = face_geometry(mesh), cell_geometry(mesh)
    else:
        fgeo, cgeo = geo
    if local is None:
        local = paper_local(mesh, fgeo, cgeo, k, nq)
    nu = np.ones(nc) if nu is None else np.asarray(nu, dtype=np.float64)
    nfd, ng, ncx, npd = counts(k)
    nint = ng + ncx
    Nu, Np = nf * nfd + nc * nint, nc * npd
    rows, cols, vals, br, bc, bv = [], [], [], [], [], []
    for P, loc in enumerate(local):
        F = len(loc["faces"])
        gid = np.concatenate([np.repeat(loc["faces"] * nfd, nfd) + np.tile(np.arange(nfd), F),
                              nf * nfd + P * nint + np.arange(nint)])
        sg = np.concatenate([np.repeat(loc["sign"], nfd), np.ones(nint)])
        Mg = nu[P] * loc["M1"] * sg[:, None] * sg[None, :]
        rows.append(np.repeat(gid, len(gid)))
        cols.append(np.tile(gid, len(gid)))
        vals.append(Mg.ravel())
        br.append(np.repeat(P * npd + np.arange(npd), len(gid)))
        bc.append(np.tile(gid, npd))
        bv.append((loc["Bdiv"] * sg[None, :]).ravel())
    M = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(Nu, Nu))
    Bdiv = sp.csr_matrix((np.concatenate(bv), (np.concatenate(br), np.concatenate(bc))), shape=(Np, Nu))
    M.sum_duplicates()
    Bdiv.sum_duplicates()
    B = -Bdiv
    K = sp.bmat([[M, B.T], [B, None]], format="csr")
    g = np.zeros(Nu)
    Fl = np.zeros(Np)
    if rhs is not None:
        Fl = paper_loads(mesh, cgeo, local, k, rhs.f, nq_load)
        bnd, bsg = boundary_faces(mesh)
        Fk = exps2(k)
        for f, s in zip(bnd, bsg):
            Xf, Wf = _face_quadrature(mesh, f, nq_load)
            mf = mono2(Xf, fgeo["centroid"][f], fgeo["diam"][f], fgeo["e1"][f], fgeo["e2"][f], Fk)
            ipd = (Wf * rhs.pD(Xf))[:, None] * mf
            # the face function phi_(f,b).n_f = sum_d T[d, b] m^f_d, T = |f| H_f^{-1}
            Hf = (Wf[:, None, None] * mf[:, :, None] * mf[:, None, :]).sum(0)
            Tf = fgeo["area"][f] * np.linalg.inv(Hf)
            g[f * nfd:(f + 1) * nfd] = -s * (Tf.T @ ipd.sum(0))
    return {"fgeo": fgeo, "cgeo": cgeo, "local": local, "nu": nu, "M": M, "Bdiv": Bdiv, "B": B, "K": K,
            "g": g, "F": Fl, "b": np.concatenate([g, -Fl]), "Nu": Nu, "Np": Np, "k": k,
            "nfd": nfd, "nint": nint, "npd": npd}


def interpolate_paper(mesh, d, sol, nq=None):
    """DOFs of the exact flux (face moments w.r.t. n_f, gradient and cross moments) and pressure moments."""
    k = d["k"]
    nq = nq if nq is not None else k + 3
    fgeo, cgeo = d["fgeo"], d["cgeo"]
    nfd, nint, npd = d["nfd"], d["nint"], d["npd"]
    nf = len(mesh["face_ptr"]) - 1
    nc = len(mesh["cell_ptr"]) - 1
    Fk, Mk1 = exps2(k), exps3(k - 1)
    grad_set, xset = Mk1[1:], cross_set(k)
    u = np.zeros(d["Nu"])
    p = np.zeros(d["Np"])
    for f in range(nf):
        Xf, Wf = _face_quadrature(mesh, f, nq)
        mf = mono2(Xf, fgeo["centroid"][f], fgeo["diam"][f], fgeo["e1"][f], fgeo["e2"][f], Fk)
        un = sol.u(Xf) @ fgeo["normal"][f]
        u[f * nfd:(f + 1) * nfd] = ((Wf * un)[:, None] * mf).sum(0) / fgeo["area"][f]
    for P in range(nc):
        X, W = _cell_quadrature(mesh, cgeo, P, nq)
        xP, hP, vol = cgeo["centroid"][P], cgeo["diam"][P], cgeo["volume"][P]
        U = sol.u(X)
        Y = (X - xP) / hP
        o = nf * nfd + P * nint
        for g, ga in enumerate(grad_set):
            grad = np.zeros_like(X)
            for c in range(3):
                if ga[c] > 0:
                    e = list(ga)
                    e[c] -= 1
                    grad[:, c] = ga[c] / hP * Y[:, 0] ** e[0] * Y[:, 1] ** e[1] * Y[:, 2] ** e[2]
            u[o + g] = hP / vol * (W * (U * grad).sum(1)).sum()
        for x, (dd, mu) in enumerate(xset):
            m = Y[:, 0] ** mu[0] * Y[:, 1] ** mu[1] * Y[:, 2] ** mu[2]
            ev = np.zeros_like(X)
            ev[:, dd] = m
            w = np.cross(Y, ev)
            u[o + len(grad_set) + x] = (W * (U * w).sum(1)).sum() / vol
        mq = mono3(X, xP, hP, Mk1)
        p[P * npd:(P + 1) * npd] = ((W * sol.p(X))[:, None] * mq).sum(0) / vol
    return u, p
