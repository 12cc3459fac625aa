"""Python binding of the C ABI in include/vem.h (argument marshalling only).

Device memory and streams come from PyTorch: every device argument is a
torch CUDA (HIP) tensor.  A Solver is bound to the stream that is current when
it is created (or the one it is given); each wrapper runs on that stream,
ordered after the caller's current stream, and the caller's stream then waits
for it.  All
numerical work runs in the HIP library; if the library is not built, loading
fails with an error (there is no fallback).
"""

from __future__ import annotations

import ctypes
import functools
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_int64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvem_mi355x.so")

VEM_LO, VEM_PAPER = 0, 1
PREC = {"schur": 0, "reg": 1, "none": 2}
MATS = {"K": 0, "schur": 1, "reg": 2, "reg_face": 3, "reg_schwarz": 4}
STATUS = {0: "VEM_OK", 1: "VEM_NOT_CONVERGED", -1: "VEM_EINVAL", -2: "VEM_EBADMESH", -3: "VEM_ENOMEM",
          -4: "VEM_EHIP", -5: "VEM_EBREAKDOWN", -6: "VEM_ENAN"}


class VemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Sizes(ctypes.Structure):
    _fields_ = [
        ("n_vertices", c_int64), ("n_faces", c_int64), ("n_cells", c_int64),
        ("n_u", c_int64), ("n_p", c_int64), ("n", c_int64),
        ("nnz_K", c_int64), ("nnz_schur", c_int64), ("nnz_reg", c_int64),
        ("n_qp_cell", c_int64), ("n_qp_face", c_int64),
        ("load_points", ctypes.c_int32), ("max_cell_faces", ctypes.c_int32),
        ("h", c_double), ("gamma", c_double), ("n_face_dofs", c_int64),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("precond", ctypes.c_int32), ("restart", ctypes.c_int32), ("maxit", ctypes.c_int32),
        ("use_x0", ctypes.c_int32), ("tol", c_double), ("inner_tol", c_double),
        ("inner_maxit", ctypes.c_int32), ("inner_check", ctypes.c_int32), ("gamma", c_double),
        ("precision", ctypes.c_int32), ("use_graphs", ctypes.c_int32), ("inner_form", ctypes.c_int32),
        ("reg_inner", ctypes.c_int32), ("cheb_lo", c_double),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32), ("restarts", ctypes.c_int32), ("inner_iterations", c_int64),
        ("relres", c_double), ("solve_ms", c_double), ("status", ctypes.c_int32),
    ]


_lib = None


def load():
    """Load the HIP library (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime the library binds to)

    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    H = c_void_p
    P = c_void_p
    sigs = {
        "vem_create": ([POINTER(c_void_p), c_void_p], c_int),
        "vem_destroy": ([H], c_int),
        "vem_set_mesh": ([H, c_int64, P, c_int64, P, P, c_int64, P, P, P, c_int], c_int),
        "vem_discretize": ([H, c_int, c_int, c_int], c_int),
        "vem_get_sizes": ([H, POINTER(Sizes)], c_int),
        "vem_get_quadrature": ([H, P, P], c_int),
        "vem_set_coefficient": ([H, P], c_int),
        "vem_set_rhs": ([H, P, P], c_int),
        "vem_solve": ([H, POINTER(SolveOpts), P, P, POINTER(SolveInfo)], c_int),
        "vem_apply": ([H, P, P], c_int),
        "vem_export_csr": ([H, c_int, P, P, P], c_int),
        "vem_get_rhs": ([H, P], c_int),
        "vem_get_geometry": ([H, P, P, P, P, P, P], c_int),
        "vem_status_string": ([c_int], c_char_p),
        "vem_last_error": ([H], c_char_p),
        "vem_solve_opts_default": ([POINTER(SolveOpts)], None),
        "vem_time_kernel": ([H, c_int, c_int, POINTER(c_double), POINTER(c_double)], c_int),
        "vem_solve_rhs": ([H, POINTER(SolveOpts), P, P, P, POINTER(SolveInfo)], c_int),
        "vem_coefficient_gradient": ([H, P, P, P], c_int),
        "vem_set_boundary": ([H, c_int], c_int),
        "vem_set_rhs_flux": ([H, P, P], c_int),
        "vem_set_rhs_noalloc": ([H, P, P], c_int),
        "vem_set_coefficient_batch": ([H, c_int64, P], c_int),
        "vem_set_rhs_batch": ([H, c_int64, P, P], c_int),
        "vem_solve_batch": ([H, POINTER(SolveOpts), c_int64, P, P, POINTER(SolveInfo)], c_int),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _ordered(method):
    """Run a wrapper on the handle's stream, ordered after the caller's current stream, and make the
    caller's stream wait for it afterwards: inputs converted by the caller are complete before the
    library reads them, and outputs (or temporaries freed on return) are not touched by the caller's
    later work before the library's kernels finish.  Without this, entry points that return before
    their kernels end (vem_apply, vem_get_quadrature, ...) could race with a caller on another stream."""

    @functools.wraps(method)
    def run(self, *args, **kwargs):
        t = self.torch
        cur = t.cuda.current_stream(self.device)
        if cur == self.stream:
            return method(self, *args, **kwargs)
        self.stream.wait_stream(cur)
        try:
            with t.cuda.stream(self.stream):
                return method(self, *args, **kwargs)
        finally:
            cur.wait_stream(self.stream)

    return run


class Solver:
    """One mesh + discretisation + solver state on the current device and stream."""

    def __init__(self, stream=None):
        import torch

        self.torch = torch
        self.lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible")
        self.device = torch.device("cuda", torch.cuda.current_device())
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        self.h = c_void_p()
        self._check(self.lib.vem_create(byref(self.h), c_void_p(s.cuda_stream)))
        self._sizes = None
        self.boundary = "pressure"

    # -- helpers
    def _check(self, code):
        if code < 0:
            msg = self.lib.vem_last_error(self.h).decode() if self.h else ""
            raise VemError(code, msg)
        return code

    def close(self):
        if self.h:
            self.lib.vem_destroy(self.h)
            self.h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, dtype):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.device, dtype=dtype).contiguous()
        return t.as_tensor(a, dtype=dtype, device=self.device).contiguous()

    # -- C ABI wrappers
    @_ordered
    def set_mesh(self, mesh):
        t = self.torch
        xyz = self._dev(mesh["xyz"], t.float64)
        fp = self._dev(mesh["face_ptr"], t.int32)
        fv = self._dev(mesh["face_vtx"], t.int32)
        cp = self._dev(mesh["cell_ptr"], t.int32)
        cf = self._dev(mesh["cell_face"], t.int32)
        cs = self._dev(mesh["cell_face_sign"], t.int8)
        self._check(self.lib.vem_set_mesh(self.h, xyz.shape[0], _ptr(xyz), fp.numel() - 1, _ptr(fp), _ptr(fv),
                                          cp.numel() - 1, _ptr(cp), _ptr(cf), _ptr(cs), 1))
        self._sizes = None

    @_ordered
    def discretize(self, family="lo", k=0, load_points=3):
        fam = {"lo": VEM_LO, "paper": VEM_PAPER}[family]
        self._check(self.lib.vem_discretize(self.h, fam, int(k), int(load_points)))
        self._sizes = None

    @_ordered
    def sizes(self):
        if self._sizes is None:
            s = Sizes()
            self._check(self.lib.vem_get_sizes(self.h, byref(s)))
            self._sizes = {f: getattr(s, f) for f, _ in Sizes._fields_}
        return self._sizes

    @_ordered
    def quadrature(self):
        t = self.torch
        sz = self.sizes()
        # the library writes x, y, z as separate arrays; the (n, 3) views keep each column contiguous
        qc = t.empty((3, sz["n_qp_cell"]), dtype=t.float64, device=self.device)
        qf = t.empty((3, sz["n_qp_face"]), dtype=t.float64, device=self.device)
        self._check(self.lib.vem_get_quadrature(self.h, _ptr(qc) if qc.numel() else None,
                                                _ptr(qf) if qf.numel() else None))
        return qc.t(), qf.t()

    @_ordered
    def set_coefficient(self, nu):
        nu = self._dev(nu, self.torch.float64)
        self._check(self.lib.vem_set_coefficient(self.h, _ptr(nu)))

    @_ordered
    def set_rhs(self, f_qp, pD_qp=None):
        f_qp = self._dev(f_qp, self.torch.float64)
        pD = None if pD_qp is None else self._dev(pD_qp, self.torch.float64)
        self._check(self.lib.vem_set_rhs(self.h, _ptr(f_qp), _ptr(pD) if pD is not None and pD.numel() else None))

    @_ordered
    def set_boundary(self, kind):
        """'pressure' (p_D given, the default) or 'flux' (u.n given and zero-mean pressure, the paper's
        model problem)."""
        self._check(self.lib.vem_set_boundary(self.h, {"pressure": 0, "flux": 1}[kind]))
        self.boundary = kind

    @_ordered
    def set_rhs_flux(self, f_qp, u_qp):
        """f at the cell points and the flux field u (n_qp_face, 3) at the boundary points."""
        f_qp = self._dev(f_qp, self.torch.float64)
        u = self._dev(u_qp, self.torch.float64).t().contiguous()  # x, y, z components as separate arrays
        self._check(self.lib.vem_set_rhs_flux(self.h, _ptr(f_qp), _ptr(u) if u.numel() else None))

    def set_rhs_functions(self, f, g=None):
        """Evaluate f, and g at the boundary points, with torch at the library's quadrature points, then
        load them: g is p_D with pressure data, the flux field u (returning (n, 3)) with flux data."""
        qc, qf = self.quadrature()
        fv = f(qc)
        gv = None if g is None else g(qf)
        del qc, qf
        if self.boundary == "flux":
            if gv is None:
                raise ValueError("flux boundary data need the flux field u")
            self.set_rhs_flux(fv, gv)
        else:
            self.set_rhs(fv, gv)

    def _opts(self, precond="schur", tol=1e-8, restart=30, maxit=5000, inner_tol=1e-6, inner_maxit=5000,
              inner_check=32, gamma=0.0, precision="fp64", graphs=False, inner_form="pipelined",
              reg_inner="schwarz", cheb_lo=0.0):
        o = SolveOpts()
        self.lib.vem_solve_opts_default(byref(o))
        o.precond = PREC[precond]
        o.restart, o.maxit, o.tol = int(restart), int(maxit), float(tol)
        o.inner_tol, o.inner_maxit, o.inner_check = float(inner_tol), int(inner_maxit), int(inner_check)
        o.gamma = float(gamma)
        o.precision = {"fp64": 0, "mixed": 1}[precision]
        o.use_graphs = 1 if graphs else 0
        o.inner_form = {"pipelined": 0, "classical": 1, "chebyshev": 2}[inner_form]
        o.reg_inner = {"jacobi": 0, "schwarz": 1}[reg_inner]
        o.cheb_lo = float(cheb_lo)
        return o

    @_ordered
    def set_coefficient_batch(self, nus):
        """nbatch coefficient fields (nbatch, n_cells) for solve_batch."""
        nus = self._dev(nus, self.torch.float64)
        self._check(self.lib.vem_set_coefficient_batch(self.h, nus.shape[0], _ptr(nus)))

    @_ordered
    def set_rhs_batch(self, f_qp, pD_qp=None):
        """nbatch right-hand sides from point values: f_qp (nbatch, n_qp_cell), pD_qp (nbatch, n_qp_face)."""
        f = self._dev(f_qp, self.torch.float64)
        pD = None if pD_qp is None else self._dev(pD_qp, self.torch.float64)
        self._check(self.lib.vem_set_rhs_batch(self.h, f.shape[0], _ptr(f), _ptr(pD) if pD is not None else None))

    @_ordered
    def solve_batch(self, nbatch, **kw):
        """Solve the nbatch systems set by set_coefficient_batch / set_rhs_batch: u (nbatch, n_u),
        p (nbatch, n_p) and one info dict per system."""
        t = self.torch
        sz = self.sizes()
        o = self._opts(**kw)
        u = t.empty((nbatch, sz["n_u"]), dtype=t.float64, device=self.device)
        p = t.empty((nbatch, sz["n_p"]), dtype=t.float64, device=self.device)
        infos = (SolveInfo * nbatch)()
        self._check(self.lib.vem_solve_batch(self.h, byref(o), nbatch, _ptr(u), _ptr(p), infos))
        out = []
        for i in infos:
            d = {f: getattr(i, f) for f, _ in SolveInfo._fields_}
            d["converged"] = d["status"] == 0
            out.append(d)
        return u, p, out

    @_ordered
    def solve(self, precond="schur", tol=1e-8, restart=30, maxit=5000, inner_tol=1e-6, inner_maxit=5000,
              inner_check=32, gamma=0.0, x0=None, precision="fp64", rhs=None, graphs=False,
              inner_form="pipelined", reg_inner="schwarz", cheb_lo=0.0):
        t = self.torch
        sz = self.sizes()
        o = self._opts(precond=precond, tol=tol, restart=restart, maxit=maxit, inner_tol=inner_tol,
                       inner_maxit=inner_maxit, inner_check=inner_check, gamma=gamma, precision=precision,
                       graphs=graphs, inner_form=inner_form, reg_inner=reg_inner, cheb_lo=cheb_lo)
        if x0 is not None:
            u = self._dev(x0[0], t.float64).clone()
            p = self._dev(x0[1], t.float64).clone()
            o.use_x0 = 1
        else:
            u = t.empty(sz["n_u"], dtype=t.float64, device=self.device)
            p = t.empty(sz["n_p"], dtype=t.float64, device=self.device)
        info = SolveInfo()
        if rhs is None:
            code = self._check(self.lib.vem_solve(self.h, byref(o), _ptr(u), _ptr(p), byref(info)))
        else:
            rhs = self._dev(rhs, t.float64)
            assert rhs.numel() == sz["n"]
            code = self._check(self.lib.vem_solve_rhs(self.h, byref(o), _ptr(rhs), _ptr(u), _ptr(p), byref(info)))
        out = {f: getattr(info, f) for f, _ in SolveInfo._fields_}
        out["converged"] = code == 0
        return u, p, out

    @_ordered
    def coefficient_gradient(self, u, lam):
        """g[P] = nu_P lambda_P^T M1_P u_P (flux parts u, lam of length n_u)."""
        t = self.torch
        u = self._dev(u, t.float64)
        lam = self._dev(lam, t.float64)
        g = t.empty(self.sizes()["n_cells"], dtype=t.float64, device=self.device)
        self._check(self.lib.vem_coefficient_gradient(self.h, _ptr(u), _ptr(lam), _ptr(g)))
        return g

    @_ordered
    def apply(self, x):
        t = self.torch
        x = self._dev(x, t.float64)
        y = t.empty_like(x)
        self._check(self.lib.vem_apply(self.h, _ptr(x), _ptr(y)))
        return y

    @_ordered
    def export_csr(self, which="K"):
        t = self.torch
        sz = self.sizes()
        rows = {"K": sz["n"], "schur": sz["n_p"], "reg": sz["n_u"], "reg_face": sz["n_face_dofs"],
                "reg_schwarz": sz["n_face_dofs"]}[which]
        rp = t.empty(rows + 1, dtype=t.int32, device=self.device)
        if which in ("reg_face", "reg_schwarz"):
            # the Schwarz patterns are built on first use: the row offsets give their size
            self._check(self.lib.vem_export_csr(self.h, MATS[which], _ptr(rp), None, None))
            nnz = int(rp[-1].item())
        else:
            nnz = {"K": sz["nnz_K"], "schur": sz["nnz_schur"], "reg": sz["nnz_reg"]}[which]
        col = t.empty(nnz, dtype=t.int32, device=self.device)
        val = t.empty(nnz, dtype=t.float64, device=self.device)
        self._check(self.lib.vem_export_csr(self.h, MATS[which], _ptr(rp), _ptr(col), _ptr(val)))
        return rp, col, val

    @_ordered
    def rhs(self):
        t = self.torch
        b = t.empty(self.sizes()["n"], dtype=t.float64, device=self.device)
        self._check(self.lib.vem_get_rhs(self.h, _ptr(b)))
        return b

    @_ordered
    def time_kernel(self, which="cg_schur", reps=50):
        """Mean duration (ms) of one launch of a hot kernel, timed with HIP events, and its algorithmic bytes."""
        code = {"spmv": 0, "cg_schur": 1, "cg_reg": 2, "cg_schur32": 3, "cg_reg32": 4, "cg_schur32p": 5,
                "cg_reg32p": 6, "cg_reg_schwarz": 7, "cg_reg_schwarz32": 8, "cheb_schur": 9, "cheb_schur32": 10}[which]
        ms, nb = c_double(), c_double()
        self._check(self.lib.vem_time_kernel(self.h, code, int(reps), byref(ms), byref(nb)))
        return ms.value, nb.value

    @_ordered
    def geometry(self):
        t = self.torch
        sz = self.sizes()
        nf, nc = sz["n_faces"], sz["n_cells"]
        out = {
            "area": t.empty(nf, dtype=t.float64, device=self.device),
            "normal": t.empty((nf, 3), dtype=t.float64, device=self.device),
            "fcentroid": t.empty((nf, 3), dtype=t.float64, device=self.device),
            "volume": t.empty(nc, dtype=t.float64, device=self.device),
            "centroid": t.empty((nc, 3), dtype=t.float64, device=self.device),
            "diam": t.empty(nc, dtype=t.float64, device=self.device),
        }
        self._check(self.lib.vem_get_geometry(self.h, _ptr(out["area"]), _ptr(out["normal"]),
                                              _ptr(out["fcentroid"]), _ptr(out["volume"]), _ptr(out["centroid"]),
                                              _ptr(out["diam"])))
        return out


EXPORTED = [
    "vem_solve_opts_default", "vem_create", "vem_destroy", "vem_set_mesh", "vem_discretize", "vem_get_sizes",
    "vem_get_quadrature", "vem_set_coefficient", "vem_set_rhs", "vem_solve", "vem_apply", "vem_export_csr",
    "vem_get_rhs", "vem_get_geometry", "vem_status_string", "vem_last_error", "vem_time_kernel",
    "vem_solve_rhs", "vem_coefficient_gradient", "vem_set_boundary", "vem_set_rhs_flux", "vem_set_rhs_noalloc",
    "vem_set_coefficient_batch", "vem_set_rhs_batch", "vem_solve_batch",
]
