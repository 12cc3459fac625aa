"""The solver driven from plain C (tests/capi_c/cube_solve.c: include/vem.h and the HIP runtime's C
API only, no Python or PyTorch in the process).

CPU: the C program's cube mesh equals the Python input generator's, array for array.
GPU: its Block-Schur and Block-Reg solutions of the lowest-order sine problem with a log-normal
coefficient equal the oracle's direct solve of the same system (the program runs as a child
process; this process never touches the GPU).
"""
import os
import subprocess

import numpy as np
import pytest

from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "capi_c", "cube_solve")


def _exe():
    if not os.path.exists(EXE):
        pytest.skip("C driver not built (run __graft_entry__.build())")
    return EXE


def _read_mesh(path):
    raw = open(path, "rb").read()
    nv, nf, nc = np.frombuffer(raw, dtype=np.int64, count=3)
    off = 24
    out = {}
    for name, dt, cnt in (("xyz", np.float64, 3 * nv), ("face_ptr", np.int32, nf + 1),
                          ("face_vtx", np.int32, 4 * nf), ("cell_ptr", np.int32, nc + 1),
                          ("cell_face", np.int32, 6 * nc), ("cell_face_sign", np.int8, 6 * nc)):
        a = np.frombuffer(raw, dtype=dt, count=int(cnt), offset=off)
        off += a.nbytes
        out[name] = a
    assert off == len(raw)
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_c_driver_mesh_matches_generator(n, tmp_path):
    path = tmp_path / "mesh.bin"
    r = subprocess.run([_exe(), "--mesh", str(n), str(path)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    c = _read_mesh(path)
    m = cube_mesh(n)
    np.testing.assert_array_equal(c["xyz"].reshape(-1, 3), np.asarray(m["xyz"]))
    for k in ("face_ptr", "face_vtx", "cell_ptr", "cell_face", "cell_face_sign"):
        np.testing.assert_array_equal(c[k].astype(np.int64), np.asarray(m[k]).astype(np.int64).ravel(), err_msg=k)


@pytest.mark.gpu
@pytest.mark.parametrize("n,precond", [(6, "schur"), (9, "schur"), (6, "reg")])
def test_c_driver_solve_matches_oracle(n, precond, tmp_path):
    from oracle.assemble import discretize
    from oracle.solvers import direct_solve

    exe = _exe()
    nu = 1.0 / lognormal_field(n**3, 1.0, 3)
    nu_file, out_file = tmp_path / "nu.bin", tmp_path / "x.bin"
    nu.astype(np.float64).tofile(nu_file)
    print(f"C driver: n={n} precond={precond}", flush=True)
    r = subprocess.run([exe, str(n), str(nu_file), str(out_file), precond], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    n_u, n_p, its, relres, status = r.stdout.split()
    n_u, n_p = int(n_u), int(n_p)
    assert int(status) == 0 and float(relres) <= 1e-12, r.stdout
    x = np.fromfile(out_file, dtype=np.float64)
    assert x.size == n_u + n_p

    d = discretize(cube_mesh(n), nu=nu, rhs=SineSolution())
    assert (d["Nu"], d["K"].shape[0] - d["Nu"]) == (n_u, n_p)
    xo = direct_solve(d["K"], d["b"])
    eu = np.linalg.norm(x[:n_u] - xo[:n_u]) / np.linalg.norm(xo[:n_u])
    ep = np.linalg.norm(x[n_u:] - xo[n_u:]) / np.linalg.norm(xo[n_u:])
    print(f"  iterations={its} relres={relres} err_u={eu:.2e} err_p={ep:.2e}", flush=True)
    assert eu < 1e-9 and ep < 1e-9


@pytest.mark.gpu
def test_c_driver_batched_fields_match_oracle(tmp_path):
    """The batched call from plain C: three coefficient fields set with vem_set_coefficient_batch (host
    memory) and solved with vem_solve_batch; every field against the oracle's direct solve."""
    from oracle.assemble import discretize
    from oracle.solvers import direct_solve

    exe = _exe()
    n, B = 5, 3
    nus = np.stack([1.0 / lognormal_field(n**3, 1.0, 30 + b) for b in range(B)])
    nu_file, out_file = tmp_path / "nu.bin", tmp_path / "x.bin"
    nus.astype(np.float64).tofile(nu_file)
    print(f"C driver batch: n={n} fields={B}", flush=True)
    r = subprocess.run([exe, str(n), str(nu_file), str(out_file), "schur", "batch", str(B)], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.split("\n")
    lines = [l for l in lines if l.strip()]
    assert len(lines) == B
    x = np.fromfile(out_file, dtype=np.float64)
    for b, line in enumerate(lines):
        n_u, n_p, its, relres, status = line.split()
        n_u, n_p = int(n_u), int(n_p)
        assert int(status) == 0 and float(relres) <= 1e-12, line
        xb = x[b * (n_u + n_p):(b + 1) * (n_u + n_p)]
        d = discretize(cube_mesh(n), nu=nus[b], rhs=SineSolution())
        xo = direct_solve(d["K"], d["b"])
        eu = np.linalg.norm(xb[:n_u] - xo[:n_u]) / np.linalg.norm(xo[:n_u])
        ep = np.linalg.norm(xb[n_u:] - xo[n_u:]) / np.linalg.norm(xo[n_u:])
        print(f"  field {b}: iterations={its} err_u={eu:.2e} err_p={ep:.2e}", flush=True)
        assert eu < 1e-9 and ep < 1e-9
