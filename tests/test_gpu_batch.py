"""Batched solves over many coefficient fields, run concurrently on separate streams, give the same
bits as one-at-a-time solves, and the first field's solution matches the oracle's direct solve."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_batch_matches_sequential():
    import torch

    from paper_1901_02330_amd.batch import BatchSolver, percentiles
    from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field
    from paper_1901_02330_amd.vem import Solver

    print("batch", flush=True)
    m = cube_mesh(12, 10, 9)
    nc = 12 * 10 * 9
    nus = [torch.as_tensor(1.0 / lognormal_field(nc, 1.5, seed), device="cuda") for seed in range(6)]
    torch.cuda.synchronize()
    kw = dict(precond="schur", tol=1e-10, inner_tol=1e-12, inner_maxit=32)
    bs = BatchSolver(m, lanes=3, rhs=SineSolution())
    us, ps, infos = bs.solve(nus, **kw)
    s = Solver()
    s.set_mesh(m)
    s.discretize("lo")
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    for b, nu in enumerate(nus):
        s.set_coefficient(nu)
        u, p, info = s.solve(**kw)
        assert infos[b]["converged"] and infos[b]["iterations"] == info["iterations"]
        assert torch.equal(us[b], u) and torch.equal(ps[b], p)
    print(percentiles(infos), flush=True)
    bs.close()
    # field 0 against the oracle: backward error in the oracle's K within the tolerance, and the
    # solution within the tolerance times this small system's conditioning
    from oracle.assemble import discretize
    from oracle.solvers import direct_solve

    d = discretize(m, nu=nus[0].cpu().numpy(), rhs=SineSolution())
    xg = np.concatenate([us[0].cpu().numpy(), ps[0].cpu().numpy()])
    berr = np.linalg.norm(d["b"] - d["K"] @ xg) / np.linalg.norm(d["b"])
    x = direct_solve(d["K"], d["b"])
    eu = np.linalg.norm(xg[: d["Nu"]] - x[: d["Nu"]]) / np.linalg.norm(x[: d["Nu"]])
    ep = np.linalg.norm(xg[d["Nu"]:] - x[d["Nu"]:]) / np.linalg.norm(x[d["Nu"]:])
    print("field 0 vs oracle: backward error", berr, "u", eu, "p", ep, flush=True)
    assert berr <= 1.01e-10
    assert eu <= 1e-7 and ep <= 1e-7


def test_native_batch_matches_single_solves_and_oracle():
    """vem_set_coefficient_batch / vem_set_rhs_batch / vem_solve_batch: each system of the batch gives the
    same bits as a single solve with that coefficient and right-hand side, the handle's own coefficient
    and right-hand side are unchanged afterwards, and system 0 matches the oracle's direct solve."""
    import torch

    from oracle.assemble import discretize
    from oracle.solvers import direct_solve
    from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field
    from paper_1901_02330_amd.vem import Solver

    print("native batch", flush=True)
    m = cube_mesh(7, 6, 5)
    nc = 210
    B = 4
    nus = np.stack([1.0 / lognormal_field(nc, 1.5, 20 + b) for b in range(B)])
    s = Solver()
    s.set_mesh(m)
    s.discretize("lo")
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    qc, qf = s.quadrature()
    scale = torch.arange(1, B + 1, dtype=torch.float64, device=qc.device)[:, None]
    fb = scale * SineSolution.f(qc)[None, :]          # system b: load (b + 1) f
    pDb = (qf[:, 0] * qf[:, 1])[None, :] * scale       # and p_D = (b + 1) x y
    s.set_coefficient_batch(torch.as_tensor(nus))
    s.set_rhs_batch(fb, pDb)
    b_before = s.rhs().clone()
    kw = dict(precond="schur", tol=1e-12, inner_tol=1e-12, inner_maxit=32)
    ub, pb, infos = s.solve_batch(B, **kw)
    assert all(i["converged"] for i in infos), infos
    assert torch.equal(s.rhs(), b_before)
    ref = Solver()
    ref.set_mesh(m)
    ref.discretize("lo")
    for b in range(B):
        ref.set_coefficient(torch.as_tensor(nus[b]))
        ref.set_rhs(fb[b], pDb[b])
        u, p, info = ref.solve(**kw)
        assert info["iterations"] == infos[b]["iterations"]
        assert torch.equal(u, ub[b]) and torch.equal(p, pb[b]), b
    # system 0 against the oracle (load f, p_D = x y)
    class Rhs0:
        f = staticmethod(SineSolution.f)

        @staticmethod
        def pD(x):
            return x[..., 0] * x[..., 1]

    d = discretize(m, nu=nus[0], rhs=Rhs0())
    x = direct_solve(d["K"], d["b"])
    eu = np.linalg.norm(ub[0].cpu().numpy() - x[: d["Nu"]]) / np.linalg.norm(x[: d["Nu"]])
    ep = np.linalg.norm(pb[0].cpu().numpy() - x[d["Nu"]:]) / np.linalg.norm(x[d["Nu"]:])
    print("system 0 vs oracle", eu, ep, flush=True)
    assert eu <= 1e-9 and ep <= 1e-9
    # the handle's own coefficient (nu = 1) still solves its own system
    u1, p1, i1 = s.solve(**kw)
    d1 = discretize(m, rhs=SineSolution())
    x1 = direct_solve(d1["K"], d1["b"])
    assert np.linalg.norm(u1.cpu().numpy() - x1[: d1["Nu"]]) <= 1e-9 * np.linalg.norm(x1[: d1["Nu"]])
    s.close()
    ref.close()


def test_native_batch_rejects_mismatched_counts():
    """vem_solve_batch needs nbatch coefficient fields or nbatch right-hand sides; other counts are
    rejected with VEM_EINVAL and leave the handle usable."""
    import torch

    from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field
    from paper_1901_02330_amd.vem import Solver, VemError

    m = cube_mesh(4)
    s = Solver()
    s.set_mesh(m)
    s.discretize("lo")
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    with pytest.raises(VemError) as e:
        s.solve_batch(2, precond="schur", tol=1e-10)  # nothing batched yet
    assert e.value.code == -1
    s.set_coefficient_batch(torch.as_tensor(np.stack([1.0 / lognormal_field(64, 1.0, b) for b in range(3)])))
    with pytest.raises(VemError) as e:
        s.solve_batch(2, precond="schur", tol=1e-10)  # 3 fields, 2 systems
    assert e.value.code == -1
    with pytest.raises(VemError) as e:
        s.set_coefficient_batch(torch.as_tensor(np.full((2, 64), -1.0)))  # not positive
    assert e.value.code == -1
    u, p, infos = s.solve_batch(3, precond="schur", tol=1e-10)
    assert all(i["converged"] for i in infos)
    s.close()


def test_native_batch_order2_block_reg_matches_single_solves_and_oracle():
    """The batched order-2 workload in small: the paper's k = 2 element, three log-normal fields,
    Block-Reg with FP32 inner Schwarz-CG (face-block storage) under FP64 FGMRES through
    vem_solve_batch.  Each system gives the same bits as a single solve with its field, and each
    matches the oracle's direct solve: backward error in the oracle's matrix within the tolerance
    (the order-2 matrices agree to about 1e-11 of their largest entries), solution within 1e-7."""
    import torch

    from oracle.assemble import discretize
    from oracle.solvers import direct_solve
    from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field
    from paper_1901_02330_amd.vem import Solver

    print("native batch, order 2", flush=True)
    m = cube_mesh(3, 3, 2)
    nc = 18
    B = 3
    nus = np.stack([1.0 / lognormal_field(nc, 1.5, 40 + b) for b in range(B)])
    s = Solver()
    s.set_mesh(m)
    s.discretize("paper", k=2)
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    kw = dict(precond="reg", tol=1e-10, maxit=1000, inner_tol=1e-2, precision="mixed")
    s.set_coefficient_batch(torch.as_tensor(nus))
    ub, pb, infos = s.solve_batch(B, **kw)
    assert all(i["converged"] for i in infos), infos
    ref = Solver()
    ref.set_mesh(m)
    ref.discretize("paper", k=2)
    ref.set_rhs_functions(SineSolution.f, SineSolution.pD)
    for b in range(B):
        ref.set_coefficient(torch.as_tensor(nus[b]))
        u, p, info = ref.solve(**kw)
        assert info["iterations"] == infos[b]["iterations"]
        assert torch.equal(u, ub[b]) and torch.equal(p, pb[b]), b
        d = discretize(m, nu=nus[b], rhs=SineSolution(), family="paper", k=2)
        xg = np.concatenate([ub[b].cpu().numpy(), pb[b].cpu().numpy()])
        berr = np.linalg.norm(d["b"] - d["K"] @ xg) / np.linalg.norm(d["b"])
        x = direct_solve(d["K"], d["b"])
        eu = np.linalg.norm(xg[: d["Nu"]] - x[: d["Nu"]]) / np.linalg.norm(x[: d["Nu"]])
        ep = np.linalg.norm(xg[d["Nu"]:] - x[d["Nu"]:]) / np.linalg.norm(x[d["Nu"]:])
        print("system", b, infos[b]["iterations"], "backward error", berr, "u", eu, "p", ep, flush=True)
        assert berr <= 1e-10 and eu <= 1e-7 and ep <= 1e-7
    s.close()
    ref.close()
