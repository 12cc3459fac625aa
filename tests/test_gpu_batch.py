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
