"""Batched solves: many coefficient fields on one mesh, run concurrently on one GPU.

Each field gets its own library handle bound to its own HIP stream (default
priority), so the latency-bound kernels of independent solves (small inner
CG systems, reductions, host convergence checks) overlap on the device's
hardware queues.  Host threads drive the handles (the C ABI releases the
Python interpreter while it runs); every numerical step runs in the HIP
library.  Handles are reused across batches: a field only changes the
coefficient (vem_set_coefficient), not the discretisation.
"""

from __future__ import annotations

import concurrent.futures as cf
import time

import numpy as np


class BatchSolver:
    def __init__(self, mesh, lanes=8, family="lo", k=0, load_points=3, rhs=None):
        import torch

        from .vem import Solver

        self.torch = torch
        self.lanes = lanes
        self.streams = [torch.cuda.Stream() for _ in range(lanes)]
        self.solvers = []
        for st in self.streams:
            with torch.cuda.stream(st):
                s = Solver(stream=st)
                s.set_mesh(mesh)
                s.discretize(family, k=k, load_points=load_points)
                if rhs is not None:
                    s.set_rhs_functions(rhs.f, rhs.pD)
            self.solvers.append(s)
        torch.cuda.synchronize()

    def _one(self, lane, nu, kw):
        torch = self.torch
        s, st = self.solvers[lane], self.streams[lane]
        with torch.cuda.stream(st):
            t0 = time.perf_counter()
            s.set_coefficient(nu)
            u, p, info = s.solve(**kw)
            st.synchronize()
            info["wall_s"] = time.perf_counter() - t0
        return u, p, info

    def solve(self, nus, **kw):
        """Solve for every coefficient field nus[b] (nu = 1/K per cell); returns (us, ps, infos)."""
        B = len(nus)
        out = [None] * B
        with cf.ThreadPoolExecutor(max_workers=self.lanes) as ex:
            futs = {}
            next_b = 0
            free = list(range(self.lanes))
            while next_b < B or futs:
                while free and next_b < B:
                    lane = free.pop()
                    futs[ex.submit(self._one, lane, nus[next_b], kw)] = (lane, next_b)
                    next_b += 1
                done, _ = cf.wait(list(futs), return_when=cf.FIRST_COMPLETED)
                for f in done:
                    lane, b = futs.pop(f)
                    out[b] = f.result()
                    free.append(lane)
        return [o[0] for o in out], [o[1] for o in out], [o[2] for o in out]

    def close(self):
        for s in self.solvers:
            s.close()


def percentiles(infos):
    t = np.array([i["wall_s"] for i in infos])
    return {"p50_s": float(np.percentile(t, 50)), "p99_s": float(np.percentile(t, 99)), "mean_s": float(t.mean())}
