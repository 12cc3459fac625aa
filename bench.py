"""Benchmark: time to a relative residual of 1e-8 for the mixed-VEM saddle-point solve on one MI355X.

Workload (the path's headline configuration): Cube mesh of [0,1]^3 with 64^3
hexahedra, lowest-order element (one flux moment per face, one pressure per
cell: 798,720 + 262,144 unknowns), per-cell K = exp(g), g ~ N(0, 2^2) i.i.d.
(seed 0), nu = 1/K, f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z), p = 0 on the
boundary, FP64 throughout, FGMRES(30) to ||b - Kx|| <= 1e-8 ||b|| with each
of the paper's two block preconditioners.

One step = the whole hot path on inputs already resident in HBM: mesh in ->
geometry, local matrices, assembly, both preconditioner set-ups
(vem_set_mesh, vem_discretize, vem_set_coefficient), load integration at
the library's quadrature points (vem_set_rhs), then a Block-Schur solve and a
Block-Reg solve (vem_solve), flux and pressure out.

Printed JSON (one line):
  value        seconds per step of assembly + the Block-Schur solve (the
               paper's Schur-complement preconditioner, the faster of the two);
  ms_per_step  the whole step, both solves included;
  solves       per-preconditioner solve times, iterations, true residuals;
  roofline     the dominant kernel, timed live with HIP events;
  cpu_baseline the FP64 CPU oracle on a bounded sample of the same recipe.
"""

from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=64, help="cells per direction of the Cube mesh")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--schur-inner-tol", type=float, default=1e-2)
    ap.add_argument("--reg-inner-tol", type=float, default=1e-1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=32, help="Cube size of the CPU oracle sample")
    ap.add_argument("--summarize", metavar="PREFIX", default=None,
                    help="print a markdown summary of rocprofv3 CSV output PREFIX_kernel_stats.csv / "
                         "PREFIX_kernel_trace.csv and exit")
    return ap.parse_args()


def summarize(prefix: str):
    """Markdown summary of a rocprofv3 --kernel-trace --stats --output-format csv run."""
    import csv
    import statistics

    stats = list(csv.DictReader(open(prefix + "_kernel_stats.csv")))
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| total ms | calls | avg us | min us | max us | % | kernel |", "|---|---|---|---|---|---|---|"]
    for r in stats[:12]:
        out.append(f"| {float(r['TotalDurationNs']) / 1e6:.2f} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} | "
                   f"`{r['Name'][:80]}` |")
    trace = prefix + "_kernel_trace.csv"
    if os.path.exists(trace):
        out += ["", "Per launch grid (threads) of the hot kernels; 'working' launches exclude the ones that found",
                "their solve already converged and returned at once (< 5 us):", "",
                "| kernel | grid | launches | working | avg working us | median us |", "|---|---|---|---|---|---|"]
        by = {}
        for r in csv.DictReader(open(trace)):
            mt = re.search(r"(k_[A-Za-z0-9_]+(?:<[^>]*>)?)\(", r["Kernel_Name"])
            name = mt.group(1) if mt else r["Kernel_Name"][:40]
            if not any(k in name for k in ("k_ppcg_iter", "k_spmv")):
                continue
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            by.setdefault((name, int(r["Grid_Size_X"])), []).append(d)
        for (name, g), ds in sorted(by.items()):
            w = [d for d in ds if d > 5.0] or ds
            out.append(f"| `{name}` | {g} | {len(ds)} | {len(w)} | {sum(w) / len(w):.2f} | "
                       f"{statistics.median(w):.2f} |")
    print("\n".join(out))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(n_gpu: int, n_cpu: int):
    """The oracle (the paper's algorithm: FGMRES + Block-Schur with an exact sparse LU of S) on the
    n_cpu^3 cube of the same recipe, scaled to the n_gpu^3 workload by the number of unknowns."""
    import numpy as np

    from oracle.assemble import discretize
    from oracle.solvers import block_schur, fgmres
    from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field

    m = cube_mesh(n_cpu)
    nu = 1.0 / lognormal_field(n_cpu**3, 2.0, 0)
    t0 = time.perf_counter()
    d = discretize(m, nu=nu, rhs=SineSolution())
    t1 = time.perf_counter()
    pre = block_schur(d["M"], d["B"], inner="exact")
    x, info = fgmres(d["K"], d["b"], pre, m=30, tol=1e-8)
    t2 = time.perf_counter()
    n_small = d["Nu"] + d["Np"]
    n_big = 3 * n_gpu * n_gpu * (n_gpu + 1) + n_gpu**3
    scale = n_big / n_small
    return {
        "value": (t2 - t0) * scale,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle FP64 (NumPy/SciPy, single-threaded sparse phases) on the {n_cpu}^3 cube of the same "
                   f"recipe ({n_small} unknowns): assembly {t1 - t0:.2f} s + FGMRES(30)/Block-Schur with exact "
                   f"sparse LU of S {t2 - t1:.2f} s ({info['iterations']} iterations, relres "
                   f"{info['relres']:.1e}); scaled x{scale:.2f} to {n_big} unknowns by unknown count "
                   f"(a lower bound: the LU grows faster than linearly)"),
        "host_cpus_available": len(os.sched_getaffinity(0)),
    }


def main():
    args = parse()
    if args.summarize:
        summarize(args.summarize)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (the design note on sharding "
              "describes how it would split); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field
    from paper_1901_02330_amd.vem import Solver

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n = args.n
    mesh = cube_mesh(n)
    # inputs resident in HBM before the timed region
    mdev = {k: torch.as_tensor(mesh[k]).to(dev) for k in
            ("xyz", "face_ptr", "face_vtx", "cell_ptr", "cell_face", "cell_face_sign")}
    nu = torch.as_tensor(1.0 / lognormal_field(n**3, 2.0, 0), device=dev)
    solver = Solver()

    def step():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.set_mesh(mdev)
        solver.discretize("lo", load_points=3)
        solver.set_coefficient(nu)
        solver.set_rhs_functions(SineSolution.f, SineSolution.pD)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        u, p, i_s = solver.solve("schur", tol=args.tol, inner_tol=args.schur_inner_tol)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        u2, p2, i_r = solver.solve("reg", tol=args.tol, inner_tol=args.reg_inner_tol, maxit=5000)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        return {"t_ass": t1 - t0, "t_schur": t2 - t1, "t_reg": t3 - t2, "info_schur": i_s, "info_reg": i_r}

    for w in range(args.warmup):
        r = step()
        log(f"warmup {w}: ass {r['t_ass']:.4f}s schur {r['t_schur']:.4f}s reg {r['t_reg']:.4f}s")
    torch.cuda.synchronize()
    results = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        r = step()
        results.append(r)
        log(f"step {k}: ass {r['t_ass']:.4f}s schur {r['t_schur']:.4f}s ({r['info_schur']['iterations']} it, "
            f"{r['info_schur']['inner_iterations']} inner) reg {r['t_reg']:.4f}s "
            f"({r['info_reg']['iterations']} it, {r['info_reg']['inner_iterations']} inner)")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    K = args.steps
    mean = lambda key: sum(r[key] for r in results) / K  # noqa: E731
    for r in results:
        assert r["info_schur"]["converged"] and r["info_reg"]["converged"], "solve did not reach the tolerance"

    # dominant kernel: one pipelined inner-CG iteration; the Block-Reg one carries most of the step
    kern = {}
    for which in ("cg_reg", "cg_schur", "spmv"):
        ms, nbytes = solver.time_kernel(which, reps=200)
        kern[which] = {"avg_us": ms * 1e3, "bytes": nbytes, "gbs": nbytes / (ms * 1e-3) / 1e9}
    dom = kern["cg_reg"]
    sz = solver.sizes()
    line = {
        "metric": "solve time to rel. residual 1e-8 (s) + HBM GB/s in SpMV/precond",
        "value": mean("t_ass") + mean("t_schur"),
        "unit": "s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / K,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"cube{n}^3 lowest-order mixed VEM, K=exp(N(0,2^2)) seed 0, sine manufactured rhs, "
                        f"FGMRES(30) tol {args.tol:g}, Block-Schur and Block-Reg",
            "n_u": sz["n_u"], "n_p": sz["n_p"], "nnz_K": sz["nnz_K"],
        },
        "phases_s": {"assembly": mean("t_ass"), "solve_schur": mean("t_schur"), "solve_reg": mean("t_reg")},
        "solves": {
            "schur": {"iterations": results[-1]["info_schur"]["iterations"],
                      "inner_iterations": results[-1]["info_schur"]["inner_iterations"],
                      "relres": results[-1]["info_schur"]["relres"], "inner_tol": args.schur_inner_tol},
            "reg": {"iterations": results[-1]["info_reg"]["iterations"],
                    "inner_iterations": results[-1]["info_reg"]["inner_iterations"],
                    "relres": results[-1]["info_reg"]["relres"], "inner_tol": args.reg_inner_tol},
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_ppcg_iter (pipelined inner CG iteration on M + B^T B/gamma)",
            "achieved": dom["gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": dom["gbs"] / HBM_PEAK_GBS,
            "traffic": None,
            "avg_launch_us": dom["avg_us"],
            "algorithmic_bytes_per_launch": dom["bytes"],
        },
        "kernels": kern,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline(n, args.cpu_n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
