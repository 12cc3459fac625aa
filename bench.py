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

Inner solves: Block-Schur applies S^{-1} by a Chebyshev-Jacobi polynomial of degree 24 on
[hi/400, hi] (hi the Gershgorin bound of D^{-1}S); Block-Reg applies A_gamma^{-1} by CG with the
edge-patch Schwarz preconditioner to a relative tolerance of 0.1, capped at 24 iterations.

Printed JSON (one line):
  value          seconds per step of assembly + the Block-Schur solve (the
                 paper's Schur-complement preconditioner, the faster of the two);
  ms_per_step    the whole step, both solves included;
  solves         per-preconditioner solve times, iterations, true residuals;
  roofline       the step's dominant kernel (Block-Reg's inner iteration), timed live with HIP events;
  roofline_value the kernel that dominates `value` (the Chebyshev product on S);
  kernels        every hot kernel's live rate, with its algorithmic bytes;
  cpu_baseline   the FP64 CPU oracle on the same 64^3 workload (assembly + Block-Schur solve).
"""

from __future__ import annotations

import argparse
import json
import os
import re
import statistics
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
    ap.add_argument("--schur-inner-form", default="chebyshev", choices=("chebyshev", "pipelined", "classical"))
    ap.add_argument("--schur-inner-tol", type=float, default=1e-12, help="CG inner forms only")
    ap.add_argument("--schur-inner-maxit", type=int, default=24, help="degree (Chebyshev) or iteration cap (CG)")
    ap.add_argument("--cheb-lo", type=float, default=1.0 / 400.0)
    ap.add_argument("--reg-inner-tol", type=float, default=1e-1)
    ap.add_argument("--reg-inner-maxit", type=int, default=24)
    ap.add_argument("--reg-inner", default="schwarz", choices=("schwarz", "jacobi"))
    ap.add_argument("--no-extras", action="store_true", help="skip the adjoint / mixed / batch / 128^3 measurements")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="short run for rocprofv3 --pmc: discretize, 20 launches of each hot kernel, and a plain "
                         "256 MiB device copy that calibrates FETCH_SIZE / WRITE_SIZE")
    ap.add_argument("--k2-batch", type=int, default=0, metavar="FIELDS",
                    help="also time FIELDS log-normal fields (sigma 1.5, seeds 0..) on the Cube 32^3 k=2 mesh: "
                         "Block-Reg with FP32 inner solves, sequential and on FIELDS concurrent lanes (minutes)")
    ap.add_argument("--voronoi-checkerboard", action="store_true",
                    help="also solve the mixed-precision workload: Random Voronoi 20,000 cells, the paper's k = 2, "
                         "checkerboard K in {1e-3, 1e3}, Block-Reg with FP32 and FP64 inner solves (minutes)")
    ap.add_argument("--k2-fields-only", type=int, default=0, metavar="FIELDS",
                    help="run only the batched order-2 workload (FIELDS fields on Cube 32^3 through "
                         "vem_solve_batch), print its JSON and exit (for kernel traces)")
    ap.add_argument("--voronoi-sweep", action="store_true",
                    help="also run the order-2 sweep on Random Voronoi meshes of 1,000 to 16,000 cells, flux data (minutes)")
    ap.add_argument("--voronoi-checkerboard-only", action="store_true",
                    help="run only the Voronoi checkerboard solve with FP32 inner solves, print its JSON and exit "
                         "(for kernel traces)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=0, help="Cube size of the CPU oracle run (default: the workload's)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="print the HBM-traffic summary of two rocprofv3 --pmc runs of --pmc-probe and exit")
    ap.add_argument("--summarize", metavar="PREFIX", default=None,
                    help="print a markdown summary of rocprofv3 CSV output PREFIX_kernel_stats.csv / "
                         "PREFIX_kernel_trace.csv and exit")
    return ap.parse_args()


def kernel_short(full: str):
    """A kernel's name with its template arguments (nested brackets kept), without the namespaces;
    None when the name holds no library kernel."""
    t = full.replace("vem::(anonymous namespace)::", "")
    m = re.search(r"\bk_[A-Za-z0-9_]+", t)
    if not m:
        return None
    i = m.end()
    if i < len(t) and t[i] == "<":
        depth = 0
        for j in range(i, len(t)):
            depth += {"<": 1, ">": -1}.get(t[j], 0)
            if depth == 0:
                return t[m.start():j + 1]
    return m.group(0)


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
        out += ["", "Per launch grid (threads) of the hot kernels; 'working' excludes launches under 3 us (launches",
                "enqueued after their inner solve converged return at once):", "",
                "| kernel | grid | launches | working | avg working us | median us |", "|---|---|---|---|---|---|"]
        by = {}
        for r in csv.DictReader(open(trace)):
            name = kernel_short(r["Kernel_Name"]) or r["Kernel_Name"][:40]
            if not any(k in name for k in ("k_ppcg_iter", "k_spmv", "k_scg_", "k_cheb_iter")):
                continue
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            by.setdefault((name, int(r["Grid_Size_X"])), []).append(d)
        for (name, g), ds in sorted(by.items()):
            w = [d for d in ds if d > 3.0] or ds
            out.append(f"| `{name}` | {g} | {len(ds)} | {len(w)} | {sum(w) / len(w):.2f} | "
                       f"{statistics.median(w):.2f} |")
        # the live timing loops (vem_time_kernel, 200 launches each) run after the solves: the last 200
        # launches of each roofline kernel (FP64), the Chebyshev product's middle variant
        out += ["", "The live timing loops (the last 200 launches of each roofline kernel, FP64):", "",
                "| kernel | grid | mean us | median us |", "|---|---|---|---|"]
        pair = 0.0
        # the Chebyshev product's middle variant, whatever its row form (fixed count, masked or loop)
        for pref in ("k_scg_prod<double,", "k_scg_update<double,", r"k_cheb_iter<double, [^,]+, false, false>"):
            it = [k for k in by if re.match(re.escape(pref) if pref.startswith("k_scg") else pref, k[0])]
            if not it:
                continue
            key = max(it, key=lambda k: k[1])
            last = by[key][-200:]
            mean = sum(last) / len(last)
            if pref.startswith("k_scg_"):
                pair += mean
            out.append(f"| `{key[0]}` | {key[1]} | {mean:.2f} | {statistics.median(last):.2f} |")
        if pair:
            out += ["", f"One Schwarz-CG iteration (k_scg_prod + k_scg_update): {pair:.2f} us."]
        out += schur_window(trace)
    print("\n".join(out))


def schur_window(trace: str):
    """Kernel time inside the first Block-Schur solve of a traced step: from its value build (the
    k_values launch that builds K, just before the first k_schur_values) to the launch before the
    Block-Reg solve's own value build (the next k_values).  Template arguments that only count
    Krylov vectors are folded into one row."""
    import csv

    rows = sorted(csv.DictReader(open(trace)), key=lambda r: int(r["Start_Timestamp"]))
    names = [r["Kernel_Name"] for r in rows]

    def is_values(n):
        return re.search(r"\bk_values\(", n) is not None

    try:
        sv = next(i for i, n in enumerate(names) if "k_schur_values" in n)
        s = max(i for i in range(sv) if is_values(names[i]))
        e = next(i for i in range(sv, len(names)) if is_values(names[i]))
    except (StopIteration, ValueError):
        return []
    seg = rows[s:e]
    busy, calls = {}, {}
    for r in seg:
        name = kernel_short(r["Kernel_Name"]) or r["Kernel_Name"].split("(")[0][:40]
        name = re.sub(r"^(k_(?:dots|dots_fix|update_dots|combine))<\d+>$", r"\1<j>", name)
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        busy[name] = busy.get(name, 0.0) + d
        calls[name] = calls.get(name, 0) + 1
    span = (int(seg[-1]["End_Timestamp"]) - int(seg[0]["Start_Timestamp"])) / 1e3
    total = sum(busy.values())
    out = ["", f"First Block-Schur solve of the step (value build included): {len(seg)} launches, "
           f"{total / 1e3:.2f} ms of kernel time in a {span / 1e3:.2f} ms span (the traced run is the "
           "first, cold step: the span also holds first-use allocations and tracer gaps).", "",
           "| kernel | launches | total ms | avg us | % of kernel time |", "|---|---|---|---|---|"]
    for name, t in sorted(busy.items(), key=lambda x: -x[1])[:14]:
        out.append(f"| `{name}` | {calls[name]} | {t / 1e3:.2f} | {t / calls[name]:.2f} | "
                   f"{100.0 * t / total:.1f} |")
    return out


KERNEL_SRC = ("krylov.hip", "pcg.hip", "krylov_device.h")  # the measured kernels' sources (traffic record)
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_cube64_lo.md")


def kernel_src_digest():
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SRC:
        h.update(open(os.path.join(ROOT, "paper_1901_02330_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles():
    """HBM bytes of the two roofline kernels from the committed counter summary, if it was taken on
    the current kernel sources (their hash is recorded there); else None."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    digest = kernel_src_digest()
    for line in open(TRAFFIC_PROFILE):
        if line.startswith("{") and '"traffic"' in line:
            rec = json.loads(line)
            if rec.get("kernel_src_sha256_16") == digest:
                return rec
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(n: int, args):
    """The oracle on the workload itself (Cube n^3, the same coefficient and data): its assembly, then
    FGMRES(30) with its Block-Schur preconditioner to the same tolerance.  The oracle's exact sparse LU
    of S takes minutes at 64^3 on the host, so its inner Jacobi-CG on S is used, capped at the GPU
    run's 24 products (the same preconditioner family; the outer iteration count is stated)."""
    import numpy as np

    from oracle.assemble import discretize
    from oracle.solvers import block_schur, fgmres
    from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field

    from threadpoolctl import threadpool_limits

    m = cube_mesh(n)
    nu = 1.0 / lognormal_field(n**3, 2.0, 0)
    # one thread throughout (SciPy's sparse kernels are single-threaded; BLAS is held to one thread)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        d = discretize(m, nu=nu, rhs=SineSolution())
        t1 = time.perf_counter()
        Nu = d["Nu"]
        K = d["K"].tocsr()
        pre = block_schur(K[:Nu, :Nu], K[Nu:, :Nu], inner="cg", tol=1e-12, maxit=args.schur_inner_maxit)
        x, info = fgmres(K, d["b"], pre, m=30, tol=args.tol)
        t2 = time.perf_counter()
    return {
        "value": t2 - t0,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"the whole {n}^3 workload ({Nu + d['Np']} unknowns), unscaled, on one thread: oracle FP64 "
                   f"(NumPy/SciPy) assembly {t1 - t0:.2f} s + FGMRES(30)/Block-Schur with the oracle's inner "
                   f"Jacobi-CG on S capped at {args.schur_inner_maxit} iterations {t2 - t1:.2f} s "
                   f"({info['iterations']} iterations, relres {info['relres']:.1e})"),
        "host_cpus_available": len(os.sched_getaffinity(0)),
    }


def pmc_probe(mesh, n):
    """Counter run: a plain copy of known size, then 20 launches of each hot kernel (one
    dispatch each), so that per-dispatch FETCH_SIZE / WRITE_SIZE can be scaled by the copy's."""
    import torch

    from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field
    from paper_1901_02330_amd.vem import Solver

    src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")  # 512 MiB, twice the MALL
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)  # one elementwise kernel: 512 MiB read, 512 MiB written
    torch.cuda.synchronize()
    s = Solver()
    s.set_mesh(mesh)
    s.discretize("lo", load_points=3)
    s.set_coefficient(torch.as_tensor(1.0 / lognormal_field(n**3, 2.0, 0), device="cuda"))
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    rec = {"copy_read_bytes": src.numel() * 8, "copy_write_bytes": src.numel() * 8, "kernels": {}}
    for which in ("cg_reg_schwarz", "cheb_schur", "spmv", "cg_schur", "cg_reg"):
        ms, nb = s.time_kernel(which, reps=20)
        log(f"{which}: {ms * 1e3:.1f} us, algorithmic {nb / 1e6:.1f} MB")
        rec["kernels"][which] = {"avg_us": ms * 1e3, "algorithmic_bytes": nb}
    s.close()
    # the order-k Schwarz-CG on face blocks: Cube 32^3, the paper's k = 2, log K = 1.5 N(0,1)
    s = Solver()
    s.set_mesh(cube_mesh(32))
    s.discretize("paper", k=2)
    s.set_coefficient(torch.as_tensor(1.0 / lognormal_field(32**3, 1.5, 0), device="cuda"))
    for which in ("cg_reg_schwarz", "cg_reg_schwarz32"):
        ms, nb = s.time_kernel(which, reps=20)
        log(f"{which} (cube 32^3, k = 2): {ms * 1e3:.1f} us, algorithmic {nb / 1e6:.1f} MB")
        rec["kernels"][which + "_k2"] = {"avg_us": ms * 1e3, "algorithmic_bytes": nb}
    s.close()
    print(json.dumps(rec), flush=True)


def summarize_pmc(fetch_dir: str, write_dir: str):
    """HBM traffic per launch from two rocprofv3 --pmc runs of --pmc-probe (FETCH_SIZE, then
    WRITE_SIZE; both in KiB per dispatch), each scaled by what the same counter reads for the
    probe's plain 512 MiB elementwise copy."""
    import csv
    import glob
    import statistics

    def per_kernel(d, counter):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        by = {}
        for f in files:
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                name = kernel_short(r["Kernel_Name"]) or ("copy" if "neg" in r["Kernel_Name"] else None)
                if name is None:
                    continue
                by.setdefault((name, int(r["Grid_Size"])), []).append(float(r["Counter_Value"]) * 1024.0)
        return by

    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    probe = json.loads(open(os.path.join(fetch_dir, "probe.json")).read())
    cf = [v for (n, _), vs in fetch.items() if n == "copy" for v in vs]
    cw = [v for (n, _), vs in write.items() if n == "copy" for v in vs]
    f_fetch = probe["copy_read_bytes"] / statistics.median(cf)
    f_write = probe["copy_write_bytes"] / statistics.median(cw)
    out = ["Calibration (plain 512 MiB elementwise copy): FETCH_SIZE reads "
           f"{statistics.median(cf) / 2**20:.1f} MiB (factor {f_fetch:.4f}), WRITE_SIZE "
           f"{statistics.median(cw) / 2**20:.1f} MiB (factor {f_write:.4f}).", "",
           "| kernel | grid (threads) | dispatches | fetch MB (scaled) | write MB (scaled) | total MB |",
           "|---|---|---|---|---|---|"]
    rows = {}
    for key in sorted(set(fetch) & set(write)):
        if key[0] == "copy" or not any(k in key[0] for k in ("k_ppcg_iter", "k_spmv", "k_scg_", "k_cheb_iter")):
            continue
        fm = statistics.median(fetch[key]) * f_fetch
        wm = statistics.median(write[key]) * f_write
        rows[key] = (fm, wm, len(fetch[key]))
        out.append(f"| `{key[0]}` | {key[1]} | {len(fetch[key])} | {fm / 1e6:.1f} | {wm / 1e6:.1f} | "
                   f"{(fm + wm) / 1e6:.1f} |")

    def most(prefix):  # the variant of a kernel with the most dispatches (the timing loop's)
        ks = [k for k in rows if k[0].startswith(prefix)]
        return max(ks, key=lambda k: rows[k][2]) if ks else None

    measured = {}
    for which, prefixes in (("spmv", ["k_spmv"]), ("cheb_schur", ["k_cheb_iter<double"]),
                            ("cg_schur", ["k_ppcg_iter<double, false, 1024"]),
                            ("cg_reg", ["k_ppcg_iter<double, false, 256"]),
                            ("cg_reg_schwarz", ["k_scg_prod<double, 256, SellViewT", "k_scg_update<double, 256, SellViewT"]),
                            ("cg_reg_schwarz_k2", ["k_scg_prod<double, 256, BlockViewT<double, 6>",
                                                   "k_scg_update<double, 256, BlockViewT<double, 6>"]),
                            ("cg_reg_schwarz32_k2", ["k_scg_prod<float, 256, BlockViewT<float, 6>",
                                                     "k_scg_update<float, 256, BlockViewT<float, 6>"])):
        keys = [most(p) for p in prefixes]
        if any(k is None for k in keys) or which not in probe["kernels"]:
            continue
        fm = sum(rows[k][0] for k in keys)
        wm = sum(rows[k][1] for k in keys)
        alg = probe["kernels"][which]["algorithmic_bytes"]
        measured[which] = {"bytes": fm + wm, "fetch_bytes": fm, "write_bytes": wm, "algorithmic_bytes": alg,
                           "ratio_to_algorithmic": (fm + wm) / alg, "kernels": [k[0] for k in keys]}
    out += ["", "Per iteration or launch, against the algorithmic bytes (every matrix entry and vector element "
            "once):", "", "| timed unit | kernels | algorithmic MB | measured MB | ratio |", "|---|---|---|---|---|"]
    for which, m in measured.items():
        out.append(f"| {which} | {', '.join('`' + k + '`' for k in m['kernels'])} | {m['algorithmic_bytes'] / 1e6:.1f} "
                   f"| {m['bytes'] / 1e6:.1f} | {m['ratio_to_algorithmic']:.3f} |")
    note = "FETCH_SIZE + WRITE_SIZE, cube 64^3 LO, each scaled by a 512 MiB copy; L2-to-fabric traffic (MALL hits included)"
    rec = {"traffic": dict(measured.get("cg_reg_schwarz", {}), note=note),
           "traffic_value": dict(measured.get("cheb_schur", {}), note=note),
           "kernel_src_sha256_16": kernel_src_digest()}
    out += ["", json.dumps(rec)]
    print("\n".join(out))


def extras(args, torch, dev):
    """Measurements outside the timed region (each states its own workload)."""
    import numpy as np

    from paper_1901_02330_amd.adjoint import solve_logk
    from paper_1901_02330_amd.batch import BatchSolver, percentiles
    from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field
    from paper_1901_02330_amd.vem import Solver

    out = {}
    sk = dict(inner_form=args.schur_inner_form, inner_tol=args.schur_inner_tol, inner_maxit=args.schur_inner_maxit,
              cheb_lo=args.cheb_lo)
    rk = dict(reg_inner=args.reg_inner, inner_tol=args.reg_inner_tol, inner_maxit=args.reg_inner_maxit)
    # adjoint: Cube 48^3, log K ~ N(0,1) seed 0, p_obs from the seed-1 field, J = 1/2 ||p - p_obs||^2
    m48 = cube_mesh(48)
    s = Solver()
    s.set_mesh(m48)
    s.discretize("lo")
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    kw = dict(precond="schur", tol=1e-10, **sk)
    s.set_coefficient(torch.as_tensor(1.0 / lognormal_field(48**3, 1.0, 1), device=dev))
    _, p_obs, _ = s.solve(**kw)
    logk = torch.tensor(np.log(lognormal_field(48**3, 1.0, 0)), dtype=torch.float64, device=dev,
                        requires_grad=True)
    ts = []
    for _ in range(3):
        logk.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, p = solve_logk(s, logk, **kw)
        J = 0.5 * torch.sum((p - p_obs) ** 2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        ts.append((t1 - t0, time.perf_counter() - t1))
    fw, bw = min(t[0] for t in ts), min(t[1] for t in ts)
    out["adjoint_cube48"] = {"forward_s": fw, "backward_s": bw, "backward_over_forward": bw / fw,
                             "note": "forward = set coefficient + Block-Schur solve to 1e-10; backward = adjoint "
                                     "solve + per-cell gradient kernel"}
    s.close()
    # mixed precision against the FP64 oracle's direct solve, Cube 24^3 of the same recipe (the oracle
    # solves it in seconds); then on the headline workload, against the GPU's FP64 solution (which the
    # full-size test matches to the oracle's 1e-13 solution within 4e-15)
    from oracle.assemble import discretize
    from oracle.solvers import direct_solve

    s = Solver()
    m24 = cube_mesh(24)
    nu24 = 1.0 / lognormal_field(24**3, 2.0, 0)
    s.set_mesh(m24)
    s.discretize("lo")
    s.set_coefficient(torch.as_tensor(nu24, device=dev))
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    d24 = discretize(m24, nu=nu24, rhs=SineSolution())
    x24 = direct_solve(d24["K"], d24["b"])
    vs_or = {}
    for prec, kwp in (("schur", sk), ("reg", rk)):
        for precision in ("mixed", "fp64"):
            u, p, info = s.solve(prec, tol=1e-10, precision=precision, maxit=3000, **kwp)
            uc, pc = u.cpu().numpy(), p.cpu().numpy()
            vs_or[f"{prec}_{precision}"] = {
                "iterations": info["iterations"], "relres": info["relres"],
                "rel_err_u_vs_oracle": float(np.linalg.norm(uc - x24[: d24["Nu"]]) / np.linalg.norm(x24[: d24["Nu"]])),
                "rel_err_p_vs_oracle": float(np.linalg.norm(pc - x24[d24["Nu"]:]) / np.linalg.norm(x24[d24["Nu"]:]))}
    out["precision_vs_oracle_cube24_tol1e-10"] = vs_or
    s.close()
    n = args.n
    s = Solver()
    s.set_mesh(cube_mesh(n))
    s.discretize("lo")
    s.set_coefficient(torch.as_tensor(1.0 / lognormal_field(n**3, 2.0, 0), device=dev))
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    mixed = {}
    for prec, kwp in (("schur", sk), ("reg", rk)):
        u64, p64, i64 = s.solve(prec, tol=1e-10, **kwp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u32, p32, i32 = s.solve(prec, tol=1e-10, precision="mixed", **kwp)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        u64b, p64b, _ = s.solve(prec, tol=1e-10, **kwp)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        mixed[prec] = {"mixed_s": t1 - t0, "fp64_s": t2 - t1, "mixed_iterations": i32["iterations"],
                       "fp64_iterations": i64["iterations"], "mixed_relres": i32["relres"],
                       "rel_err_u_vs_fp64": float(torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64)),
                       "rel_err_p_vs_fp64": float(torch.linalg.norm(p32 - p64) / torch.linalg.norm(p64))}
    out["mixed_precision_cube64_tol1e-10"] = mixed
    s.close()
    # batched: 16 log-normal fields (sigma 1.5, seeds 0..15) on the 64^3 mesh, Block-Schur
    nus = [torch.as_tensor(1.0 / lognormal_field(n**3, 1.5, sd), device=dev) for sd in range(16)]
    torch.cuda.synchronize()
    bat = {}
    for lanes in (1, 8):
        bs = BatchSolver(cube_mesh(n), lanes=lanes, rhs=SineSolution())
        bs.solve(nus[:lanes], precond="schur", tol=1e-8, **sk)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, infos = bs.solve(nus, precond="schur", tol=1e-8, **sk)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        bat[f"lanes{lanes}"] = {"solves_per_s": len(nus) / wall, "wall_s": wall, **percentiles(infos)}
        bs.close()
    out["batch_cube64_16fields"] = bat
    out["batch_cube32_k2_64fields"] = k2_fields(args, torch, dev, 64)
    # one 128^3 solve (8.4M unknowns), log-normal sigma 1.5 seed 0
    s = Solver()
    m128 = cube_mesh(128)
    mdev = {k: torch.as_tensor(m128[k]).to(dev) for k in
            ("xyz", "face_ptr", "face_vtx", "cell_ptr", "cell_face", "cell_face_sign")}
    nu128 = torch.as_tensor(1.0 / lognormal_field(128**3, 1.5, 0), device=dev)
    big = {}
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_mesh(mdev)
        s.discretize("lo")
        s.set_coefficient(nu128)
        s.set_rhs_functions(SineSolution.f, SineSolution.pD)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        u, p, info = s.solve("schur", tol=1e-8, **sk)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        big = {"n_unknowns": s.sizes()["n"], "assembly_s": t1 - t0, "solve_schur_s": t2 - t1,
               "iterations": info["iterations"], "relres": info["relres"]}
    out["cube128_lo"] = big
    s.close()
    # the paper's boundary data on the benchmark mesh (Section 3): u.n of the sine solution's flux
    # prescribed on the whole boundary, zero-mean pressure; the step's coefficient field
    s = Solver()
    s.set_mesh(cube_mesh(args.n))
    s.set_boundary("flux")
    s.discretize("lo")
    s.set_coefficient(torch.as_tensor(1.0 / lognormal_field(args.n**3, 2.0, 0), device=dev))
    s.set_rhs_functions(SineSolution.f, SineSolution.u)
    fl = {"boundary_data": "flux, zero-mean pressure"}
    for prec, kw in (("schur", sk), ("reg", rk)):
        for rep in range(2):  # the second solve is timed
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, info = s.solve(prec, tol=args.tol, maxit=3000, **kw)
            torch.cuda.synchronize()
            fl[prec] = {"iterations": info["iterations"], "inner_iterations": info["inner_iterations"],
                        "solve_s": time.perf_counter() - t0, "relres": info["relres"]}
    out[f"cube{args.n}_lo_flux"] = fl
    s.close()
    # the paper's element on the paper's Cube meshes (Table 1: 32^3 at k = 1, 24^3 at k = 2, 20^3 at
    # k = 3), nu = 1,
    # the paper's polynomial solution, with the paper's boundary data (flux, zero-mean pressure; its
    # counts carry one more unknown, the multiplier of the mean) and with pressure data.  The paper
    # does not state its GMRES tolerance or restart: iteration counts are context.
    from paper_1901_02330_amd.inputs import PolynomialSolution

    paper = {(32, 1): {"dofs": 435201, "T_ass_p1_s": 68, "T_ass_p32_s": 3, "schur_its": 66, "schur_T_sol_p1_s": 50,
                       "schur_T_sol_p32_s": 9, "reg_its_p1": 84, "reg_T_sol_p1_s": 53, "reg_T_sol_p32_s": 26},
             (24, 2): {"dofs": 508033, "T_ass_p1_s": 271, "T_ass_p32_s": 13, "schur_its": 72, "schur_T_sol_p1_s": 347,
                       "schur_T_sol_p32_s": 40, "reg_its_p1": 98, "reg_T_sol_p1_s": 138, "reg_T_sol_p32_s": 58},
             # k = 3: the paper's smallest run is on 4 processes
             (20, 3): {"dofs": 612001, "T_ass_p4_s": 623, "T_ass_p32_s": 97, "schur_its": 147, "schur_T_sol_p4_s": 570,
                       "schur_T_sol_p32_s": 192, "reg_its_p4": 720, "reg_T_sol_p4_s": 450, "reg_T_sol_p32_s": 197}}
    tab = {}
    for (nn, k), ref in paper.items():
      for bc in ("flux", "pressure"):
        s = Solver()
        s.set_mesh(cube_mesh(nn))
        s.set_boundary(bc)
        for rep in range(2):  # the second discretisation is timed (warm)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.discretize("paper", k=k)
            s.set_rhs_functions(PolynomialSolution.f, PolynomialSolution.u if bc == "flux" else PolynomialSolution.pD)
            torch.cuda.synchronize()
            t_ass = time.perf_counter() - t0
        row = {"boundary_data": bc, "n_unknowns": s.sizes()["n"], "assembly_s": t_ass}
        precs = (("schur", dict(inner_tol=1e-8, inner_maxit=2000)), ("reg", dict(inner_tol=1e-1)))
        if k == 3 and bc == "pressure":
            # Block-Schur with diag(M) does not reach 1e-8 in 3,000 iterations here (about a minute)
            precs = precs[1:]
        for prec, kw in precs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, info = s.solve(prec, tol=1e-8, maxit=3000, **kw)
            torch.cuda.synchronize()
            row[prec] = {"iterations": info["iterations"], "solve_s": time.perf_counter() - t0,
                         "relres": info["relres"]}
        row["paper_cluster_context"] = ref
        tab[f"cube{nn}_k{k}_{bc}"] = row
        s.close()
    out["paper_cube_table1"] = tab
    # the paper's optimality sweep on Cube meshes (its Table 4: k = 2, 512 to 21,952 cells, flux data,
    # nu = 1, the polynomial solution; the paper's counts at 8 processes are context)
    paper4 = {8: (19585, 113, 86), 16: (152065, 78, 123), 20: (295201, 76, 145), 24: (508033, 72, 168),
              28: (804385, 69, 188)}
    opt = {}
    for nn, (dofs, its_s, its_r) in paper4.items():
        s = Solver()
        s.set_mesh(cube_mesh(nn))
        s.set_boundary("flux")
        s.discretize("paper", k=2)
        s.set_rhs_functions(PolynomialSolution.f, PolynomialSolution.u)
        row = {"n_unknowns": s.sizes()["n"], "paper": {"dofs": dofs, "schur_its": its_s, "reg_its": its_r}}
        for prec, kw in (("schur", dict(inner_tol=1e-8, inner_maxit=2000)), ("reg", dict(inner_tol=1e-1))):
            _, _, info = s.solve(prec, tol=1e-8, maxit=3000, **kw)  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, info = s.solve(prec, tol=1e-8, maxit=3000, **kw)
            torch.cuda.synchronize()
            row[prec] = {"iterations": info["iterations"], "inner_iterations": info["inner_iterations"],
                         "solve_s": time.perf_counter() - t0}
        opt[f"cube{nn}_k2_flux"] = row
        s.close()
    out["paper_cube_table4_k2"] = opt
    return out


def copy_ceiling(torch, nbytes, reps=200):
    """Rate of a plain device copy that moves the same bytes (half read, half written), timed like the
    kernels (events around `reps` back-to-back copies on torch's stream): what a kernel with this
    working set can reach on this part, beside the 8 TB/s peak."""
    n = max(1, int(nbytes / 16))
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"copy_bytes": 16.0 * n, "copy_us": ms * 1e3, "gbs": 16.0 * n / (ms * 1e-3) / 1e9}


def schwarz_rates(s, reps=100):
    """One Schwarz-CG iteration (both launches), FP64 and FP32: mean time over `reps` back-to-back
    iterations (HIP events), algorithmic bytes (every stored matrix entry, index and vector element
    once) and the fraction of the HBM peak."""
    out = {}
    for which in ("cg_reg_schwarz", "cg_reg_schwarz32"):
        ms, nb = s.time_kernel(which, reps=reps)
        gbs = nb / (ms * 1e-3) / 1e9
        out[which] = {"avg_us": ms * 1e3, "bytes": nb, "gbs": gbs, "frac": gbs / HBM_PEAK_GBS}
    return out


def k2_fields(args, torch, dev, fields):
    """The batched workload: `fields` log-normal coefficient fields (log K = 1.5 N(0,1), seeds 0..) on the
    Cube 32^3 mesh with the paper's k = 2 element, one handle, vem_set_coefficient_batch +
    vem_solve_batch: Block-Reg (Schwarz inner CG in FP32, FP64 FGMRES) to 1e-8.  Per-system times
    include each field's value and preconditioner build.  Field 0 is also solved in FP64."""
    import numpy as np

    from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field
    from paper_1901_02330_amd.vem import Solver

    s = Solver()
    s.set_mesh(cube_mesh(32))
    s.discretize("paper", k=2)
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    nus = np.stack([1.0 / lognormal_field(32**3, 1.5, sd) for sd in range(fields)])
    # polled inner solves: at order 2 an application needs about 16 iterations, and a cap of 24 would
    # enqueue launches past convergence (32^3: 0.10 s polled against 0.12 s capped)
    kw = dict(precond="reg", tol=1e-8, maxit=1000, inner_tol=args.reg_inner_tol, precision="mixed")
    s.set_coefficient(torch.as_tensor(nus[0], device=dev))
    u64, p64, i64 = s.solve(**dict(kw, precision="fp64"))  # also builds the Schwarz patterns
    s.set_coefficient_batch(torch.as_tensor(nus, device=dev))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, p, infos = s.solve_batch(fields, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([i["solve_ms"] for i in infos])
    out = {"fields": fields, "n_unknowns_per_field": s.sizes()["n"], "solves_per_s": fields / wall, "wall_s": wall,
           "p50_s": float(np.percentile(ms, 50)) / 1e3, "p99_s": float(np.percentile(ms, 99)) / 1e3,
           "iterations_min_max": [min(i["iterations"] for i in infos), max(i["iterations"] for i in infos)],
           "all_converged": all(i["converged"] for i in infos),
           "field0_fp64": {"iterations": i64["iterations"], "relres": i64["relres"]},
           "field0_rel_err_u_vs_fp64": float(torch.linalg.norm(u[0] - u64) / torch.linalg.norm(u64)),
           "field0_rel_err_p_vs_fp64": float(torch.linalg.norm(p[0] - p64) / torch.linalg.norm(p64))}
    out["schwarz_iteration"] = schwarz_rates(s)
    s.close()
    return out


def voronoi_checkerboard(torch, dev, precisions=("mixed", "fp64")):
    """The mixed-precision workload: Random Voronoi mesh of 20,000 seeded uniform points, the paper's k = 2,
    checkerboard K in {1e-3, 1e3} on 4x4x4 blocks, Block-Reg to 1e-8 with FP32 inner Schwarz-CG under FP64
    FGMRES, then with FP64 inner solves; the difference between the two solutions."""
    from paper_1901_02330_amd.inputs import SineSolution, checkerboard_field, voronoi_mesh
    from paper_1901_02330_amd.vem import Solver

    t0 = time.perf_counter()
    m = voronoi_mesh(20000, seed=0)
    t_mesh = time.perf_counter() - t0
    s = Solver()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.set_mesh(m)
    s.discretize("paper", k=2)
    s.set_coefficient(torch.as_tensor(1.0 / checkerboard_field(m["seeds"]), device=dev))
    s.set_rhs_functions(SineSolution.f, SineSolution.pD)
    torch.cuda.synchronize()
    out = {"mesh_generation_s": t_mesh, "assembly_s": time.perf_counter() - t0, "n_unknowns": s.sizes()["n"],
           "nnz_K": s.sizes()["nnz_K"]}
    xs = {}
    for prec in precisions:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, p, info = s.solve("reg", tol=1e-8, maxit=1500, inner_tol=1e-2, precision=prec)
        torch.cuda.synchronize()
        out[prec] = {"solve_s": time.perf_counter() - t0, "iterations": info["iterations"],
                     "inner_iterations": info["inner_iterations"], "relres": info["relres"],
                     "converged": info["converged"]}
        xs[prec] = torch.cat([u, p])
        log(f"voronoi checkerboard {prec}: {out[prec]}")
    if "mixed" in xs and "fp64" in xs:
        out["rel_diff_mixed_vs_fp64"] = float(torch.linalg.norm(xs["mixed"] - xs["fp64"]) /
                                              torch.linalg.norm(xs["fp64"]))
    out["schwarz_iteration"] = schwarz_rates(s, reps=50)
    s.close()
    return out


def voronoi_sweep(torch, dev):
    """The optimality trend on Random Voronoi meshes (the paper's sweep is on CVT meshes, whose recipe it
    does not give): the paper's k = 2, nu = 1, its polynomial solution with its flux data, 1,000 to
    16,000 seeded uniform points; Block-Reg (Schwarz-CG to 0.1) and Block-Schur (inner CG to 1e-8)."""
    from paper_1901_02330_amd.inputs import PolynomialSolution, voronoi_mesh
    from paper_1901_02330_amd.vem import Solver

    out = {}
    for cells in (1000, 2000, 4000, 8000, 16000):
        m = voronoi_mesh(cells, seed=0)
        s = Solver()
        s.set_mesh(m)
        s.set_boundary("flux")
        s.discretize("paper", k=2)
        s.set_rhs_functions(PolynomialSolution.f, PolynomialSolution.u)
        row = {"n_unknowns": s.sizes()["n"]}
        for prec, kw in (("reg", dict(inner_tol=1e-1)), ("schur", dict(inner_tol=1e-8, inner_maxit=2000))):
            s.solve(prec, tol=1e-8, maxit=3000, **kw)  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, info = s.solve(prec, tol=1e-8, maxit=3000, **kw)
            torch.cuda.synchronize()
            row[prec] = {"iterations": info["iterations"], "inner_iterations": info["inner_iterations"],
                         "solve_s": time.perf_counter() - t0, "converged": info["converged"]}
        log(f"voronoi {cells}: {row}")
        out[f"voronoi{cells}_k2_flux"] = row
        s.close()
    return out


def k2_batch(fields, torch, dev):
    """Fields seeds 0..fields-1 (log K = 1.5 N(0,1)) on the Cube 32^3 mesh, the paper's k = 2, Block-Reg
    with FP32 inner solves to 1e-8: one lane (sequential) and `fields` concurrent lanes."""
    from paper_1901_02330_amd.batch import BatchSolver, percentiles
    from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field

    nus = [torch.as_tensor(1.0 / lognormal_field(32**3, 1.5, sd), device=dev) for sd in range(fields)]
    kw = dict(precond="reg", tol=1e-8, inner_tol=1e-1, precision="mixed", maxit=1000)
    out = {"fields": fields, "note": "a sample of the 64-field batch; each solve takes seconds"}
    for lanes in (1, fields):
        bs = BatchSolver(cube_mesh(32), lanes=lanes, family="paper", k=2, rhs=SineSolution())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, infos = bs.solve(nus, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[f"lanes{lanes}"] = {"solves_per_s": fields / wall, "wall_s": wall,
                                "iterations": [i["iterations"] for i in infos],
                                "converged": all(i["converged"] for i in infos), **percentiles(infos)}
        log(f"k2 batch lanes {lanes}: {wall:.1f} s")
        bs.close()
    return out


def main():
    args = parse()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return
    if args.summarize:
        summarize(args.summarize)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the design note on sharding "
              "describes how it would split); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1901_02330_amd.inputs import SineSolution, cube_mesh, lognormal_field
    from paper_1901_02330_amd.vem import Solver

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n = args.n
    mesh = cube_mesh(n)
    if args.pmc_probe:
        pmc_probe(mesh, n)
        return
    if args.voronoi_checkerboard_only:
        print(json.dumps({"voronoi20k_k2_checkerboard": voronoi_checkerboard(torch, dev, ("mixed",))}), flush=True)
        return
    if args.k2_fields_only > 0:
        print(json.dumps({"batch_cube32_k2": k2_fields(args, torch, dev, args.k2_fields_only)}), flush=True)
        return
    # inputs resident in HBM before the timed region
    mdev = {k: torch.as_tensor(mesh[k]).to(dev) for k in
            ("xyz", "face_ptr", "face_vtx", "cell_ptr", "cell_face", "cell_face_sign")}
    nu = torch.as_tensor(1.0 / lognormal_field(n**3, 2.0, 0), device=dev)
    solver = Solver()
    schur_kw = dict(inner_form=args.schur_inner_form, inner_tol=args.schur_inner_tol,
                    inner_maxit=args.schur_inner_maxit, cheb_lo=args.cheb_lo)
    reg_kw = dict(reg_inner=args.reg_inner, inner_tol=args.reg_inner_tol, inner_maxit=args.reg_inner_maxit)

    def step():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.set_mesh(mdev)
        solver.discretize("lo", load_points=3)
        solver.set_coefficient(nu)
        solver.set_rhs_functions(SineSolution.f, SineSolution.pD)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        u, p, i_s = solver.solve("schur", tol=args.tol, **schur_kw)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        u2, p2, i_r = solver.solve("reg", tol=args.tol, maxit=5000, **reg_kw)
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

    # live kernel rates (HIP events on the library's stream, 200 back-to-back launches each)
    sz = solver.sizes()
    kern = {}
    for which in ("cg_reg_schwarz", "cheb_schur", "spmv", "cg_schur", "cg_reg", "cheb_schur32", "cg_reg_schwarz32",
                  "cg_schur32p"):
        ms, nbytes = solver.time_kernel(which, reps=200)
        gbs = nbytes / (ms * 1e-3) / 1e9
        kern[which] = {"avg_us": ms * 1e3, "bytes": nbytes, "gbs": gbs, "frac": gbs / HBM_PEAK_GBS}
    # the pipelined Jacobi-CG iterations also against the blueprint's inner-PCG count, 12 nnz + 68 n
    # (matrix once, D^{-1}, r, x read and written, z, p, q ... as a textbook PCG step), beside their own
    # 12 nnz + 104 n (the pipelined form's 13 vector streams)
    for which, nnz, rows in (("cg_schur", sz["nnz_schur"], sz["n_p"]), ("cg_reg", sz["nnz_reg"], sz["n_u"])):
        b3 = 12.0 * nnz + 68.0 * rows
        kern[which]["bytes_pcg_12nnz_68n"] = b3
        kern[which]["frac_pcg_12nnz_68n"] = b3 / (kern[which]["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS
    dom, val = kern["cg_reg_schwarz"], kern["cheb_schur"]
    line = {
        "metric": "solve time to rel. residual 1e-8 (s) + HBM GB/s in SpMV/precond; adjoint/fwd",
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
        "value_per_step_s": {"min": min(r["t_ass"] + r["t_schur"] for r in results),
                             "median": statistics.median(r["t_ass"] + r["t_schur"] for r in results),
                             "max": max(r["t_ass"] + r["t_schur"] for r in results)},
        "solves": {
            "schur": {"iterations": results[-1]["info_schur"]["iterations"],
                      "inner_iterations": results[-1]["info_schur"]["inner_iterations"],
                      "relres": results[-1]["info_schur"]["relres"], **schur_kw},
            "reg": {"iterations": results[-1]["info_reg"]["iterations"],
                    "inner_iterations": results[-1]["info_reg"]["inner_iterations"],
                    "relres": results[-1]["info_reg"]["relres"], **reg_kw},
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_scg_prod + k_scg_update: one iteration of Block-Reg's inner CG on A_gamma with the "
                      "edge-patch Schwarz preconditioner (two launches; the step's dominant kernel pair)",
            "achieved": dom["gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": dom["frac"],
            "traffic": None,
            "avg_iteration_us": dom["avg_us"],
            "algorithmic_bytes_per_iteration": dom["bytes"],
            "bytes_formula": "12 (nnz(A_gamma) + nnz(P)) + 13 * 8 n_u",
        },
        "roofline_value": {
            "bound": "hbm",
            "kernel": "k_cheb_iter<double>: one Chebyshev-Jacobi product on S (Block-Schur's inner polynomial, "
                      "the kernel that dominates `value`)",
            "achieved": val["gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": val["frac"],
            "traffic": None,
            "avg_launch_us": val["avg_us"],
            "algorithmic_bytes_per_launch": val["bytes"],
            "bytes_formula": "12 nnz(S) + 4 * 8 n_p",
        },
        "kernels": kern,
    }
    if not args.no_extras:
        log("extras ...")
        line["extras"] = extras(args, torch, dev)
        # the metric's third part: adjoint (backward) time over forward time, 48^3 (extras)
        line["adjoint_over_forward"] = line["extras"]["adjoint_cube48"]["backward_over_forward"]
    if args.voronoi_checkerboard:
        log("voronoi checkerboard ...")
        line.setdefault("extras", {})["voronoi20k_k2_checkerboard"] = voronoi_checkerboard(torch, dev)
    if args.voronoi_sweep:
        log("voronoi sweep ...")
        line.setdefault("extras", {})["voronoi_sweep_k2_flux"] = voronoi_sweep(torch, dev)
    if args.k2_batch > 0:
        log("k=2 batch ...")
        line.setdefault("extras", {})["batch_cube32_k2"] = k2_batch(args.k2_batch, torch, dev)
    # the same-size plain copy beside each roofline figure
    for obj in ("roofline", "roofline_value"):
        nb = line[obj].get("algorithmic_bytes_per_iteration") or line[obj]["algorithmic_bytes_per_launch"]
        cc = copy_ceiling(torch, nb)
        cc["frac_of_copy"] = line[obj]["achieved"] / cc["gbs"]
        line[obj]["copy_ceiling"] = cc
    tr = traffic_from_profiles()
    if tr is not None:
        for key, obj in (("traffic", "roofline"), ("traffic_value", "roofline_value")):
            if tr.get(key, {}).get("bytes"):
                line[obj]["traffic"] = tr[key]["bytes"]
                line[obj]["traffic_ratio_to_algorithmic"] = tr[key]["ratio_to_algorithmic"]
                line[obj]["traffic_note"] = tr[key]["note"]
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline(args.cpu_n or n, args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
