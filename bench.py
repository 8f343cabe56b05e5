"""Benchmark: V-cycles/s, smoother HBM bandwidth and time to relative residual
1e-10 for the Poisson-control KKT system at 2049^2 vertices (level 11) on one
MI355X.

One step = one complete solve from x = 0: right-hand side f = (M y_D; 0), then
multigrid iterates until ||f - A x||_{L^-1} <= 1e-10 ||f||_{L^-1}, the residual
norm weighted by L_k^-1 (the dual of the L_k norm in which section 3 measures
convergence; the Euclidean ratio has an FP64 floor near eps h^-2, about 3e-9
at this size).  The printed JSON line carries the throughput, the roofline of
the dominant kernel (the finest-level smoothing sweep, timed with HIP events
on the launch stream), per-field errors of the FP32-refinement solves, and
the FP64 CPU oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "V-cycles/s and HBM GB/s at 2049^2 Poisson control; time to rel. residual 1e-10"

# The HBM traffic of the finest-level sweep is measured with hardware counters
# (FETCH_SIZE, WRITE_SIZE) in separate profiler runs and recorded, together
# with a hash of the sources the kernel is built from, in TRAFFIC_RECORDS; the
# figure is reported only while those sources are unchanged.
# what the sweep kernel is built from: its source, the level descriptors of
# the internal header (the part before the launcher declarations) and the
# compiler flags
SWEEP_SOURCES = ("paper_1502_03917_amd/csrc/sweep.hip", "paper_1502_03917_amd/csrc/mg_internal.hpp",
                 "paper_1502_03917_amd/build.py")
TRAFFIC_RECORDS = {"fp64": os.path.join(ROOT, "profiles", "lsgs_sweep_2049sq_traffic.txt"),
                   "fp32_ir": os.path.join(ROOT, "profiles", "lsgs_sweep_2049sq_fp32_traffic.txt")}
COPY_MIB = 512  # size of the plain copy that calibrates the counters


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def words_per_cycle(level: int, coarse: int, nu1: int, nu2: int, sweep_words: float = 8.0,
                    fine_residual: bool = False) -> float:
    """Algorithmic words of one V-cycle in steady state: per level visit
    nu1+nu2 sweeps of `sweep_words` per vertex, restriction (read r: 2 words,
    write f_c: 0.5) and prolongation + residual (read x_c 0.5, x 2, f 2; write
    x 2, r 2), 43 words per vertex for V(2,2), about 57.3 per fine vertex over
    all levels.  The smoothers keep r = f - A x current, so a finest-level
    residual pass (read f, x; write r: 6 words) is added only where the solve
    moves one (fine_residual)."""
    total = 0.0
    for l in range(coarse + 1, level + 1):
        V = ((1 << l) + 1) ** 2
        total += V * ((nu1 + nu2) * sweep_words + 2.5 + 8.5)
    if fine_residual:
        total += 6 * ((1 << level) + 1) ** 2
    return total


def field_errors(got, ref, alpha, problem: str = "poisson", level: int | None = None) -> dict:
    """max |got - ref| / max |ref| per field of a solution vector (Poisson
    [y | lambda], Stokes [v1 | v2 | p | lambda1 | lambda2 | mu]) and of the
    control u = lambda / alpha; torch tensors on the device."""
    import torch

    if problem == "poisson":
        V = got.numel() // 2
        names, sizes = ("y", "lambda"), (V, V)
    else:
        n = 1 << level
        nv, npv = (2 * n - 1) ** 2, (n + 1) ** 2
        names, sizes = ("v1", "v2", "p", "lambda1", "lambda2", "mu"), (nv, nv, npv, nv, nv, npv)
    out, at = {}, 0
    for name, k in zip(names, sizes):
        g, r = got[at:at + k], ref[at:at + k]
        out["err_" + name] = float(torch.max(torch.abs(g - r)) / torch.clamp(torch.max(torch.abs(r)), min=1e-300))
        if name.startswith("lambda"):
            gu, ru = g / alpha, r / alpha
            out["err_u" + name[6:]] = float(torch.max(torch.abs(gu - ru)) /
                                            torch.clamp(torch.max(torch.abs(ru)), min=1e-300))
        at += k
    return out


def sweep_source_hash() -> str:
    h = hashlib.sha256()
    for rel in SWEEP_SOURCES:
        with open(os.path.join(ROOT, rel)) as fh:
            text = fh.read()
        if rel.endswith("mg_internal.hpp"):
            # the level descriptors and stencil tables; not the tail's or the
            # launchers' declarations
            text = text.split("// ---- batched launches")[0]
            a = text.find("// ---- coarse-level tail")
            b = text.find("__host__ __device__ inline int cls3")
            if 0 <= a < b:
                text = text[:a] + text[b:]
        elif rel.endswith("sweep.hip"):
            # the batched kernel and launcher do not affect the single-instance sweep
            text = "\n\n".join(c for c in text.split("\n\n")
                                if "kb_lsgs_tile" not in c and "launch_b_lsgs_sweep" not in c)
        elif rel.endswith("build.py"):
            text = text[text.index("FLAGS = ["):]
            text = text[: text.index("]") + 1]
        if not rel.endswith("build.py"):
            # comments and blank lines do not change the kernels
            lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines())
            text = "\n".join(ln for ln in lines if ln)
        h.update(text.encode())
    return h.hexdigest()[:16]


def read_record(path: str) -> dict:
    out = {}
    if os.path.exists(path):
        for line in open(path):
            if ":" in line and not line.startswith((" ", "#", "|")):
                k, v = line.split(":", 1)
                out[k.strip()] = v.strip()
    return out


def recorded_traffic(precision: str, level: int):
    """HBM bytes per finest-level sweep from the counter record, or None when
    the record is missing, was taken for another configuration, or the sweep
    sources have changed since."""
    rec = read_record(TRAFFIC_RECORDS.get(precision, ""))
    key = f"traffic_bytes_per_launch_{precision}"
    if rec.get("source_hash") != sweep_source_hash() or rec.get("level") != str(level) or key not in rec:
        return None
    return float(rec[key])


# --- profiler output summaries (rocprofv3 --output-format csv) ----------------

def _csv_rows(directory: str, suffix: str):
    rows = []
    for dirpath, _, files in os.walk(directory):
        for fn in files:
            if fn.endswith(suffix):
                with open(os.path.join(dirpath, fn), newline="") as fh:
                    rows.extend(csv.DictReader(fh))
    return rows


def kernel_trace_summary(directory: str):
    """Per (kernel, grid size) dispatch count and average duration in us."""
    agg = {}
    for r in _csv_rows(directory, "kernel_trace.csv"):
        key = (r["Kernel_Name"], int(r.get("Grid_Size_X") or r.get("Grid_Size")))
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
        a = agg.setdefault(key, [0, 0.0])
        a[0] += 1
        a[1] += d
    return {k: (n, t / n) for k, (n, t) in agg.items()}


def counter_summary(directory: str):
    """Per (kernel, grid size, counter) dispatch count and average value."""
    agg = {}
    for r in _csv_rows(directory, "counter_collection.csv"):
        key = (r["Kernel_Name"], int(r["Grid_Size"]), r["Counter_Name"])
        a = agg.setdefault(key, [0, 0.0])
        a[0] += 1
        a[1] += float(r["Counter_Value"])
    return {k: (n, v / n) for k, (n, v) in agg.items()}


# finest-level tile shape (tile width, threads per workgroup) per precision
def sweep_tile(level: int, precision: str) -> tuple[int, int]:
    """(tile edge, threads) of the sweep on a level: the per-level table of
    the sweep launcher (csrc/sweep.hip, launch_tile_cfg)."""
    n = 1 << level
    if precision == "fp64":
        if n <= 256:
            return 16, 256
        if n in (1024, 2048):
            return 65, 1024
        return (56, 1024) if n >= 4096 else (48, 1024)
    if n <= 512:
        return 16, 256
    return (46, 512) if n == 2048 else (48, 512)


def finest_sweep_grid(level: int, precision: str) -> int:
    """Work-items launched by the finest-level sweep: one workgroup per
    TW x TW tile, the workgroup count rounded up to a multiple of 8."""
    tw, nt = sweep_tile(level, precision)
    side = -(-((1 << level) + 1) // tw)
    return nt * (-(-side * side // 8) * 8)


def print_summary(args) -> int:
    """Summarise a kernel trace (--trace DIR) or write the traffic record from
    four counter runs (--fetch/--write over the bench, --copy-fetch/--copy-write
    over `bench.py --copy-probe`)."""
    if args.trace:
        rows = sorted(kernel_trace_summary(args.trace).items(), key=lambda kv: -kv[1][0] * kv[1][1])
        print(f"{'kernel':100s} {'grid':>9s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s}")
        for (name, grid), (n, avg) in rows:
            print(f"{name[:100]:100s} {grid:9d} {n:7d} {avg:10.2f} {n * avg * 1e-3:10.3f}")
        return 0
    fetch, write = counter_summary(args.fetch), counter_summary(args.write)
    cfetch, cwrite = counter_summary(args.copy_fetch), counter_summary(args.copy_write)
    copy_bytes = COPY_MIB << 20

    def copy_kib(table, counter):
        # the copy probe's dispatches that move COPY_MIB (the largest copy kernel entries)
        vals = [(n * v, n) for (name, _, c), (n, v) in table.items() if c == counter and "copy" in name.lower()]
        tot, n = max(vals)
        return tot / n

    f_fetch = copy_bytes / (copy_kib(cfetch, "FETCH_SIZE") * 1024.0)
    f_write = copy_bytes / (copy_kib(cwrite, "WRITE_SIZE") * 1024.0)
    grid = finest_sweep_grid(args.level, args.precision)
    # the plain sweep (transfer argument IO = 0), not the launches that carry
    # the prolongation or the restriction
    def plain(name):
        return "k_lsgs_tile<" in name and ", 0>(" in name

    sweep = [(k, v) for k, v in fetch.items() if plain(k[0]) and k[1] == grid]
    wsweep = [(k, v) for k, v in write.items() if plain(k[0]) and k[1] == grid]
    if len(sweep) != 1 or len(wsweep) != 1:
        print("expected one finest-level sweep entry per counter run", sweep, wsweep, file=sys.stderr)
        return 1
    (kname, _, _), (nf, fk) = sweep[0]
    (_, (nw, wk)) = wsweep[0]
    rd, wr = fk * 1024.0 * f_fetch, wk * 1024.0 * f_write
    V = ((1 << args.level) + 1) ** 2
    wb = 4 if args.precision == "fp32_ir" else 8
    print(f"# HBM traffic of the finest-level LSGS sweep, {(1 << args.level) + 1}^2 vertices, {args.precision}")
    print(f"kernel: {kname}")
    print(f"grid: {grid}")
    print(f"level: {args.level}")
    print(f"source_hash: {sweep_source_hash()}")
    print(f"copy_fetch_factor: {f_fetch:.4f}")
    print(f"copy_write_factor: {f_write:.4f}")
    print(f"fetch_kib_per_dispatch: {fk:.1f}  (dispatches: {nf})")
    print(f"write_kib_per_dispatch: {wk:.1f}  (dispatches: {nw})")
    print(f"read_bytes_per_launch: {rd:.0f}")
    print(f"write_bytes_per_launch: {wr:.0f}")
    print(f"traffic_bytes_per_launch_{args.precision}: {rd + wr:.0f}")
    print(f"algorithmic_bytes_per_launch: {8 * V * wb}")
    print(f"traffic_over_algorithmic: {(rd + wr) / (8 * V * wb):.3f}")
    return 0


def copy_probe() -> int:
    """A plain device-to-device copy of COPY_MIB, five times: the reference
    that scales the traffic counters."""
    import torch

    n = (COPY_MIB << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 8, "copies": 5}), flush=True)
    return 0


def batch_measure(steps: int, tol: float):
    """64 independent instances (257^2, 513^2 or 1025^2 vertices, alpha
    log-uniform in [1e-8, 1], y_D seeds 3000 + i), FP32 cycles inside FP64
    refinement, solved together from x = 0; timed with the batched iterate
    replayed from a HIP graph and launched eagerly."""
    import torch

    import paper_1502_03917_amd as mg
    import workloads

    inst = workloads.batch_instances(64, seed=3)
    levels = [l for l, _, _ in inst]
    alphas = [a for _, a, _ in inst]
    yds = [torch.from_numpy(workloads.desired_state(l, sd)).cuda() for l, _, sd in inst]
    out = {"instances": len(inst), "levels": {str(l): levels.count(l) for l in sorted(set(levels))},
           "unknowns": sum(2 * ((1 << l) + 1) ** 2 for l in levels), "precision": "fp32_ir", "tol": tol}

    def timed(graph: bool):
        if not graph:
            os.environ["MGKKT_NO_GRAPH"] = "1"
        try:
            b = mg.Batch(levels, alphas, precision="fp32_ir")
        finally:
            os.environ.pop("MGKKT_NO_GRAPH", None)
        fs = b.rhs(yds)
        xs = [torch.zeros(b.vec_len(i), dtype=torch.float64, device="cuda") for i in range(len(inst))]
        b.solve(fs, xs, tol=tol, raise_on_error=False)  # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cyc_total, st = 0, 0
        for _ in range(steps):
            for x in xs:
                x.zero_()
            _, cyc, rel, _, st = b.solve(fs, xs, tol=tol, raise_on_error=False)
            cyc_total += sum(cyc)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        tiles = {str(l): b.sweep_tile(l) for l in sorted(set(levels))}
        b.close()
        return dt, cyc_total / steps, cyc, rel, st, tiles

    dt, cyc_sum, cyc, rel, st, tiles = timed(True)
    dt_eager, _, _, _, _, _ = timed(False)
    out["sweep_tiles_autotuned"] = tiles
    # final error of every instance's FP32-refinement solution against its
    # FP64 one-instance solve, per field (y, lambda, u = lambda / alpha)
    b = mg.Batch(levels, alphas, precision="fp32_ir")
    fs = b.rhs(yds)
    xs, _, _, _, _ = b.solve(fs, tol=tol, raise_on_error=False)
    errs = []
    for i, (l, a) in enumerate(zip(levels, alphas)):
        s1 = mg.Solver(l, a)
        x1, _, _, _ = s1.solve(s1.rhs(yds[i]), tol=tol, raise_on_error=False)
        e = field_errors(xs[i], x1, a)
        errs.append([float(f"{e['err_y']:.2e}"), float(f"{e['err_lambda']:.2e}"), float(f"{e['err_u']:.2e}")])
        s1.close()
    b.close()
    out["fp32_ir_err_vs_fp64_per_instance"] = {"fields": ["y", "lambda", "u"], "errors": errs,
                                               "max": [max(e[k] for e in errs) for k in range(3)]}
    nbytes = 0.0
    for l, c in zip(levels, cyc):
        V = ((1 << l) + 1) ** 2
        nbytes += c * (words_per_cycle(l, 1, 2, 2) * 4 + V * 2 * (8 + 8 + 8 + 4 + 8))
    out.update({"ms_per_solve": 1e3 * dt, "ms_per_solve_eager": 1e3 * dt_eager,
                "instance_vcycles_per_s": cyc_sum / dt, "cycles_min_max": [min(cyc), max(cyc)],
                "max_relres": max(rel), "status": mg.lib().mg_strerror(st).decode(),
                "aggregate_algorithmic_GBps": nbytes / dt / 1e9})
    return out


def stokes_measure(steps: int, tol: float, level: int = 9):
    """Stokes control (Taylor-Hood) on 513^2 vertices (4,712,454 unknowns),
    desired velocity from a seeded stream function (seed 7), V(2,2) cycles
    from x = 0 to relative residual tol: LSGS in FP64 and FP32 refinement for
    alpha in {1e-2, 1e-6}, and the patch smoother (FP64, alpha = 1e-2)."""
    import torch

    import paper_1502_03917_amd as mg
    import workloads

    vd = torch.from_numpy(workloads.desired_velocity(level, 7)).cuda()
    out = {"workload": f"Stokes control, {(1 << level) + 1}^2 vertices, Taylor-Hood, V(2,2), tol {tol:g}"}
    runs = [("lsgs", "fp64", 1e-2), ("lsgs", "fp32_ir", 1e-2), ("lsgs", "fp64", 1e-6), ("lsgs", "fp32_ir", 1e-6),
            ("vanka", "fp64", 1e-2)]
    keep = {}
    for sm, pr, al in runs:
        t0 = time.perf_counter()
        s = mg.Solver(level, al, problem="stokes", smoother=sm, precision=pr)
        setup = time.perf_counter() - t0
        n = s.vec_len()
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        f = s.rhs(vd)
        s.solve(f, x, tol=tol, raise_on_error=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cyc = 0
        for _ in range(steps):
            x.zero_()
            _, it, rel, st = s.solve(f, x, tol=tol, raise_on_error=False)
            cyc += it
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        rec = {"unknowns": n, "cycles": cyc / steps, "ms_per_solve": 1e3 * dt, "vcycles_per_s": cyc / steps / dt,
               "final_relres": rel, "status": mg.lib().mg_strerror(st).decode(), "setup_s": setup}
        if sm == "lsgs":
            keep[(pr, al)] = x.clone()
        if sm == "lsgs" and pr == "fp64" and al == 1e-2:
            # the finest-level LSGS sweep (59 colour phases) timed with events
            # on the launch stream: 4 words (read x, r; write x, r) per unknown
            r = s.residual(f, x)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            nsw = 8
            s.smooth(x, r, steps=1)
            ev0.record()
            s.smooth(x, r, steps=nsw)
            ev1.record()
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / nsw
            nbytes = 4 * n * 8
            rec["roofline"] = {"bound": "hbm", "kernel": "finest-level LSGS sweep (59 colour-phase launches)",
                               "sweep_ms": ms, "algorithmic_bytes_per_sweep": nbytes,
                               "achieved": nbytes / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        s.close()
        out[f"{sm}/{pr}/alpha={al:g}"] = rec
    for al in (1e-2, 1e-6):
        if ("fp64", al) in keep and ("fp32_ir", al) in keep:
            out[f"lsgs/fp32_ir/alpha={al:g}"]["field_errors_vs_fp64"] = field_errors(
                keep[("fp32_ir", al)], keep[("fp64", al)], al, "stokes", level)
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(level: int, alpha: float, seed: int, smoother: str, reps: int, gpu_cycles: float | None):
    """The FP64 CPU oracle on the host: V(2,2) cycles of the same workload in
    the same 7-colour order, from x = 0 (setup excluded), each timed alone,
    median of `reps`; (1) the OpenMP build on all host threads (the groups of
    one colour, the sparse products and the transfers in parallel; results
    bit-identical to the single-threaded build), (2) the single-threaded
    build.  Time to 1e-10 is extrapolated: the oracle's cycles equal the GPU
    FP64 cycles to 1e-12 at this size, so it needs the same number of cycles."""
    import statistics

    import numpy as np

    import oracle
    import workloads

    def leg(threaded: bool):
        h = oracle.Hierarchy(level, alpha, coarse=1, threaded=threaded)
        f = h.rhs(workloads.desired_state(level, seed))
        x = np.zeros(h.ndof())
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            h.cycle(f, x, smoother=smoother, order="col7")
            times.append(time.perf_counter() - t0)
        nthr = oracle.threads(threaded)
        h.close()
        med = statistics.median(times)
        rec = {"value": 1.0 / med, "unit": "V-cycles/s", "cores": nthr, "cycle_s_median": med,
               "cycle_s_all": times}
        if gpu_cycles:
            rec["cycles_to_tol"] = gpu_cycles
            rec["time_to_tol_s_extrapolated"] = gpu_cycles * med
        return rec

    log("bench: CPU oracle, all host threads")
    multi = leg(True)
    log("bench: CPU oracle, one thread")
    single = leg(False)
    host = {"nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)), "model": cpu_model()}
    out = dict(multi)
    out.update({"kind": "oracle",
                "sample": f"{reps} V(2,2) {smoother.upper()} cycles (7-colour order) of the {(1 << level) + 1}^2 "
                          f"workload, alpha={alpha:g}, from x=0, setup excluded, each timed, median; FP64 C "
                          f"oracle built with OpenMP on {multi['cores']} threads; time to 1e-10 = GPU cycle "
                          f"count x median cycle time (extrapolated)",
                "host": host, "single_core": single})
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--level", type=int, default=11)
    ap.add_argument("--alpha", type=float, default=1e-4)
    ap.add_argument("--smoother", default="lsgs")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--cpu-reps", type=int, default=3, help="oracle cycles timed per CPU leg (median)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance batched solve")
    ap.add_argument("--no-fp32-ir", action="store_true", help="skip the FP32-refinement rerun of the main workload")
    ap.add_argument("--no-cgs", action="store_true", help="skip the collective-smoother solves of the main workload")
    ap.add_argument("--batch-only", action="store_true", help="run only the 64-instance batched solve")
    ap.add_argument("--no-stokes", action="store_true", help="skip the Stokes-control solves")
    ap.add_argument("--stokes-only", action="store_true", help="run only the Stokes-control solves")
    ap.add_argument("--variants", action="store_true", help="also time the other smoother/precision/alpha variants")
    ap.add_argument("--copy-probe", action="store_true", help="run only the plain copy that calibrates the counters")
    ap.add_argument("--trace", help="summarise a rocprofv3 kernel-trace CSV directory and exit")
    ap.add_argument("--fetch", help="FETCH_SIZE counter CSV directory of a bench run (with --write, --copy-*)")
    ap.add_argument("--write", help="WRITE_SIZE counter CSV directory of a bench run")
    ap.add_argument("--copy-fetch", help="FETCH_SIZE counter CSV directory of --copy-probe")
    ap.add_argument("--copy-write", help="WRITE_SIZE counter CSV directory of --copy-probe")
    args = ap.parse_args()

    if args.trace or args.fetch:
        return print_summary(args)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this solver runs on one GPU; --gpus must be 1 (multi-GPU sharding is design only)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1502_03917_amd as mg
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        return copy_probe()
    if args.stokes_only:
        print(json.dumps(stokes_measure(max(1, args.steps // 5), args.tol)), flush=True)
        return 0
    if args.batch_only:
        print(json.dumps(batch_measure(max(2, args.steps // 3), args.tol)), flush=True)
        return 0
    yd = torch.from_numpy(workloads.desired_state(args.level, args.seed)).cuda()

    def run(smoother, precision, alpha, steps, warmup, timing=False, keep=False, gamma=1):
        nu = 1 if smoother == "slsgs" else 2
        s = mg.Solver(args.level, alpha, smoother=smoother, precision=precision, gamma=gamma, nu1=nu, nu2=nu)
        inner = s.opts().inner_cycles
        x = torch.zeros(s.vec_len(), dtype=torch.float64, device="cuda")
        for _ in range(warmup):
            x.zero_()
            f = s.rhs(yd)
            s.solve(f, x, tol=args.tol, raise_on_error=False)
        torch.cuda.synchronize()
        if timing:
            s.timing_enable(True)
        cycles = 0
        rel = None
        st = mg.MG_OK
        t0 = time.perf_counter()
        for _ in range(steps):
            x.zero_()
            f = s.rhs(yd)
            _, it, rel, st = s.solve(f, x, tol=args.tol, raise_on_error=False)
            cycles += it * (inner if precision == "fp32_ir" else 1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out = {"cycles_per_solve": cycles / steps, "ms_per_solve": 1e3 * dt / steps, "relres": rel,
               "vcycles_per_s": cycles / dt, "status": mg.lib().mg_strerror(st).decode()}
        if timing:
            ms, n = s.timing_read()
            s.timing_enable(False)
            out["sweep_ms"] = ms / max(n, 1)
            out["sweeps_timed"] = n
        if keep:
            out["x"] = x.clone()
        s.close()
        return out

    log(f"bench: level {args.level}, alpha {args.alpha:g}, {args.smoother}/{args.precision}, "
        f"{args.warmup} warmup + {args.steps} timed solves to {args.tol:g}")
    # pass 1: the timed solves (one HIP graph per iterate) give the throughput;
    # pass 2: the same solves launched eagerly with HIP events around every
    # finest-level smoothing sweep give the dominant kernel's duration
    main_run = run(args.smoother, args.precision, args.alpha, args.steps, args.warmup, timing=False)
    sweep_run = run(args.smoother, args.precision, args.alpha, max(2, args.steps // 2), 0, timing=True)
    main_run["sweep_ms"] = sweep_run["sweep_ms"]
    main_run["sweeps_timed"] = sweep_run["sweeps_timed"]
    if main_run["status"] != "success":
        log(f"bench: the timed solve ended with status '{main_run['status']}' at relres {main_run['relres']:.3e}")
    V = ((1 << args.level) + 1) ** 2
    wbytes = 4 if args.precision == "fp32_ir" else 8
    sweep_bytes = 8 * V * wbytes  # read and write x and r, both fields
    achieved = sweep_bytes / (main_run["sweep_ms"] * 1e-3) / 1e9
    traffic = recorded_traffic(args.precision, args.level)
    # the LSGS solve takes its residual norm from the last sweep (no residual pass)
    cyc_bytes = words_per_cycle(args.level, 1, 2, 2, fine_residual=args.smoother not in ("lsgs", "slsgs")) * wbytes
    if args.precision == "fp32_ir":
        cyc_bytes += V * 2 * (8 + 8 + 8 + 4 + 8)  # FP64 residual (f, x -> r), scaled cast, FP64 update
    result = {
        "metric": METRIC,
        "value": main_run["vcycles_per_s"],
        "unit": "V-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"Poisson control KKT, {(1 << args.level) + 1}^2 vertices, alpha={args.alpha:g}, "
                               f"y_D = 8 seeded sine modes (seed {args.seed}), x0 = 0, tol {args.tol:g}",
                   "level": args.level, "unknowns": 2 * V, "smoother": args.smoother, "cycle": "V(2,2)",
                   "precision": args.precision, "coarse_level": 1},
        "time_to_tol_ms": main_run["ms_per_solve"],
        "cycles_per_solve": main_run["cycles_per_solve"],
        "final_relres": main_run["relres"],
        "residual_norm": "L_k^-1 weighted (dual of the paper's L_k error norm)",
        "solve_status": main_run["status"],
        "unknown_updates_per_s": main_run["vcycles_per_s"] * sum(4 * 2 * ((1 << l) + 1) ** 2 for l in range(2, args.level + 1)),
        "cycle_algorithmic_GBps": main_run["vcycles_per_s"] * cyc_bytes / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "finest-level smoothing sweep", "sweep_ms": main_run["sweep_ms"],
                     "sweeps_timed": main_run["sweeps_timed"], "algorithmic_bytes_per_sweep": sweep_bytes,
                     "traffic_unit": "bytes per launch"},
    }
    if args.precision == "fp64" and not args.no_fp32_ir:
        # the same workload with FP32 cycles inside FP64 refinement (same FP64 tolerance)
        log("bench: the same solves with FP32 cycles inside FP64 refinement")
        ir = run(args.smoother, "fp32_ir", args.alpha, args.steps, args.warmup, timing=False)
        ir_sweep = run(args.smoother, "fp32_ir", args.alpha, max(2, args.steps // 2), 0, timing=True)
        ach = 8 * V * 4 / (ir_sweep["sweep_ms"] * 1e-3) / 1e9
        result["fp32_ir"] = {"vcycles_per_s": ir["vcycles_per_s"], "ms_per_solve": ir["ms_per_solve"],
                             "cycles_per_solve": ir["cycles_per_solve"], "final_relres": ir["relres"],
                             "status": ir["status"], "speedup_time_to_tol_vs_fp64": main_run["ms_per_solve"] / ir["ms_per_solve"],
                             "finest_sweep_ms": ir_sweep["sweep_ms"], "finest_sweep_GBps": ach,
                             "finest_sweep_frac_of_8TBps": ach / HBM_PEAK_GBS,
                             "finest_sweep_traffic": recorded_traffic("fp32_ir", args.level)}
        # final error of the FP32-refinement solve against the FP64 solve (whose
        # cycles match the oracle's at this size), per field, for each alpha
        errs = {}
        for al in (1e-8, 1e-4, 1.0):
            log(f"bench: FP32-refinement field errors, alpha {al:g}")
            x64 = run(args.smoother, "fp64", al, 1, 0, keep=True)["x"]
            x32 = run(args.smoother, "fp32_ir", al, 1, 0, keep=True)["x"]
            errs[f"alpha={al:g}"] = field_errors(x32, x64, al)
        result["fp32_ir"]["field_errors_vs_fp64"] = errs
    if args.smoother == "lsgs" and not args.no_cgs:
        # the collective point smoother (section 2) on the same workload: the
        # paper's fastest smoother for Poisson control (Table 1), one fused
        # tile kernel per sweep moving the same 8 words per vertex
        log("bench: the same solves with the collective point smoother")
        cg = {}
        for pr in ("fp64", "fp32_ir"):
            rr = run("cgs", pr, args.alpha, max(2, args.steps // 2), max(1, args.warmup // 2))
            rt = run("cgs", pr, args.alpha, 2, 0, timing=True)
            wb = 4 if pr == "fp32_ir" else 8
            ach = 8 * V * wb / (rt["sweep_ms"] * 1e-3) / 1e9
            cg[pr] = {"vcycles_per_s": rr["vcycles_per_s"], "ms_per_solve": rr["ms_per_solve"],
                      "cycles_per_solve": rr["cycles_per_solve"], "final_relres": rr["relres"], "status": rr["status"],
                      "finest_sweep_ms": rt["sweep_ms"], "finest_sweep_GBps": ach,
                      "finest_sweep_frac_of_8TBps": ach / HBM_PEAK_GBS,
                      "time_to_tol_speedup_vs_lsgs_fp64": main_run["ms_per_solve"] / rr["ms_per_solve"]}
        result["cgs"] = cg
    if args.variants:
        # NE and LSGS, FP64 and FP32 refinement, alpha 1e-8 / 1e-4 / 1 on the same
        # workload; the FP32-refinement iterate is compared with the FP64 one
        # (whose cycles match the oracle's at this size)
        var = {}
        for sm, gamma in (("ne", 1), ("lsgs", 1), ("cgs", 1), ("slsgs", 1), ("lsgs", 2)):
            for al in (1e-8, 1e-4, 1.0):
                tag = sm + ("/W" if gamma == 2 else "")
                log(f"bench: variants {tag}, alpha {al:g}")
                r64 = run(sm, "fp64", al, 2, 1, keep=True, gamma=gamma)
                r32 = run(sm, "fp32_ir", al, 2, 1, keep=True, gamma=gamma)
                t64 = run(sm, "fp64", al, 1, 0, timing=True, gamma=gamma)
                x64, x32 = r64.pop("x"), r32.pop("x")
                r32.update(field_errors(x32, x64, al))
                r32["speedup_time_to_tol_vs_fp64"] = r64["ms_per_solve"] / r32["ms_per_solve"]
                # finest-level smoothing step: HIP events around its launches
                r64["finest_step_ms"] = t64["sweep_ms"]
                var[f"{tag}/fp64/alpha={al:g}"] = r64
                var[f"{tag}/fp32_ir/alpha={al:g}"] = r32
        result["variants"] = var
    if not args.no_batch:
        log("bench: batched solve of 64 instances (fp32_ir)")
        result["batch"] = batch_measure(max(2, args.steps // 3), args.tol)
    if not args.no_stokes:
        log("bench: Stokes-control solves (513^2 vertices)")
        result["stokes"] = stokes_measure(max(1, args.steps // 5), args.tol)
    if not args.no_cpu_baseline:
        log(f"bench: CPU oracle baseline ({args.cpu_reps} cycles per leg)")
        result["cpu_baseline"] = cpu_baseline(args.level, args.alpha, args.seed, args.smoother, args.cpu_reps,
                                              main_run["cycles_per_solve"])
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
