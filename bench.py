"""Benchmark: DOF-solves/s of the hierarchical lattice solver on one MI355X.

Prints one JSON line.  One step is one complete pass of the hot path over one
batch of synthetic input (update, float64 residual, relaxation, upper-level
assembly and solve, stop test, until every solve meets its tolerance), with
the inputs already resident in HBM.

Workloads (--workload):
  default  the batched workload as the headline, with the 1024^2 single-lattice
           workload and a sample of the served stream measured beside it:
  c4       256 independent lattices (sides U{32..512}, aspect U[0.5, 2], shape
           seed 1000, lattice b seed 2000 + b, EA lognormal(0, 0.5), left edge
           clamped, loads N(0, 1), set edge chosen by the library per shape)
           solved together by tl_solve_batch to a relative residual of 1e-8;
           one step = the whole batch; the mixed form is the value, the float64
           form beside it; latency percentiles are those of the 256 solves
           within each batch;
  c2       1024 x 1024 nodes (2,097,152 DOF), EA = 1, sets of 32 x 32,
           float64 and mixed forms, relative residual 1e-8;
  c1       64 x 64 nodes, sets of 16 x 16, relative residual 1e-10;
  c3       16384 x 16384 nodes (536,870,912 DOF), EA lognormal(0, 0.5), sets
           of 64 x 64, mixed form, relative residual 1e-10;
  c5       served stream: square lattices with sides log-uniform in [64, 2048],
           EA lognormal(0, 0.5), submitted to a tl_server with a 200 GB budget,
           first closed-loop (saturation), then Poisson arrivals at 0.5, 0.8 and
           0.95 of the saturation rate; p50/p99 latency per offered load, on a
           bounded sample of the stream (--requests per load).

The roofline object covers the tile kernel (update, residual, relaxation and
the set rows of the upper level), the kernel that streams the lattice: its
algorithmic bytes per launch over its average launch duration, both from one
extra pass with every launch timed by HIP events on the launches' stream.
The CPU baseline times the CPU oracle on the host's cores for a bounded
sample (cpu_baseline_batch / cpu_baseline_single).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF·solves/s to 1e-8 rel. residual, mixed vs FP64 form; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# Kernel durations of single solves are taken with HIP events on every
# PROFILE_STRIDE-th outer iteration of the timed solves: an event record
# between two kernels costs a few microseconds, about 4 % of the 1024^2 solve
# when every launch is timed.  The kernel split comes from one more solve
# after the timed ones with every launch timed.
PROFILE_STRIDE = 8
# Host cores the CPU baseline may use: at most 16 (the CPU share of one GPU on
# an MI355X node).
MAX_CPU_WORKERS = 16

SINGLE = {
    "c1": dict(n=64, E=16, ea="unit", rtol=1e-10, headline="fp64",
               desc="triangle lattice 64x64 nodes (8,192 DOF), EA=1, L=1, nodes i=0 clamped, "
                    "loads N(0,1) seed 0, sets 16x16 nodes, stop at rel. residual 1e-10"),
    # traffic_bytes: HBM bytes per tile-kernel launch of the headline form from
    # the FETCH_SIZE / WRITE_SIZE counter runs (FETCH x 2.0, WRITE x 1.0,
    # calibrated on copy kernels); None when the kernel has changed since the
    # counters were taken.
    "c2": dict(n=1024, E=32, ea="unit", rtol=1e-8, headline="fp64", traffic_bytes=130.97e6,
               desc="triangle lattice 1024x1024 nodes (2,097,152 DOF), EA=1, L=1, left edge "
                    "clamped, loads N(0,1) seed 0, sets 32x32 nodes, stop at rel. residual 1e-8"),
    "c3": dict(n=16384, E=64, ea="lognormal", rtol=1e-10, headline="mixed", traffic_bytes=22.09e9,
               desc="triangle lattice 16384x16384 nodes (536,870,912 DOF), EA lognormal(0,0.5), "
                    "left edge clamped, loads N(0,1) seed 0, sets 64x64 nodes, mixed precision, "
                    "stop at rel. residual 1e-10"),
}
# HBM bytes per launch of the batched workload's dominant tile kernel
# (k_tile_batch<float, 32, 512, 2>) relative to its algorithmic bytes, from the
# FETCH_SIZE / WRITE_SIZE counter runs; None when the kernel has changed since.
C4_TRAFFIC_RATIO = 1.683


# Algorithmic HBM bytes of one tile-kernel launch per lattice node: read u
# (16) and write u (16), read f (16), read three rod stiffnesses (12), read
# the clamp mask (1), read and write the relaxation increment (2 x 8 mixed,
# 2 x 16 float64).  Halo re-reads are not counted.
def tile_bytes_per_node(mixed: bool) -> int:
    return 16 + 16 + 16 + 12 + 1 + (16 if mixed else 32)


def band_factor_bytes(n: int, E: int, ov: int = 2) -> int:
    """Bytes of band factor an exact-relaxation tile launch reads: every set's
    region (its tile widened by ov nodes, clipped to the lattice) has 2 rw rh
    DOFs, each a column of 2 R + 2 doubles (R = E + 2 ov), read once by the
    forward and once by the backward triangular solve."""
    R = E + 2 * ov
    total = 0
    for i0 in range(0, n, E):
        rw = min(i0 + E + ov, n) - max(i0 - ov, 0)
        for j0 in range(0, n, E):
            rh = min(j0 + E + ov, n) - max(j0 - ov, 0)
            total += 2 * (2 * rw * rh) * (2 * R + 2) * 8
    return total


T0 = time.perf_counter()


def progress(*a):
    print("[bench %7.1fs]" % (time.perf_counter() - T0), *a, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_workers():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, MAX_CPU_WORKERS))


# ----------------------------------------------------------- CPU baselines

def _oracle_one(job):
    """One oracle solve in a worker process (single-threaded BLAS/LAPACK):
    CSR assembly, then the exact constrained solve (dense, banded Cholesky
    or PCG by size), then its relative residual."""
    from threadpoolctl import threadpool_limits
    from oracle.solve import rel_residuals, solve, system_of
    from workloads import make_instance
    nx, ny, seed = job
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        inst = make_instance(nx, ny, seed=seed, ea="lognormal")
        S = system_of(inst)
        u = solve(S)
        R = max(rel_residuals(S, u))
        return inst.dof, time.perf_counter() - t0, R


def cpu_baseline_batch(shapes, budget_s):
    """The oracle on the batched workload's lattices, in their order, one
    single-threaded process per host core, for about budget_s seconds of wall
    time: the aggregate DOF-solves/s of the lattices completed by then."""
    import multiprocessing as mp
    n = cpu_workers()
    jobs = [(nx, ny, 2000 + b) for b, (nx, ny) in enumerate(shapes)]
    ctx = mp.get_context("spawn")
    done, dof, worst = 0, 0, 0.0
    t0 = time.perf_counter()
    t_last = t0
    # the workers start with one BLAS/OpenMP thread each (their environment is
    # this process's at the time they are spawned)
    saved = {v: os.environ.get(v) for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                             "MKL_NUM_THREADS")}
    os.environ.update({v: "1" for v in saved})
    try:
        pool = ctx.Pool(n)
    finally:
        for v, val in saved.items():
            if val is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = val
    with pool:
        it = pool.imap_unordered(_oracle_one, jobs, chunksize=1)
        while True:
            left = budget_s - (time.perf_counter() - t0)
            if left <= 0.0:
                break
            try:
                d, _, R = it.next(timeout=left)
            except (StopIteration, mp.TimeoutError):
                break
            done += 1
            dof += d
            worst = max(worst, R)
            t_last = time.perf_counter()
        pool.terminate()
    wall = t_last - t0
    return {
        "value": dof / wall,
        "unit": "DOF·solves/s",
        "cores": n,
        "kind": "oracle",
        "sample": (f"{done} of the {len(shapes)} batched lattices (taken in order) completed by "
                   f"the oracle (CSR assembly + exact banded/dense Cholesky, max rel. residual "
                   f"{worst:.1e}) in {n} single-threaded processes, {wall:.1f} s wall to the last "
                   f"completion; "
                   f"{os.cpu_count()} host cores, {cpu_model()}"),
    }


def cpu_baseline_single(inst, rtol, budget_s=20.0):
    """The oracle (CSR assembly + block-Jacobi PCG, one thread) on one large
    instance for a bounded sample: solve time = assembly + (time per PCG
    iteration) x (iterations a complete oracle run needed, recorded by
    oracle/record_pcg_iterations.py), else extrapolated log-linearly."""
    from threadpoolctl import threadpool_limits
    import numpy as np
    from oracle.solve import solve_pcg, system_of
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        S = system_of(inst)
        t_asm = time.perf_counter() - t0
        hist = []
        t1 = time.perf_counter()
        solve_pcg(S, rtol=rtol, max_seconds=budget_s, history=hist)
        t_pcg = time.perf_counter() - t1
    n = len(hist)
    its = np.array([h[0] for h in hist], dtype=float)
    rel = np.array([h[1] for h in hist])
    reached = np.flatnonzero(rel <= rtol)
    rec_path = os.path.join(ROOT, "tests", "golden", f"oracle_pcg_{inst.nx}.json")
    rec = None
    if os.path.exists(rec_path):
        with open(rec_path) as fh:
            rec = json.load(fh)
        if rec.get("lattice") != [inst.nx, inst.ny] or rec.get("rtol") != rtol:
            rec = None
    if reached.size:
        n_needed, how = float(its[reached[0]]), "converged within the sample"
    elif rec is not None:
        n_needed = float(rec["iterations_to_rtol"])
        how = (f"{n} PCG iterations timed; iteration count to {rtol:g} from a complete oracle "
               f"run on the same instance (tests/golden/{os.path.basename(rec_path)})")
    else:
        half = slice(n // 2, n)
        slope = np.polyfit(its[half], np.log10(rel[half]), 1)[0]
        n_needed = n + (math.log10(rtol) - math.log10(rel[-1])) / min(slope, -1e-12)
        how = f"{n} PCG iterations timed, iteration count extrapolated log-linearly"
    t_solve = t_asm + t_pcg / max(n, 1) * n_needed
    return {
        "value": inst.dof / t_solve, "unit": "DOF·solves/s", "cores": 1, "kind": "oracle",
        "sample": (f"oracle CSR assembly ({t_asm:.1f} s) + block-Jacobi PCG on the same "
                   f"{inst.nx}x{inst.ny} instance ({t_pcg:.1f} s); {how}; {n_needed:.0f} "
                   f"iterations; one thread; {os.cpu_count()} host cores, {cpu_model()}"),
    }


def common_fields(args, value, ms_per_step, dtype, config):
    return {
        "metric": METRIC, "value": value, "unit": "DOF·solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic", "config": config,
    }


# ------------------------------------------------------ single lattices

def sampled_error_vs_reference(wl, u):
    """Relative 2-norm error of the solution u (a device tensor) at the
    sampled DOFs of the oracle's stored reference solution of this workload
    (tests/golden/oracle_u_1024_sample.json: the 1024 x 1024 lattice only), or
    None when there is no reference for it."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                        "oracle_u_1024_sample.json")
    if wl["n"] != 1024 or wl["ea"] != "unit" or not os.path.exists(path):
        return None
    import numpy as np
    ref = json.load(open(path))
    idx = np.asarray(ref["dof"])
    want = np.asarray(ref["u"])
    got = u.reshape(-1).cpu().numpy()[idx]
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


def run_single(args, wl, steps=None, warmup=None):
    import torch
    from paper_1208_4093_amd import tl
    from workloads import make_instance
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    n, E = wl["n"], wl["E"]
    progress(f"generating {n}x{n} instance")
    inst = make_instance(n, n, seed=0, ea=wl["ea"])
    lat = tl.tl_lattice_create(n, n, ea=inst.ea, fixed=inst.fixed, set_edge=E)
    f = torch.from_numpy(inst.f).to("cuda")
    u = torch.zeros_like(f)
    stream = torch.cuda.current_stream()
    bad = []
    exact = getattr(args, "local_solve", "pcg") == "exact"
    local = tl.TL_LOCAL_EXACT if exact else tl.TL_LOCAL_PCG

    def run_form(precision):
        mixed = precision == tl.TL_MIXED
        name = "mixed" if mixed else "fp64"
        for w in range(warmup):   # the first exact solve also factors the regions
            u.zero_()
            tl.tl_solve(lat, f, u, stream=stream, precision=precision, rtol=wl["rtol"],
                        local_solve=local)
        torch.cuda.synchronize()
        lat_ms, infos = [], []
        t0 = time.perf_counter()
        for k in range(steps):
            ts = time.perf_counter()
            u.zero_()
            info = tl.tl_solve(lat, f, u, stream=stream, check=False, precision=precision,
                               rtol=wl["rtol"], profile=PROFILE_STRIDE, local_solve=local)
            torch.cuda.synchronize()
            lat_ms.append(1000.0 * (time.perf_counter() - ts))
            infos.append(info)
            progress(f"{n}^2 {name} step {k + 1}/{steps}: {lat_ms[-1]:.1f} ms, "
                     f"{info['iters']} iterations, status {info['status']}")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ok = [i for i in infos if i["status"] == tl.TL_OK]
        bad.extend(i for i in infos if i["status"] != tl.TL_OK or
                   max(i["rel_res_l1"], i["rel_res_l2"]) > wl["rtol"])
        launches = sum(i["tile_launches"] for i in infos)
        tile_ms = sum(i["tile_ms"] for i in infos) / max(launches, 1)
        nodes = n * n
        tile_bytes = tile_bytes_per_node(mixed) * nodes + (band_factor_bytes(n, E) if exact else 0)
        tile_gbs = tile_bytes / (tile_ms * 1e-3) / 1e9
        u.zero_()
        full = tl.tl_solve(lat, f, u, stream=stream, precision=precision, rtol=wl["rtol"], profile=1,
                           local_solve=local)
        torch.cuda.synchronize()
        kern = {"tile": full["tile_ms"], "offdiag": full["offdiag_ms"], "coarse": full["coarse_ms"]}
        per_launch = {k: v / max(full["tile_launches"], 1) for k, v in kern.items()}
        per_launch["tile"] = tile_ms
        err = sampled_error_vs_reference(wl, u)
        return {
            "rel_err_vs_oracle_sample": err,
            "value": inst.dof * len(ok) / wall, "ms_per_step": 1000.0 * wall / steps,
            "p50_ms": percentile(lat_ms, 50), "p99_ms": percentile(lat_ms, 99),
            "iters": infos[-1]["iters"], "coarse_iters": infos[-1]["coarse_iters"],
            "rel_res": max(max(i["rel_res_l1"], i["rel_res_l2"]) for i in infos),
            "failed": len(infos) - len(ok),
            "kernel_ms_per_launch": per_launch,
            "kernel_share": {k: v / max(sum(kern.values()), 1e-30) for k, v in kern.items()},
            "tile_gbs": tile_gbs, "tile_bytes_per_launch": tile_bytes,
            "coarse_us_per_pcg_iteration": 1000.0 * full["coarse_ms"] / max(full["coarse_iters"], 1),
        }

    forms = [tl.TL_FP64, tl.TL_MIXED] if wl["headline"] == "fp64" else [tl.TL_MIXED, tl.TL_FP64]
    if args.headline_only:
        forms = forms[:1]
    if exact:   # exact local solves exist in the float64 form only
        forms = [tl.TL_FP64]
    res = {p: run_form(p) for p in forms}
    head = res[forms[0]]
    tile_ms = head["kernel_ms_per_launch"]["tile"]
    tb = wl.get("traffic_bytes")
    out = {
        "value": head["value"], "ms_per_step": head["ms_per_step"],
        "dtype": "f64" if wl["headline"] == "fp64" or exact else "f32+f64",
        "config": {"workload": wl["desc"] + (", exact local solves" if exact else ""),
                   "dof": inst.dof, "set_edge": E, "form": "fp64" if exact else wl["headline"],
                   "local_solve": "exact" if exact else "pcg"},
        "latency_ms": {"p50": head["p50_ms"], "p99": head["p99_ms"]},
        "iters": head["iters"], "coarse_iters": head["coarse_iters"], "rel_res": head["rel_res"],
        "rel_err_vs_oracle_sample": head["rel_err_vs_oracle_sample"],
        "failed": head["failed"], "kernel_ms_per_launch": head["kernel_ms_per_launch"],
        "kernel_share": head["kernel_share"],
        "coarse_us_per_pcg_iteration": head["coarse_us_per_pcg_iteration"],
        "roofline": {
            "kernel": ("k_tile (update + float64 residual + exact relaxation with the band factor "
                       "streamed from HBM + set rows of the upper level)" if exact else
                       "k_tile (update + float64 residual + LDS relaxation + set rows of the upper level)"),
            "bound": "hbm", "achieved": head["tile_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": head["tile_gbs"] / HBM_PEAK_GBS,
            "traffic": tb / (tile_ms * 1e-3) / 1e9 if tb and not exact else None,
            "avg_launch_us": 1000.0 * tile_ms,
            "algorithmic_bytes_per_launch": head["tile_bytes_per_launch"],
            "time_share": head["kernel_share"]["tile"],
        },
    }
    if len(forms) > 1:
        other = res[forms[1]]
        out["mixed" if wl["headline"] == "fp64" else "fp64"] = {
            k: other[k] for k in ("value", "ms_per_step", "p50_ms", "p99_ms", "iters", "rel_res",
                                  "rel_err_vs_oracle_sample", "failed", "kernel_ms_per_launch",
                                  "tile_gbs")}
        m, d = (res[tl.TL_MIXED], res[tl.TL_FP64])
        out["mixed_over_fp64"] = m["value"] / d["value"]
    lat.close()
    return out, inst, bad


# ---------------------------------------------------- batched lattices

def run_batch(args):
    """The batched workload: all lattices in one tl_solve_batch per step."""
    import torch
    from paper_1208_4093_amd import tl
    from workloads import batch_shapes, make_instance

    shapes = batch_shapes(args.lattices)
    lats, fs, us, dof, nodes = [], [], [], 0, []
    for b, (nx, ny) in enumerate(shapes):
        inst = make_instance(nx, ny, seed=2000 + b, ea="lognormal")
        lats.append(tl.tl_lattice_create(nx, ny, ea=inst.ea, fixed=inst.fixed))
        fs.append(torch.from_numpy(inst.f).cuda())
        us.append(torch.zeros_like(fs[-1]))
        dof += inst.dof
        nodes.append(nx * ny)
    edges = {e: sum(1 for l in lats if l.set_edge == e) for e in (16, 32, 64)}
    progress(f"{len(lats)} lattices on the device, {dof} DOF, set edges {edges}")
    bad = []

    def run_form(precision):
        mixed = precision == tl.TL_MIXED
        name = "mixed" if mixed else "fp64"
        for w in range(args.warmup):
            tl.tl_solve_batch(lats, fs, us, check=False, precision=precision, rtol=1e-8)
            torch.cuda.synchronize()
            progress(f"batch {name} warmup {w + 1}/{args.warmup}")
        walls, per_solve_ms, ok_dof, failed, worst = [], [], 0, 0, 0.0
        infos = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            ts = time.perf_counter()
            st, infos = tl.tl_solve_batch(lats, fs, us, check=False, precision=precision, rtol=1e-8)
            torch.cuda.synchronize()
            walls.append(1000.0 * (time.perf_counter() - ts))
            for l, i in zip(lats, infos):
                good = i["status"] == tl.TL_OK and max(i["rel_res_l1"], i["rel_res_l2"]) <= 1e-8
                ok_dof += l.dof if good else 0
                failed += 0 if good else 1
                worst = max(worst, i["rel_res_l1"], i["rel_res_l2"])
                per_solve_ms.append(i["ms"])
            progress(f"batch {name} step {k + 1}/{args.steps}: {walls[-1]:.1f} ms, status {st}")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if failed:
            bad.append({"form": name, "failed": failed})
        return {
            "value": ok_dof / wall, "ms_per_step": 1000.0 * wall / args.steps,
            "batch_ms": {"p50": percentile(walls, 50), "p99": percentile(walls, 99)},
            "latency_ms": {"p50": percentile(per_solve_ms, 50), "p99": percentile(per_solve_ms, 99)},
            "iters": {"max": max(i["iters"] for i in infos),
                      "median": statistics.median(i["iters"] for i in infos)},
            "max_rel_res": worst, "failed": failed, "infos": infos,
        }

    def roofline(precision, infos):
        """One more batch outside the timed steps with every launch timed:
        the dominant tile kernel (the set edge with the most tile time)."""
        mixed = precision == tl.TL_MIXED
        _, pinf = tl.tl_solve_batch(lats, fs, us, check=False, precision=precision, rtol=1e-8,
                                    profile=1)
        torch.cuda.synchronize()
        by_edge = {}
        for l, i in zip(lats, pinf):
            e = by_edge.setdefault(l.set_edge, {"ms": i["tile_ms"], "launches": i["tile_launches"],
                                               "bytes": 0})
            e["bytes"] += (i["iters"] + 1) * l.nx * l.ny * tile_bytes_per_node(mixed)
        total_tile = sum(e["ms"] for e in by_edge.values())
        E, dom = max(by_edge.items(), key=lambda kv: kv[1]["ms"])
        avg_ms = dom["ms"] / max(dom["launches"], 1)
        per_launch = dom["bytes"] / max(dom["launches"], 1)
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        coarse = pinf[0]["coarse_ms"]
        offd = pinf[0]["offdiag_ms"]
        tf = C4_TRAFFIC_RATIO if mixed else None
        return {
            "kernel": (f"k_tile_batch<{'float' if mixed else 'double'}, {E}, 512, 2> (update + "
                       "float64 residual + LDS relaxation + set rows of the upper level; the "
                       "batch's lattices with that set edge)"),
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": achieved * tf if tf else None,
            "avg_launch_us": 1000.0 * avg_ms, "launches": dom["launches"],
            "algorithmic_bytes_per_launch": per_launch,
            "time_share": dom["ms"] / max(total_tile + coarse + offd, 1e-30),
            "kernel_ms_per_batch": {"tile": total_tile, "offdiag_blockinv": offd, "coarse": coarse},
        }

    mixed = run_form(tl.TL_MIXED)
    roof = roofline(tl.TL_MIXED, mixed["infos"])
    fp64 = None
    if not args.headline_only:
        fp64 = run_form(tl.TL_FP64)
        fp64["roofline"] = roofline(tl.TL_FP64, fp64["infos"])
    config = {
        "workload": (f"{len(lats)} independent triangle lattices, sides U{{32..512}} with aspect "
                     "U[0.5,2] (shape seed 1000, lattice b seed 2000+b), EA lognormal(0,0.5), left "
                     "edge clamped, loads N(0,1), set edge chosen by the library per shape, mixed "
                     "precision, stop at rel. residual 1e-8, fused launches with hipGraph replay"),
        "dof": dof, "lattices": len(lats), "set_edges": edges, "form": "mixed"}
    out = {
        "value": mixed["value"], "ms_per_step": mixed["ms_per_step"], "dtype": "f32+f64",
        "config": config, "latency_ms": mixed["latency_ms"], "batch_ms": mixed["batch_ms"],
        "iters": mixed["iters"], "rel_res": mixed["max_rel_res"], "failed": mixed["failed"],
        "roofline": roof,
    }
    if fp64 is not None:
        out["fp64"] = {k: fp64[k] for k in ("value", "ms_per_step", "latency_ms", "batch_ms",
                                            "iters", "max_rel_res", "failed", "roofline")}
        out["mixed_over_fp64"] = mixed["value"] / fp64["value"]
    for l in lats:
        l.close()
    return out, shapes, bad


# ------------------------------------------------------------- served

def run_served(args):
    """Served workload: requests through tl_server, closed loop then Poisson."""
    import torch
    from paper_1208_4093_amd import tl
    from workloads import make_instance, poisson_arrivals, served_sides

    R = args.requests
    sides = served_sides(R)
    reqs, dof_total = [], 0
    for k, side in enumerate(sides):
        inst = make_instance(side, side, seed=3000 + k, ea="lognormal")
        lat = tl.tl_lattice_create(side, side, ea=inst.ea, fixed=inst.fixed)
        f = torch.from_numpy(inst.f).cuda()
        reqs.append((lat, f, torch.zeros_like(f), inst.dof))
        dof_total += inst.dof
    torch.cuda.synchronize()
    mean_dof = dof_total / R
    progress(f"{R} requests prepared, mean {mean_dof:.3g} DOF, largest side {max(sides)}")
    budget = 200 * 10**9
    bad = []

    def serve(precision, arrivals, label):
        srv = tl.tl_server_create(budget, args.max_slots)
        pending, lat_ms, iters = {}, [], []
        failed, ok_dof = 0, 0
        t0 = time.perf_counter()
        nxt, done = 0, 0
        last_note = t0
        while done < R:
            now = time.perf_counter() - t0
            while nxt < R and (arrivals is None or arrivals[nxt] <= now):
                lat, f, u, _ = reqs[nxt]
                pending[tl.tl_submit(srv, lat, f, u, precision=precision, rtol=1e-8)] = nxt
                nxt += 1
            for t in list(pending):
                st, info = tl.tl_poll(srv, t)
                if st != tl.TL_PENDING:
                    k = pending.pop(t)
                    done += 1
                    good = st == tl.TL_OK and max(info["rel_res_l1"], info["rel_res_l2"]) <= 1e-8
                    failed += 0 if good else 1
                    ok_dof += reqs[k][3] if good else 0
                    lat_ms.append(info["ms"])
                    iters.append(info["iters"])
            if time.perf_counter() - last_note > 5.0:
                last_note = time.perf_counter()
                progress(f"{label}: {done}/{R} finished, {len(pending)} in flight")
            time.sleep(0.0005)
        wall = time.perf_counter() - t0
        srv.close()
        progress(f"{label}: {R} requests in {wall:.1f} s")
        if failed:
            bad.append({"served": label, "failed": failed})
        return {"dof_solves_per_s": ok_dof / wall, "wall_s": wall, "requests": R,
                "p50_ms": percentile(lat_ms, 50), "p99_ms": percentile(lat_ms, 99),
                "max_iters": max(iters), "failed": failed}

    for w in range(args.warmup):
        serve(tl.TL_MIXED, None, f"served warmup {w + 1}")
    sat = serve(tl.TL_MIXED, None, "served mixed closed loop")
    sat64 = None if args.headline_only else serve(tl.TL_FP64, None, "served fp64 closed loop")
    loads = []
    for k, rho in enumerate((0.5, 0.8, 0.95)):
        rate = rho * sat["dof_solves_per_s"] / mean_dof
        arr = poisson_arrivals(R, rate, seed=3000 + k)
        r = serve(tl.TL_MIXED, arr, f"served offered load {rho}")
        r.update({"offered_load": rho, "arrival_rate_per_s": rate})
        loads.append(r)
    out = {
        "value": sat["dof_solves_per_s"], "ms_per_step": 1000.0 * sat["wall_s"], "dtype": "f32+f64",
        "config": {
            "workload": (f"served stream sample: {R} square triangle lattices, sides log-uniform in "
                         "[64,2048] (seed 3000, request k seed 3000+k), EA lognormal(0,0.5), left "
                         "edge clamped, loads N(0,1), stop at rel. residual 1e-8, HBM budget 200 GB, "
                         f"{args.max_slots} slots; Poisson arrivals at 0.5/0.8/0.95 of the "
                         "closed-loop rate"),
            "requests": R, "mean_dof": mean_dof, "form": "mixed"},
        "latency_ms": {"p50": loads[-1]["p50_ms"], "p99": loads[-1]["p99_ms"],
                       "offered_load": loads[-1]["offered_load"]},
        "closed_loop": sat, "offered_loads": loads,
    }
    if sat64 is not None:
        out["fp64_closed_loop"] = sat64
        out["mixed_over_fp64"] = sat["dof_solves_per_s"] / sat64["dof_solves_per_s"]
    for lat, _, _, _ in reqs:
        lat.close()
    return out, bad


# ---------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="default",
                    choices=["default", "c4", "c5"] + sorted(SINGLE))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--headline-only", action="store_true",
                    help="measure only the headline precision form")
    ap.add_argument("--lattices", type=int, default=256, help="batched workload: lattices per batch")
    ap.add_argument("--requests", type=int, default=80, help="served workload: requests per load")
    ap.add_argument("--max-slots", type=int, default=64, help="served workload: server slots")
    ap.add_argument("--local-solve", choices=["pcg", "exact"], default="pcg",
                    help="single-lattice workloads: relaxation by PCG sweeps, or exact with "
                         "band Cholesky factors (float64 form only)")
    args = ap.parse_args()
    if args.local_solve == "exact" and args.workload not in SINGLE:
        print("--local-solve exact applies to the single-lattice workloads "
              f"({', '.join(sorted(SINGLE))})", file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the solver "
              "runs on a single MI355X and nothing in it uses a second GPU", file=sys.stderr)
        sys.exit(2)
    bad = []
    if args.workload in ("default", "c4"):
        from workloads import batch_shapes
        cpu = None
        if not args.no_cpu_baseline:
            # before any GPU work: the oracle's worker processes start clean
            progress(f"timing the CPU oracle on the batched lattices ({args.cpu_budget:.0f} s)")
            cpu = cpu_baseline_batch(batch_shapes(args.lattices), args.cpu_budget)
            progress(f"CPU oracle: {cpu['value']:.3g} DOF·solves/s on {cpu['cores']} cores")
        res, shapes, b = run_batch(args)
        bad += b
        out = common_fields(args, res.pop("value"), res.pop("ms_per_step"), res.pop("dtype"),
                            res.pop("config"))
        out.update(res)
        out["cpu_baseline"] = cpu
        if args.workload == "default":
            c2, _, b = run_single(args, SINGLE["c2"], steps=args.steps, warmup=args.warmup)
            bad += b
            out["c2_1024"] = c2
            c5, b = run_served(args)
            bad += b
            out["c5_served"] = c5
    elif args.workload == "c5":
        res, bad = run_served(args)
        out = common_fields(args, res.pop("value"), res.pop("ms_per_step"), res.pop("dtype"),
                            res.pop("config"))
        out["steps"] = 1
        out.update(res)
        out["roofline"] = None
        out["roofline_note"] = "kernel figures come from the kernel trace of this workload"
        out["cpu_baseline"] = None
    else:
        wl = SINGLE[args.workload]
        res, inst, bad = run_single(args, wl)
        out = common_fields(args, res.pop("value"), res.pop("ms_per_step"), res.pop("dtype"),
                            res.pop("config"))
        out.update(res)
        if not args.no_cpu_baseline and wl["n"] <= 4096:
            progress("timing the CPU oracle on a bounded sample")
            out["cpu_baseline"] = cpu_baseline_single(inst, min(wl["rtol"], 1e-8), args.cpu_budget)
        else:
            out["cpu_baseline"] = None
            if wl["n"] > 4096:
                out["cpu_baseline_note"] = ("not run: the oracle's CSR matrix of this lattice "
                                            "would not fit host memory")
    out["valid"] = not bad
    if bad:
        out["invalid_because"] = bad[:8]
    print(json.dumps(out), flush=True)
    if bad:
        sys.exit(3)


if __name__ == "__main__":
    main()
