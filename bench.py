"""Benchmark: DOF-solves/s of the hierarchical lattice solver on one MI355X.

One step = one complete solve (to a relative residual of 1e-8 unless the
workload says otherwise) of the workload's lattice, inputs already resident
in HBM.  Prints one JSON line.

Workloads (--workload):
  c2 (default)  1024 x 1024 nodes (2,097,152 DOF), EA = 1, left edge clamped,
                loads N(0, 1) (seed 0), sets of 32 x 32 nodes, float64 form
                as the headline value, the mixed form measured beside it;
  c1            64 x 64 nodes, sets of 16 x 16, relative residual 1e-10;
  c3            16384 x 16384 nodes (536,870,912 DOF), EA lognormal(0, 0.5),
                sets of 64 x 64, mixed form as the headline, residual 1e-10;
  c4            256 independent lattices (sides U{32..512}, aspect U[0.5, 2],
                EA lognormal(0, 0.5), set edge chosen per shape) solved together
                by tl_solve_batch; one step = the whole batch; mixed headline;
  c5            served stream: square lattices with sides log-uniform in
                [64, 2048], EA lognormal(0, 0.5), submitted to a tl_server with a
                200 GB budget, first closed-loop (saturation), then Poisson
                arrivals at 0.5, 0.8 and 0.95 of the saturation rate; p50/p99
                latency per offered load.  A bounded sample of the stream
                (--requests per load) keeps the run to about a minute.

The roofline object is computed from per-launch kernel durations measured
with HIP events on the solve's stream inside the timed steps (the launches of
every PROFILE_STRIDE-th outer iteration); the CPU
baseline times the CPU oracle on the host for a bounded sample (see
cpu_baseline()).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF·solves/s to 1e-8 rel. residual, mixed vs FP64 form; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# Kernel durations are taken with HIP events on every PROFILE_STRIDE-th outer
# iteration of the timed solves: an event record between two kernels costs a
# few microseconds, about 4 % of the 1024^2 solve when every launch is timed.
# The tile kernel's launches all do the same work, so that sample gives its
# average; the upper level's launch time follows its PCG iteration count,
# which varies from one outer iteration to the next in a pattern that a fixed
# stride can miss, so the kernel split comes from one more solve after the
# timed ones with every launch timed.
PROFILE_STRIDE = 8

WORKLOADS = {
    "c1": dict(n=64, E=16, ea="unit", rtol=1e-10, headline="fp64",
               desc="triangle lattice 64x64 nodes (8,192 DOF), EA=1, L=1, nodes i=0 clamped, "
                    "loads N(0,1) seed 0, sets 16x16 nodes, stop at rel. residual 1e-10"),
    # traffic: HBM bytes per k_tile launch of the headline form from the
    # FETCH_SIZE / WRITE_SIZE counter runs in profiles/counters_k_tile_c2_1024.md
    # and profiles/counters_k_tile_c3_16384.md (FETCH x 2.0, WRITE x 1.0,
    # calibrated on copy kernels); None when the kernel has changed since the
    # counters were taken.
    "c2": dict(n=1024, E=32, ea="unit", rtol=1e-8, headline="fp64",
               traffic_bytes=(62557.5 * 2.0 + 84345.8) * 1024,
               desc="triangle lattice 1024x1024 nodes (2,097,152 DOF), EA=1, L=1, left edge "
                    "clamped, loads N(0,1) seed 0, sets 32x32 nodes, stop at rel. residual 1e-8"),
    "c3": dict(n=16384, E=64, ea="lognormal", rtol=1e-10, headline="mixed",
               traffic_bytes=(7575317.2 * 2.0 + 6315497.0) * 1024,
               desc="triangle lattice 16384x16384 nodes (536,870,912 DOF), EA lognormal(0,0.5), "
                    "left edge clamped, loads N(0,1) seed 0, sets 64x64 nodes, mixed precision, "
                    "stop at rel. residual 1e-10"),
}

# Algorithmic HBM bytes of one tile-kernel launch per lattice node: read u
# (16) and write u (16), read f (16), read three rod stiffnesses (12), read
# the clamp mask (1), read and write the relaxation increment (2 x 8 mixed,
# 2 x 16 float64).  Halo re-reads are not counted.
def tile_bytes_per_node(mixed: bool) -> int:
    return 16 + 16 + 16 + 12 + 1 + (16 if mixed else 32)


def progress(*a):
    print("[bench %7.1fs]" % (time.perf_counter() - T0), *a, file=sys.stderr, flush=True)


T0 = time.perf_counter()


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_baseline(inst, rtol, budget_s=20.0):
    """The CPU oracle (plain FP64 CSR assembly + block-Jacobi PCG, one thread)
    on the same instance, for a bounded sample: the assembly in full, then
    PCG iterations for about budget_s seconds.  A complete oracle solve of a
    large lattice takes too long for a benchmark run, so the solve time is
    assembly + (measured time per PCG iteration) x (iterations the oracle
    needs to reach rtol on this instance), the count taken from the record
    written by oracle/record_pcg_iterations.py when it exists and otherwise
    extrapolated from the log-linear decay of the sampled residuals."""
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
        how = (f"{n} PCG iterations timed, reaching {rel[-1]:.2e}; iteration count "
               f"extrapolated log-linearly (no complete-run record)")
    t_solve = t_asm + t_pcg / max(n, 1) * n_needed
    return {
        "value": inst.dof / t_solve,
        "unit": "DOF·solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle CSR assembly ({t_asm:.1f} s) + block-Jacobi PCG on the same "
                   f"{inst.nx}x{inst.ny} instance ({t_pcg:.1f} s); {how}; "
                   f"{n_needed:.0f} iterations; one thread of {os.cpu_count()} host cores "
                   f"({platform.processor() or platform.machine()})"),
    }


def common_fields(args, metric_value, ms_per_step, dtype, config):
    return {
        "metric": METRIC,
        "value": metric_value,
        "unit": "DOF·solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": config,
    }


def run_single(args, wl):
    import torch
    from paper_1208_4093_amd import tl
    from workloads import make_instance

    n, E = wl["n"], wl["E"]
    progress(f"generating {n}x{n} instance")
    inst = make_instance(n, n, seed=0, ea=wl["ea"])
    lat = tl.tl_lattice_create(n, n, ea=inst.ea, fixed=inst.fixed, set_edge=E)
    f = torch.from_numpy(inst.f).to("cuda")
    u = torch.zeros_like(f)
    stream = torch.cuda.current_stream()
    progress("lattice on the device")

    def run_form(precision):
        mixed = precision == tl.TL_MIXED
        name = "mixed" if mixed else "fp64"
        for w in range(args.warmup):
            u.zero_()
            info = tl.tl_solve(lat, f, u, stream=stream, precision=precision, rtol=wl["rtol"])
            progress(f"{name} warmup {w + 1}/{args.warmup}: {info['iters']} iterations")
        torch.cuda.synchronize()
        lat_ms, infos = [], []
        t0 = time.perf_counter()
        for k in range(args.steps):
            ts = time.perf_counter()
            u.zero_()
            info = tl.tl_solve(lat, f, u, stream=stream, precision=precision, rtol=wl["rtol"],
                               profile=PROFILE_STRIDE)
            torch.cuda.synchronize()
            lat_ms.append(1000.0 * (time.perf_counter() - ts))
            infos.append(info)
            progress(f"{name} step {k + 1}/{args.steps}: {lat_ms[-1]:.1f} ms, "
                     f"{info['iters']} iterations")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        launches = sum(i["tile_launches"] for i in infos)
        nodes = n * n
        tile_ms = sum(i["tile_ms"] for i in infos) / max(launches, 1)
        tile_gbs = tile_bytes_per_node(mixed) * nodes / (tile_ms * 1e-3) / 1e9
        # kernel split: one more solve, outside the timed region, every launch timed
        u.zero_()
        full = tl.tl_solve(lat, f, u, stream=stream, precision=precision, rtol=wl["rtol"], profile=1)
        torch.cuda.synchronize()
        kern = {"tile": full["tile_ms"], "offdiag": full["offdiag_ms"], "coarse": full["coarse_ms"]}
        per_launch = {k: v / max(full["tile_launches"], 1) for k, v in kern.items()}
        per_launch["tile"] = tile_ms
        return {
            "value": inst.dof * args.steps / wall,
            "ms_per_step": 1000.0 * wall / args.steps,
            "p50_ms": percentile(lat_ms, 50),
            "p99_ms": percentile(lat_ms, 99),
            "iters": infos[-1]["iters"],
            "coarse_iters": infos[-1]["coarse_iters"],
            "rel_res": max(infos[-1]["rel_res_l1"], infos[-1]["rel_res_l2"]),
            "kernel_ms_per_launch": per_launch,
            "kernel_share": {k: v / max(sum(kern.values()), 1e-30) for k, v in kern.items()},
            "tile_gbs": tile_gbs,
            "tile_bytes_per_launch": tile_bytes_per_node(mixed) * nodes,
            # the upper-level kernel is bound by its grid synchronisations: time
            # per PCG iteration (launch prologue included), from the fully
            # timed solve
            "coarse_us_per_pcg_iteration": 1000.0 * full["coarse_ms"] / max(full["coarse_iters"], 1),
        }

    forms = [tl.TL_FP64, tl.TL_MIXED] if wl["headline"] == "fp64" else [tl.TL_MIXED, tl.TL_FP64]
    if args.headline_only:
        forms = forms[:1]
    res = {p: run_form(p) for p in forms}
    head = res[forms[0]]
    tile_ms = head["kernel_ms_per_launch"]["tile"]
    roof = {
        "kernel": "k_tile (update + float64 residual + LDS relaxation + set rows of the upper level)",
        "bound": "hbm",
        "achieved": head["tile_gbs"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": head["tile_gbs"] / HBM_PEAK_GBS,
        "traffic": (wl["traffic_bytes"] / (tile_ms * 1e-3) / 1e9
                    if wl.get("traffic_bytes") else None),
        "traffic_bytes_per_launch": wl.get("traffic_bytes"),
        "avg_launch_us": 1000.0 * tile_ms,
        "algorithmic_bytes_per_launch": head["tile_bytes_per_launch"],
        "time_share": head["kernel_share"]["tile"],
    }
    out = common_fields(args, head["value"], head["ms_per_step"],
                        "f64" if wl["headline"] == "fp64" else "f32+f64",
                        {"workload": wl["desc"], "dof": inst.dof, "set_edge": E,
                         "form": wl["headline"]})
    out.update({
        "latency_ms": {"p50": head["p50_ms"], "p99": head["p99_ms"]},
        "iters": head["iters"],
        "coarse_iters": head["coarse_iters"],
        "rel_res": head["rel_res"],
        "kernel_ms_per_launch": head["kernel_ms_per_launch"],
        "kernel_share": head["kernel_share"],
        "coarse_us_per_pcg_iteration": head["coarse_us_per_pcg_iteration"],
    })
    if len(forms) > 1:
        other = res[forms[1]]
        out["mixed" if wl["headline"] == "fp64" else "fp64"] = {
            "value": other["value"], "ms_per_step": other["ms_per_step"],
            "p50_ms": other["p50_ms"], "p99_ms": other["p99_ms"], "iters": other["iters"],
            "rel_res": other["rel_res"], "kernel_ms_per_launch": other["kernel_ms_per_launch"],
            "tile_gbs": other["tile_gbs"]}
    out["roofline"] = roof
    if not args.no_cpu_baseline and n <= 4096:
        progress("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(inst, 1e-8 if wl["rtol"] >= 1e-8 else wl["rtol"],
                                           args.cpu_budget)
    elif not args.no_cpu_baseline:
        out["cpu_baseline"] = None
        out["cpu_baseline_note"] = ("not run: the oracle's CSR matrix of this lattice would not "
                                    "fit host memory")
    lat.close()
    return out


def run_batch(args):
    """Batched workload: 256 lattices in one tl_solve_batch per step."""
    import torch
    from paper_1208_4093_amd import tl
    from workloads import batch_shapes, make_instance

    shapes = batch_shapes(args.lattices)
    lats, fs, us, dof = [], [], [], 0
    for b, (nx, ny) in enumerate(shapes):
        inst = make_instance(nx, ny, seed=2000 + b, ea="lognormal")
        lats.append(tl.tl_lattice_create(nx, ny, ea=inst.ea, fixed=inst.fixed))
        fs.append(torch.from_numpy(inst.f).cuda())
        us.append(torch.zeros_like(fs[-1]))
        dof += inst.dof
    edges = {e: sum(1 for l in lats if l.set_edge == e) for e in (16, 32, 64)}
    progress(f"{len(lats)} lattices on the device, {dof} DOF, set edges {edges}")

    def run_form(precision):
        name = "mixed" if precision == tl.TL_MIXED else "fp64"
        for w in range(args.warmup):
            tl.tl_solve_batch(lats, fs, us, check=False, precision=precision, rtol=1e-8)
            torch.cuda.synchronize()
            progress(f"{name} warmup {w + 1}/{args.warmup}")
        walls, infos = [], None
        t0 = time.perf_counter()
        for k in range(args.steps):
            ts = time.perf_counter()
            st, infos = tl.tl_solve_batch(lats, fs, us, check=False, precision=precision,
                                          rtol=1e-8)
            torch.cuda.synchronize()
            walls.append(1000.0 * (time.perf_counter() - ts))
            progress(f"{name} step {k + 1}/{args.steps}: {walls[-1]:.1f} ms, status {st}")
        wall = time.perf_counter() - t0
        bad = sum(1 for i in infos if i["status"] != 0)
        return {
            "value": dof * args.steps / wall,
            "ms_per_step": 1000.0 * wall / args.steps,
            "p50_ms": percentile(walls, 50), "p99_ms": percentile(walls, 99),
            "max_iters": max(i["iters"] for i in infos),
            "median_iters": statistics.median(i["iters"] for i in infos),
            "max_rel_res": max(max(i["rel_res_l1"], i["rel_res_l2"]) for i in infos),
            "failed": bad,
        }

    mixed = run_form(tl.TL_MIXED)
    fp64 = None if args.headline_only else run_form(tl.TL_FP64)
    out = common_fields(args, mixed["value"], mixed["ms_per_step"], "f32+f64", {
        "workload": (f"{len(lats)} independent triangle lattices, sides U{{32..512}} with aspect "
                     "U[0.5,2] (shape seed 1000, lattice b seed 2000+b), EA lognormal(0,0.5), left "
                     "edge clamped, loads N(0,1), set edge chosen per shape, mixed precision, "
                     "stop at rel. residual 1e-8, fused launches with hipGraph replay"),
        "dof": dof, "lattices": len(lats), "set_edges": edges, "form": "mixed"})
    out["batch_ms"] = {"p50": mixed["p50_ms"], "p99": mixed["p99_ms"]}
    out["iters"] = {"max": mixed["max_iters"], "median": mixed["median_iters"]}
    out["rel_res"] = mixed["max_rel_res"]
    out["failed"] = mixed["failed"]
    if fp64 is not None:
        out["fp64"] = fp64
        out["mixed_over_fp64"] = mixed["value"] / fp64["value"]
    out["roofline"] = None
    out["roofline_note"] = ("per-kernel event timing is not taken inside the graph-replayed "
                            "fused launches; the kernel trace of this workload gives it")
    out["cpu_baseline"] = None
    for l in lats:
        l.close()
    return out


def run_served(args):
    """Served workload: requests through tl_server, closed loop then Poisson."""
    import numpy as np
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
    mean_dof = dof_total / R
    progress(f"{R} requests prepared, mean {mean_dof:.3g} DOF, largest side {max(sides)}")
    budget = 200 * 10**9

    def serve(precision, arrivals, label):
        srv = tl.tl_server_create(budget, args.max_slots)
        pending, lat_ms, iters = {}, [], []
        failed = 0
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
                    del pending[t]
                    done += 1
                    failed += st != tl.TL_OK
                    lat_ms.append(info["ms"])
                    iters.append(info["iters"])
            if time.perf_counter() - last_note > 5.0:
                last_note = time.perf_counter()
                progress(f"{label}: {done}/{R} finished, {len(pending)} in flight")
            time.sleep(0.0005)
        wall = time.perf_counter() - t0
        srv.close()
        progress(f"{label}: {R} requests in {wall:.1f} s")
        return {"dof_solves_per_s": dof_total / wall, "wall_s": wall,
                "p50_ms": percentile(lat_ms, 50), "p99_ms": percentile(lat_ms, 99),
                "max_iters": max(iters), "failed": failed}

    for w in range(args.warmup):
        serve(tl.TL_MIXED, None, f"warmup {w + 1}")
    sat = serve(tl.TL_MIXED, None, "mixed closed loop")
    sat64 = None if args.headline_only else serve(tl.TL_FP64, None, "fp64 closed loop")
    loads = []
    for k, rho in enumerate((0.5, 0.8, 0.95)):
        rate = rho * sat["dof_solves_per_s"] / mean_dof
        arr = poisson_arrivals(R, rate, seed=3000 + k)
        r = serve(tl.TL_MIXED, arr, f"offered load {rho}")
        r.update({"offered_load": rho, "arrival_rate_per_s": rate})
        loads.append(r)
    out = common_fields(args, sat["dof_solves_per_s"], 1000.0 * sat["wall_s"], "f32+f64", {
        "workload": (f"served stream sample: {R} square triangle lattices, sides log-uniform in "
                     "[64,2048] (seed 3000, request k seed 3000+k), EA lognormal(0,0.5), left edge "
                     "clamped, loads N(0,1), stop at rel. residual 1e-8, HBM budget 200 GB, "
                     f"{args.max_slots} slots; Poisson arrivals at 0.5/0.8/0.95 of the "
                     "closed-loop rate"),
        "requests": R, "mean_dof": mean_dof, "form": "mixed"})
    out["steps"] = 1
    out["latency_ms"] = {"p50": loads[-1]["p50_ms"], "p99": loads[-1]["p99_ms"],
                         "offered_load": loads[-1]["offered_load"]}
    out["closed_loop"] = sat
    if sat64 is not None:
        out["fp64_closed_loop"] = sat64
        out["mixed_over_fp64"] = sat["dof_solves_per_s"] / sat64["dof_solves_per_s"]
    out["offered_loads"] = loads
    out["roofline"] = None
    out["roofline_note"] = "kernel figures come from the kernel trace of this workload"
    out["cpu_baseline"] = None
    for lat, _, _, _ in reqs:
        lat.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS) + ["c4", "c5"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--headline-only", action="store_true",
                    help="measure only the headline precision form")
    ap.add_argument("--lattices", type=int, default=256, help="c4: lattices per batch")
    ap.add_argument("--requests", type=int, default=120, help="c5: requests per offered load")
    ap.add_argument("--max-slots", type=int, default=64, help="c5: server slots")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the solver runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c4":
        out = run_batch(args)
    elif args.workload == "c5":
        out = run_served(args)
    else:
        out = run_single(args, WORKLOADS[args.workload])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
