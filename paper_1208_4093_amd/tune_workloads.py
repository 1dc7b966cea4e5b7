"""Fill the autotuning table for the shapes of a workload.

    python -m paper_1208_4093_amd.tune_workloads --workload batched --out TABLE

For every shape key of the workload (half-octave buckets of nx and ny) the
first lattice of the workload with that key is tuned with tl_tune in both
precisions (to a relative residual of 1e-8) on its own seeded load, unless
the table already holds the entry.  The table is read from and written to
the file named by --out (through TL_TUNE_CACHE).
"""
import argparse
import math
import os
import sys
import time


def shape_key(nx, ny):
    return round(2 * math.log2(nx)), round(2 * math.log2(ny))


def workload_lattices(name, count):
    """(nx, ny, seed) of the workload's lattices, in workload order."""
    from workloads import batch_shapes, served_sides
    if name == "batched":
        return [(nx, ny, 2000 + b) for b, (nx, ny) in enumerate(batch_shapes(count))]
    if name == "served":
        return [(s, s, 3000 + k) for k, s in enumerate(served_sides(count))]
    raise ValueError(name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["batched", "served"], default="batched")
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    os.environ["TL_TUNE_CACHE"] = os.path.abspath(args.out)
    import torch
    from workloads import make_instance
    from paper_1208_4093_amd import tl
    first = {}
    for nx, ny, seed in workload_lattices(args.workload, args.count):
        first.setdefault(shape_key(nx, ny), (nx, ny, seed))
    t0 = time.time()
    for k, (key, (nx, ny, seed)) in enumerate(sorted(first.items())):
        inst = make_instance(nx, ny, seed=seed, ea="lognormal")
        f = torch.from_numpy(inst.f).cuda()
        for precision in (tl.TL_MIXED, tl.TL_FP64):
            if tl.tl_tune_lookup(nx, ny, precision) is not None:
                continue
            e = tl.tl_tune(nx, ny, f, ea=inst.ea, fixed=inst.fixed, precision=precision, rtol=1e-8)
            print(f"[tune {time.time() - t0:6.1f}s] key {key} {nx}x{ny} "
                  f"{'mixed' if precision == tl.TL_MIXED else 'fp64'}: E {e['set_edge']} "
                  f"overlap {e['overlap']} sweeps {e['inner_iters']} {e['ms']:.2f} ms "
                  f"({k + 1}/{len(first)})", file=sys.stderr, flush=True)
    print(f"{len(first)} shape keys in {args.out}", flush=True)


if __name__ == "__main__":
    main()
