"""Record how many block-Jacobi PCG iterations the oracle needs to reach a
relative residual on a workload instance (test infrastructure).

The benchmark's CPU baseline times the oracle's PCG per iteration on the
benchmark host for a bounded sample and multiplies by this count, because
a complete oracle solve of the 1024 x 1024 lattice takes about an hour on
one core.  Usage:
    python -m oracle.record_pcg_iterations 1024 1e-8 tests/golden/oracle_pcg_1024.json
"""
import json
import sys
import time

from workloads import make_instance

from .solve import rel_residuals, solve_pcg, system_of


def main():
    n, rtol, out = int(sys.argv[1]), float(sys.argv[2]), sys.argv[3]
    inst = make_instance(n, n, seed=0)
    t0 = time.perf_counter()
    S = system_of(inst)
    t_asm = time.perf_counter() - t0
    hist = []
    t1 = time.perf_counter()
    u = solve_pcg(S, rtol=rtol, history=hist)
    t_pcg = time.perf_counter() - t1
    R1, R2 = rel_residuals(S, u)
    first = next(it for it, rel in hist if rel <= rtol)
    rec = {"lattice": [n, n], "seed": 0, "ea": "unit", "rtol": rtol,
           "iterations_to_rtol": first, "iterations_run": len(hist),
           "final_R1": R1, "final_R2": R2, "assembly_s": t_asm, "pcg_s": t_pcg,
           "note": "2-norm relative residual of the PCG recurrence reaches rtol at iterations_to_rtol; "
                   "the explicitly recomputed residual is checked at the end"}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
