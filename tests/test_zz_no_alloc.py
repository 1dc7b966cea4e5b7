"""tl_solve_noalloc, the entry point for callers that cannot allocate, against
tl_solve (the entry point it mirrors) and the oracle, through the C ABI.

Both entry points run the same kernels in the same order on the same inputs,
so their results must agree bit for bit; the oracle bar (1e-8 relative L2 at
a 1e-10 relative residual) is checked as well.  The calls run back to back on
one device, each lattice smaller than the one before, so every call finds the
previous call's contents in the shared array; a last call goes back to the
first lattice.
"""
import numpy as np
import pytest

from oracle.solve import solve, system_of
from workloads import make_instance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
tl = pytest.importorskip("paper_1208_4093_amd.tl")

CASES = [(200, 170, 32, "lognormal", 41), (90, 75, 16, "unit", 42), (37, 30, 16, "lognormal", 43)]


def _setup():
    out = []
    for nx, ny, E, ea, seed in CASES:
        inst = make_instance(nx, ny, seed=seed, ea=ea)
        lat = tl.tl_lattice_create(nx, ny, ea=inst.ea, fixed=inst.fixed, set_edge=E)
        out.append((inst, lat, torch.from_numpy(inst.f).cuda()))
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_tl_solve_on_calls_in_a_row(precision):
    cases = _setup()
    got = []
    for inst, lat, f in cases + cases[:1]:
        u = torch.full_like(f, float("nan"))          # the caller's u is written, not read
        info = tl.tl_solve_noalloc(lat, f, u, precision=precision, rtol=1e-10)
        torch.cuda.synchronize()
        assert info["status"] == tl.TL_OK
        got.append((u.clone(), info))
    for k, (inst, lat, f) in enumerate(cases + cases[:1]):
        ref = torch.zeros_like(f)
        info_ref = tl.tl_solve(lat, f, ref, precision=precision, rtol=1e-10)
        u, info = got[k]
        assert info["iters"] == info_ref["iters"]
        assert torch.equal(u, ref), (k, CASES[k % len(CASES)])
        us = solve(system_of(inst))
        err = np.linalg.norm(u.cpu().numpy().reshape(-1) - us) / np.linalg.norm(us)
        assert err <= 1e-8, (k, err)


def test_noalloc_rejects_what_does_not_fit_or_needs_allocation():
    inst = make_instance(2048, 2048, seed=44)
    lat = tl.tl_lattice_create(2048, 2048, ea=inst.ea, fixed=inst.fixed)
    f = torch.from_numpy(inst.f).cuda()
    u = torch.zeros_like(f)
    assert lat.solve_bytes[1] > tl.NOALLOC_SCRATCH_BYTES
    info = tl.tl_solve_noalloc(lat, f, u, check=False, precision=1)
    assert info["status"] == tl.TL_E_BUDGET
    small, slat, sf = _setup()[2]
    su = torch.zeros_like(sf)
    assert tl.tl_solve_noalloc(slat, sf, su, check=False, profile=1)["status"] == tl.TL_E_INVAL
    hist = torch.zeros(64, dtype=torch.float64, device="cuda")
    tr = tl.make_trace(residual_history=hist)
    assert tl.tl_solve_noalloc(slat, sf, su, check=False, trace=tr)["status"] == tl.TL_E_INVAL
    # and the entry point still works after the rejections
    info = tl.tl_solve_noalloc(slat, sf, su, precision=1, rtol=1e-9)
    assert info["status"] == tl.TL_OK
