"""The autotuner through the C ABI: tl_tune records a measured, converged
choice for the lattice's shape and precision; a lattice created afterwards
with set edge 0 takes the tuned set edge; solves that leave overlap and
sweeps at 0 take the tuned ones (bit for bit the solve with those options
given explicitly); batched results stay bit for bit those of tl_solve alone;
the table survives a save, clear and load."""
import numpy as np
import pytest

from oracle.solve import solve, system_of
from workloads import make_instance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
tl = pytest.importorskip("paper_1208_4093_amd.tl")


@pytest.fixture(autouse=True)
def empty_table():
    # the table is process-wide: start and leave it empty so that no other
    # test's lattices pick up these choices
    tl.tl_tune_clear()
    yield
    tl.tl_tune_clear()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("precision", [tl.TL_MIXED, tl.TL_FP64])
def test_tuned_choice_is_recorded_and_honoured(precision, tmp_path):
    nx, ny = 150, 120
    inst = make_instance(nx, ny, seed=21, ea="lognormal")
    f = _dev(inst.f)
    e = tl.tl_tune(nx, ny, f, ea=inst.ea, fixed=inst.fixed, precision=precision, rtol=1e-8)
    assert e["status"] == tl.TL_OK
    assert e["set_edge"] in (16, 32, 64) and e["overlap"] in (1, 2, 4) and e["inner_iters"] >= 4
    assert (e["nx"], e["ny"]) == (nx, ny) and e["ms"] > 0.0
    got = tl.tl_tune_lookup(nx, ny, precision)
    assert got is not None and got["set_edge"] == e["set_edge"]
    assert got["overlap"] == e["overlap"] and got["inner_iters"] == e["inner_iters"]

    # a lattice of the same shape key, created with set edge 0
    inst2 = make_instance(nx - 3, ny + 2, seed=22, ea="lognormal")
    lat = tl.tl_lattice_create(inst2.nx, inst2.ny, ea=inst2.ea, fixed=inst2.fixed)
    assert lat.set_edge == e["set_edge"]
    f2 = _dev(inst2.f)
    u_def = torch.zeros_like(f2)
    i_def = tl.tl_solve(lat, f2, u_def, precision=precision, rtol=1e-10)
    u_exp = torch.zeros_like(f2)
    i_exp = tl.tl_solve(lat, f2, u_exp, precision=precision, rtol=1e-10, overlap=e["overlap"],
                        inner_iters=e["inner_iters"])
    assert torch.equal(u_def, u_exp) and i_def["iters"] == i_exp["iters"]
    ref = solve(system_of(inst2))
    err = np.linalg.norm(u_def.cpu().numpy().reshape(-1) - ref) / np.linalg.norm(ref)
    assert err <= 1e-8, err

    # batched with an untuned shape: each result is its alone result
    inst3 = make_instance(60, 45, seed=23, ea="lognormal")
    lat3 = tl.tl_lattice_create(60, 45, ea=inst3.ea, fixed=inst3.fixed)
    f3 = _dev(inst3.f)
    u3 = torch.zeros_like(f3)
    tl.tl_solve(lat3, f3, u3, precision=precision, rtol=1e-10)
    us = [torch.zeros_like(f2), torch.zeros_like(f3)]
    st, infos = tl.tl_solve_batch([lat, lat3], [f2, f3], us, precision=precision, rtol=1e-10)
    assert st == tl.TL_OK
    assert torch.equal(us[0], u_def) and torch.equal(us[1], u3)

    # save, clear, load
    path = tmp_path / "table.txt"
    tl.tl_tune_save(str(path))
    tl.tl_tune_clear()
    assert tl.tl_tune_lookup(nx, ny, precision) is None
    tl.tl_tune_load(str(path))
    assert tl.tl_tune_lookup(nx, ny, precision) == got


def test_choice_for_another_set_edge_is_not_applied():
    nx, ny = 200, 180
    inst = make_instance(nx, ny, seed=24, ea="lognormal")
    f = _dev(inst.f)
    e = tl.tl_tune(nx, ny, f, ea=inst.ea, fixed=inst.fixed, precision=tl.TL_MIXED, rtol=1e-8)
    other = 16 if e["set_edge"] != 16 else 32
    lat = tl.tl_lattice_create(nx, ny, ea=inst.ea, fixed=inst.fixed, set_edge=other)
    u_def = torch.zeros_like(f)
    tl.tl_solve(lat, f, u_def, precision=tl.TL_MIXED, rtol=1e-10)
    tl.tl_tune_clear()
    u_builtin = torch.zeros_like(f)
    tl.tl_solve(lat, f, u_builtin, precision=tl.TL_MIXED, rtol=1e-10)
    assert torch.equal(u_def, u_builtin)
