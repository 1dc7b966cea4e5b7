"""Batched solves and the continuous-batching server, through the C ABI:
every lattice's result is the same alone and in a batch or a served mix
(bit for bit: each lattice's kernels, set edge and reduction orders depend
only on that lattice), and matches the oracle."""
import time

import numpy as np
import pytest

from oracle.solve import rel_residuals, solve, system_of
from workloads import make_instance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
tl = pytest.importorskip("paper_1208_4093_amd.tl")

SHAPES = [(40, 33, 16, "lognormal", 1), (64, 64, 16, "unit", 2), (130, 70, 32, "lognormal", 3),
          (33, 95, 16, "lognormal", 4), (90, 90, 64, "unit", 5)]


def _setup():
    lats, fs, insts = [], [], []
    for nx, ny, E, ea, seed in SHAPES:
        inst = make_instance(nx, ny, seed=seed, ea=ea)
        insts.append(inst)
        lats.append(tl.tl_lattice_create(nx, ny, ea=inst.ea, fixed=inst.fixed, set_edge=E))
        fs.append(torch.from_numpy(inst.f).cuda())
    return insts, lats, fs


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_alone_and_oracle(precision):
    insts, lats, fs = _setup()
    alone = []
    for lat, f in zip(lats, fs):
        u = torch.zeros_like(f)
        tl.tl_solve(lat, f, u, precision=precision, rtol=1e-10)
        alone.append(u.cpu().numpy())
    us = [torch.zeros_like(f) for f in fs]
    st, infos = tl.tl_solve_batch(lats, fs, us, precision=precision, rtol=1e-10)
    assert st == tl.TL_OK
    for inst, u, ua, info in zip(insts, us, alone, infos):
        ub = u.cpu().numpy()
        assert np.array_equal(ub, ua)
        S = system_of(inst)
        ref = solve(S)
        assert np.linalg.norm(ub.reshape(-1) - ref) <= 1e-8 * np.linalg.norm(ref)
        assert max(info["rel_res_l1"], info["rel_res_l2"]) <= 1e-10


@pytest.mark.parametrize("no_lds", [0, 1])
def test_batch_equals_alone_upper_level_general_path(monkeypatch, no_lds):
    """Several upper-level rows per thread with the blocks (and, with no_lds,
    the PCG vectors) in global memory: the single-lattice kernel reads a row's
    neighbour blocks branch-free, the batched one skips absent neighbours;
    the two must still agree bit for bit."""
    monkeypatch.setenv("TL_COARSE_SETS_PER_WG", "64")
    monkeypatch.setenv("TL_COARSE_NO_LDS", str(no_lds))
    shapes = [(200, 180, 16, "lognormal", 21), (150, 160, 16, "unit", 22)]
    lats, fs, insts = [], [], []
    for nx, ny, E, ea, seed in shapes:
        inst = make_instance(nx, ny, seed=seed, ea=ea)
        insts.append(inst)
        lats.append(tl.tl_lattice_create(nx, ny, ea=inst.ea, fixed=inst.fixed, set_edge=E))
        fs.append(torch.from_numpy(inst.f).cuda())
    alone = []
    for lat, f in zip(lats, fs):
        u = torch.zeros_like(f)
        info = tl.tl_solve(lat, f, u, precision=1, rtol=1e-10)
        assert info["status"] == tl.TL_OK
        alone.append(u.cpu().numpy())
    us = [torch.zeros_like(f) for f in fs]
    st, infos = tl.tl_solve_batch(lats, fs, us, precision=1, rtol=1e-10)
    assert st == tl.TL_OK
    for inst, u, ua in zip(insts, us, alone):
        ub = u.cpu().numpy()
        assert np.array_equal(ub, ua)
        ref = solve(system_of(inst))
        assert np.linalg.norm(ub.reshape(-1) - ref) <= 1e-8 * np.linalg.norm(ref)


def test_batch_with_repeated_lattice():
    insts, lats, fs = _setup()
    f2 = torch.from_numpy(make_instance(40, 33, seed=99, ea="lognormal").f).cuda()
    L = [lats[0], lats[0], lats[1]]
    F = [fs[0], f2, fs[1]]
    us = [torch.zeros_like(f) for f in F]
    st, infos = tl.tl_solve_batch(L, F, us, precision=1, rtol=1e-9)
    assert st == tl.TL_OK
    for lat, f, u in zip(L, F, us):
        ua = torch.zeros_like(f)
        tl.tl_solve(lat, f, ua, precision=1, rtol=1e-9)
        assert torch.equal(u, ua)


def test_server_results_equal_alone_under_overlap():
    insts, lats, fs = _setup()
    alone = []
    for lat, f in zip(lats, fs):
        u = torch.zeros_like(f)
        tl.tl_solve(lat, f, u, precision=1, rtol=1e-9)
        alone.append(u.cpu().numpy())
    srv = tl.tl_server_create(1 << 32, 3)
    us = [torch.zeros_like(f) for f in fs]
    tickets = []
    for k, (lat, f, u) in enumerate(zip(lats, fs, us)):
        tickets.append(tl.tl_submit(srv, lat, f, u, precision=1, rtol=1e-9))
        time.sleep(0.002 * k)          # staggered arrivals join running rounds
    done = {}
    t0 = time.time()
    while len(done) < len(tickets) and time.time() - t0 < 60:
        for tk in tickets:
            if tk in done:
                continue
            st, info = tl.tl_poll(srv, tk)
            if st != tl.TL_PENDING:
                done[tk] = (st, info)
        time.sleep(0.001)
    srv.close()
    assert len(done) == len(tickets)
    for tk, u, ua in zip(tickets, us, alone):
        st, info = done[tk]
        assert st == tl.TL_OK and info["ms"] > 0.0
        assert np.array_equal(u.cpu().numpy(), ua)


def test_server_budget_limits():
    insts, lats, fs = _setup()
    srv = tl.tl_server_create(1 << 16, 2)          # 64 KiB: the 130 x 70 lattice never fits
    u = torch.zeros_like(fs[2])
    with pytest.raises(tl.TLError) as ei:
        tl.tl_submit(srv, lats[2], fs[2], u, precision=1, rtol=1e-9)
    assert ei.value.status == tl.TL_E_BUDGET
    srv.close()


# Four 1500 x 1500 lattices with 32 x 32 sets (47 x 47 = 2209 sets each) take
# ceil(2209 / 16) = 139 upper-level workgroups apiece, 556 together: more
# than the device can hold co-resident, so a batch of them runs as groups
# and a server admits them a few at a time.
BIG = 1500


@pytest.fixture(scope="module")
def big_mix():
    insts, lats, fs = [], [], []
    for k in range(4):
        inst = make_instance(BIG, BIG, seed=500 + k, ea="lognormal")
        insts.append(inst)
        lats.append(tl.tl_lattice_create(BIG, BIG, ea=inst.ea, fixed=inst.fixed, set_edge=32))
        fs.append(torch.from_numpy(inst.f).cuda())
    for nx, ny, E, ea, seed in SHAPES[:3]:
        inst = make_instance(nx, ny, seed=seed, ea=ea)
        insts.append(inst)
        lats.append(tl.tl_lattice_create(nx, ny, ea=inst.ea, fixed=inst.fixed, set_edge=E))
        fs.append(torch.from_numpy(inst.f).cuda())
    alone = []
    for lat, f in zip(lats, fs):
        u = torch.zeros_like(f)
        tl.tl_solve(lat, f, u, precision=1, rtol=1e-8)
        alone.append(u)
    return insts, lats, fs, alone


def test_batch_beyond_coresident_capacity(big_mix):
    insts, lats, fs, alone = big_mix
    us = [torch.zeros_like(f) for f in fs]
    st, infos = tl.tl_solve_batch(lats, fs, us, precision=1, rtol=1e-8)
    assert st == tl.TL_OK
    for u, ua, info in zip(us, alone, infos):
        assert info["status"] == tl.TL_OK
        assert max(info["rel_res_l1"], info["rel_res_l2"]) <= 1e-8
        assert torch.equal(u, ua)


def test_server_admits_by_coresidency(big_mix):
    insts, lats, fs, alone = big_mix
    srv = tl.tl_server_create(1 << 36, 8)
    us = [torch.zeros_like(f) for f in fs]
    tickets = [tl.tl_submit(srv, lat, f, u, precision=1, rtol=1e-8)
               for lat, f, u in zip(lats, fs, us)]
    done = {}
    t0 = time.time()
    while len(done) < len(tickets) and time.time() - t0 < 100:
        for tk in tickets:
            if tk not in done:
                st, info = tl.tl_poll(srv, tk)
                if st != tl.TL_PENDING:
                    done[tk] = (st, info)
        time.sleep(0.001)
    srv.close()
    assert len(done) == len(tickets)
    for tk, u, ua in zip(tickets, us, alone):
        st, info = done[tk]
        assert st == tl.TL_OK
        assert torch.equal(u, ua)


# Many lattices of 200 x 200 nodes with 16 x 16 sets: 169 sets, 11 upper-level
# workgroups each, 616 in all, more than the device holds at once at two
# workgroups per CU (512): the fused upper-level launch is over-subscribed
# and its workgroups take their places in start order.
MANY = 56


@pytest.fixture(scope="module")
def many_small():
    lats, fs, alone = [], [], []
    for k in range(MANY):
        inst = make_instance(200, 200, seed=700 + k, ea="lognormal")
        lats.append(tl.tl_lattice_create(200, 200, ea=inst.ea, fixed=inst.fixed, set_edge=16))
        fs.append(torch.from_numpy(inst.f).cuda())
    for lat, f in zip(lats, fs):
        u = torch.zeros_like(f)
        tl.tl_solve(lat, f, u, precision=1, rtol=1e-8)
        alone.append(u)
    return lats, fs, alone


def test_oversubscribed_upper_level_batch_equals_alone(many_small):
    lats, fs, alone = many_small
    assert lats[0].sets == 169
    us = [torch.zeros_like(f) for f in fs]
    st, infos = tl.tl_solve_batch(lats, fs, us, precision=1, rtol=1e-8)
    assert st == tl.TL_OK
    for u, ua, info in zip(us, alone, infos):
        assert info["status"] == tl.TL_OK
        assert torch.equal(u, ua)


def test_oversubscribed_server_equals_alone(many_small):
    lats, fs, alone = many_small
    srv = tl.tl_server_create(1 << 36, 64)
    us = [torch.zeros_like(f) for f in fs]
    tickets = [tl.tl_submit(srv, lat, f, u, precision=1, rtol=1e-8)
               for lat, f, u in zip(lats, fs, us)]
    done = {}
    t0 = time.time()
    while len(done) < len(tickets) and time.time() - t0 < 100:
        for tk in tickets:
            if tk not in done:
                st, info = tl.tl_poll(srv, tk)
                if st != tl.TL_PENDING:
                    done[tk] = (st, info)
        time.sleep(0.001)
    srv.close()
    assert len(done) == len(tickets)
    for tk, u, ua in zip(tickets, us, alone):
        assert done[tk][0] == tl.TL_OK
        assert torch.equal(u, ua)
