"""GPU parity of the paths the first tests leave out, through the C ABI:

* the served results against the oracle (not only against tl_solve alone);
* a request whose load is still being produced on the caller's stream when
  it is submitted;
* tl_solve on a second stream while the server's worker runs (the
  process-wide admission of persistent upper-level grids);
* one outer iteration of the mixed form: the float32 relaxation increment of
  every set against the oracle's exact local solve (Eq. 12-13) at a float32
  tolerance, and the upper-level blocks and force it yields against the
  oracle's assembly (Eq. 6-7) at float64 tolerance;
* batched lattices of the batched workload's shapes at the library's own set
  edge, against the oracle;
* the upper level without its coarse space (one-level block-Jacobi PCG);
* profiled batches (per-launch timing) give the unprofiled results;
* a device-side descriptor with a free node no rod holds is rejected.

Float32 tolerance of the relaxation increment: the inner PCG runs 2 R^2
sweeps (R = region edge), far past convergence, so the float32 iterate sits
at its attainable accuracy, about kappa x 2^-24 with kappa the condition
number of the Jacobi-scaled local matrix (the right-hand side's rounding to
float32 alone costs that much).  The test computes kappa for every region of
its lattice (from 5e2 to 6.4e3 for these cases) and allows 5 kappa 2^-24,
relative, per lattice, in the 2-norm.
"""
import threading
import time

import numpy as np
import pytest

import oracle.method as om
from oracle.solve import rel_residuals, solve, solve_banded, system_of
from workloads import batch_shapes, make_instance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
tl = pytest.importorskip("paper_1208_4093_amd.tl")

F32_EPS = 2.0 ** -24


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def make_lattice(inst, E=0):
    return tl.tl_lattice_create(inst.nx, inst.ny, ea=inst.ea, fixed=inst.fixed,
                                u_fixed=inst.u_fixed, set_edge=E)


def oracle_u(inst):
    S = system_of(inst)
    return solve(S) if int(S.free.sum()) < 200_000 else solve_banded(S)


def wait_all(srv, tickets, limit_s=120):
    done = {}
    t0 = time.time()
    while len(done) < len(tickets) and time.time() - t0 < limit_s:
        for tk in tickets:
            if tk not in done:
                st, info = tl.tl_poll(srv, tk)
                if st != tl.TL_PENDING:
                    done[tk] = (st, info)
        time.sleep(0.001)
    return done


SERVED = [(40, 33, 16, "lognormal", 61), (64, 64, 16, "unit", 62), (130, 70, 32, "lognormal", 63),
          (33, 95, 16, "lognormal", 64), (90, 90, 64, "unit", 65), (150, 121, 0, "lognormal", 66)]


def test_served_results_match_oracle():
    """Both forms served together (one fused batch per form), staggered
    arrivals, each result against the oracle's exact solution."""
    insts = [make_instance(nx, ny, seed=s, ea=ea) for nx, ny, E, ea, s in SERVED]
    lats = [make_lattice(i, E) for i, (_, _, E, _, _) in zip(insts, SERVED)]
    fs = [dev(i.f) for i in insts]
    srv = tl.tl_server_create(1 << 32, 4)
    us, tickets = [], []
    for k, (lat, f) in enumerate(zip(lats, fs)):
        for precision in (0, 1):
            u = torch.zeros_like(f)
            us.append((k, u))
            tickets.append(tl.tl_submit(srv, lat, f, u, precision=precision, rtol=1e-10))
        time.sleep(0.003)
    done = wait_all(srv, tickets)
    srv.close()
    assert len(done) == len(tickets)
    refs = [oracle_u(i) for i in insts]
    for tk, (k, u) in zip(tickets, us):
        st, info = done[tk]
        assert st == tl.TL_OK, (SERVED[k], info)
        assert max(info["rel_res_l1"], info["rel_res_l2"]) <= 1e-10
        err = np.linalg.norm(u.cpu().numpy().reshape(-1) - refs[k]) / np.linalg.norm(refs[k])
        assert err <= 1e-8, (SERVED[k], err)


def test_submit_waits_for_the_load_on_the_callers_stream():
    """The load is written by a kernel queued behind a long computation on
    torch's stream, and submitted before that kernel has run."""
    inst = make_instance(96, 80, seed=67, ea="lognormal")
    lat = make_lattice(inst, 32)
    f_src = dev(inst.f)
    u_ref = torch.zeros_like(f_src)
    tl.tl_solve(lat, f_src, u_ref, precision=1, rtol=1e-9)
    torch.cuda.synchronize()
    srv = tl.tl_server_create(1 << 32, 2)
    f = torch.zeros_like(f_src)
    x = torch.randn(4096, 4096, device="cuda")
    for _ in range(30):                       # tens of milliseconds of queued work
        x = torch.tanh(x @ x)
    f.copy_(f_src + 0.0 * x[0, 0])            # the load, produced after that work
    u = torch.zeros_like(f)
    tk = tl.tl_submit(srv, lat, f, u, precision=1, rtol=1e-9)
    done = wait_all(srv, [tk])
    srv.close()
    st, info = done[tk]
    assert st == tl.TL_OK
    assert torch.equal(u, u_ref)


def test_solve_on_a_second_stream_while_the_server_runs():
    """Persistent upper-level grids of a served batch and of a tl_solve on
    another stream: both finish, with the results they give alone."""
    insts = [make_instance(1500, 1500, seed=70 + k, ea="lognormal") for k in range(3)]
    lats = [make_lattice(i, 32) for i in insts]
    fs = [dev(i.f) for i in insts]
    alone = []
    for lat, f in zip(lats, fs):
        u = torch.zeros_like(f)
        tl.tl_solve(lat, f, u, precision=1, rtol=1e-8)
        alone.append(u)
    torch.cuda.synchronize()
    srv = tl.tl_server_create(1 << 36, 4)
    us = [torch.zeros_like(f) for f in fs[:2]]
    tickets = [tl.tl_submit(srv, lat, f, u, precision=1, rtol=1e-8)
               for lat, f, u in zip(lats[:2], fs[:2], us)]
    side = torch.cuda.Stream()
    u2 = torch.zeros_like(fs[2])
    with torch.cuda.stream(side):
        info = tl.tl_solve(lats[2], fs[2], u2, stream=side, check=False, precision=1, rtol=1e-8)
    side.synchronize()
    done = wait_all(srv, tickets)
    srv.close()
    assert info["status"] == tl.TL_OK
    assert torch.equal(u2, alone[2])
    assert len(done) == 2
    for tk, u, ua in zip(tickets, us, alone[:2]):
        assert done[tk][0] == tl.TL_OK
        assert torch.equal(u, ua)


def test_concurrent_solves_from_two_threads():
    """Two host threads, two lattices, two streams, small enough that their
    upper-level grids run side by side."""
    insts = [make_instance(300, 260, seed=75 + k, ea="lognormal") for k in range(2)]
    lats = [make_lattice(i, 32) for i in insts]
    fs = [dev(i.f) for i in insts]
    alone = []
    for lat, f in zip(lats, fs):
        u = torch.zeros_like(f)
        tl.tl_solve(lat, f, u, precision=0, rtol=1e-9)
        alone.append(u)
    torch.cuda.synchronize()
    outs, infos = [torch.zeros_like(f) for f in fs], [None, None]

    def run(k):
        s = torch.cuda.Stream()
        for _ in range(3):
            outs[k].zero_()
            s.wait_stream(torch.cuda.current_stream())
            infos[k] = tl.tl_solve(lats[k], fs[k], outs[k], stream=s, check=False, precision=0,
                                   rtol=1e-9)
        s.synchronize()
    th = [threading.Thread(target=run, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join(120)
    for k in range(2):
        assert infos[k]["status"] == tl.TL_OK
        assert torch.equal(outs[k], alone[k])


def _kappa_max(S, sets, ov):
    """Largest condition number, over the relaxation regions, of the
    Jacobi-scaled region matrix k^Inner."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    kmax = 1.0
    for I in range(sets.M):
        nodes = om.relaxation_region(sets, I, ov)
        dofs = np.sort(np.concatenate([2 * nodes, 2 * nodes + 1]))
        idx = dofs[S.free[dofs]]
        if idx.size < 4:
            continue
        K = S.K[idx][:, idx].tocsc()
        Dm = sp.diags(1.0 / np.sqrt(K.diagonal()))
        A = (Dm @ K @ Dm).tocsc()
        lmax = spla.eigsh(A, k=1, which="LA", return_eigenvectors=False)[0]
        lmin = spla.eigsh(A, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
        kmax = max(kmax, lmax / lmin)
    return kmax


def _scale_of_set(S, sets, r, I, ov):
    """2^-e with e = ilogb of max |r| over the free DOFs of set I's region."""
    nodes = om.relaxation_region(sets, I, ov)
    dofs = np.concatenate([2 * nodes, 2 * nodes + 1])
    dofs = dofs[S.free[dofs]]
    rm = np.abs(r[dofs]).max() if dofs.size else 0.0
    if rm == 0.0:
        return 1.0
    _, e = np.frexp(rm)            # rm = m 2^e, 0.5 <= m < 1: ilogb(rm) = e - 1
    return float(np.ldexp(1.0, -(int(e) - 1)))


@pytest.mark.parametrize("nx,ny,E,ea,seed,ov", [
    (64, 48, 16, "lognormal", 7, 0), (45, 37, 16, "unit", 8, 2), (70, 66, 32, "lognormal", 9, 2),
    (100, 72, 32, "lognormal", 10, 1), (70, 130, 64, "lognormal", 3, 2)])
def test_one_iteration_mixed_matches_method_model(nx, ny, E, ea, seed, ov):
    inst = make_instance(nx, ny, seed=seed, ea=ea)
    S = system_of(inst)
    sets = om.make_sets(nx, ny, E)
    local = om.LocalSolver(S, sets, overlap=ov)
    r0 = om.residual(S, S.u_c.copy())
    d_exact = local.relax(r0)
    M, Q = sets.M, om.Q
    tr_t = dict(delta=torch.zeros((ny, nx, 2), dtype=torch.float64, device="cuda"),
                kdiag=torch.zeros((M, Q, Q), dtype=torch.float64, device="cuda"),
                koff=torch.zeros((M, 6, Q, Q), dtype=torch.float64, device="cuda"),
                force=torch.zeros((M, Q), dtype=torch.float64, device="cuda"),
                coef=torch.zeros((M, Q), dtype=torch.float64, device="cuda"),
                residual_history=torch.zeros(4, dtype=torch.float64, device="cuda"))
    lat = make_lattice(inst, E)
    f = dev(inst.f)
    u = torch.zeros_like(f)
    R = E + 2 * ov
    info = tl.tl_solve(lat, f, u, check=False, precision=1, rtol=1e-300, max_iters=1,
                       inner_iters=2 * R * R, coarse_iters=20000, coarse_rtol=1e-15,
                       trace=tl.make_trace(**tr_t), overlap=ov if ov > 0 else -1)
    torch.cuda.synchronize()
    assert info["status"] == tl.TL_E_NOCONV and info["iters"] == 1
    # the stored increment is the float32 solve of the set's scaled residual
    d_g = tr_t["delta"].cpu().numpy().reshape(-1)
    want = np.zeros_like(d_exact)
    node_set = np.repeat(sets.of_node, 2)
    for I in range(M):
        own = node_set == I
        want[own] = _scale_of_set(S, sets, r0, I, ov) * d_exact[own]
    err = np.linalg.norm(d_g - want) / np.linalg.norm(want)
    kappa = _kappa_max(S, sets, ov)
    assert err <= 5.0 * kappa * F32_EPS, (err, kappa)
    # blocks and force of the upper level assembled (float64) from that increment
    U = om.mode_matrix(S, sets, d_g)
    Kc, P = om.upper_level(S, U, S.u_c.copy())
    kd, ko = tr_t["kdiag"].cpu().numpy(), tr_t["koff"].cpu().numpy()
    Pg = tr_t["force"].cpu().numpy().reshape(-1)
    assert np.linalg.norm(Pg - P) <= 1e-9 * np.linalg.norm(P)
    dirs = [(1, 0), (0, 1), (-1, 1), (-1, 0), (0, -1), (1, -1)]
    for s in range(M):
        I, J = s % sets.mx, s // sets.mx
        diag = Kc[Q * s:Q * s + Q, Q * s:Q * s + Q]
        nrm = np.abs(diag).max()
        assert np.abs(kd[s] - diag).max() <= 1e-9 * nrm, s
        for d, (di, dj) in enumerate(dirs):
            if 0 <= I + di < sets.mx and 0 <= J + dj < sets.my:
                s2 = (J + dj) * sets.mx + I + di
                assert np.abs(ko[s][d] - Kc[Q * s:Q * s + Q, Q * s2:Q * s2 + Q]).max() <= 1e-9 * nrm
    # the coefficients solve that system, and the update applies them (Eq. 3, 8)
    a_g = tr_t["coef"].cpu().numpy().reshape(-1)
    assert np.linalg.norm(Kc @ a_g - P) <= 1e-8 * np.linalg.norm(P)
    u_exp = S.u_c + U @ a_g
    assert np.linalg.norm(u.cpu().numpy().reshape(-1) - u_exp) <= 1e-9 * np.linalg.norm(u_exp)


def _subset_indices():
    shapes = batch_shapes(256)
    area = np.array([nx * ny for nx, ny in shapes])
    aspect = np.array([max(nx / ny, ny / nx) for nx, ny in shapes])
    pick = [int(area.argmax()), int(aspect.argmax()), int(area.argmin())]
    for k in np.linspace(0, 255, 8).astype(int):
        if len(pick) < 8 and int(k) not in pick:
            pick.append(int(k))
    return shapes, pick


@pytest.mark.slow
@pytest.mark.parametrize("precision", [0, 1])
def test_batched_workload_subset_at_library_set_edge(precision):
    """Eight lattices of the 256-lattice batched workload (its largest, its
    most elongated, its smallest and five more), seeds 2000 + b, set edge
    chosen by the library, solved in one batch against the oracle."""
    shapes, pick = _subset_indices()
    insts = [make_instance(*shapes[b], seed=2000 + b, ea="lognormal") for b in pick]
    lats = [make_lattice(i, 0) for i in insts]
    fs = [dev(i.f) for i in insts]
    us = [torch.zeros_like(f) for f in fs]
    st, infos = tl.tl_solve_batch(lats, fs, us, check=False, precision=precision, rtol=1e-10)
    assert st == tl.TL_OK, [i["status"] for i in infos]
    for b, inst, u, info in zip(pick, insts, us, infos):
        ref = oracle_u(inst)
        err = np.linalg.norm(u.cpu().numpy().reshape(-1) - ref) / np.linalg.norm(ref)
        assert err <= 1e-8, (b, shapes[b], err, info)


@pytest.mark.parametrize("precision", [0, 1])
def test_upper_level_without_coarse_space_matches_oracle(monkeypatch, precision):
    monkeypatch.setenv("TL_COARSE_2LEVEL", "0")
    inst = make_instance(150, 140, seed=80, ea="lognormal")
    lat = make_lattice(inst, 16)
    f = dev(inst.f)
    u = torch.zeros_like(f)
    info = tl.tl_solve(lat, f, u, precision=precision, rtol=1e-10)
    assert info["status"] == tl.TL_OK
    ref = oracle_u(inst)
    assert np.linalg.norm(u.cpu().numpy().reshape(-1) - ref) <= 1e-8 * np.linalg.norm(ref)


def test_profiled_batch_gives_unprofiled_results():
    shapes = [(90, 70, 16), (200, 150, 32), (120, 230, 32)]
    insts = [make_instance(nx, ny, seed=90 + k, ea="lognormal") for k, (nx, ny, _) in enumerate(shapes)]
    lats = [make_lattice(i, E) for i, (_, _, E) in zip(insts, shapes)]
    fs = [dev(i.f) for i in insts]
    u0 = [torch.zeros_like(f) for f in fs]
    u1 = [torch.zeros_like(f) for f in fs]
    st0, inf0 = tl.tl_solve_batch(lats, fs, u0, precision=1, rtol=1e-9)
    st1, inf1 = tl.tl_solve_batch(lats, fs, u1, precision=1, rtol=1e-9, profile=1)
    assert st0 == st1 == tl.TL_OK
    for a, b, i0, i1, (_, _, E) in zip(u0, u1, inf0, inf1, shapes):
        assert torch.equal(a, b)
        assert i0["iters"] == i1["iters"]
        assert i1["tile_ms"] > 0.0 and i1["coarse_ms"] > 0.0
        last = max(i["iters"] for i, (_, _, e) in zip(inf1, shapes) if e == E)
        assert i1["tile_launches"] == last + 1
        assert 0.0 < i0["ms"] and 0.0 < i1["ms"]


def test_device_descriptor_with_unheld_node_is_rejected():
    inst = make_instance(12, 10, seed=95)
    ea = inst.ea.copy()
    # every rod of node (i, j) = (5, 4) ([d, j, i] layout)
    ea[0, 4, 5] = ea[0, 4, 4] = ea[1, 4, 5] = ea[1, 3, 5] = ea[2, 4, 5] = ea[2, 3, 6] = 0.0
    with pytest.raises(tl.TLError) as ei:
        tl.tl_lattice_create(12, 10, ea=dev(ea), fixed=dev(inst.fixed))
    assert ei.value.status == tl.TL_E_INVAL
    lat = tl.tl_lattice_create(12, 10, ea=dev(inst.ea), fixed=dev(inst.fixed))
    assert lat.sets == 1
