"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Tolerances:
* the residual kernel is float64 arithmetic on the same data in a different
  summation order, so it agrees with the oracle's CSR product to a few ulps
  of the largest term: 1e-12 relative to ||f||_inf + ||K||_1 ||u||_inf;
* converged displacements: 1e-8 relative L2 (the stated target), with the
  solve run to a 1e-10 relative residual since the error of an iterate can
  exceed its relative residual by the lattice's conditioning (about
  13 n^2 for n x n), see the solve tests;
* one outer iteration with near-exact inner solves: relaxation increment,
  upper-level blocks and force to 1e-9 relative (inner PCG to convergence),
  the updated displacement to 1e-9.
"""
import numpy as np
import pytest

import oracle.method as om
from oracle.solve import rel_residuals, residual, solve, system_of
from workloads import make_instance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

tl = pytest.importorskip("paper_1208_4093_amd.tl")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def make_lattice(inst, E):
    return tl.tl_lattice_create(inst.nx, inst.ny, ea=inst.ea, fixed=inst.fixed,
                                u_fixed=inst.u_fixed, set_edge=E)


def gpu_solve(inst, E, precision, rtol, **kw):
    lat = make_lattice(inst, E)
    f = dev(inst.f)
    u = torch.zeros_like(f)
    info = tl.tl_solve(lat, f, u, precision=precision, rtol=rtol, **kw)
    torch.cuda.synchronize()
    return u.cpu().numpy(), info, lat


CASES = [
    # (nx, ny, E, ea, seed)  -- C1 exactly, then ragged and lognormal shapes
    (64, 64, 16, "unit", 0),
    (100, 72, 32, "lognormal", 1),
    (45, 37, 16, "lognormal", 2),
    (70, 130, 64, "lognormal", 3),
    (2, 2, 16, "unit", 4),
    (17, 33, 16, "unit", 5),
]


@pytest.mark.parametrize("nx,ny,E,ea,seed", CASES)
def test_residual_kernel_matches_oracle(nx, ny, E, ea, seed):
    inst = make_instance(nx, ny, seed=seed, ea=ea)
    S = system_of(inst)
    rng = np.random.default_rng(100 + seed)
    u = rng.standard_normal((ny, nx, 2))
    u[inst.fixed.astype(bool)] = 0.0
    lat = make_lattice(inst, E)
    f_d, u_d = dev(inst.f), dev(u)
    r_d = torch.empty_like(f_d)
    R1, R2, en = tl.tl_residual(lat, f_d, u_d, r_d)
    r_o = residual(S, u.reshape(-1))
    scale = np.abs(inst.f).max() + abs(S.K).sum(axis=1).max() * np.abs(u).max()
    assert np.abs(r_d.cpu().numpy().reshape(-1) - r_o).max() <= 1e-12 * scale
    R1o, R2o = rel_residuals(S, u.reshape(-1))
    assert R1 == pytest.approx(R1o, rel=1e-12)
    assert R2 == pytest.approx(R2o, rel=1e-12)
    uf = u.reshape(-1)
    assert en == pytest.approx(0.5 * uf @ (S.K @ uf) - uf @ S.f, rel=1e-11)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("nx,ny,E,ea,seed", CASES)
def test_solve_matches_oracle(nx, ny, E, ea, seed, precision):
    inst = make_instance(nx, ny, seed=seed, ea=ea)
    S = system_of(inst)
    us = solve(S)
    u, info, _ = gpu_solve(inst, E, precision, 1e-10)
    assert info["status"] == tl.TL_OK
    assert max(info["rel_res_l1"], info["rel_res_l2"]) <= 1e-10
    err = np.linalg.norm(u.reshape(-1) - us) / np.linalg.norm(us)
    assert err <= 1e-8, (err, info)
    # the library's own certificate agrees with the oracle's residual of u;
    # both carry a rounding error of a few ulps of |K||u| / |f| from f - K u
    R1o, R2o = rel_residuals(S, u.reshape(-1))
    assert info["rel_res_l1"] == pytest.approx(R1o, rel=1e-3, abs=1e-13)
    assert info["rel_res_l2"] == pytest.approx(R2o, rel=1e-3, abs=1e-13)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("sets_per_wg,no_lds", [(64, 0), (64, 1)])
def test_upper_level_general_path_matches_oracle(monkeypatch, sets_per_wg, no_lds, precision):
    """The upper level with several rows per thread and its blocks (and, with
    no_lds, its PCG vectors) in global memory, the form large lattices take,
    forced on a lattice the oracle solves in seconds."""
    monkeypatch.setenv("TL_COARSE_SETS_PER_WG", str(sets_per_wg))
    monkeypatch.setenv("TL_COARSE_NO_LDS", str(no_lds))
    inst = make_instance(200, 180, seed=11, ea="lognormal")
    S = system_of(inst)
    us = solve(S)
    u, info, _ = gpu_solve(inst, 16, precision, 1e-10)
    assert info["status"] == tl.TL_OK
    assert max(info["rel_res_l1"], info["rel_res_l2"]) <= 1e-10
    err = np.linalg.norm(u.reshape(-1) - us) / np.linalg.norm(us)
    assert err <= 1e-8, (err, info)


def _oracle_blocks(Kc, sets, s):
    Q = om.Q
    I, J = s % sets.mx, s // sets.mx
    diag = Kc[Q * s:Q * s + Q, Q * s:Q * s + Q]
    off = np.zeros((6, Q, Q))
    for d, (di, dj) in enumerate([(1, 0), (0, 1), (-1, 1), (-1, 0), (0, -1), (1, -1)]):
        I2, J2 = I + di, J + dj
        if 0 <= I2 < sets.mx and 0 <= J2 < sets.my:
            s2 = J2 * sets.mx + I2
            off[d] = Kc[Q * s:Q * s + Q, Q * s2:Q * s2 + Q]
    return diag, off


@pytest.mark.parametrize("nx,ny,E,ea,seed,ov", [
    (64, 48, 16, "lognormal", 7, 0), (45, 37, 16, "unit", 8, 0), (70, 66, 32, "lognormal", 9, 0),
    # relaxation on widened regions (section 2.2 end), ragged and clipped
    (64, 48, 16, "lognormal", 7, 2), (45, 37, 16, "unit", 8, 4), (70, 66, 32, "lognormal", 9, 1),
    (100, 72, 32, "lognormal", 10, 2), (70, 130, 64, "lognormal", 3, 2)])
def test_one_iteration_matches_method_model(nx, ny, E, ea, seed, ov):
    """Every intermediate of one outer iteration (Eqs. 3, 6, 7, 8, 13) with
    the GPU's inner solves driven to convergence, against the oracle's exact
    step."""
    inst = make_instance(nx, ny, seed=seed, ea=ea)
    S = system_of(inst)
    sets = om.make_sets(nx, ny, E)
    step = om.Method(S, sets, overlap=ov).step(S.u_c.copy())
    M, Q = sets.M, om.Q
    tr_t = dict(delta=torch.zeros((ny, nx, 2), dtype=torch.float64, device="cuda"),
                kdiag=torch.zeros((M, Q, Q), dtype=torch.float64, device="cuda"),
                koff=torch.zeros((M, 6, Q, Q), dtype=torch.float64, device="cuda"),
                force=torch.zeros((M, Q), dtype=torch.float64, device="cuda"),
                coef=torch.zeros((M, Q), dtype=torch.float64, device="cuda"),
                residual_history=torch.zeros(4, dtype=torch.float64, device="cuda"))
    trace = tl.make_trace(**tr_t)
    lat = make_lattice(inst, E)
    f = dev(inst.f)
    u = torch.zeros_like(f)
    R = E + 2 * ov
    info = tl.tl_solve(lat, f, u, check=False, precision=0, rtol=1e-300, max_iters=1,
                       inner_iters=2 * R * R, coarse_iters=20000, coarse_rtol=1e-15, trace=trace,
                       overlap=ov if ov > 0 else -1)
    torch.cuda.synchronize()
    assert info["status"] == tl.TL_E_NOCONV and info["iters"] == 1
    d_g = tr_t["delta"].cpu().numpy().reshape(-1)
    assert np.linalg.norm(d_g - step.delta) <= 1e-9 * np.linalg.norm(step.delta)
    kd, ko = tr_t["kdiag"].cpu().numpy(), tr_t["koff"].cpu().numpy()
    P = tr_t["force"].cpu().numpy().reshape(-1)
    assert np.linalg.norm(P - step.P) <= 1e-9 * np.linalg.norm(step.P)
    for s in range(M):
        diag, off = _oracle_blocks(step.Kc, sets, s)
        nrm = np.abs(diag).max()
        assert np.abs(kd[s] - diag).max() <= 1e-9 * nrm, s
        assert np.abs(ko[s] - off).max() <= 1e-9 * nrm, s
    # Eq. 8: the coefficients solve the GPU's own upper-level system K_a a = P
    # to the upper-level PCG's reach, and the oracle's to the blocks' agreement
    a_g = tr_t["coef"].cpu().numpy().reshape(-1)
    Kg = np.zeros((M * Q, M * Q))
    dirs = [(1, 0), (0, 1), (-1, 1), (-1, 0), (0, -1), (1, -1)]
    for sidx in range(M):
        I, J = sidx % sets.mx, sidx // sets.mx
        Kg[Q * sidx:Q * sidx + Q, Q * sidx:Q * sidx + Q] = kd[sidx]
        for d, (di, dj) in enumerate(dirs):
            if 0 <= I + di < sets.mx and 0 <= J + dj < sets.my:
                s2 = (J + dj) * sets.mx + I + di
                Kg[Q * sidx:Q * sidx + Q, Q * s2:Q * s2 + Q] = ko[sidx][d]
    # (the pipelined PCG's recurrences reach a true relative residual of about
    # 1e-10 before rounding stalls them: its attainable accuracy)
    res_g = np.linalg.norm(Kg @ a_g - P) / np.linalg.norm(P)
    assert res_g <= 1e-9, res_g
    res_o = np.linalg.norm(step.Kc @ a_g - step.P) / np.linalg.norm(step.P)
    assert res_o <= 1e-8, res_o
    # Eq. 3: the update applies exactly those coefficients to the modes
    u1 = u.cpu().numpy().reshape(-1)
    u_exp = S.u_c + step.U @ a_g
    assert np.linalg.norm(u1 - u_exp) <= 1e-9 * np.linalg.norm(u_exp)
    # and agrees with the oracle's exact step, to the accuracy the residual of
    # Eq. 8 allows.  With D = diag(K_a), S = D^-1/2, A = S K_a S, y = S^-1 a:
    # the energy norm of U (a - a*) is |A^{1/2} (y - y*)| = |A^{+1/2} S (K_a a - P)|
    # <= |S (K_a a - P)| / sqrt(lambda_min(A)) (lambda_min over A's range).
    d = np.diag(step.Kc).copy()
    sc = np.where(d > 0.0, 1.0 / np.sqrt(np.where(d > 0.0, d, 1.0)), 0.0)
    w = np.linalg.eigvalsh(step.Kc * sc[:, None] * sc[None, :])
    lam_min = w[w > 1e-13 * w.max()].min()
    res_s = np.linalg.norm(sc * (step.Kc @ a_g - step.P))
    du = u1 - step.u_new
    err_k = np.sqrt(max(du @ (S.K @ du), 0.0))
    norm_k = np.sqrt(step.u_new @ (S.K @ step.u_new))
    assert err_k <= 1.01 * res_s / np.sqrt(lam_min) + 1e-9 * norm_k, (err_k, res_s, lam_min)
    assert np.linalg.norm(du) <= 1e-7 * np.linalg.norm(step.u_new)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("nx,ny,E,ea,seed,ov", [
    (64, 64, 16, "unit", 0, 2), (100, 72, 32, "lognormal", 1, 2), (45, 37, 16, "lognormal", 2, 4),
    (70, 130, 64, "lognormal", 3, 2), (17, 33, 16, "unit", 5, 1), (2, 2, 16, "unit", 4, 2)])
def test_overlap_solve_matches_oracle(nx, ny, E, ea, seed, ov, precision):
    inst = make_instance(nx, ny, seed=seed, ea=ea)
    S = system_of(inst)
    us = solve(S)
    u, info, _ = gpu_solve(inst, E, precision, 1e-10, overlap=ov)
    assert info["status"] == tl.TL_OK
    assert max(info["rel_res_l1"], info["rel_res_l2"]) <= 1e-10
    err = np.linalg.norm(u.reshape(-1) - us) / np.linalg.norm(us)
    assert err <= 1e-8, (err, info)


# Every tile kernel the library can launch: set edge 16, 32 or 64 (as a caller
# or the autotuner picks it), each thread count the launcher takes for it
# (its default, or TL_TILE_THREADS), relaxation overlap 0, 1, 2 or 4 (section
# 2.2 end), in both forms, solved against the oracle on a ragged lattice of
# several sets.
TILE_LATTICES = {16: (45, 37), 32: (75, 70), 64: (140, 70)}
TILE_SHAPES = [(16, 256, ov) for ov in (0, 1, 2, 4)] + \
    [(32, 256, ov) for ov in (0, 1, 2, 4)] + [(32, 512, ov) for ov in (0, 1, 2, 4)] + \
    [(32, 1024, 0)] + [(64, nt, ov) for nt in (512, 1024) for ov in (0, 1, 2, 4)]
_tile_refs = {}


def _tile_case(E):
    if E not in _tile_refs:
        nx, ny = TILE_LATTICES[E]
        inst = make_instance(nx, ny, seed=100 + E, ea="lognormal")
        _tile_refs[E] = (inst, solve(system_of(inst)))
    return _tile_refs[E]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("E,nt,ov", TILE_SHAPES)
def test_every_tile_instantiation_matches_oracle(E, nt, ov, precision, monkeypatch):
    monkeypatch.setenv("TL_TILE_THREADS", str(nt))
    inst, us = _tile_case(E)
    u, info, _ = gpu_solve(inst, E, precision, 1e-10, overlap=ov if ov > 0 else -1)
    assert info["status"] == tl.TL_OK
    assert max(info["rel_res_l1"], info["rel_res_l2"]) <= 1e-10
    err = np.linalg.norm(u.reshape(-1) - us) / np.linalg.norm(us)
    assert err <= 1e-8, (err, info)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("ov", [0, 1, 2, 4])
def test_every_batched_tile_instantiation_matches_oracle(ov, precision):
    """The fused batch's tile kernels at each overlap, one lattice per set edge
    in one call, against the same oracle solutions."""
    cases = [_tile_case(E) for E in (16, 32, 64)]
    lats = [make_lattice(inst, E) for E, (inst, _) in zip((16, 32, 64), cases)]
    fs = [dev(inst.f) for inst, _ in cases]
    us = [torch.zeros_like(f) for f in fs]
    st, infos = tl.tl_solve_batch(lats, fs, us, precision=precision, rtol=1e-10,
                                  overlap=ov if ov > 0 else -1)
    torch.cuda.synchronize()
    assert st == tl.TL_OK
    for (inst, ref), u, info in zip(cases, us, infos):
        assert info["status"] == tl.TL_OK
        assert max(info["rel_res_l1"], info["rel_res_l2"]) <= 1e-10
        err = np.linalg.norm(u.cpu().numpy().reshape(-1) - ref) / np.linalg.norm(ref)
        assert err <= 1e-8, (err, info)


@pytest.mark.parametrize("precision,cap", [(0, 20), (1, 25)])
def test_small_lattice_upper_level_cap(precision, cap):
    """Lattices of at most 256 sets stop the upper-level PCG after 20
    (float64) or 25 (mixed) iterations by default and still reach the oracle's
    solution; an explicit cap overrides it."""
    inst = make_instance(200, 150, seed=21, ea="lognormal")
    us = solve(system_of(inst))
    u, info, lat = gpu_solve(inst, 16, precision, 1e-10)
    assert lat.sets <= 256
    assert info["status"] == tl.TL_OK
    assert info["coarse_iters"] <= cap * info["iters"]
    err = np.linalg.norm(u.reshape(-1) - us) / np.linalg.norm(us)
    assert err <= 1e-8, (err, info)
    u2, info2, _ = gpu_solve(inst, 16, precision, 1e-10, coarse_iters=3)
    assert info2["status"] == tl.TL_OK
    assert info2["coarse_iters"] <= 3 * info2["iters"]
    assert np.linalg.norm(u2.reshape(-1) - us) <= 1e-8 * np.linalg.norm(us)


def test_energy_decreases_every_iteration():
    inst = make_instance(50, 41, seed=11, ea="lognormal")
    lat = make_lattice(inst, 16)
    f = dev(inst.f)
    energies = []
    for k in range(1, 9):
        u = torch.zeros_like(f)
        info = tl.tl_solve(lat, f, u, check=False, precision=1, rtol=1e-300, max_iters=k,
                           coarse_iters=200, coarse_rtol=1e-12)
        assert info["iters"] == k
        energies.append(info["energy"])
    assert all(energies[i + 1] <= energies[i] + 1e-12 * abs(energies[i]) for i in range(len(energies) - 1))
    assert energies[-1] < energies[0] < 0.0


def test_affine_patch_on_gpu():
    """Unit EA, boundary nodes prescribed an affine field, no load inside:
    the solver reproduces the field (a non-default support mask and
    prescribed displacements through the ABI)."""
    nx, ny = 40, 35
    inst = make_instance(nx, ny, seed=12)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    xy = np.stack([i + 0.5 * j, j * np.sqrt(3) / 2], -1)
    A, b = np.array([[0.3, -0.2], [0.1, 0.4]]), np.array([0.5, -1.0])
    field = xy @ A.T + b
    inst.fixed[:] = 0
    inst.fixed[[0, -1], :] = 1
    inst.fixed[:, [0, -1]] = 1
    inst.u_fixed[:] = np.where(inst.fixed[..., None].astype(bool), field, 0.0)
    inst.f[:] = 0.0
    S = system_of(inst)
    us = solve(S)
    assert np.abs(us.reshape(ny, nx, 2) - field).max() <= 1e-12 * np.abs(field).max()
    for precision in (0, 1):
        u, info, _ = gpu_solve(inst, 16, precision, 1e-11)
        assert info["status"] == tl.TL_OK
        assert np.abs(u - field).max() <= 1e-8 * np.abs(field).max()


def test_nonfinite_load_is_reported():
    inst = make_instance(32, 32, seed=13)
    inst.f[5, 5, 1] = np.nan
    lat = make_lattice(inst, 16)
    f = dev(inst.f)
    u = torch.zeros_like(f)
    info = tl.tl_solve(lat, f, u, check=False, precision=0, rtol=1e-8)
    assert info["status"] == tl.TL_E_NONFINITE


def test_max_iters_gives_noconv_with_filled_result():
    inst = make_instance(64, 64, seed=14)
    S = system_of(inst)
    lat = make_lattice(inst, 16)
    f = dev(inst.f)
    u = torch.zeros_like(f)
    info = tl.tl_solve(lat, f, u, check=False, precision=0, rtol=1e-12, max_iters=5)
    assert info["status"] == tl.TL_E_NOCONV and info["iters"] == 5
    R1, R2 = rel_residuals(S, u.cpu().numpy().reshape(-1))
    assert R1 == pytest.approx(info["rel_res_l1"], rel=1e-9) and R1 < 1.0


def test_repeat_solves_are_bitwise_identical():
    inst = make_instance(96, 80, seed=15, ea="lognormal")
    lat = make_lattice(inst, 32)
    f = dev(inst.f)
    outs = []
    for _ in range(2):
        u = torch.zeros_like(f)
        tl.tl_solve(lat, f, u, precision=1, rtol=1e-9)
        outs.append(u.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_1024_certified(precision):
    """The 1024 x 1024 workload at its own settings (E = 32, library defaults,
    1e-8), in both forms: certified by the oracle's residual of the returned
    u (no CPU solve at this size finishes in a test's time) and the energy
    identity."""
    inst = make_instance(1024, 1024, seed=0)
    u, info, _ = gpu_solve(inst, 32, precision, 1e-8)
    assert info["status"] == tl.TL_OK
    S = system_of(inst)
    uf = u.reshape(-1)
    R1, R2 = rel_residuals(S, uf)
    assert max(R1, R2) <= 1e-8
    fu, uKu = S.f @ uf, uf @ (S.K @ uf)
    assert abs(fu - uKu) <= 1e-6 * abs(fu)


@pytest.mark.parametrize("precision", [tl.TL_FP64, tl.TL_MIXED])
def test_full_size_1024_against_oracle_solution(precision):
    """The 1024 x 1024 workload against the oracle's own solution of it (block-
    Jacobi PCG to a recomputed relative residual of 1e-11, written by
    tests/golden/make_oracle_1024.py) at its 4,000 sampled free DOFs: solved
    to 1e-10 (the parity tolerance of the method's readings) the relative
    error over the sample is at most 1e-8; at the benchmark's 1e-8 it is
    reported and held to 1e-6 (the relative error of CG-type iterates runs at
    a fraction of the relative residual here, far below kappa(K) times it)."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_u_1024_sample.json")
    if not os.path.exists(path):
        pytest.skip("tests/golden/oracle_u_1024_sample.json not written yet "
                    "(python tests/golden/make_oracle_1024.py tests/golden/oracle_u_1024_sample.json)")
    ref = json.load(open(path))
    assert ref["rel_residual_2norm"] <= 1e-11 and ref["lattice"] == [1024, 1024]
    idx = np.asarray(ref["dof"])
    want = np.asarray(ref["u"])
    inst = make_instance(1024, 1024, seed=0)
    for rtol, bound in ((1e-10, 1e-8), (1e-8, 1e-6)):
        u, info, _ = gpu_solve(inst, 32, precision, rtol)
        assert info["status"] == tl.TL_OK
        got = u.reshape(-1)[idx]
        err = np.linalg.norm(got - want) / np.linalg.norm(want)
        print(f"precision {precision} rtol {rtol:g}: sampled relative error {err:.3e}")
        assert err <= bound, (rtol, err)


def test_unsupported_overlap_is_rejected():
    inst = make_instance(40, 30, seed=13)
    lat = make_lattice(inst, 16)
    f = dev(inst.f)
    u = torch.zeros_like(f)
    for ov in (3, 5, 64):
        info = tl.tl_solve(lat, f, u, check=False, overlap=ov)
        assert info["status"] == tl.TL_E_INVAL


@pytest.mark.slow
def test_full_size_16384_mixed_sampled():
    """The 16384 x 16384 workload (537M DOF, lognormal EA, 64 x 64 sets,
    mixed, 1e-10) in the launch configuration the benchmark times.  No CPU
    solve or full CSR fits at this size, so the result is checked through
    properties that hold at any size: the library's float64 certificate meets
    1e-10, and its residual r = f - K u agrees, at 2000 sampled nodes, with
    the oracle's stiffness assembled on the 3 x 3 patch around each node
    (which holds every rod of that node, so its row is the global row)."""
    from oracle.lattice import assemble
    n = 16384
    inst = make_instance(n, n, seed=0, ea="lognormal")
    lat = make_lattice(inst, 64)
    f = dev(inst.f)
    u = torch.zeros_like(f)
    info = tl.tl_solve(lat, f, u, precision=1, rtol=1e-10)
    assert info["status"] == tl.TL_OK
    assert max(info["rel_res_l1"], info["rel_res_l2"]) <= 1e-10
    r = torch.empty_like(f)
    R1, R2, _ = tl.tl_residual(lat, f, u, r)
    assert max(R1, R2) <= 1e-10
    rng = np.random.default_rng(7)
    js, is_ = rng.integers(0, n, 2000), rng.integers(1, n, 2000)   # free nodes (i >= 1)
    idx = torch.from_numpy(js * n + is_).cuda()
    u_s = u.reshape(-1, 2)
    r_g = r.reshape(-1, 2)[idx].cpu().numpy()
    for k, (j, i) in enumerate(zip(js, is_)):
        j0, j1, i0, i1 = max(j - 1, 0), min(j + 2, n), max(i - 1, 0), min(i + 2, n)
        py, px = j1 - j0, i1 - i0
        Kp = assemble(px, py, np.ascontiguousarray(inst.ea[:, j0:j1, i0:i1]))
        rows = torch.from_numpy(np.array([(jj * n + ii) for jj in range(j0, j1) for ii in range(i0, i1)])).cuda()
        up = u_s[rows].cpu().numpy().reshape(-1)
        c = (j - j0) * px + (i - i0)
        r_o = inst.f[j, i] - (Kp @ up)[2 * c:2 * c + 2]
        scale = np.abs(inst.f[j, i]).max() + np.abs(Kp[2 * c:2 * c + 2]).sum(axis=1).max() * np.abs(up).max()
        assert np.abs(r_g[k] - r_o).max() <= 1e-12 * scale, (j, i, r_g[k], r_o)
