"""Pins of the oracle's relaxation with fixed-force boundary (Eq. 15-18),
against facts that do not come from the oracle's own code:

* k^Inner + Delta k of Eq. 15 is the stiffness of the isolated region: the
  rods with both ends in the region, assembled here by an explicit loop;
* the increment u^RF - u^old equals the literal solve of Eq. 16;
* a region with no clamped node has exactly the three rigid motions as null
  space (dense eigenvalues), a region holding a clamped column has none;
* for a floating region the increment is the minimum-norm solution: the
  isolated stiffness maps it to the residual minus its rigid-motion part, and
  it is orthogonal to the rigid motions;
* on every region of a lattice with a ragged set row one node thick and two
  clamped corners (strips, floating regions, regions pinned at one node) the
  increment is the dense pseudo-inverse of the loop-built isolated stiffness
  applied to the residual;
* modes 10-12 span {d_F, x d_F, y d_F} on each set (Eq. 17-18);
* with q = 12 the method keeps its invariants (the energy of Eq. 2 never
  rises, Galerkin orthogonality to all twelve modes, convergence to the plain
  solution) and needs fewer outer iterations than with q = 9.
The planted slips at the end fail these pins.
"""
import math

import numpy as np
import pytest

import oracle.method as om
from oracle.solve import rel_residuals, residual, solve, system_of
from workloads import make_instance


def _positions(nx, ny):
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([(i + 0.5 * j).reshape(-1), (j * math.sqrt(3.0) / 2.0).reshape(-1)], 1)


def _isolated_by_loops(inst, nodes):
    """Stiffness of the rods with both ends in `nodes`, on the free DOFs of
    those nodes (sorted DOF order), by an explicit loop over the rods."""
    nx, ny = inst.nx, inst.ny
    xy = _positions(nx, ny)
    inside = set(int(n) for n in nodes)
    free = ~inst.fixed.astype(bool).reshape(-1)
    dofs = sorted(2 * n + c for n in inside for c in (0, 1) if free[n])
    pos = {d: k for k, d in enumerate(dofs)}
    Kd = np.zeros((len(dofs), len(dofs)))
    for a in inside:
        i, j = a % nx, a // nx
        for d, (di, dj) in enumerate(((1, 0), (0, 1), (-1, 1))):
            i2, j2 = i + di, j + dj
            if not (0 <= i2 < nx and 0 <= j2 < ny):
                continue
            b = j2 * nx + i2
            if b not in inside:
                continue
            k = float(inst.ea[d, j, i])
            n = xy[b] - xy[a]
            ke = k * np.outer(n, n)
            for p, q, sgn in ((a, a, 1.0), (b, b, 1.0), (a, b, -1.0), (b, a, -1.0)):
                for c1 in range(2):
                    for c2 in range(2):
                        r, c = 2 * p + c1, 2 * q + c2
                        if r in pos and c in pos:
                            Kd[pos[r], pos[c]] += sgn * ke[c1, c2]
    return np.array(dofs), Kd


CASE = dict(nx=40, ny=37, E=16, seed=51)


def _solver(overlap):
    inst = make_instance(CASE["nx"], CASE["ny"], seed=CASE["seed"], ea="lognormal")
    S = system_of(inst)
    sets = om.make_sets(CASE["nx"], CASE["ny"], CASE["E"])
    return inst, S, sets, om.ForceLocalSolver(S, sets, overlap)


@pytest.mark.parametrize("overlap", [0, 2])
def test_isolated_stiffness_is_the_rods_inside_the_region(overlap):
    inst, S, sets, fs = _solver(overlap)
    for I in range(sets.M):
        nodes = om.relaxation_region(sets, I, overlap)
        dofs, Kd = _isolated_by_loops(inst, nodes)
        assert np.array_equal(dofs, fs.idx[I])
        Kg = fs.kiso[I].toarray()
        assert np.abs(Kg - Kd).max() <= 1e-13 * np.abs(Kd).max(), I


def test_increment_equals_the_literal_solve_of_eq16():
    inst, S, sets, fs = _solver(2)
    rng = np.random.default_rng(52)
    u_old = rng.standard_normal(S.f.size) * S.free
    r = residual(S, u_old)
    d = fs.relax(r)
    K = S.K.toarray()
    checked = 0
    for I in range(sets.M):
        if fs.null[I].shape[1]:
            continue                       # the literal form needs a regular matrix
        idx = fs.idx[I]
        nodes = om.relaxation_region(sets, I, 2)
        inside_dofs = np.concatenate([2 * nodes, 2 * nodes + 1])
        outer = np.setdiff1d(np.arange(S.f.size), inside_dofs)
        # p^Inner - k^Outer u^Outer,old + Delta k u^Inner,old   (Eq. 16; the
        # clamped DOFs of the region carry their prescribed values, here 0)
        pbar = S.f[idx] - K[np.ix_(idx, outer)] @ u_old[outer] + fs.dk[I] @ u_old[idx]
        u_rf = np.linalg.solve(fs.kiso[I].toarray(), pbar)
        own = fs.own[I]
        mode10 = (u_rf - u_old[idx])[own]
        assert np.allclose(d[idx[own]], mode10, rtol=1e-9, atol=1e-12 * np.abs(mode10).max())
        checked += 1
    assert checked >= 3


def test_null_space_of_isolated_regions():
    inst, S, sets, fs = _solver(0)
    for I in range(sets.M):
        w = np.linalg.eigvalsh(fs.kiso[I].toarray())
        nzero = int((w < 1e-10 * w.max()).sum())
        holds_clamped = (I % sets.mx) == 0     # the tile column on the clamped edge
        assert nzero == (0 if holds_clamped else 3), (I, nzero)
        assert fs.null[I].shape[1] == nzero


def test_floating_region_gives_the_minimum_norm_increment():
    inst, S, sets, fs = _solver(0)
    rng = np.random.default_rng(53)
    r = rng.standard_normal(S.f.size) * S.free
    floating = [I for I in range(sets.M) if fs.null[I].shape[1] == 3]
    assert floating
    xy = _positions(CASE["nx"], CASE["ny"])
    for I in floating:
        idx = fs.idx[I]
        x = fs.relax_region(I, r)
        node, comp = idx // 2, idx % 2
        rigid = np.stack([comp == 0, comp == 1,
                          np.where(comp == 0, -xy[node, 1], xy[node, 0])], 1).astype(float)
        Q, _ = np.linalg.qr(rigid)
        rhs = r[idx] - Q @ (Q.T @ r[idx])
        Kd = fs.kiso[I].toarray()
        assert np.linalg.norm(Kd @ x - rhs) <= 1e-10 * np.linalg.norm(rhs)
        assert np.linalg.norm(Q.T @ x) <= 1e-10 * np.linalg.norm(x)


def test_every_region_increment_is_the_pseudo_inverse_solution():
    """Regions one node thick (the ragged top row of 16 x 16 sets on 33 rows,
    w = 0), regions with no clamped node and with exactly one (two opposite
    corners clamped): on each, the increment is the minimum-norm solution,
    the dense pseudo-inverse of the rods inside the region (assembled by the
    loop above) applied to the residual."""
    nx, ny = 40, 33
    inst = make_instance(nx, ny, seed=56, ea="lognormal", clamp="none")
    inst.fixed[:] = 0
    inst.fixed[0, 0] = inst.fixed[-1, -1] = 1
    inst.f[inst.fixed.astype(bool)] = 0.0
    S = system_of(inst)
    sets = om.make_sets(nx, ny, 16)
    fs = om.ForceLocalSolver(S, sets, 0)
    r = np.random.default_rng(57).standard_normal(S.f.size) * S.free
    kinds = set()
    for I in range(sets.M):
        nodes = om.relaxation_region(sets, I, 0)
        dofs, Kd = _isolated_by_loops(inst, nodes)
        assert np.array_equal(dofs, fs.idx[I])
        w = np.linalg.eigvalsh(Kd)
        nzero = int((w < 1e-10 * w.max()).sum())
        kinds.add(nzero)
        want = np.linalg.pinv(Kd, rcond=1e-10, hermitian=True) @ r[dofs]
        got = fs.relax_region(I, r)
        assert np.linalg.norm(got - want) <= 1e-9 * np.linalg.norm(want), (I, nzero)
    # strips (each free node's motion across the strip, and a slide along it
    # unless the strip holds a clamped node), floating regions (3) and regions
    # pinned at one node (1) all occur
    assert {1, 3} <= kinds and max(kinds) > 3, kinds
    # the method's twelve-mode step runs on this lattice
    m = om.Method(S, sets, overlap=0, modes=12)
    st = m.step(S.u_c.copy())
    assert np.all(np.isfinite(st.u_new))


def test_modes_10_to_12_span_the_force_increment_products():
    inst, S, sets, fs = _solver(2)
    rng = np.random.default_rng(54)
    d = rng.standard_normal(S.f.size) * S.free
    dF = rng.standard_normal(S.f.size) * S.free
    U = om.mode_matrix(S, sets, d, dF)
    assert U.shape[1] == om.Q12 * sets.M
    xy = _positions(CASE["nx"], CASE["ny"])
    node_set = np.repeat(sets.of_node, 2)
    for I in range(sets.M):
        rows = np.flatnonzero((node_set == I) & S.free)
        B = U[:, om.Q12 * I:om.Q12 * I + om.Q12].toarray()[rows]
        assert np.array_equal(B[:, 9], dF[rows])
        R = B[:, 9:12]
        nodes = rows // 2
        for v in (dF[rows], xy[nodes, 0] * dF[rows], xy[nodes, 1] * dF[rows]):
            c, *_ = np.linalg.lstsq(R, v, rcond=None)
            assert np.linalg.norm(R @ c - v) <= 1e-12 * np.linalg.norm(v)
        # the first nine modes are those of the q = 9 matrix
        B9 = om.mode_matrix(S, sets, d)[:, om.Q * I:om.Q * I + om.Q].toarray()[rows]
        assert np.array_equal(B[:, :9], B9)


def _method(modes, overlap=0, nx=50, ny=41, E=16, seed=55):
    inst = make_instance(nx, ny, seed=seed, ea="lognormal")
    S = system_of(inst)
    return S, om.Method(S, om.make_sets(nx, ny, E), overlap=overlap, modes=modes)


def test_twelve_modes_keep_the_method_invariants():
    S, m = _method(12)
    u = S.u_c.copy()
    Pi = []
    for _ in range(6):
        st = m.step(u)
        g_old = st.U.T @ st.r
        g_new = st.U.T @ residual(S, st.u_new)
        assert st.U.shape[1] == 12 * m.sets.M
        assert np.linalg.norm(g_new) <= 1e-9 * np.linalg.norm(g_old)
        Pi.append(om.energy(S, u))
        u = st.u_new
    Pi.append(om.energy(S, u))
    assert all(Pi[k + 1] <= Pi[k] + 1e-13 * abs(Pi[k]) for k in range(len(Pi) - 1))


@pytest.mark.parametrize("overlap", [0, 2])
def test_twelve_modes_converge_faster_to_the_plain_solution(overlap):
    S, m12 = _method(12, overlap)
    _, m9 = _method(9, overlap)
    u12, it12, h12 = m12.run(tol=1e-10, max_iters=2000)
    _, it9, _ = m9.run(tol=1e-10, max_iters=2000)
    ref = solve(S)
    assert max(h12[-1][:2]) <= 1e-10
    assert np.linalg.norm(u12 - ref) <= 1e-8 * np.linalg.norm(ref)
    assert it12 < it9, (it12, it9)


# ------------------------------------------------------------- planted slips

def test_planted_sign_slip_in_delta_k_is_caught(monkeypatch):
    real = om.isolation_correction
    monkeypatch.setattr(om, "isolation_correction", lambda K, idx, inside: -real(K, idx, inside))
    with pytest.raises(AssertionError):
        test_isolated_stiffness_is_the_rods_inside_the_region(0)


def test_planted_cut_clamped_rods_are_caught(monkeypatch):
    """Counting the region's clamped nodes as outside it, so that their rods
    are cut too."""
    inst = make_instance(CASE["nx"], CASE["ny"], seed=CASE["seed"], ea="lognormal")
    free_node = ~inst.fixed.astype(bool).reshape(-1)
    real = om.isolation_correction
    monkeypatch.setattr(om, "isolation_correction",
                        lambda K, idx, inside: real(K, idx, inside & free_node))
    with pytest.raises(AssertionError):
        test_isolated_stiffness_is_the_rods_inside_the_region(0)


def test_planted_copy_of_mode_11_is_caught(monkeypatch):
    real = om.mode_matrix

    def copy11(S, sets, delta, delta_f=None):
        U = real(S, sets, delta, delta_f).tolil()
        if delta_f is not None:
            U[:, 11::om.Q12] = U[:, 10::om.Q12]
        return U.tocsr()
    monkeypatch.setattr(om, "mode_matrix", copy11)
    with pytest.raises(AssertionError):
        test_modes_10_to_12_span_the_force_increment_products()
