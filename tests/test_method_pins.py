"""Pins of the oracle's step-by-step method model against the properties the
paper states or that follow from its equations:

* the total energy (Eq. 2) never increases (section 2.1 end);
* the upper-level solve makes the new residual orthogonal to every mode
  (Eq. 5 set to zero);
* one set with an exact local solve reaches the solution in one iteration
  (the relaxation increment of Eq. 13 is then the exact correction);
* the exact solution is a fixed point (zero relaxation, zero coefficients);
* the upper-level matrix of Eq. 6 is symmetric positive semidefinite and the
  force of Eq. 7 lies in its range;
* the iterates do not depend on the representative node of Eq. 10 and 14;
* the iteration converges to the plain solution of Eq. 1.

Iteration counts are not pinned: the paper prints none.
"""
import numpy as np
import pytest

import oracle.method as om
from oracle.solve import energy, rel_residuals, residual, solve, system_of
from workloads import make_instance


def _setup(nx, ny, E, seed=0, ea="lognormal", shift=(0.0, 0.0)):
    inst = make_instance(nx, ny, seed=seed, ea=ea)
    S = system_of(inst)
    return S, om.Method(S, om.make_sets(nx, ny, E, rep_shift=shift))


def test_energy_never_increases_ragged_sets():
    S, m = _setup(50, 37, 16, seed=1)
    u, it, hist = m.run(tol=0.0, max_iters=25)
    Pi = [h[2] for h in hist]
    assert all(Pi[k + 1] <= Pi[k] + 1e-13 * abs(Pi[k]) for k in range(len(Pi) - 1))
    assert Pi[-1] < Pi[0]


def test_galerkin_orthogonality_after_update():
    S, m = _setup(40, 33, 16, seed=2)
    u = S.u_c.copy()
    for _ in range(3):
        st = m.step(u)
        g_old = st.U.T @ st.r
        g_new = st.U.T @ residual(S, st.u_new)
        assert np.linalg.norm(g_new) <= 1e-9 * np.linalg.norm(g_old)
        u = st.u_new


def test_single_set_converges_in_one_iteration():
    S, m = _setup(20, 14, 32, seed=3)
    assert m.sets.M == 1
    st = m.step(S.u_c.copy())
    assert max(rel_residuals(S, st.u_new)) <= 1e-12


def test_exact_solution_is_fixed_point():
    S, m = _setup(33, 20, 16, seed=4)
    u = solve(S)
    st = m.step(u)
    assert np.linalg.norm(st.U @ st.a) <= 1e-10 * np.linalg.norm(u)
    assert np.linalg.norm(st.delta) <= 1e-10 * np.linalg.norm(u)


def test_upper_level_matrix_psd_and_force_consistent():
    S, m = _setup(48, 40, 16, seed=5)
    u = S.u_c.copy()
    for _ in range(2):
        st = m.step(u)
        assert np.array_equal(st.Kc, st.Kc.T) or np.abs(st.Kc - st.Kc.T).max() <= 1e-14 * np.abs(st.Kc).max()
        w, V = np.linalg.eigh(st.Kc)
        assert w.min() >= -1e-11 * w.max()
        null = V[:, w <= 1e-11 * w.max()]
        assert np.linalg.norm(null.T @ st.P) <= 1e-9 * np.linalg.norm(st.P)
        u = st.u_new


def test_iterates_independent_of_representative_node():
    S, m0 = _setup(45, 30, 16, seed=6)
    _, m1 = _setup(45, 30, 16, seed=6, shift=(0.37, -1.3))
    u0, _, _ = m0.run(tol=0.0, max_iters=4)
    u1, _, _ = m1.run(tol=0.0, max_iters=4)
    assert np.linalg.norm(u1 - u0) <= 1e-9 * np.linalg.norm(u0)


def test_converges_to_plain_solution():
    S, m = _setup(45, 37, 16, seed=7)
    u, it, hist = m.run(tol=1e-10, max_iters=2000)
    assert max(hist[-1][:2]) <= 1e-10
    us = solve(S)
    assert np.linalg.norm(u - us) <= 1e-8 * np.linalg.norm(us)


def test_planted_sign_slip_in_force_is_caught(monkeypatch):
    """A sign slip in Eq. 7 makes the update climb the energy."""
    real = om.upper_level
    monkeypatch.setattr(om, "upper_level", lambda S, U, u: (lambda kc, p: (kc, -p))(*real(S, U, u)))
    with pytest.raises(AssertionError):
        test_energy_never_increases_ragged_sets()


def test_planted_wrong_gradient_mode_is_caught(monkeypatch):
    """Losing the y-weighted relaxation mode of Eq. 14 (mode 9 a copy of
    mode 8) leaves the new residual not orthogonal to the intended modes."""
    real = om.mode_matrix

    def no_eta(S, sets, delta, *rest):
        U = real(S, sets, delta, *rest).tolil()
        U[:, 8::om.Q] = U[:, 7::om.Q]
        return U.tocsr()
    S, m = _setup(40, 33, 16, seed=2)
    st_good = m.step(S.u_c.copy())
    monkeypatch.setattr(om, "mode_matrix", no_eta)
    st_bad = m.step(S.u_c.copy())
    g = st_good.U.T @ residual(S, st_bad.u_new)
    assert np.linalg.norm(g) > 1e-6 * np.linalg.norm(st_good.U.T @ st_good.r)


# ------------------------------------------- overlapping relaxation regions
# Section 2.2 (end): a set may be relaxed on a larger region around it.  The
# reading here: the region is the set's tile widened by w nodes on every side
# (clipped to the lattice), solved with everything outside it held fixed, and
# the increment is kept on the set's own DOFs.

def _region_by_loops(nx, ny, E, I, w):
    """Free-or-not node ids of set I's widened tile, by explicit loops."""
    mx = -(-nx // E)
    i0, j0 = (I % mx) * E, (I // mx) * E
    out = []
    for j in range(ny):
        for i in range(nx):
            di = max(i0 - i, 0, i - (min(i0 + E, nx) - 1))
            dj = max(j0 - j, 0, j - (min(j0 + E, ny) - 1))
            if di <= w and dj <= w:
                out.append(j * nx + i)
    return out


@pytest.mark.parametrize("w", [1, 2, 5])
def test_overlap_increment_equals_dense_region_solve(w):
    nx, ny, E = 13, 11, 4
    inst = make_instance(nx, ny, seed=21, ea="lognormal")
    S = system_of(inst)
    sets = om.make_sets(nx, ny, E)
    r = residual(S, S.u_c.copy())
    d = om.LocalSolver(S, sets, overlap=w).relax(r)
    Kd = S.K.toarray()
    for I in (0, 5, sets.M - 1):
        nodes = _region_by_loops(nx, ny, E, I, w)
        dofs = [2 * n + c for n in nodes for c in (0, 1) if S.free[2 * n + c]]
        x = np.linalg.solve(Kd[np.ix_(dofs, dofs)], r[dofs])
        own = [k for k, q in enumerate(dofs) if sets.of_node[q // 2] == I]
        got = d[[dofs[k] for k in own]]
        assert np.allclose(got, x[own], rtol=1e-11, atol=1e-14 * np.abs(x).max())
        # nothing outside the set
        mine = np.repeat(sets.of_node == I, 2)
        assert np.all(d[mine & ~np.isin(np.arange(d.size), dofs)] == 0.0)


def test_overlap_covering_lattice_converges_in_one_iteration():
    # every region is the whole lattice: each set's increment is the exact
    # correction restricted to the set, and a_7 = 1 on every set rebuilds it
    inst = make_instance(30, 22, seed=22, ea="lognormal")
    S = system_of(inst)
    m = om.Method(S, om.make_sets(30, 22, 8), overlap=40)
    assert m.sets.M == 12
    st = m.step(S.u_c.copy())
    assert max(rel_residuals(S, st.u_new)) <= 1e-11


def test_overlap_energy_monotone_and_converges():
    inst = make_instance(40, 33, seed=23, ea="lognormal")
    S = system_of(inst)
    m0 = om.Method(S, om.make_sets(40, 33, 16))
    m3 = om.Method(S, om.make_sets(40, 33, 16), overlap=3)
    u3, it3, hist3 = m3.run(tol=1e-11, max_iters=400)
    _, it0, _ = m0.run(tol=1e-11, max_iters=400)
    Pi = [h[2] for h in hist3]
    assert all(Pi[k + 1] <= Pi[k] + 1e-13 * abs(Pi[k]) for k in range(len(Pi) - 1))
    ref = solve(S)
    assert np.linalg.norm(u3 - ref) <= 1e-9 * np.linalg.norm(ref)
    assert it3 < it0          # the larger region relaxes better (section 2.2 end)


def test_planted_region_off_by_one_is_caught(monkeypatch):
    real = om.relaxation_region
    monkeypatch.setattr(om, "relaxation_region", lambda sets, I, w: real(sets, I, max(w - 1, 0)))
    with pytest.raises(AssertionError):
        test_overlap_increment_equals_dense_region_solve(2)


# ----------------------------------------------- the modes themselves (Eq. 9-14)
# The iterates depend only on the span of each set's modes (the representative
# node and the gradient scale are free, Eq. 10 and 14), so the modes are pinned
# by their spans, computed from node positions written out here:
#   modes 1-6 span the affine fields b + A x on the set's free nodes (Eq. 9-10);
#   mode 7 is the relaxation increment itself (Eq. 13);
#   modes 7-9 span {d, x d, y d} for the increment d (Eq. 13-14);
# and every mode vanishes outside its set and on clamped nodes.

def _positions(nx, ny):
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return (i + 0.5 * j).reshape(-1), (j * np.sqrt(3.0) / 2.0).reshape(-1)


def _set_columns(U, Q, I):
    return U[:, Q * I:Q * I + Q].toarray()


def _in_span(B, v):
    """Relative distance of v from the column span of B."""
    c, *_ = np.linalg.lstsq(B, v, rcond=None)
    return np.linalg.norm(B @ c - v) / max(np.linalg.norm(v), 1e-300)


def _mode_case():
    nx, ny, E = 37, 29, 16                    # ragged sets, a clamped left edge
    inst = make_instance(nx, ny, seed=31, ea="lognormal")
    S = system_of(inst)
    sets = om.make_sets(nx, ny, E)
    delta = np.random.default_rng(32).standard_normal(2 * nx * ny) * S.free
    return nx, ny, S, sets, delta


def test_modes_span_affine_fields_and_relaxation_products():
    nx, ny, S, sets, delta = _mode_case()
    Q = om.Q
    U = om.mode_matrix(S, sets, delta)
    x, y = _positions(nx, ny)
    rng = np.random.default_rng(33)
    node_set = np.repeat(sets.of_node, 2)
    for I in range(sets.M):
        rows = np.flatnonzero((node_set == I) & S.free)
        B = _set_columns(U, Q, I)
        # support: the set's free DOFs only
        outside = np.ones(U.shape[0], bool)
        outside[rows] = False
        assert np.all(B[outside] == 0.0)
        nodes = rows[0::2] // 2
        if nodes.size < 3:
            continue
        G = B[rows, :6]
        assert np.linalg.matrix_rank(G, tol=1e-10 * np.abs(G).max()) == 6
        for _ in range(3):
            A, b = rng.standard_normal((2, 2)), rng.standard_normal(2)
            field = np.empty(rows.size)
            field[0::2] = b[0] + A[0, 0] * x[nodes] + A[0, 1] * y[nodes]
            field[1::2] = b[1] + A[1, 0] * x[nodes] + A[1, 1] * y[nodes]
            assert _in_span(G, field) <= 1e-12
        d = delta[rows]
        assert np.array_equal(B[rows, 6], d)
        xd, yd = np.repeat(x[nodes], 2) * d, np.repeat(y[nodes], 2) * d
        R = B[rows, 6:9]
        assert np.linalg.matrix_rank(R, tol=1e-10 * np.abs(R).max()) == 3
        for v in (d, xd, yd):
            assert _in_span(R, v) <= 1e-12


def test_planted_duplicate_gradient_mode_is_caught(monkeypatch):
    """Mode 4, (y - y_I, 0), replaced by a copy of mode 3, (x - x_I, 0)."""
    real = om.mode_matrix

    def dup(S, sets, delta, *rest):
        U = real(S, sets, delta, *rest).tolil()
        U[:, 3::om.Q] = U[:, 2::om.Q]
        return U.tocsr()
    monkeypatch.setattr(om, "mode_matrix", dup)
    with pytest.raises(AssertionError):
        test_modes_span_affine_fields_and_relaxation_products()


def test_planted_transposed_gradient_mode_is_caught(monkeypatch):
    """Mode 6, (0, y - y_I), built as (0, x - x_I): a copy of mode 5."""
    real = om.mode_matrix

    def tr(S, sets, delta, *rest):
        U = real(S, sets, delta, *rest).tolil()
        U[:, 5::om.Q] = U[:, 4::om.Q]
        return U.tocsr()
    monkeypatch.setattr(om, "mode_matrix", tr)
    with pytest.raises(AssertionError):
        test_modes_span_affine_fields_and_relaxation_products()


def test_planted_wrong_weight_in_relaxation_mode_is_caught(monkeypatch):
    """Mode 9 weighted by x (a copy of mode 8) instead of y (Eq. 14)."""
    real = om.mode_matrix

    def wrong(S, sets, delta, *rest):
        U = real(S, sets, delta, *rest).tolil()
        U[:, 8::om.Q] = U[:, 7::om.Q]
        return U.tocsr()
    monkeypatch.setattr(om, "mode_matrix", wrong)
    with pytest.raises(AssertionError):
        test_modes_span_affine_fields_and_relaxation_products()


def test_planted_mode_on_clamped_node_is_caught(monkeypatch):
    """Translation mode left non-zero on the clamped nodes of a set."""
    real = om.mode_matrix

    def leaky(S, sets, delta, *rest):
        U = real(S, sets, delta, *rest).tolil()
        clamped = np.flatnonzero(~S.free)
        for d in clamped[0::2]:
            U[d, om.Q * sets.of_node[d // 2]] = 1.0
        return U.tocsr()
    monkeypatch.setattr(om, "mode_matrix", leaky)
    with pytest.raises(AssertionError):
        test_modes_span_affine_fields_and_relaxation_products()
