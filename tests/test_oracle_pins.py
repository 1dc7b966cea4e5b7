"""Pins of the CPU oracle's assembly and plain solve against facts that do
not come from the oracle itself: closed forms, invariants of linear
elasticity, hand-derived small systems and brute force on tiny lattices.

Each check is chosen so that a plausible slip in the oracle (a wrong bar
direction, a dropped bar, a wrong sign or factor, a transposed block, a
solver bug) fails at least one of them; the planted-mistake tests at the end
show that for the most likely slips.
"""
import math
from fractions import Fraction
from pathlib import Path

import numpy as np
import pytest

from oracle import lattice as L
from oracle.solve import (energy, rel_residuals, residual, solve, solve_banded,
                          solve_dense, solve_pcg, system_of)
from workloads import make_instance

GOLDEN = Path(__file__).parent / "golden"


def positions(nx, ny):
    """Node positions (i + j/2, j*sqrt(3)/2) of the workload, written out here."""
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([i + 0.5 * j, j * math.sqrt(3.0) / 2.0], -1).reshape(-1, 2)


# ----------------------------------------------------------------- geometry

def test_bars_are_unit_rods_between_nearest_neighbours():
    nx, ny = 7, 6
    inst = make_instance(nx, ny, seed=1, ea="lognormal")
    a, b, k, n = L.bar_list(nx, ny, inst.ea)
    xy = positions(nx, ny)
    d = xy[b] - xy[a]
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)   # L = 1
    assert np.allclose(n, d, atol=1e-15)                              # n along the rod
    # every pair of nodes at distance 1 is joined by exactly one rod
    dist = np.linalg.norm(xy[:, None] - xy[None], axis=-1)
    pairs = {tuple(p) for p in np.argwhere(np.isclose(dist, 1.0)) if p[0] < p[1]}
    bars = {tuple(sorted(p)) for p in zip(a.tolist(), b.tolist())}
    assert bars == pairs
    assert len(bars) == (nx - 1) * ny + nx * (ny - 1) + (nx - 1) * (ny - 1)


# --------------------------------------------------------------- stiffness

def test_stiffness_symmetric_bitwise():
    inst = make_instance(9, 8, seed=2, ea="lognormal")
    K = L.assemble(9, 8, inst.ea)
    D = (K - K.T).tocoo()
    assert D.nnz == 0 or np.abs(D.data).max() == 0.0


@pytest.mark.parametrize("n", [2, 5, 10])
def test_unconstrained_null_space_is_rigid_motion(n):
    """Unsupported truss: exactly 3 zero modes (two translations, rotation)."""
    inst = make_instance(n, n, seed=3, ea="lognormal", clamp="none")
    K = L.assemble(n, n, inst.ea).toarray()
    w = np.linalg.eigvalsh(K)
    assert int((w < 1e-10 * w.max()).sum()) == 3
    xy = positions(n, n)
    tx = np.zeros(2 * n * n); tx[0::2] = 1
    ty = np.zeros(2 * n * n); ty[1::2] = 1
    rot = np.zeros(2 * n * n); rot[0::2] = -xy[:, 1]; rot[1::2] = xy[:, 0]
    normK = np.abs(w).max()
    for v in (tx, ty, rot):
        assert np.linalg.norm(K @ v) <= 1e-13 * normK * np.linalg.norm(v)


def test_interior_node_block_closed_form():
    """Six unit rods around a node: sum of n n^T over the six directions = 3 I."""
    inst = make_instance(5, 5, seed=0)
    K = L.assemble(5, 5, inst.ea).toarray()
    node = 2 * 5 + 2
    blk = K[2 * node:2 * node + 2, 2 * node:2 * node + 2]
    assert np.allclose(blk, 3.0 * np.eye(2), atol=1e-15)


@pytest.mark.parametrize("ea", ["unit", "lognormal"])
def test_affine_field_energy_closed_form(ea):
    """u = A x elongates a rod along n (L = 1) by n.A.n, so
    u.K.u = sum over rods of EA (n.A.n)^2, a sum per bar direction."""
    nx, ny = 11, 7
    inst = make_instance(nx, ny, seed=4, ea=ea)
    K = L.assemble(nx, ny, inst.ea)
    rng = np.random.default_rng(5)
    A = rng.standard_normal((2, 2))
    xy = positions(nx, ny)
    u = (xy @ A.T).reshape(-1)
    dirs = [np.array([1.0, 0.0]), np.array([0.5, math.sqrt(3) / 2]),
            np.array([-0.5, math.sqrt(3) / 2])]
    want = sum(float(inst.ea[d].astype(np.float64).sum()) * float(dirs[d] @ A @ dirs[d]) ** 2
               for d in range(3))
    assert u @ (K @ u) == pytest.approx(want, rel=1e-13)


# ------------------------------------------------------------ hand solutions

def _read_golden_sqrt3(path):
    rows = []
    for line in path.read_text().splitlines():
        if not line.strip() or line.startswith("#"):
            continue
        t = line.split()
        rows.append([float(Fraction(t[2 * k])) + float(Fraction(t[2 * k + 1])) * math.sqrt(3)
                     for k in range(len(t) // 2)])
    return np.array(rows)


def test_2x2_compliance_matches_hand_derivation():
    inst = make_instance(2, 2, seed=0)
    S = system_of(inst)
    Kff = S.Kff.toarray()
    C = _read_golden_sqrt3(GOLDEN / "lattice_2x2_compliance.txt")
    assert np.allclose(np.linalg.inv(Kff), C, atol=1e-14)
    # and the solver's answer for a load case equals the compliance column
    inst.f[:] = 0.0
    inst.f[1, 1, 1] = 1.0                         # unit load on B_y
    u = solve(system_of(inst)).reshape(2, 2, 2)
    assert np.allclose([u[0, 1, 0], u[0, 1, 1], u[1, 1, 0], u[1, 1, 1]], C[:, 3], atol=1e-14)


def test_3x3_centre_node_closed_form():
    """All eight outer nodes clamped, unit EA: the centre moves by f / 3."""
    inst = make_instance(3, 3, seed=6)
    inst.fixed[:] = 1
    inst.fixed[1, 1] = 0
    inst.f[:] = 0.0
    inst.f[1, 1] = (0.7, -1.9)
    u = solve(system_of(inst)).reshape(3, 3, 2)
    assert np.allclose(u[1, 1], np.array([0.7, -1.9]) / 3.0, atol=1e-15)


def test_affine_patch_test():
    """Unit EA, every boundary node prescribed u = A x + b, no interior load:
    the interior reproduces the affine field (opposite rods cancel)."""
    nx, ny = 12, 9
    inst = make_instance(nx, ny, seed=7)
    rng = np.random.default_rng(8)
    A, b = rng.standard_normal((2, 2)), rng.standard_normal(2)
    xy = positions(nx, ny)
    field = (xy @ A.T + b).reshape(ny, nx, 2)
    inst.fixed[:] = 0
    inst.fixed[[0, -1], :] = 1
    inst.fixed[:, [0, -1]] = 1
    inst.u_fixed[:] = np.where(inst.fixed[..., None].astype(bool), field, 0.0)
    inst.f[:] = 0.0
    u = solve(system_of(inst)).reshape(ny, nx, 2)
    assert np.abs(u - field).max() <= 1e-12 * np.abs(field).max()


# --------------------------------------------------------- solver and energy

def test_brute_force_dense_agrees_on_small_lattices():
    for (nx, ny, seed) in [(2, 2, 0), (4, 3, 1), (6, 7, 2), (10, 10, 3)]:
        inst = make_instance(nx, ny, seed=seed, ea="lognormal")
        S = system_of(inst)
        x = np.linalg.solve(S.Kff.toarray(), S.rhs)            # brute force
        for u in (solve_dense(S), solve_banded(S), solve_pcg(S, rtol=1e-14)):
            assert np.linalg.norm(u[S.free] - x) <= 1e-12 * np.linalg.norm(x)


def test_banded_and_pcg_agree_mid_size():
    inst = make_instance(48, 30, seed=9, ea="lognormal")
    S = system_of(inst)
    ub, up = solve_banded(S), solve_pcg(S, rtol=1e-13)
    assert np.linalg.norm(ub - up) <= 1e-10 * np.linalg.norm(ub)
    assert max(rel_residuals(S, ub)) <= 1e-12


def test_energy_identity_and_minimum():
    """Clapeyron: f.u* = u*.K.u*, so Pi(u*) = -1/2 f.u*; and u* is a minimum."""
    inst = make_instance(20, 16, seed=10, ea="lognormal")
    S = system_of(inst)
    u = solve(S)
    fu = S.f @ u
    assert u @ (S.K @ u) == pytest.approx(fu, rel=1e-12)
    assert energy(S, u) == pytest.approx(-0.5 * fu, rel=1e-12)
    rng = np.random.default_rng(11)
    for _ in range(3):
        v = rng.standard_normal(u.size) * S.free * 1e-3
        assert energy(S, u + v) > energy(S, u)


def test_relative_residual_of_zero_is_one_and_reactions_excluded():
    inst = make_instance(8, 6, seed=12)
    S = system_of(inst)
    R1, R2 = rel_residuals(S, np.zeros(S.f.size))
    assert R1 == pytest.approx(1.0) and R2 == pytest.approx(1.0)
    u = solve(S)
    assert np.all(residual(S, u)[~S.free] == 0.0)


# ------------------------------------------------------------ planted slips

def test_planted_wrong_bar_direction_is_caught(monkeypatch):
    """A sign slip in the third bar direction breaks the rotation null mode."""
    good = L.bar_unit_vector
    monkeypatch.setattr(L, "bar_unit_vector",
                        lambda d: (abs(good(d)[0]), good(d)[1]) if d == 2 else good(d))
    with pytest.raises(AssertionError):
        test_unconstrained_null_space_is_rigid_motion(5)


def test_planted_dropped_bar_is_caught(monkeypatch):
    """Forgetting the diagonal rods breaks the affine-energy closed form."""
    real = L.bar_list

    def no_diagonals(nx, ny, ea):
        a, b, k, n = real(nx, ny, ea)
        keep = n[:, 0] >= 0.0
        return a[keep], b[keep], k[keep], n[keep]
    monkeypatch.setattr(L, "bar_list", no_diagonals)
    with pytest.raises(AssertionError):
        test_affine_field_energy_closed_form("unit")


def test_planted_wrong_sign_in_offdiagonal_is_caught(monkeypatch):
    """Assembling +k_e off the diagonal (instead of -k_e) breaks the 2x2 hand solution."""
    import scipy.sparse as sp
    real = L.assemble

    def flipped(nx, ny, ea):
        K = real(nx, ny, ea).tocoo()
        blk_r, blk_c = K.row // 2, K.col // 2
        data = np.where(blk_r != blk_c, -K.data, K.data)
        return sp.csr_matrix((data, (K.row, K.col)), shape=K.shape)
    monkeypatch.setattr(L, "assemble", flipped)
    import oracle.solve as osolve
    monkeypatch.setattr(osolve, "assemble", flipped)
    with pytest.raises(AssertionError):
        test_2x2_compliance_matches_hand_derivation()


# ------------------------------------------------ Eq. 19 at a non-zero iterate

def _golden_residual_cases():
    cases = {}
    for line in (GOLDEN / "lattice_2x2_residual.txt").read_text().splitlines():
        if not line.strip() or line.startswith("#"):
            continue
        t = line.split()
        R1 = float(Fraction(t[1])) + float(Fraction(t[2])) * math.sqrt(3)
        R2 = math.sqrt(float(Fraction(t[3])))
        en = None if t[4] == "-" else float(Fraction(t[4]))
        cases[int(t[0])] = (R1, R2, en)
    return cases


def _case_2x2(case):
    """The two hand-derived states of tests/golden/lattice_2x2_residual.txt."""
    inst = make_instance(2, 2, seed=0)
    inst.f[:] = 0.0
    inst.f[0, 1] = (2.0, 1.0)                 # load on node A = (i=1, j=0)
    if case == 2:
        inst.u_fixed[0, 0] = (0.5, 0.0)       # clamped node O = (0, 0) prescribed
    S = system_of(inst)
    u = S.u_c.copy()
    u[2 * 1] = 1.0                            # u_A = (1, 0)
    return S, u


@pytest.mark.parametrize("case", [1, 2])
def test_relative_residuals_at_nonzero_iterate_match_hand_values(case):
    import oracle.solve as osolve
    R1, R2, en = _golden_residual_cases()[case]
    S, u = _case_2x2(case)
    got1, got2 = osolve.rel_residuals(S, u)
    assert got1 == pytest.approx(R1, rel=1e-14)
    assert got2 == pytest.approx(R2, rel=1e-14)
    if en is not None:
        assert osolve.energy(S, u) == pytest.approx(en, rel=1e-14)


def _plant(monkeypatch, fn):
    import oracle.solve as osolve
    monkeypatch.setattr(osolve, "rel_residuals", fn)


def test_planted_squared_r2_is_caught(monkeypatch):
    import oracle.solve as osolve
    real = osolve.rel_residuals
    _plant(monkeypatch, lambda S, u: (real(S, u)[0], real(S, u)[1] ** 2))
    with pytest.raises(AssertionError):
        test_relative_residuals_at_nonzero_iterate_match_hand_values(1)


def test_planted_max_norm_r1_is_caught(monkeypatch):
    import oracle.solve as osolve
    real = osolve.rel_residuals

    def max_norm(S, u):
        r = osolve.residual(S, u)[S.free]
        return float(np.abs(r).max() / np.abs(S.rhs).max()), real(S, u)[1]
    _plant(monkeypatch, max_norm)
    with pytest.raises(AssertionError):
        test_relative_residuals_at_nonzero_iterate_match_hand_values(1)


def test_planted_unconstrained_normaliser_is_caught(monkeypatch):
    """Dividing by the load f_f instead of the constrained right-hand side
    f_f - K_fc u_c (the two differ only with prescribed displacements)."""
    import oracle.solve as osolve
    real = osolve.rel_residuals

    def by_load(S, u):
        r = osolve.residual(S, u)[S.free]
        f = S.f[S.free]
        return (float(np.abs(r).sum() / np.abs(f).sum()),
                float(np.sqrt((r * r).sum() / (f * f).sum())))
    _plant(monkeypatch, by_load)
    with pytest.raises(AssertionError):
        test_relative_residuals_at_nonzero_iterate_match_hand_values(2)
