"""The hierarchical master/slave iteration, step by step (oracle).

Test infrastructure only (see the package docstring).

One outer iteration, in the paper's order (section 2, section 3 flowchart
description):

  1. residual of the current displacement and the stop test of Eq. 19;
  2. per set I, local relaxation with the displacements outside the set held
     at their last values (Eq. 11-12), giving the relaxation increment
     u^RD - u^old (Eq. 13);
  3. the q = 9 incremental modes of every set: translations (Eq. 9),
     constant-gradient modes about the set's representative node (Eq. 10),
     the relaxation increment and its two gradient-weighted copies (Eq. 13-14);
     with q = 12 also the increment of the relaxation with fixed-force
     boundary and its two gradient-weighted copies (Eq. 15-18);
  4. upper-level stiffness K_a = U^T K U (Eq. 6) and force
     P_a = U^T (p - K u^old) (Eq. 7);
  5. solve the upper-level system (Eq. 8);
  6. update u = u^old + U a (Eq. 3).

Both inner solves are exact here, as in the paper (a direct sparse solver
for the local relaxation, section 2.2 end; a single-processor solver for the
upper level, section 2.1).  Sets are E x E node tiles of the (i, j) index
grid; the last row/column of tiles is narrower when E does not divide the
lattice side.  Every mode is zero on clamped DOFs, so supports never move.

Readings where the paper is silent (stated, not derived):
  * the fixed-force relaxation (Eq. 15-17) isolates the same region as the
    fixed-displacement one: every rod that crosses the region's edge is cut
    (Eq. 15 moves its coupling onto the diagonal with the opposite sign),
    rods to clamped nodes inside the region stay; where the isolated region
    can move rigidly (no clamped node inside it) Eq. 16 is singular and in
    general inconsistent, and its minimum-norm least-squares solution is
    taken, i.e. the right-hand side and the increment are both taken off
    the region's rigid motions (which modes 1-6 already represent);
  * representative node of a set = centroid of the tile's nodes in physical
    coordinates, and the gradient modes are scaled by 1/(E/2); in exact
    arithmetic neither choice changes the iterates (span{1, x - c} =
    span{1, x}, span{d, (x - c) d} = span{d, x d});
  * the upper-level matrix can be singular (dependent modes, e.g. a set
    whose relaxation increment is zero); it is consistent, so its
    minimum-norm solution is taken after a symmetric Jacobi scaling, and
    U a is then the same for every minimiser.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .lattice import node_xy
from .solve import System, energy, rel_residuals, residual

Q = 9   # modes per set on the hot path: Eq. 9 (2), Eq. 10 (4), Eq. 13-14 (3)
Q12 = 12  # with the fixed-force relaxation modes of Eq. 17-18


@dataclasses.dataclass
class Sets:
    nx: int
    ny: int
    E: int
    mx: int                  # tiles along i
    my: int                  # tiles along j
    of_node: np.ndarray      # int [ny*nx] set id of every node, id = J*mx + I
    xc: np.ndarray           # float [M] representative node x
    yc: np.ndarray           # float [M] representative node y
    scale: float             # gradient-mode length scale

    @property
    def M(self) -> int:
        return self.mx * self.my


def make_sets(nx: int, ny: int, E: int, rep_shift=(0.0, 0.0)) -> Sets:
    """E x E tiles of the node index grid; the representative node is the
    tile's centroid, optionally shifted by rep_shift (for invariance checks)."""
    mx, my = -(-nx // E), -(-ny // E)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    of_node = ((j // E) * mx + (i // E)).reshape(-1)
    x, y = node_xy(nx, ny)
    M = mx * my
    cnt = np.bincount(of_node, minlength=M).astype(np.float64)
    xc = np.bincount(of_node, weights=x.reshape(-1), minlength=M) / cnt + rep_shift[0]
    yc = np.bincount(of_node, weights=y.reshape(-1), minlength=M) / cnt + rep_shift[1]
    return Sets(nx, ny, E, mx, my, of_node, xc, yc, E / 2.0)


def relaxation_region(sets: Sets, I: int, overlap: int) -> np.ndarray:
    """Node ids of set I's relaxation region: its tile, widened by `overlap`
    nodes on every side in index space and clipped to the lattice (section
    2.2 end: relaxing a larger region around the set)."""
    E, nx, ny = sets.E, sets.nx, sets.ny
    i0, j0 = (I % sets.mx) * E, (I // sets.mx) * E
    i1, j1 = min(i0 + E, nx), min(j0 + E, ny)
    a0, a1 = max(i0 - overlap, 0), min(i1 + overlap, nx)
    b0, b1 = max(j0 - overlap, 0), min(j1 + overlap, ny)
    jj, ii = np.meshgrid(np.arange(b0, b1), np.arange(a0, a1), indexing="ij")
    return (jj * nx + ii).reshape(-1)


class LocalSolver:
    """Exact local relaxation of Eq. 12 for every set.

    For set I, k^Inner is the block of K on the free DOFs of the relaxation
    region (its entries are those of the global matrix, section 2.2), so
        k^Inner u^RD = p^Inner - k^Outer u^Outer,old
    gives u^RD - u^old = (k^Inner)^-1 (p - K u^old)|_region.  With overlap 0
    the region is the set itself; with overlap w > 0 it is the set widened by
    w nodes (section 2.2 end) and the increment is kept on the set's own
    DOFs only, so the modes of different sets still have disjoint supports.
    The factors are computed once and reused, as section 2.2 describes."""

    def __init__(self, sys_: System, sets: Sets, overlap: int = 0):
        self.idx = []      # region free DOFs
        self.own = []      # positions (within idx) of the set's own DOFs
        self.lu = []
        dof_set = np.repeat(sets.of_node, 2)
        for I in range(sets.M):
            nodes = relaxation_region(sets, I, overlap)
            dofs = np.sort(np.concatenate([2 * nodes, 2 * nodes + 1]))
            idx = dofs[sys_.free[dofs]]
            self.idx.append(idx)
            self.own.append(np.flatnonzero(dof_set[idx] == I))
            if idx.size:
                kin = sys_.K[idx][:, idx].tocsc()
                self.lu.append(spla.splu(kin))
            else:
                self.lu.append(None)

    def relax(self, r: np.ndarray) -> np.ndarray:
        """Relaxation increment (Eq. 13) of every set, stacked into one vector."""
        d = np.zeros_like(r)
        for idx, own, lu in zip(self.idx, self.own, self.lu):
            if lu is not None:
                d[idx[own]] = lu.solve(r[idx])[own]
        return d


def isolation_correction(K: sp.csr_matrix, idx: np.ndarray, inside: np.ndarray) -> sp.csr_matrix:
    """Delta k of Eq. 15 on the region's free DOFs idx: block diagonal, the
    2 x 2 block of node i the sum of K's (i, l) blocks over every node l
    outside the region (inside: bool per node)."""
    rows = K[idx].tocoo()
    out = ~inside[rows.col // 2]
    sums = np.zeros((idx.size, 2))
    np.add.at(sums, (rows.row[out], rows.col[out] % 2), rows.data[out])
    pos = {int(d): k for k, d in enumerate(idx)}
    r, c, v = [], [], []
    for k, d in enumerate(idx):
        base = 2 * (int(d) // 2)
        for cp in range(2):
            r.append(k)
            c.append(pos[base + cp])
            v.append(sums[k, cp])
    return sp.csr_matrix((v, (r, c)), shape=(idx.size, idx.size))


class ForceLocalSolver:
    """Exact local relaxation with fixed-force boundary (Eq. 15-17) for every
    set, on the same region as LocalSolver.

    (k^Inner + Delta k) is the stiffness of the isolated region (Eq. 15).
    Subtracting (k^Inner + Delta k) u^Inner,old from both sides of Eq. 16
    gives the increment of Eq. 17 directly:
        (k^Inner + Delta k) (u^RF - u^old) = (p - K u^old)|_region,
    whose right-hand side is the residual on the region.  Where the isolated
    stiffness is singular, the minimum-norm solution is taken: with N an
    orthonormal basis of what it does not resist (the region's rigid motions,
    and for a region one node thick also the motions across the strip), the
    bordered system
        [[K_iso, N], [N^T, 0]] [x; l] = [r; 0]
    gives K_iso x = r - N N^T r with N^T x = 0.  Factors are computed once and
    reused.  The increment is kept on the set's own DOFs."""

    def __init__(self, sys_: System, sets: Sets, overlap: int = 0):
        self.idx, self.own, self.lu, self.kiso, self.dk, self.null = [], [], [], [], [], []
        dof_set = np.repeat(sets.of_node, 2)
        K = sys_.K.tocsr()
        x, y = node_xy(sets.nx, sets.ny)
        x, y = x.reshape(-1), y.reshape(-1)
        nn = sets.nx * sets.ny
        for I in range(sets.M):
            nodes = relaxation_region(sets, I, overlap)
            inside = np.zeros(nn, dtype=bool)
            inside[nodes] = True
            dofs = np.sort(np.concatenate([2 * nodes, 2 * nodes + 1]))
            idx = dofs[sys_.free[dofs]]
            self.idx.append(idx)
            self.own.append(np.flatnonzero(dof_set[idx] == I))
            if idx.size == 0:
                for lst in (self.lu, self.kiso, self.dk, self.null):
                    lst.append(None)
                continue
            dk = isolation_correction(K, idx, inside)
            kiso = (K[idx][:, idx] + dk).tocsc()
            N = self._null_space(kiso, idx, x, y)
            self.dk.append(dk)
            self.kiso.append(kiso)
            self.null.append(N)
            if N.shape[1]:
                Nsp = sp.csc_matrix(N)
                A = sp.bmat([[kiso, Nsp], [Nsp.T, None]], format="csc")
                self.lu.append(spla.splu(A))
            else:
                self.lu.append(spla.splu(kiso))

    @staticmethod
    def _null_space(kiso, idx, x, y):
        """Orthonormal basis of the displacements of the region's free DOFs
        that kiso does not resist.  A region of at most 256 free DOFs, which
        includes every region one node thick (a strip of rods along one line
        resists nothing across it, a mechanism beyond the rigid motions),
        takes it from kiso's dense eigenvectors; a larger region, at least
        two nodes thick and so triangulated, can only move rigidly, and the
        rigid motions are tested."""
        if idx.size <= 256:
            scale = abs(kiso).sum(axis=1).max()
            w, V = np.linalg.eigh(kiso.toarray())
            return V[:, w <= 1e-10 * scale]
        return ForceLocalSolver._rigid_null_space(kiso, idx, x, y)

    @staticmethod
    def _rigid_null_space(kiso, idx, x, y):
        """Orthonormal basis of the rigid motions (two translations, rotation
        about the region's centroid) of the region's free nodes that kiso
        does not resist."""
        node = idx // 2
        comp = idx % 2
        xc, yc = x[node].mean(), y[node].mean()
        cand = np.stack([comp == 0, comp == 1,
                         np.where(comp == 0, -(y[node] - yc), x[node] - xc)], 1).astype(float)
        cand /= np.linalg.norm(cand, axis=0)
        KN = kiso @ cand
        _, sv, Vt = np.linalg.svd(KN, full_matrices=True)
        scale = abs(kiso).sum(axis=1).max()
        sv = np.concatenate([sv, np.zeros(3 - sv.size)])
        V = Vt.T[:, sv <= 1e-10 * scale]
        if V.shape[1] == 0:
            return np.zeros((idx.size, 0))
        Q, _ = np.linalg.qr(cand @ V)
        return Q

    def relax_region(self, I: int, r: np.ndarray) -> np.ndarray:
        """The increment on set I's whole region (free DOFs self.idx[I])."""
        idx, lu, N = self.idx[I], self.lu[I], self.null[I]
        if lu is None:
            return np.zeros(0)
        rhs = r[idx]
        if N.shape[1]:
            return lu.solve(np.concatenate([rhs, np.zeros(N.shape[1])]))[:idx.size]
        return lu.solve(rhs)

    def relax(self, r: np.ndarray) -> np.ndarray:
        """Fixed-force relaxation increment (Eq. 17) of every set, stacked."""
        d = np.zeros_like(r)
        for I, (idx, own) in enumerate(zip(self.idx, self.own)):
            if self.lu[I] is not None:
                d[idx[own]] = self.relax_region(I, r)[own]
        return d


def mode_matrix(sys_: System, sets: Sets, delta: np.ndarray,
                delta_f: np.ndarray | None = None) -> sp.csr_matrix:
    """U = [u_hat_k^(I)] as a sparse 2N x (q*M) matrix, column q*I + (k-1),
    q = 9, or 12 when the fixed-force increment delta_f is given.

    Modes 1-2 translations (Eq. 9); 3-6 (x - x_I, 0), (y - y_I, 0),
    (0, x - x_I), (0, y - y_I) (Eq. 10), scaled; 7 the relaxation increment
    (Eq. 13); 8-9 its copies weighted by (x - x_I) and (y - y_I) (Eq. 14);
    10 the fixed-force increment (Eq. 17); 11-12 its weighted copies (Eq. 18)."""
    q = Q if delta_f is None else Q12
    nn = sets.nx * sets.ny
    x, y = node_xy(sets.nx, sets.ny)
    I = sets.of_node
    xi = (x.reshape(-1) - sets.xc[I]) / sets.scale
    eta = (y.reshape(-1) - sets.yc[I]) / sets.scale
    free_node = sys_.free[0::2]
    dx, dy = delta[0::2], delta[1::2]
    one, zero = np.ones(nn), np.zeros(nn)
    comps = [  # (x-component, y-component) of modes 1..9 at every node
        (one, zero), (zero, one),
        (xi, zero), (eta, zero), (zero, xi), (zero, eta),
        (dx, dy), (xi * dx, xi * dy), (eta * dx, eta * dy),
    ]
    if delta_f is not None:
        fx, fy = delta_f[0::2], delta_f[1::2]
        comps += [(fx, fy), (xi * fx, xi * fy), (eta * fx, eta * fy)]
    rows, cols, vals = [], [], []
    node = np.arange(nn)
    for k, (cx, cy) in enumerate(comps):
        for c, comp in ((0, cx), (1, cy)):
            v = np.where(free_node, comp, 0.0)
            nz = v != 0.0
            rows.append(2 * node[nz] + c)
            cols.append(q * I[nz] + k)
            vals.append(v[nz])
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(2 * nn, q * sets.M)).tocsr()


def upper_level(sys_: System, U: sp.csr_matrix, u_old: np.ndarray):
    """K_a = U^T K U (Eq. 6) and P_a = U^T (p - K u^old) (Eq. 7)."""
    Kc = (U.T @ (sys_.K @ U)).toarray()
    P = U.T @ residual(sys_, u_old)
    return Kc, P


def solve_upper(Kc: np.ndarray, P: np.ndarray, rcond: float = 1e-13) -> np.ndarray:
    """Minimum-norm solution of Eq. 8 after symmetric Jacobi scaling.

    K_a is symmetric positive semidefinite and P lies in its range, so every
    least-squares solution is exact and all give the same U a."""
    d = np.diag(Kc).copy()
    s = np.where(d > 0.0, 1.0 / np.sqrt(np.where(d > 0.0, d, 1.0)), 0.0)
    Ks = Kc * s[:, None] * s[None, :]
    w, V = sla.eigh(Ks)
    keep = w > rcond * max(w.max(), 0.0)
    y = V[:, keep] @ ((V[:, keep].T @ (P * s)) / w[keep])
    return s * y


@dataclasses.dataclass
class Step:
    """Every intermediate quantity of one outer iteration."""
    r: np.ndarray            # residual at u_old
    R1: float
    R2: float
    delta: np.ndarray        # relaxation increments (Eq. 13)
    delta_f: np.ndarray | None   # fixed-force relaxation increments (Eq. 17), q = 12
    U: sp.csr_matrix         # modes
    Kc: np.ndarray           # Eq. 6
    P: np.ndarray            # Eq. 7
    a: np.ndarray            # Eq. 8
    u_new: np.ndarray        # Eq. 3


class Method:
    """Outer loop of the hierarchical solver with exact inner solves."""

    def __init__(self, sys_: System, sets: Sets, overlap: int = 0, modes: int = Q):
        if modes not in (Q, Q12):
            raise ValueError("modes must be 9 or 12")
        self.sys = sys_
        self.sets = sets
        self.q = modes
        self.local = LocalSolver(sys_, sets, overlap)
        self.local_f = ForceLocalSolver(sys_, sets, overlap) if modes == Q12 else None

    def step(self, u_old: np.ndarray) -> Step:
        r = residual(self.sys, u_old)
        R1, R2 = rel_residuals(self.sys, u_old)
        delta = self.local.relax(r)
        delta_f = self.local_f.relax(r) if self.local_f is not None else None
        U = mode_matrix(self.sys, self.sets, delta, delta_f)
        Kc, P = upper_level(self.sys, U, u_old)
        a = solve_upper(Kc, P)
        return Step(r, R1, R2, delta, delta_f, U, Kc, P, a, u_old + U @ a)

    def run(self, tol: float, max_iters: int, u0: np.ndarray | None = None):
        """Iterate from u0 (default: prescribed values, zero elsewhere) until
        max(R1, R2) <= tol.  Returns (u, iterations, history), history rows
        (R1, R2, energy) per iteration before its update."""
        u = self.sys.u_c.copy() if u0 is None else u0.copy()
        hist = []
        for it in range(max_iters + 1):
            R1, R2 = rel_residuals(self.sys, u)
            hist.append((R1, R2, energy(self.sys, u)))
            if max(R1, R2) <= tol or it == max_iters:
                return u, it, hist
            u = self.step(u).u_new
        return u, max_iters, hist
