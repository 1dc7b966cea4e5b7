"""Plain solve of the lattice equations (oracle).

Test infrastructure only (see the package docstring).

The method converges to the unique minimiser of the total energy (Eq. 2),
i.e. to the solution of Eq. 1 restricted to the free DOFs:

    K_ff u_f = f_f - K_fc u_c ,      u = u_c on clamped DOFs,

with K_ff symmetric positive definite (section 2.1 assumes an SPD matrix;
clamping the left edge removes the rigid motions).  This module computes
that definition directly: dense Cholesky for small systems, banded Cholesky
(LAPACK, natural DOF order) for mid-size ones and block-Jacobi PCG for the
rest, with the final residual always recomputed from the assembled matrix.

Also: the relative residuals of Eq. 19 (1-norm, as the paper stops on, and
2-norm), both over free DOFs, and the energy of Eq. 2.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .lattice import assemble, free_mask


@dataclasses.dataclass
class System:
    """The constrained system of one instance."""
    K: sp.csr_matrix          # full 2N x 2N stiffness
    free: np.ndarray          # bool [2N]
    u_c: np.ndarray           # float64 [2N], prescribed values (0 on free DOFs)
    f: np.ndarray             # float64 [2N], loads (0 on clamped DOFs)

    @property
    def Kff(self) -> sp.csr_matrix:
        return self.K[self.free][:, self.free].tocsr()

    @property
    def rhs(self) -> np.ndarray:
        """f_f - K_fc u_c."""
        return (self.f - self.K @ self.u_c)[self.free]


def system_of(inst) -> System:
    free = free_mask(inst.fixed)
    u_c = np.where(free, 0.0, inst.u_fixed.reshape(-1))
    f = np.where(free, inst.f.reshape(-1), 0.0)
    return System(assemble(inst.nx, inst.ny, inst.ea), free, u_c, f)


def residual(sys_: System, u: np.ndarray) -> np.ndarray:
    """r = f - K u on free DOFs, 0 on clamped DOFs (reactions are not loads)."""
    r = sys_.f - sys_.K @ u
    r[~sys_.free] = 0.0
    return r


def rel_residuals(sys_: System, u: np.ndarray):
    """(R1, R2): ||f - K u|| / ||p|| over free DOFs in the 1- and 2-norm (Eq. 19).

    p is the right-hand side of the constrained system, f_f - K_fc u_c; with
    no prescribed displacement (the paper's setting) it is the load f."""
    r = residual(sys_, u)[sys_.free]
    f = sys_.rhs
    return (float(np.abs(r).sum() / np.abs(f).sum()),
            float(np.sqrt((r * r).sum()) / np.sqrt((f * f).sum())))


def energy(sys_: System, u: np.ndarray) -> float:
    """Total energy of Eq. 2, Pi = 1/2 u.K.u - u.p, with the clamped DOFs'
    prescribed values inside u and no load on them."""
    return float(0.5 * u @ (sys_.K @ u) - u @ sys_.f)


def _bandwidth(A: sp.csr_matrix) -> int:
    coo = A.tocoo()
    return int(np.abs(coo.row - coo.col).max()) if coo.nnz else 0


def solve_dense(sys_: System) -> np.ndarray:
    """Dense Cholesky of K_ff."""
    A = sys_.Kff.toarray()
    x = sla.cho_solve(sla.cho_factor(A, lower=True), sys_.rhs)
    u = sys_.u_c.copy()
    u[sys_.free] = x
    return u


def solve_banded(sys_: System) -> np.ndarray:
    """Banded Cholesky of K_ff in natural DOF order (LAPACK pbsv)."""
    A = sys_.Kff.tocoo()
    n = A.shape[0]
    bw = _bandwidth(A)
    ab = np.zeros((bw + 1, n))
    up = A.row <= A.col
    ab[bw + A.row[up] - A.col[up], A.col[up]] = A.data[up]
    x = sla.solveh_banded(ab, sys_.rhs, lower=False, check_finite=True)
    u = sys_.u_c.copy()
    u[sys_.free] = x
    return u


def block_jacobi(Kff: sp.csr_matrix):
    """Inverse of the 2x2 node-block diagonal of K_ff, as a callable.

    Free DOFs come in node pairs (a clamped node removes both of its DOFs),
    so the block of free DOFs (2k, 2k+1) is one node's."""
    d = Kff.diagonal()
    off = np.asarray(Kff[np.arange(0, Kff.shape[0], 2), np.arange(1, Kff.shape[0], 2)]).ravel()
    a, c = d[0::2], d[1::2]
    det = a * c - off * off

    def apply(r):
        rx, ry = r[0::2], r[1::2]
        z = np.empty_like(r)
        z[0::2] = (c * rx - off * ry) / det
        z[1::2] = (a * ry - off * rx) / det
        return z
    return apply


def solve_pcg(sys_: System, rtol: float = 1e-13, maxiter: int = 10_000_000,
              x0: np.ndarray | None = None, max_seconds: float | None = None,
              history: list | None = None) -> np.ndarray:
    """Block-Jacobi preconditioned CG on K_ff from x0 (default 0).

    Stops when the recomputed relative 2-norm residual ||b - K x|| / ||b||
    is <= rtol; the recurrence residual only triggers the recomputation.
    ``history`` (optional) receives (iteration, recurrence relative residual).
    ``max_seconds`` bounds the run (the result is then not converged)."""
    import time
    A = sys_.Kff
    b = sys_.rhs
    M = block_jacobi(A)
    x = np.zeros_like(b) if x0 is None else x0[sys_.free].copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        u = sys_.u_c.copy()
        return u
    t0 = time.perf_counter()
    r = b - A @ x
    it = 0
    while it < maxiter:
        z = M(r)
        p = z.copy()
        rz = r @ z
        while it < maxiter:
            q = A @ p
            alpha = rz / (p @ q)
            x += alpha * p
            r -= alpha * q
            it += 1
            rel = np.linalg.norm(r) / bnorm
            if history is not None:
                history.append((it, rel))
            if rel <= rtol:
                break
            if max_seconds is not None and time.perf_counter() - t0 > max_seconds:
                break
            z = M(r)
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
        r = b - A @ x                     # explicit recomputation
        if np.linalg.norm(r) / bnorm <= rtol:
            break
        if max_seconds is not None and time.perf_counter() - t0 > max_seconds:
            break
    u = sys_.u_c.copy()
    u[sys_.free] = x
    return u


def solve(sys_: System, rtol: float = 1e-13) -> np.ndarray:
    """u* of the constrained Eq. 1 by the cheapest exact route for its size."""
    n = int(sys_.free.sum())
    if n <= 6000:
        return solve_dense(sys_)
    bw = _bandwidth(sys_.Kff)
    if n * (bw + 1) * 8 <= 6 << 30 and n * bw * bw <= 1e12:
        return solve_banded(sys_)
    return solve_pcg(sys_, rtol=rtol)
