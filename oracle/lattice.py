"""Triangle-lattice truss: geometry and assembled stiffness (oracle).

Test infrastructure only (see the package docstring).

The paper's test problem (section 3.1) is a 2-D triangle-lattice truss whose
nodes are joined to their neighbours by elastic rods; its stiffness comes
from standard FEM.  A rod of axial stiffness EA and length L along unit
vector n contributes the element matrix (EA/L) n n^T, assembled as
[[k_e, -k_e], [-k_e, k_e]] on its two end nodes.  The global matrix of
Eq. 1 is the sum of these blocks; it has 2 DOFs per node (s = 2).

DOF numbering: dof = 2 * (j * nx + i) + c, c = 0 for x and 1 for y.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

# Forward bars stored at node (i, j): (di, dj) of the other end.  The unit
# vector of each follows from the node positions (i + j/2, j*sqrt(3)/2)
# and is evaluated below from those positions, not typed in.
BAR_OFFSETS = ((1, 0), (0, 1), (-1, 1))
SQRT3_HALF = math.sqrt(3.0) / 2.0


def node_xy(nx: int, ny: int):
    """Physical coordinates x[j, i], y[j, i] of every node."""
    j, i = np.meshgrid(np.arange(ny, dtype=np.float64),
                       np.arange(nx, dtype=np.float64), indexing="ij")
    return i + 0.5 * j, SQRT3_HALF * j


def bar_unit_vector(d: int):
    """Unit vector from node (i, j) towards the other end of forward bar d.

    Taken from the coordinate difference of the two end nodes; the rod length
    of every nearest-neighbour bar is exactly 1, which the pins check."""
    di, dj = BAR_OFFSETS[d]
    return (di + 0.5 * dj, SQRT3_HALF * dj)


def bar_list(nx: int, ny: int, ea: np.ndarray):
    """All rods of the lattice as flat arrays.

    Returns (a, b, k, n): end node ids a -> b, axial stiffness k = EA / L with
    L = 1, and unit vector n (shape [nbars, 2]) pointing from a to b.  A rod
    exists when both ends lie in the lattice; its EA is read from the plane
    of the end that stores it."""
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    A, B, K, N = [], [], [], []
    for d, (di, dj) in enumerate(BAR_OFFSETS):
        I2, J2 = I + di, J + dj
        inside = (I2 >= 0) & (I2 < nx) & (J2 >= 0) & (J2 < ny)
        A.append((J * nx + I)[inside])
        B.append((J2 * nx + I2)[inside])
        K.append(ea[d][inside].astype(np.float64))
        N.append(np.tile(np.asarray(bar_unit_vector(d)), (int(inside.sum()), 1)))
    return (np.concatenate(A).astype(np.int64), np.concatenate(B).astype(np.int64),
            np.concatenate(K), np.concatenate(N).reshape(-1, 2))


def assemble(nx: int, ny: int, ea: np.ndarray) -> sp.csr_matrix:
    """Global stiffness K of Eq. 1 (2*nx*ny square, CSR, duplicates summed)."""
    a, b, k, n = bar_list(nx, ny, ea)
    rows, cols, vals = [], [], []
    for c1 in range(2):
        for c2 in range(2):
            ke = k * (n[:, c1] * n[:, c2])          # (EA/L) n n^T entry
            for p, q, s in ((a, a, 1.0), (b, b, 1.0), (a, b, -1.0), (b, a, -1.0)):
                rows.append(2 * p + c1)
                cols.append(2 * q + c2)
                vals.append(s * ke)
    ndof = 2 * nx * ny
    r, c, v = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    # Sum duplicates in a fixed order (the order the element blocks were
    # listed), so that mirrored entries add the same terms in the same order.
    order = np.argsort(r * ndof + c, kind="stable")
    r, c, v = r[order], c[order], v[order]
    key = r * ndof + c
    start = np.flatnonzero(np.r_[True, key[1:] != key[:-1]])
    rows_u, cols_u = r[start], c[start]              # sorted by (row, col), unique
    indptr = np.r_[0, np.cumsum(np.bincount(rows_u, minlength=ndof))]
    return sp.csr_matrix((np.add.reduceat(v, start), cols_u, indptr), shape=(ndof, ndof))


def free_mask(fixed: np.ndarray) -> np.ndarray:
    """Boolean over DOFs: True where the DOF is free (its node is not clamped)."""
    return np.repeat(~fixed.astype(bool).reshape(-1), 2)
