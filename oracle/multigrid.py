"""Aggregation multigrid preconditioner (oracle, FP64).

Test infrastructure: a plain CPU statement of the multigrid V-cycle the
library offers as a preconditioner of the projection's conjugate-gradient
solve (Introduction: preconditioned conjugate gradients; the preconditioner
is not named -- Jacobi is the default, this is the stronger option).

Hierarchy.  Level 0 is the merged operator A' over the reduced unknowns (the
cells that carry an unknown).  A level's cells are aggregated in blocks of
2 x 2 x 2 (the last block along an odd axis holds one layer); an unknown of
level 0 belongs to the block of its own cell.  With P_l the 0/1 matrix that
maps a block to its unknowns, the next operator is the Galerkin product
A_{l+1} = P_l^T A_l P_l, kept on the full block grid (blocks without an
unknown have empty rows).  There is always at least one coarse level.  Couplings of A_1 between blocks that are not
neighbours (|offset| > 1 along an axis, possible only through long merge
chains) are dropped, the diagonal kept -- each such face then adds a
positive semidefinite term, so A_1 stays symmetric positive semidefinite;
coarser levels are exact Galerkin products (their couplings never reach
further).  Coarsening stops at `min_coarse` cells or fewer.

V-cycle (symmetric, so it preconditions CG): on level l with right-hand
side r,
    z = omega D^-1 r;  r_c = P^T (r - A z);  z += alpha P V(r_c);
    z += omega D^-1 (r - A z)
with D the diagonal (rows without an unknown get z = 0) and alpha the scale
of the coarse correction (1: the plain cycle; 0 < alpha < 2 keeps the cycle
symmetric positive definite, since the coarse step then contracts in the
energy norm).

With coef="bf16" the cycle's level 0 applies the operator assembled from
the face coefficients rounded to FP32 and then to BF16 (nearest even), and
smooths with D^-1 rounded the same way; level 1 is still the Galerkin
product of the exact operator.  The cycle stays symmetric (each face keeps
one coefficient).  The coarsest level
is solved exactly: empty rows become identity rows and, when every boundary
is Neumann, c v v^T is added (v the indicator of the non-empty rows, c their
mean diagonal), which leaves A x = b for every compatible b.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

OMEGA = 0.9
ALPHA = 1.0
MIN_COARSE = 600


def _blocks(shape):
    nz, ny, nx = shape
    cz, cy, cx = (nz + 1) // 2, (ny + 1) // 2, (nx + 1) // 2
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    blk = ((k // 2) * cy + j // 2) * cx + i // 2
    return blk.reshape(-1), (cz, cy, cx)


def _drop_far(A, shape):
    """Remove the off-diagonal entries between blocks more than one apart
    along an axis (the diagonal is kept)."""
    nz, ny, nx = shape
    A = A.tocoo()
    rk, rem = np.divmod(A.row, nx * ny)
    rj, ri = np.divmod(rem, nx)
    ck, rem = np.divmod(A.col, nx * ny)
    cj, ci = np.divmod(rem, nx)
    near = (np.abs(rk - ck) <= 1) & (np.abs(rj - cj) <= 1) & (np.abs(ri - ci) <= 1)
    return sp.csr_matrix((A.data[near], (A.row[near], A.col[near])), shape=A.shape), int(np.count_nonzero(~near))


def bf16(x):
    """Round to FP32, then to the nearest BF16 (ties to even); float64 values."""
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


class Hierarchy:
    """Operators, shapes and aggregation maps of every level."""

    def __init__(self, op, min_coarse=MIN_COARSE, omega=OMEGA, alpha=ALPHA, coef="f64"):
        self.op = op
        self.omega = omega
        self.alpha = alpha
        g = op.grid
        shape = g.shape
        A = op.csr()
        red = op.reduced_mask().reshape(-1) > 0
        self.A, self.shapes, self.maps = [A], [shape], []
        self.dropped = 0
        rows_mask = red
        while (len(self.A) == 1 or A.shape[0] > min_coarse) and max(shape) > 1:
            blk, cshape = _blocks(shape)
            nc = int(np.prod(cshape))
            rows = np.nonzero(rows_mask)[0]
            P = sp.csr_matrix((np.ones(len(rows)), (rows, blk[rows])), shape=(A.shape[0], nc))
            Ac = (P.T @ A @ P).tocsr()
            Ac, nd = _drop_far(Ac, cshape)
            self.dropped += nd
            self.maps.append(P)
            self.A.append(Ac)
            self.shapes.append(cshape)
            A, shape = Ac, cshape
            rows_mask = np.ones(nc, dtype=bool)
        self.diag = [a.diagonal() for a in self.A]
        self.dinv = [np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0) for d in self.diag]
        self.coarse_inv = self._coarsest(g.all_neumann)
        if coef == "bf16":
            # the cycle's level 0 (the coarse levels above were built exactly)
            self.A[0] = op.csr(coeffs=(bf16(op.tx), bf16(op.ty), bf16(op.tz)))
            self.dinv[0] = bf16(op.dinv).reshape(-1)
        elif coef != "f64":
            raise ValueError("coef must be 'f64' or 'bf16'")

    def _coarsest(self, singular):
        A = self.A[-1].toarray()
        d = np.diag(A).copy()
        empty = ~(d > 0)
        M = A.copy()
        if singular and np.any(~empty):
            v = (~empty).astype(np.float64)
            M = M + np.mean(d[~empty]) * np.outer(v, v)
        M[empty, :] = 0.0
        M[:, empty] = 0.0
        M[empty, empty] = 1.0
        return np.linalg.inv(M)

    def vcycle(self, r, level=0):
        if level == len(self.A) - 1:
            return self.coarse_inv @ r
        A, P, dinv, w = self.A[level], self.maps[level], self.dinv[level], self.omega
        z = w * (dinv * r)
        rc = P.T @ (r - A @ z)
        z = z + self.alpha * (P @ self.vcycle(rc, level + 1))
        return z + w * (dinv * (r - A @ z))

    def precond(self, r):
        """z = V(r) on cell arrays (zeros off the reduced unknowns)."""
        shape = np.shape(r)
        return self.vcycle(np.asarray(r, dtype=np.float64).reshape(-1)).reshape(shape)
