"""Krylov solvers for the merged pressure system A' x = b' (oracle).

The paper solves the Poisson equation by a preconditioned conjugate-gradient
method (Introduction) without naming the preconditioner; the reading taken
is Jacobi, M = diag(A').  Vectors live on the cell array: the solution and
search directions are expanded (slaves carry their root's value), residuals
are gathered (slaves zero), so every dot product over all cells equals the
dot product over the reduced unknowns.  Dots are np.add.reduce(a*b)
(pairwise, single thread), never BLAS.

Stopping: recursive ||r||/||b'|| <= tol, then the true residual b' - A'x is
recomputed; if it is above tol the iteration restarts from x (at most three
times).  The reported relative residual is always the true one.

Residual replacement (the scheme the GPU's mixed-precision solve runs, here
in FP64): whenever the recursive residual has fallen by `drop` since the last
replacement, it is replaced by the true residual b' - A'x and CG goes on with
the same direction; the next direction's beta divides the replaced residual's
r.z by the r.z the recursion's own beta divides by, so in exact arithmetic
the iteration is CG's.

Flexible CG follows Notay's truncated FCG(m): the new direction is the
preconditioned residual A'-orthogonalised against the last m directions, and
the step is alpha = (p.r)/(p.q).  A stagnation monitor switches once to
Jacobi-PCG from the current iterate when the mean residual reduction factor
over a window of W iterations exceeds `ratio`.
"""
from __future__ import annotations

import math

import numpy as np


def dot(a, b):
    return float(np.add.reduce((np.asarray(a) * np.asarray(b)).ravel()))


def norm(a):
    return math.sqrt(dot(a, a))


class Result:
    def __init__(self, x, iterations, relres, history, fallback=False, restarts=0):
        self.x, self.iterations, self.relres = x, iterations, relres
        self.history, self.fallback, self.restarts = history, fallback, restarts


def true_relres(op, b, x):
    return norm(b - op.apply(x)) / norm(b)


def pcg(op, b, x0=None, tol=1e-10, maxit=100000, precond="jacobi", max_restarts=3,
        record=None, callback=None):
    """Jacobi (or unpreconditioned) CG on A' x = b'.

    record: optional list of iteration numbers k at which (x_k, r_k) copies
    are appended to `callback(k, x, r)`.
    """
    b = np.asarray(b, dtype=np.float64)
    bnorm = norm(b)
    x = np.zeros_like(b) if x0 is None else op.expand(np.array(x0, dtype=np.float64))
    if bnorm == 0.0:
        return Result(np.zeros_like(b), 0, 0.0, [0.0])
    if precond == "jacobi":
        M = lambda r: op.expand(op.dinv * r)
    elif precond == "none":
        M = lambda r: op.expand(r)
    else:
        raise ValueError(precond)
    history = []
    it = 0
    restarts = 0
    while True:
        r = b - op.apply(x)
        rn = norm(r)
        history.append(rn / bnorm)
        if rn / bnorm <= tol or it >= maxit:
            return Result(x, it, rn / bnorm, history, restarts=restarts)
        if restarts > max_restarts:
            return Result(x, it, rn / bnorm, history, restarts=restarts)
        z = M(r)
        p = z.copy()
        rz = dot(r, z)
        while it < maxit:
            if callback is not None and record is not None and it in record:
                callback(it, x.copy(), r.copy())
            q = op.apply(p)
            pq = dot(p, q)
            if pq <= 0.0:
                break
            alpha = rz / pq
            x = x + alpha * p
            r = r - alpha * q
            it += 1
            rn = norm(r)
            history.append(rn / bnorm)
            if rn / bnorm <= tol:
                break
            z = M(r)
            rz_new = dot(r, z)
            beta = rz_new / rz
            rz = rz_new
            p = z + beta * p
        restarts += 1


def pcg_replaced(op, b, tol=1e-8, drop=0.1, maxit=100000):
    """Jacobi-PCG (Introduction) with residual replacement every `drop` of
    reduction.  Returns the Result with `restarts` = the number of true
    residuals formed after the first."""
    b = np.asarray(b, dtype=np.float64)
    bnorm = norm(b)
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return Result(x, 0, 0.0, [0.0])
    M = lambda v: op.expand(op.dinv * v)
    r = b - op.apply(x)
    p = np.zeros_like(b)
    history, it, replaced = [], 0, -1
    rz_prev = None            # r.z before the last update: beta's denominator
    while True:
        replaced += 1
        rn = norm(r)
        history.append(rn / bnorm)
        if rn / bnorm <= tol or it >= maxit:
            return Result(x, it, rn / bnorm, history, restarts=replaced)
        z = M(r)
        rz = dot(r, z)
        rr_ref = rn * rn
        beta = 0.0 if rz_prev is None else rz / rz_prev
        while it < maxit:
            p = z + beta * p
            q = op.apply(p)
            pq = dot(p, q)
            if pq <= 0.0:
                break
            alpha = rz / pq
            x = x + alpha * p
            r = r - alpha * q
            it += 1
            z = M(r)
            rzn = dot(r, z)
            beta = rzn / rz
            rz_prev, rz = rz, rzn
            rr = dot(r, r)
            if rr <= drop * drop * rr_ref or math.sqrt(rr) / bnorm <= tol:
                break
        r = b - op.apply(x)


def fcg(op, b, precond, x0=None, tol=1e-8, maxit=100000, m=1, ratio=0.99, window=10,
        fallback=True):
    """Flexible CG (Notay FCG(m)) with an arbitrary preconditioner callable
    z = precond(r) (cell arrays), a stagnation fallback to Jacobi-PCG, and a
    true-residual check."""
    b = np.asarray(b, dtype=np.float64)
    bnorm = norm(b)
    x = np.zeros_like(b) if x0 is None else op.expand(np.array(x0, dtype=np.float64))
    if bnorm == 0.0:
        return Result(np.zeros_like(b), 0, 0.0, [0.0])
    r = b - op.apply(x)
    hist = [norm(r) / bnorm]
    P, Q, PQ = [], [], []
    it = 0
    while it < maxit:
        if hist[-1] <= tol:
            tr = true_relres(op, b, x)
            if tr <= tol:
                return Result(x, it, tr, hist)
            r = b - op.apply(x)
            P, Q, PQ = [], [], []
        z = op.expand(precond(r))
        p = z.copy()
        for pj, qj, pqj in zip(P, Q, PQ):
            p = p - (dot(z, qj) / pqj) * pj
        q = op.apply(p)
        pq = dot(p, q)
        if not pq > 0.0:               # breakdown: restart with plain Jacobi step
            P, Q, PQ = [], [], []
            z = op.expand(op.dinv * r)
            p, q = z, op.apply(z)
            pq = dot(p, q)
        alpha = dot(p, r) / pq
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        P.append(p)
        Q.append(q)
        PQ.append(pq)
        if len(P) > m:
            P.pop(0), Q.pop(0), PQ.pop(0)
        hist.append(norm(r) / bnorm)
        if fallback and len(hist) > 2 * window:
            rate = (hist[-1] / hist[-1 - window]) ** (1.0 / window)
            if not rate <= ratio:
                res = pcg(op, b, x0=x, tol=tol, maxit=maxit - it)
                return Result(res.x, it + res.iterations, res.relres, hist + res.history[1:],
                              fallback=True)
    return Result(x, it, true_relres(op, b, x), hist)


def gauge_fixed(op, x):
    return op.gauge(x)
