"""One-dimensional grid stretching (oracle, FP64).

Test infrastructure: a plain CPU statement of the Gridding section for
checking the library's grid generator against.  Along one axis the nodes
x(xi), xi in [0, 1], satisfy eq. grid,

    x_xixi + (w_xi / w) x_xi = 0,   i.e.  (w x_xi)_xi = 0,

with x(0) = a, x(1) = b and a weight w(x) given in physical space: constant
levels joined by the cosine transitions of the section,

    w(x) = (w0 - w1)/2 (1 + cos(pi (x - x0)/(x1 - x0))) + w1   on [x0, x1],

w0 before the zone and w1 after it (several zones chain the levels).  A
large weight clusters nodes: w x_xi is constant, so the spacing is
inversely proportional to w.

Discretization and iteration (the paper says only that the nonlinear
equation is solved iteratively; readings): the conservative form on the
N + 1 nodes, w(m_{i+1/2}) (x_{i+1} - x_i) - w(m_{i-1/2}) (x_i - x_{i-1}) = 0
with m the midpoints, solved by Picard iteration -- the weights frozen at the
current midpoints, the tridiagonal system for the interior nodes solved
exactly -- from uniform nodes until no node moves by more than
tol * (b - a), at most max_iter sweeps.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded


def weight(x, levels, zones):
    """w at the points x: levels[0] before zones[0], the cosine transition
    from levels[k] to levels[k+1] across zones[k] = (x0, x1), levels[k+1]
    after it."""
    x = np.asarray(x, dtype=np.float64)
    w = np.full(x.shape, float(levels[0]))
    for k, (x0, x1) in enumerate(zones):
        wa, wb = float(levels[k]), float(levels[k + 1])
        t = np.pi * (x - x0) / (x1 - x0)
        inside = (wa - wb) / 2.0 * (1.0 + np.cos(t)) + wb
        w = np.where(x < x0, w, np.where(x <= x1, inside, wb))
    return w


def stretch(a, b, n, levels, zones, tol=1e-13, max_iter=500):
    """The n + 1 nodes of [a, b] and the number of Picard sweeps taken."""
    x = a + (b - a) * np.arange(n + 1) / n
    for it in range(1, max_iter + 1):
        wm = weight(0.5 * (x[:-1] + x[1:]), levels, zones)      # w at the n midpoints
        if n == 1:
            return x, it
        # rows i = 1..n-1: -wm[i-1] x[i-1] + (wm[i-1] + wm[i]) x[i] - wm[i] x[i+1] = 0
        ab = np.zeros((3, n - 1))
        ab[0, 1:] = -wm[1:n - 1]          # super-diagonal
        ab[1, :] = wm[:n - 1] + wm[1:]    # diagonal
        ab[2, :-1] = -wm[1:n - 1]         # sub-diagonal
        rhs = np.zeros(n - 1)
        rhs[0] += wm[0] * a
        rhs[-1] += wm[n - 1] * b
        new = x.copy()
        new[1:-1] = solve_banded((1, 1), ab, rhs)
        moved = np.max(np.abs(new - x))
        x = new
        if moved <= tol * (b - a):
            return x, it
    return x, max_iter
