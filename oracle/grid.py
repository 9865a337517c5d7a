"""Grid metrics of a stretched cartesian grid (oracle).

Follows the Gridding section: the grid is a tensor product of three
one-dimensional stretched axes, given here by their face coordinates.
"""
from __future__ import annotations

import numpy as np


class Axis:
    """Metrics of one axis from its n+1 strictly increasing face coordinates.

    d[i]  = f[i+1] - f[i]           cell width (i = 0..n-1)
    c[i]  = 0.5 * (f[i] + f[i+1])   cell centre
    h[i]  = distance associated with face i (i = 0..n):
            interior faces: c[i] - c[i-1]  (centre to centre)
            boundary faces: 0.5 * d        (centre to face, used by a
                                            Dirichlet face only)
    """

    def __init__(self, f):
        f = np.asarray(f, dtype=np.float64)
        if f.ndim != 1 or len(f) < 2 or not np.all(np.diff(f) > 0):
            raise ValueError("face coordinates must be strictly increasing")
        self.f = f
        self.n = len(f) - 1
        self.d = f[1:] - f[:-1]
        self.c = 0.5 * (f[:-1] + f[1:])
        h = np.empty(self.n + 1)
        h[1:-1] = self.c[1:] - self.c[:-1]
        h[0] = 0.5 * self.d[0]
        h[-1] = 0.5 * self.d[-1]
        self.h = h


class Grid:
    """bc = (-x, +x, -y, +y, -z, +z), 0 = Neumann (no flux), 1 = Dirichlet p = 0."""

    def __init__(self, xf, yf, zf, bc):
        self.ax = Axis(xf)
        self.ay = Axis(yf)
        self.az = Axis(zf)
        self.bc = tuple(int(b) for b in bc)
        if len(self.bc) != 6 or any(b not in (0, 1) for b in self.bc):
            raise ValueError("bc must hold six 0/1 flags")
        self.nx, self.ny, self.nz = self.ax.n, self.ay.n, self.az.n
        self.shape = (self.nz, self.ny, self.nx)
        self.n = self.nx * self.ny * self.nz

    @property
    def all_neumann(self):
        return not any(self.bc)

    def face_areas(self):
        """Full (uncut) face areas on the three face sets."""
        dx, dy, dz = self.ax.d, self.ay.d, self.az.d
        ax = np.broadcast_to((dz[:, None] * dy[None, :])[:, :, None], (self.nz, self.ny, self.nx + 1))
        ay = np.broadcast_to((dz[:, None] * dx[None, :])[:, None, :], (self.nz, self.ny + 1, self.nx))
        az = np.broadcast_to((dy[:, None] * dx[None, :])[None, :, :], (self.nz + 1, self.ny, self.nx))
        return ax, ay, az

    def volumes(self):
        return (self.az.d[:, None, None] * self.ay.d[None, :, None]) * self.ax.d[None, None, :]
