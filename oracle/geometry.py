"""Immersed body on the cartesian grid (oracle).

Follows "Enforcement of Body Boundary Conditions": the body is the region
psi < 0 of a signed-distance function given at the grid nodes; the finite-
volume equation of a cut cell uses the fractional areas of its faces (method
of fractional areas); cells whose cut volume is below a threshold (25 % in
the paper) are merged with a neighbour along the steepest gradient of psi.
The face flux is A_i (u_i - v_i) with A_i = 0 inside the hull
(Interface reconstruction and advection section).

Readings (the paper defers the details to a reference that is not given):
  * a face's fraction = share of S x S midpoint samples where the bilinear
    interpolant of its four corner psi values is > 0; a cell's fraction =
    share of S^3 midpoint samples where the trilinear interpolant is > 0.
    When all corners are > 0 (<= 0) every sample is, because the weights are
    strictly positive, so the fraction is exactly 1 (0) without sampling.
  * a cell is active iff its fraction is > 0 and it has an open coupling:
    a face with fraction > 0 to a neighbour of fraction > 0, or an open
    Dirichlet boundary face.  Every face touching an inactive cell is closed.
  * merge direction: the axis of largest |d psi/d x_d| at the cell centre
    (gradient of the trilinear interpolant: mean of the four edge
    differences over the cell width), ties to the lower axis, toward larger
    psi; if that face is closed or on the domain boundary the next axis is
    tried; no candidate leaves the cell unmerged.  Roots follow the target
    chain; in a cycle the member with the largest fraction (then the lowest
    index) is the root.
"""
from __future__ import annotations

import numpy as np


def _samples(S):
    return (np.arange(S, dtype=np.float64) + 0.5) / S


def _bilinear_fraction(c00, c10, c01, c11, S):
    """Fraction of S*S samples with bilinear interpolant > 0.

    c_ab: corner values, a along the first local axis (s), b along the second (t).
    Interpolant: ((w00*c00 + w10*c10) + w01*c01) + w11*c11 with
    w00 = (1-s)*(1-t), w10 = s*(1-t), w01 = (1-s)*t, w11 = s*t.
    """
    shape = c00.shape
    out = np.ones(shape)
    allpos = (c00 > 0) & (c10 > 0) & (c01 > 0) & (c11 > 0)
    allneg = (c00 <= 0) & (c10 <= 0) & (c01 <= 0) & (c11 <= 0)
    out[allneg] = 0.0
    mixed = ~(allpos | allneg)
    if np.any(mixed):
        a00, a10, a01, a11 = c00[mixed], c10[mixed], c01[mixed], c11[mixed]
        cnt = np.zeros(a00.shape, dtype=np.int64)
        sv = _samples(S)
        for t in sv:
            for s in sv:
                w00 = (1.0 - s) * (1.0 - t)
                w10 = s * (1.0 - t)
                w01 = (1.0 - s) * t
                w11 = s * t
                val = ((w00 * a00 + w10 * a10) + w01 * a01) + w11 * a11
                cnt += val > 0
        out[mixed] = cnt / float(S * S)
    return out


def face_fractions(psi, S=8):
    """Fractional areas of the x-, y- and z-faces from nodal psi (nz+1, ny+1, nx+1)."""
    # x-face (k, j, i): corners over (y, z): s along y, t along z
    fx = _bilinear_fraction(psi[:-1, :-1, :], psi[:-1, 1:, :], psi[1:, :-1, :], psi[1:, 1:, :], S)
    # y-face (k, j, i): s along x, t along z
    fy = _bilinear_fraction(psi[:-1, :, :-1], psi[:-1, :, 1:], psi[1:, :, :-1], psi[1:, :, 1:], S)
    # z-face (k, j, i): s along x, t along y
    fz = _bilinear_fraction(psi[:, :-1, :-1], psi[:, :-1, 1:], psi[:, 1:, :-1], psi[:, 1:, 1:], S)
    return fx, fy, fz


def cell_fractions(psi, S=8):
    """Fluid fraction of each cell: share of S^3 samples where the trilinear
    interpolant of its 8 corner psi values is > 0.

    Interpolant: sum over corners in the order (a, b, c) = (0,0,0), (1,0,0),
    (0,1,0), (1,1,0), (0,0,1), (1,0,1), (0,1,1), (1,1,1) (a along x, b along
    y, c along z), each weight (wx_a * wy_b) * wz_c, summed left to right.
    """
    corners = []
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                corners.append(psi[c:psi.shape[0] - 1 + c, b:psi.shape[1] - 1 + b, a:psi.shape[2] - 1 + a])
    out = np.ones(corners[0].shape)
    allpos = np.ones(out.shape, dtype=bool)
    allneg = np.ones(out.shape, dtype=bool)
    for q in corners:
        allpos &= q > 0
        allneg &= q <= 0
    out[allneg] = 0.0
    mixed = ~(allpos | allneg)
    if np.any(mixed):
        cm = [q[mixed] for q in corners]
        cnt = np.zeros(cm[0].shape, dtype=np.int64)
        sv = _samples(S)
        for u in sv:
            for t in sv:
                for s in sv:
                    wx = (1.0 - s, s)
                    wy = (1.0 - t, t)
                    wz = (1.0 - u, u)
                    val = None
                    idx = 0
                    for c in (0, 1):
                        for b in (0, 1):
                            for a in (0, 1):
                                term = ((wx[a] * wy[b]) * wz[c]) * cm[idx]
                                val = term if val is None else val + term
                                idx += 1
                    cnt += val > 0
        out[mixed] = cnt / float(S * S * S)
    return out


class Body:
    """Static body geometry on a grid: open face areas, fractions, active set,
    merge groups.  `psi=None` means no body."""

    def __init__(self, grid, psi=None, theta=0.25, S=8):
        g = grid
        ax, ay, az = g.face_areas()
        if psi is None:
            fx = np.ones(ax.shape)
            fy = np.ones(ay.shape)
            fz = np.ones(az.shape)
            vol = np.ones(g.shape)
        else:
            psi = np.asarray(psi, dtype=np.float64)
            if psi.shape != (g.nz + 1, g.ny + 1, g.nx + 1):
                raise ValueError("psi must have the node shape")
            fx, fy, fz = face_fractions(psi, S)
            vol = cell_fractions(psi, S)
        self.frac_x, self.frac_y, self.frac_z = fx, fy, fz
        self.vfrac = vol
        self.active = self._active_set(g, fx, fy, fz, vol)
        act = self.active
        # close every face that touches an inactive cell
        ox = fx.copy()
        ox[:, :, 1:] *= act
        ox[:, :, :-1] *= act
        oy = fy.copy()
        oy[:, 1:, :] *= act
        oy[:, :-1, :] *= act
        oz = fz.copy()
        oz[1:, :, :] *= act
        oz[:-1, :, :] *= act
        # open face area a_f * Area_f
        self.open_x = ox * ax
        self.open_y = oy * ay
        self.open_z = oz * az
        self.root = self._merge(g, psi, theta)
        self._groups()

    @staticmethod
    def _active_set(g, fx, fy, fz, vol):
        wet = vol > 0
        coupled = np.zeros(g.shape, dtype=bool)
        # interior faces
        ix = (fx[:, :, 1:-1] > 0) & wet[:, :, :-1] & wet[:, :, 1:]
        coupled[:, :, :-1] |= ix
        coupled[:, :, 1:] |= ix
        iy = (fy[:, 1:-1, :] > 0) & wet[:, :-1, :] & wet[:, 1:, :]
        coupled[:, :-1, :] |= iy
        coupled[:, 1:, :] |= iy
        iz = (fz[1:-1, :, :] > 0) & wet[:-1, :, :] & wet[1:, :, :]
        coupled[:-1, :, :] |= iz
        coupled[1:, :, :] |= iz
        # open Dirichlet boundary faces
        bc = g.bc
        if bc[0]:
            coupled[:, :, 0] |= fx[:, :, 0] > 0
        if bc[1]:
            coupled[:, :, -1] |= fx[:, :, -1] > 0
        if bc[2]:
            coupled[:, 0, :] |= fy[:, 0, :] > 0
        if bc[3]:
            coupled[:, -1, :] |= fy[:, -1, :] > 0
        if bc[4]:
            coupled[0, :, :] |= fz[0, :, :] > 0
        if bc[5]:
            coupled[-1, :, :] |= fz[-1, :, :] > 0
        return (wet & coupled).astype(np.float64)

    def _merge(self, g, psi, theta):
        """root[c] = linear index of the cell that c is merged into (itself if
        not merged; -1 if inactive)."""
        nz, ny, nx = g.shape
        n = g.n
        act = self.active.reshape(-1) > 0
        v = self.vfrac.reshape(-1)
        root = np.where(act, np.arange(n), -1)
        if psi is None:
            return root.reshape(g.shape)
        small = np.nonzero(act & (v < theta))[0]
        target = {}
        dxs = (g.ax.d, g.ay.d, g.az.d)
        for c in small:
            k, r = divmod(int(c), nx * ny)
            j, i = divmod(r, nx)
            P = psi[k:k + 2, j:j + 2, i:i + 2]  # P[c][b][a]
            # edge differences of the trilinear interpolant, averaged: gradient at the centre
            gx = ((((P[0, 0, 1] - P[0, 0, 0]) + (P[0, 1, 1] - P[0, 1, 0])) + (P[1, 0, 1] - P[1, 0, 0]))
                  + (P[1, 1, 1] - P[1, 1, 0])) * 0.25 / dxs[0][i]
            gy = ((((P[0, 1, 0] - P[0, 0, 0]) + (P[0, 1, 1] - P[0, 0, 1])) + (P[1, 1, 0] - P[1, 0, 0]))
                  + (P[1, 1, 1] - P[1, 0, 1])) * 0.25 / dxs[1][j]
            gz = ((((P[1, 0, 0] - P[0, 0, 0]) + (P[1, 0, 1] - P[0, 0, 1])) + (P[1, 1, 0] - P[0, 1, 0]))
                  + (P[1, 1, 1] - P[0, 1, 1])) * 0.25 / dxs[2][k]
            grad = (gx, gy, gz)
            order = sorted(range(3), key=lambda d: (-abs(grad[d]), d))
            for d in order:
                if grad[d] == 0.0:
                    continue
                s = 1 if grad[d] > 0 else -1
                if d == 0:
                    fi = i + (1 if s > 0 else 0)
                    if fi == 0 or fi == nx or self.open_x[k, j, fi] <= 0:
                        continue
                    t = c + s
                elif d == 1:
                    fj = j + (1 if s > 0 else 0)
                    if fj == 0 or fj == ny or self.open_y[k, fj, i] <= 0:
                        continue
                    t = c + s * nx
                else:
                    fk = k + (1 if s > 0 else 0)
                    if fk == 0 or fk == nz or self.open_z[fk, j, i] <= 0:
                        continue
                    t = c + s * nx * ny
                target[int(c)] = int(t)
                break
        # resolve roots along the target chains
        resolved = {}
        for c in target:
            path = []
            cur = c
            while cur in target and cur not in resolved and cur not in path:
                path.append(cur)
                cur = target[cur]
            if cur in resolved:
                r = resolved[cur]
            elif cur in path:          # cycle: cur .. end of path
                cyc = path[path.index(cur):]
                r = min(cyc, key=lambda m: (-v[m], m))
            else:                      # reached a cell that is not merged further
                r = cur
            for m in path:
                resolved[m] = r
        for c, r in resolved.items():
            root[c] = r
        return root.reshape(g.shape)

    def _groups(self):
        """Reduced unknowns: one per root.  members[r] = [r, slaves ascending]."""
        root = self.root.reshape(-1)
        n = root.size
        idx = np.arange(n)
        slaves = np.nonzero((root >= 0) & (root != idx))[0]
        self.slaves = slaves
        self.slave_root = root[slaves]
        groups = {}
        for s in slaves:        # ascending
            groups.setdefault(int(root[s]), []).append(int(s))
        self.groups = {r: [r] + sl for r, sl in sorted(groups.items())}
        self.reduced = ((root >= 0) & (root == idx)).reshape(self.root.shape)   # one cell per unknown
        self.n_reduced = int(self.reduced.sum())
