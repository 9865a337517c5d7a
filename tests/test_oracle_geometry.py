"""Pins of the oracle's body geometry (no GPU): exact fractions for a planar
body, sphere volume and surface area, merge targets along the steepest
gradient of psi."""
import math

import numpy as np

from paper_1410_1937_amd import fixtures as fx
from oracle.geometry import Body, cell_fractions, face_fractions
from oracle.grid import Grid


def test_planar_body_fractions_are_exact():
    """psi = z - z0 with z0 between two sample rows: vertical faces and cells of
    the cut layer have wet fraction exactly 5/8 (S = 8), z-faces 0 or 1."""
    n = 6
    xf = fx.uniform_faces(0, 1, n)
    yf = fx.uniform_faces(0, 2, n)
    zf = fx.uniform_faces(0, 1, n)
    k = 2
    z0 = zf[k] + (3.0 / 8.0) * (zf[k + 1] - zf[k])
    psi = fx.psi_plane_z(xf, yf, zf, z0)
    fxa, fya, fza = face_fractions(psi, 8)
    v = cell_fractions(psi, 8)
    assert np.all(v[:k] == 0) and np.all(v[k] == 5 / 8) and np.all(v[k + 1:] == 1)
    assert np.all(fxa[k] == 5 / 8) and np.all(fya[k] == 5 / 8)
    assert np.all(fxa[:k] == 0) and np.all(fxa[k + 1:] == 1)
    assert np.all(fza[:k + 1] == 0) and np.all(fza[k + 1:] == 1)


def test_sphere_volume_and_surface_area():
    """Sum of v_c V_c approaches the fluid volume (box minus 4/3 pi R^3) and the
    body-surface area vectors S_c (from the open face areas by Gauss) add up
    in magnitude to about 4 pi R^2."""
    n = 40
    xf = fx.uniform_faces(-0.5, 0.5, n)
    yf = fx.uniform_faces(-0.5, 0.5, n)
    zf = fx.uniform_faces(-0.5, 0.5, n)
    R = 0.27
    psi = fx.psi_sphere(xf, yf, zf, radius=R, centre=(0.013, -0.021, 0.007))
    g = Grid(xf, yf, zf, (0,) * 6)
    body = Body(g, psi, theta=0.25)
    vol = np.sum(body.vfrac * g.volumes())
    assert abs((1.0 - vol) - 4 / 3 * math.pi * R ** 3) <= 0.01 * 4 / 3 * math.pi * R ** 3
    for f in (body.frac_x, body.frac_y, body.frac_z):
        assert f.min() >= 0 and f.max() <= 1
    sx = -(body.open_x[:, :, 1:] - body.open_x[:, :, :-1])
    sy = -(body.open_y[:, 1:, :] - body.open_y[:, :-1, :])
    sz = -(body.open_z[1:] - body.open_z[:-1])
    area = np.sum(np.sqrt(sx ** 2 + sy ** 2 + sz ** 2))
    assert abs(area - 4 * math.pi * R ** 2) <= 0.03 * 4 * math.pi * R ** 2
    # each S_c points into the body (toward the centre)
    xc, yc, zc = g.ax.c, g.ay.c, g.az.c
    rx = xc[None, None, :] - 0.013
    ry = yc[None, :, None] + 0.021
    rz = zc[:, None, None] - 0.007
    mag = np.sqrt(sx ** 2 + sy ** 2 + sz ** 2)
    m = mag > 1e-3 * mag.max()
    assert np.all((sx * rx + sy * ry + sz * rz)[m] < 0)


def test_small_cells_merge_upward_above_a_flat_bed():
    """A cell layer cut 7/8 by a flat bed (v = 1/8 < theta) merges with the
    cell above: the steepest gradient of psi = z - z0 is +z."""
    n = 5
    xf = fx.uniform_faces(0, 1, n)
    yf = fx.uniform_faces(0, 1, n)
    zf = fx.uniform_faces(0, 1, n)
    k = 1
    z0 = zf[k] + 0.86 * (zf[k + 1] - zf[k])
    g = Grid(xf, yf, zf, (0,) * 6)
    body = Body(g, fx.psi_plane_z(xf, yf, zf, z0), theta=0.25)
    assert np.all(body.vfrac[k] == 1 / 8)
    assert np.all(body.active[:k] == 0)
    idx = np.arange(g.n).reshape(g.shape)
    assert np.array_equal(body.root[k], idx[k + 1])
    assert np.array_equal(body.root[k + 1:], idx[k + 1:])
    assert body.n_reduced == n * n * (n - k - 1)


def test_merge_groups_are_connected_through_open_faces():
    wl = fx.small(0, 24, 16, 14, body="sphere", theta=0.5)
    g = Grid(wl.xf, wl.yf, wl.zf, wl.bc)
    body = Body(g, wl.psi, wl.theta)
    assert len(body.slaves) > 10
    nz, ny, nx = g.shape
    for r, members in body.groups.items():
        assert body.active.ravel()[r] == 1
        seen = {r}
        frontier = [r]
        mset = set(members)
        while frontier:
            c = frontier.pop()
            k, rem = divmod(c, nx * ny)
            j, i = divmod(rem, nx)
            nbs = []
            if i > 0 and body.open_x[k, j, i] > 0: nbs.append(c - 1)
            if i < nx - 1 and body.open_x[k, j, i + 1] > 0: nbs.append(c + 1)
            if j > 0 and body.open_y[k, j, i] > 0: nbs.append(c - nx)
            if j < ny - 1 and body.open_y[k, j + 1, i] > 0: nbs.append(c + nx)
            if k > 0 and body.open_z[k, j, i] > 0: nbs.append(c - nx * ny)
            if k < nz - 1 and body.open_z[k + 1, j, i] > 0: nbs.append(c + nx * ny)
            for nb in nbs:
                if nb in mset and nb not in seen:
                    seen.add(nb)
                    frontier.append(nb)
        assert seen == mset
    # every small active cell is merged unless it has no open candidate face
    small = (body.active > 0) & (body.vfrac < wl.theta)
    merged = body.root != np.arange(g.n).reshape(g.shape)
    assert np.mean(merged[small]) > 0.8
