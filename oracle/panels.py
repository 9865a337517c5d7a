"""Signed distance to a triangulated body surface (oracle, FP64).

Test infrastructure: a plain CPU statement of the Enforcement of Body
Boundary Conditions section's signed distance for checking the library's
kernel against.  psi(p) is the minimal distance from p to the panels (the
closest point may lie inside a panel, on an edge or at a vertex), negative
inside the body and positive outside; inside and outside are told apart by
Gauss's theorem applied to the solid angle: the panels of a closed surface
subtend 4 pi at a point inside and 0 outside.

Readings (the section cites the method without giving it): the distance to
a triangle is the distance to the foot of the perpendicular on its plane
when that foot falls inside the triangle (barycentric coordinates all >= 0),
else the least distance to its three edges as segments; the solid angle of
a triangle (a, b, c seen from p) is Van Oosterom and Strackee's
2 atan2(a . (b x c), |a||b||c| + (a.b)|c| + (a.c)|b| + (b.c)|a|); a point is
inside when the summed solid angle exceeds 2 pi in magnitude.  Panels are
(m, 3, 3) arrays: m triangles of three vertices (x, y, z).
"""
from __future__ import annotations

import numpy as np


def _seg_dist2(p, a, b):
    """Squared distance from points p (..., 3) to segments [a, b] (..., 3)."""
    ab = b - a
    L2 = np.sum(ab * ab, axis=-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(L2 > 0, np.sum((p - a) * ab, axis=-1) / L2, 0.0)
    t = np.clip(t, 0.0, 1.0)
    d = p - (a + t[..., None] * ab)
    return np.sum(d * d, axis=-1)


def tri_dist2(p, tri):
    """Squared distance from points p (k, 3) to triangles tri (m, 3, 3):
    a (k, m) array."""
    p = np.asarray(p, dtype=np.float64)[:, None, :]
    a, b, c = (np.asarray(tri, dtype=np.float64)[None, :, v, :] for v in range(3))
    e0, e1 = b - a, c - a
    n = np.cross(e0, e1)
    nn = np.sum(n * n, axis=-1)
    ap = p - a
    # barycentric coordinates of the foot of the perpendicular
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.sum(np.cross(ap, e1) * n, axis=-1) / nn
        t = np.sum(np.cross(e0, ap) * n, axis=-1) / nn
        plane2 = np.sum(ap * n, axis=-1) ** 2 / nn
    inside = (nn > 0) & (s >= 0) & (t >= 0) & (s + t <= 1)
    edges = np.minimum(np.minimum(_seg_dist2(p, a, b), _seg_dist2(p, b, c)), _seg_dist2(p, c, a))
    return np.where(inside, plane2, edges)


def solid_angle(p, tri):
    """Solid angle of each triangle seen from each point: (k, m), signed by
    the triangle's orientation."""
    p = np.asarray(p, dtype=np.float64)[:, None, :]
    a, b, c = (np.asarray(tri, dtype=np.float64)[None, :, v, :] - p for v in range(3))
    la, lb, lc = (np.sqrt(np.sum(v * v, axis=-1)) for v in (a, b, c))
    num = np.sum(a * np.cross(b, c), axis=-1)
    den = la * lb * lc + np.sum(a * b, axis=-1) * lc + np.sum(a * c, axis=-1) * lb + np.sum(b * c, axis=-1) * la
    return 2.0 * np.arctan2(num, den)


def signed_distance(points, tri, chunk=4096):
    """psi at points (k, 3): minimal distance to the panels, negative inside."""
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.empty(len(points))
    for s in range(0, len(points), chunk):
        p = points[s:s + chunk]
        d = np.sqrt(np.min(tri_dist2(p, tri), axis=1))
        omega = np.sum(solid_angle(p, tri), axis=1)
        out[s:s + chunk] = np.where(np.abs(omega) > 2.0 * np.pi, -d, d)
    return out


def nodes_psi(xf, yf, zf, tri):
    """psi on the (nz+1, ny+1, nx+1) nodes of a grid."""
    Z, Y, X = np.meshgrid(zf, yf, xf, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return signed_distance(pts, tri).reshape(Z.shape)
