"""Pins of the oracle's grid stretching and panel signed distance (no GPU).

Grid: a constant weight gives uniform nodes; the converged nodes keep the
discrete first integral w dx constant; they converge at second order to the
continuous equidistribution x(xi) = W^-1(xi W(b)), with W the weight's
integral in closed form.  Signed distance: a box panelization reproduces the
box's closed-form signed distance (faces, edges, corners, inside); a single
triangle agrees with dense sampling; an icosphere stays within the sagitta of
the sphere's signed distance; the solid angles of a closed surface sum to
4 pi inside and 0 outside."""
import numpy as np
import pytest

from oracle import gridgen, panels
from paper_1410_1937_amd import fixtures as fx

LEVELS = (1.0, 8.0, 2.0)
ZONES = ((-0.3, -0.1), (0.2, 0.45))


def _W(x, a, levels=LEVELS, zones=ZONES):
    """Integral of the weight from a to x, by hand: levels times lengths plus
    (wa + wb)/2 (x - x0) + (wa - wb)/2 (L/pi) sin(pi (x - x0)/L) across a
    transition of length L."""
    total, pos = 0.0, a
    for k, (x0, x1) in enumerate(zones):
        wa, wb = levels[k], levels[k + 1]
        if x <= x0:
            return total + wa * (x - pos)
        total += wa * (x0 - pos)
        L = x1 - x0
        e = min(x, x1)
        total += (wa + wb) / 2 * (e - x0) + (wa - wb) / 2 * (L / np.pi) * np.sin(np.pi * (e - x0) / L)
        if x <= x1:
            return total
        pos = x1
    return total + levels[-1] * (x - pos)


def _equidistributed(a, b, n):
    WB = _W(b, a)
    out = np.empty(n + 1)
    for i in range(n + 1):
        lo, hi = a, b
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if _W(mid, a) < WB * i / n:
                lo = mid
            else:
                hi = mid
        out[i] = 0.5 * (lo + hi)
    return out


def test_constant_weight_gives_uniform_nodes():
    x, it = gridgen.stretch(-0.75, 0.75, 64, (3.0,), ())
    assert np.max(np.abs(x - np.linspace(-0.75, 0.75, 65))) <= 1e-14     # the solve's rounding
    assert it <= 2


@pytest.mark.parametrize("levels,zones", [(LEVELS, ZONES), ((4.0, 1.0, 6.0), ((-0.75, -0.2), (0.3, 0.75)))])
def test_converged_nodes_keep_the_discrete_first_integral(levels, zones):
    x, it = gridgen.stretch(-0.75, 0.75, 200, levels, zones)
    assert it < 500
    wdx = gridgen.weight(0.5 * (x[:-1] + x[1:]), levels, zones) * np.diff(x)
    assert np.max(np.abs(wdx / np.mean(wdx) - 1.0)) <= 1e-11
    if levels != LEVELS:
        return
    # spacing in the constant zones in the ratio of the levels
    dx = np.diff(x)
    m = 0.5 * (x[:-1] + x[1:])
    assert dx[m < -0.35].mean() / dx[(m > 0.0) & (m < 0.15)].mean() == pytest.approx(8.0, rel=1e-9)


def test_nodes_converge_to_the_continuous_equidistribution_at_second_order():
    errs = []
    for n in (100, 200, 400):
        x, _ = gridgen.stretch(-0.75, 0.75, n, LEVELS, ZONES)
        errs.append(np.max(np.abs(x - _equidistributed(-0.75, 0.75, n))))
    assert errs[2] < 2e-4
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


def _box_sdf(p, lo, hi):
    c, h = (lo + hi) / 2, (hi - lo) / 2
    q = np.abs(p - c) - h
    outside = np.linalg.norm(np.maximum(q, 0.0), axis=1)
    inside = np.minimum(np.max(q, axis=1), 0.0)
    return outside + inside


def test_box_panels_give_the_box_signed_distance():
    lo, hi = np.array([0.1, -0.2, 0.3]), np.array([0.9, 0.5, 0.8])
    tri = fx.box_panels(lo, hi)
    rng = np.random.default_rng(0)
    p = rng.uniform(-0.5, 1.5, (3000, 3))
    p[:500] = rng.uniform(lo, hi, (500, 3))            # inside
    p[500:600, :2] = hi[:2] + rng.uniform(0.0, 0.3, (100, 2))    # beyond an edge
    ref = _box_sdf(p, lo, hi)
    got = panels.signed_distance(p, tri)
    assert np.max(np.abs(got - ref)) <= 1e-14
    assert np.all(got[:500] < 0)


def test_single_triangle_distance_against_dense_sampling():
    rng = np.random.default_rng(1)
    tri = rng.uniform(-1, 1, (1, 3, 3))
    p = rng.uniform(-2, 2, (200, 3))
    m = 400
    u, v = np.meshgrid(np.linspace(0, 1, m + 1), np.linspace(0, 1, m + 1))
    keep = u + v <= 1
    u, v = u[keep], v[keep]
    S = tri[0, 0] + u[:, None] * (tri[0, 1] - tri[0, 0]) + v[:, None] * (tri[0, 2] - tri[0, 0])
    sampled = np.sqrt(np.min(np.sum((p[:, None, :] - S[None]) ** 2, axis=-1), axis=1))
    d = np.sqrt(panels.tri_dist2(p, tri)[:, 0])
    spacing = np.max(np.linalg.norm(tri[0] - np.roll(tri[0], 1, axis=0), axis=1)) / m
    assert np.all(d <= sampled + 1e-12)
    assert np.all(sampled - d <= spacing)


def test_icosphere_is_within_its_sagitta_of_the_sphere_distance():
    R, c = 0.1, np.array([0.0, 0.0, -0.15])
    tri = fx.icosphere_panels(R, c, levels=3)
    n = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    plane = np.abs(np.sum(n * (tri[:, 0] - c), axis=1)) / np.linalg.norm(n, axis=1)
    sag = R - plane.min()
    rng = np.random.default_rng(2)
    p = c + rng.uniform(-0.25, 0.25, (4000, 3))
    exact = np.linalg.norm(p - c, axis=1) - R
    got = panels.signed_distance(p, tri)
    assert np.max(np.abs(got - exact)) <= sag + 1e-15
    far = np.abs(exact) > sag
    assert np.array_equal(np.sign(got[far]), np.sign(exact[far]))


@pytest.mark.parametrize("mesh", ["box", "ico", "wigley"])
def test_solid_angles_of_a_closed_surface(mesh):
    tri = {"box": lambda: fx.box_panels((0, 0, 0), (1, 2, 3)), "ico": lambda: fx.icosphere_panels(levels=2),
           "wigley": lambda: fx.wigley_panels()}[mesh]()
    lo, hi = tri.reshape(-1, 3).min(axis=0), tri.reshape(-1, 3).max(axis=0)
    centre = 0.5 * (lo + hi) if mesh != "wigley" else np.array([0.0, 0.0, -0.005])
    rng = np.random.default_rng(3)
    out = hi + rng.uniform(0.05, 1.0, (50, 3)) * (hi - lo)
    inside = centre + rng.uniform(-0.1, 0.1, (50, 3)) * (hi - lo)
    om_in = panels.solid_angle(inside, tri).sum(axis=1)
    om_out = panels.solid_angle(out, tri).sum(axis=1)
    assert np.max(np.abs(om_in - 4 * np.pi)) <= 1e-11
    assert np.max(np.abs(om_out)) <= 1e-11
    assert np.all(panels.signed_distance(inside, tri) < 0) and np.all(panels.signed_distance(out, tri) > 0)
