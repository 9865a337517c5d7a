"""Pins of the oracle's Runge-Kutta projection cycle (no GPU): discrete
solenoidality after each stage, the fixed point of a projected field, a closed
column coming to rest, and the velocity update against the flux projection."""
import numpy as np

from oracle import rk2
from oracle.geometry import Body
from oracle.grid import Grid
from oracle.operator import Operator
from paper_1410_1937_amd import fixtures as fx


def _setup(seed=0, bc=(0,) * 6):
    wl = fx.small(seed, 24, 12, 10, body="sphere", bc=bc)
    g = Grid(wl.xf, wl.yf, wl.zf, wl.bc)
    body = Body(g, wl.psi, wl.theta, wl.samples)
    R = tuple(0.1 * a for a in fx.face_velocity(wl.xf, wl.yf, wl.zf, seed + 7))
    return wl, g, body, R


def _open(body):
    return body.open_x, body.open_y, body.open_z


def _div(op, body, u, vel):
    return op.merged_divergence(*[o * a for o, a in zip(_open(body), u)], vel)


def test_each_stage_leaves_a_discretely_solenoidal_field():
    wl, g, body, R = _setup()
    phi_s = np.roll(wl.phi, 1, axis=2)           # the interface moved by one cell
    out = rk2.cycle(g, body, wl.phi, phi_s, (wl.u, wl.v, wl.w), R, 0.01, wl.body_vel, tol=1e-12)
    d1_before = np.linalg.norm(_div(out["op1"], body, out["ut1"], wl.body_vel))
    d1 = np.linalg.norm(_div(out["op1"], body, out["us"], wl.body_vel))
    d2_before = np.linalg.norm(_div(out["op2"], body, out["ut2"], out["vel2"]))
    d2 = np.linalg.norm(_div(out["op2"], body, out["un"], wl.body_vel))
    assert d1_before > 1e-3 and d2_before > 1e-3
    assert d1 <= 1e-9 * d1_before and d2 <= 1e-9 * d2_before


def test_projected_field_is_a_fixed_point_without_forcing():
    wl, g, body, R = _setup(1)
    op = Operator(g, body, wl.phi)
    # a field that already satisfies the discrete constraint with the body moving
    b = op.rhs(wl.u, wl.v, wl.w, 1.0, wl.body_vel)
    p = rk2._solve(op, b, 1e-13)[0]
    uk = rk2.update_velocity(op, (wl.u, wl.v, wl.w), p, 1.0)
    zero = tuple(np.zeros_like(a) for a in uk)
    out = rk2.cycle(g, body, wl.phi, wl.phi, uk, zero, 0.01, wl.body_vel, tol=1e-13)
    for a, c, o in zip(out["un"], uk, _open(body)):
        m = o > 0
        assert np.linalg.norm(a[m] - c[m]) <= 1e-9 * np.linalg.norm(c[m])


def test_closed_column_comes_to_rest():
    nz = 40
    xf = yf = np.array([0.0, 1.0])
    zf = fx.stretched_faces(0.0, 1.0, nz, [0.5])
    g = Grid(xf, yf, zf, (0, 0, 0, 0, 0, 1))
    body = Body(g, None, 0.25, 8)
    phi = (fx.centres(zf) < 0.5).astype(np.float64).reshape(nz, 1, 1)
    rng = np.random.default_rng(3)
    u = np.zeros((nz, 1, 2)), np.zeros((nz, 2, 1)), rng.standard_normal((nz + 1, 1, 1))
    u[2][0] = 0.0                                 # closed bottom
    R = np.zeros((nz, 1, 2)), np.zeros((nz, 2, 1)), rng.standard_normal((nz + 1, 1, 1))
    R[2][0] = 0.0
    out = rk2.cycle(g, body, phi, phi, u, R, 0.05, smooth=False, tol=1e-13)
    w = out["un"][2]
    assert np.max(np.abs(w)) <= 1e-9 * np.max(np.abs(out["ut2"][2]))
    assert np.max(np.abs(out["us"][2])) <= 1e-9 * np.max(np.abs(out["ut1"][2]))


def test_velocity_update_matches_the_flux_projection():
    wl, g, body, R = _setup(2, bc=(1, 0, 0, 1, 0, 1))
    op = Operator(g, body, wl.phi)
    p = np.random.default_rng(4).standard_normal(g.shape)
    ut = (wl.u, wl.v, wl.w)
    uv = rk2.update_velocity(op, ut, p, 0.3)
    fl = op.project(*ut, p, 0.3)
    for a, f, o in zip(uv, fl, _open(body)):
        assert np.max(np.abs(o * a - f)) <= 1e-13 * np.max(np.abs(f))
    # closed faces keep the provisional velocity; scale applies to every face
    half = rk2.update_velocity(op, ut, p, 0.3, 0.5)
    for a, h, u0, o in zip(uv, half, ut, _open(body)):
        assert np.array_equal(a[o == 0], u0[o == 0])
        assert np.array_equal(h, 0.5 * a)
