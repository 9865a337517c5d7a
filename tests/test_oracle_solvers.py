"""Pins of the oracle's solvers (no GPU): dense brute force, finite
termination, PCG orthogonality, FCG == PCG for a fixed preconditioner, the
stagnation fallback, and the grid fixture's stretching law."""
import math

import numpy as np
import pytest

from paper_1410_1937_amd import fixtures as fx
from oracle.geometry import Body
from oracle.grid import Grid
from oracle.operator import Operator
from oracle import solvers


def _case(bc, seed=0, n=6, theta=0.4, body="sphere"):
    wl = fx.small(seed, n, n, n, body=body, bc=bc, theta=theta)
    g = Grid(wl.xf, wl.yf, wl.zf, wl.bc)
    bd = Body(g, wl.psi, wl.theta)
    op = Operator(g, bd, wl.phi, smooth=True)
    b = op.rhs(wl.u, wl.v, wl.w, 1.0, wl.body_vel)
    return wl, g, bd, op, b


@pytest.mark.parametrize("bc", [(0,) * 6, (0, 0, 0, 0, 0, 1), (1, 1, 0, 0, 0, 0), (1,) * 6])
def test_pcg_matches_dense_solve_6cubed(bc):
    """216 unknowns, stretched grid, 1000:1.2 jump, smoothing, a body with merges."""
    wl, g, bd, op, b = _case(bc)
    assert len(bd.slaves) > 0
    A = op.csr().toarray()
    m = bd.reduced.ravel()
    Ar = A[np.ix_(m, m)]
    br = b.ravel()[m]
    if any(bc):
        xr = np.linalg.solve(Ar, br)
    else:
        xr = np.linalg.lstsq(Ar, br, rcond=None)[0]
        xr -= xr.mean()
    xd = np.zeros(g.n)
    xd[m] = xr
    xd = op.expand(xd.reshape(g.shape))
    res = solvers.pcg(op, b, tol=1e-13)
    x = op.gauge(res.x)
    assert res.relres <= 1e-13
    assert solvers.norm(x - xd) <= 1e-10 * solvers.norm(xd)


def test_cg_terminates_in_m_steps_for_m_eigenvectors():
    """Unpreconditioned CG on a right-hand side made of m eigenvectors with
    distinct eigenvalues converges in exactly m iterations."""
    nx, ny, nz = 8, 6, 5
    g = Grid(fx.uniform_faces(0, 1, nx), fx.uniform_faces(0, 1, ny), fx.uniform_faces(0, 1, nz),
             (1, 1, 1, 1, 1, 1))
    op = Operator(g, Body(g), np.zeros(g.shape), smooth=False)
    i = [np.arange(n) + 0.5 for n in (nx, ny, nz)]
    for m, ks in ((1, [(1, 1, 1)]), (3, [(1, 1, 1), (2, 1, 1), (1, 3, 2)])):
        b = np.zeros(g.shape)
        for kx, ky, kz in ks:
            b += (np.sin(kz * math.pi * i[2] / nz)[:, None, None] * np.sin(ky * math.pi * i[1] / ny)[None, :, None]
                  * np.sin(kx * math.pi * i[0] / nx)[None, None, :])
        res = solvers.pcg(op, b, tol=1e-12, precond="none")
        assert res.iterations == m
        assert res.relres <= 1e-12


def test_pcg_residuals_are_m_orthogonal_and_directions_a_conjugate():
    wl, g, bd, op, b = _case((0, 0, 0, 0, 0, 1), n=10)
    rs, ps = [], []
    x = np.zeros(g.shape)
    r = b.copy()
    z = op.expand(op.dinv * r)
    p = z.copy()
    rz = solvers.dot(r, z)
    for _ in range(6):
        rs.append((r.copy(), z.copy()))
        ps.append(p.copy())
        q = op.apply(p)
        a = rz / solvers.dot(p, q)
        x, r = x + a * p, r - a * q
        z = op.expand(op.dinv * r)
        rzn = solvers.dot(r, z)
        p, rz = z + (rzn / rz) * p, rzn
    for i in range(len(rs)):
        for j in range(i):
            ri, zi = rs[i]
            rj, zj = rs[j]
            assert abs(solvers.dot(ri, zj)) <= 1e-9 * math.sqrt(solvers.dot(ri, zi) * solvers.dot(rj, zj))
            api = op.apply(ps[i])
            assert abs(solvers.dot(api, ps[j])) <= 1e-9 * math.sqrt(solvers.dot(api, ps[i]) * solvers.dot(op.apply(ps[j]), ps[j]))


def test_fcg_with_jacobi_reproduces_pcg():
    wl, g, bd, op, b = _case((0,) * 6, n=12)
    ref = solvers.pcg(op, b, tol=1e-30, maxit=50)
    out = solvers.fcg(op, b, lambda r: op.dinv * r, tol=1e-30, maxit=50, fallback=False)
    h1, h2 = np.array(ref.history[:51]), np.array(out.history[:51])
    assert np.max(np.abs(h1 - h2) / h1) <= 1e-8


def test_fcg_falls_back_and_still_meets_tolerance():
    """A sabotaged preconditioner (noise unrelated to r) stalls FCG; the
    stagnation monitor switches to Jacobi-PCG and the true residual is met."""
    wl, g, bd, op, b = _case((0,) * 6, n=12)
    rng = np.random.default_rng(0)
    bad = lambda r: rng.standard_normal(r.shape) * bd.reduced * 1e-6
    out = solvers.fcg(op, b, bad, tol=1e-8, maxit=5000)
    assert out.fallback
    assert solvers.true_relres(op, b, out.x) <= 1e-8


def test_pcg_reports_true_residual_and_restarts():
    wl, g, bd, op, b = _case((0,) * 6, n=12)
    res = solvers.pcg(op, b, tol=1e-11)
    assert res.relres == pytest.approx(solvers.true_relres(op, b, res.x), rel=1e-12)
    assert res.relres <= 1e-11
    short = solvers.pcg(op, b, tol=1e-11, maxit=3)
    assert short.iterations == 3 and short.relres > 1e-11


@pytest.mark.parametrize("bc", [(0,) * 6, (0, 0, 0, 0, 0, 1)])
def test_residual_replacement_continues_as_pcg(bc):
    """Replacing the recursive residual by the true one every 10x of
    reduction, with beta = (replaced r.z) / (the r.z before the last update),
    leaves CG's iteration: the same iteration count and the same solution as
    plain PCG.  (Dividing by the last r.z instead takes 2-3x the iterations
    on these grids.)"""
    wl = fx.small(0, 32, 16, 12, body="sphere", bc=bc)
    g = Grid(wl.xf, wl.yf, wl.zf, wl.bc)
    bd = Body(g, wl.psi, wl.theta, wl.samples)
    op = Operator(g, bd, wl.phi, wl.rho_l, wl.rho_g, wl.smooth)
    b = op.rhs(wl.u, wl.v, wl.w, wl.dt, wl.body_vel)
    ref = solvers.pcg(op, b, tol=1e-10)
    out = solvers.pcg_replaced(op, b, tol=1e-10, drop=0.1)
    assert out.restarts >= 5                 # the replacement path is exercised
    assert abs(out.iterations - ref.iterations) <= max(2, 0.01 * ref.iterations)
    assert out.relres <= 1e-10
    assert solvers.true_relres(op, b, out.x) == pytest.approx(out.relres, rel=1e-12)
    xr, xo = op.gauge(ref.x), op.gauge(out.x)
    assert np.linalg.norm(xo - xr) <= 1e-8 * np.linalg.norm(xr)


def test_stretched_grid_obeys_the_elliptic_grid_law():
    """Fixture grid: widths add up, the spacing ratio stays below 8, and
    w(x) dx is constant (first integral of the 1-D grid equation)."""
    for n, c in ((256, [-0.25, 0.25]), (96, [0.0]), (192, [0.0, -0.15])):
        f = fx.stretched_faces(-0.5, 0.7, n, c)
        d = np.diff(f)
        assert abs(d.sum() - 1.2) <= 1e-13
        assert d.max() / d.min() < 8.0
        xc = 0.5 * (f[1:] + f[:-1])
        dist = np.min(np.abs(xc[:, None] - np.array(c)[None, :]), axis=1)
        w = 1.0 / (1.0 + 7.0 * np.tanh(dist / 0.05))
        prod = w * d
        assert prod.max() / prod.min() < 1.05
