"""One cycle of the second-order Runge-Kutta projection (oracle, FP64).

Test infrastructure: a plain CPU statement of the cycle that wraps the
projection (Numerical Time Integration, eqs. poisson1, runge1, poisson2,
runge2), for checking the GPU path against.

    stage 1:  u~1 = u^k + dt R
              div((1/rho(phi^k)) grad P*) = div(u~1)/dt        (eq. poisson1)
              u*  = u~1 - dt (1/rho(phi^k)) grad P*             (eq. runge1)
    stage 2:  u~2 = (u* + u^k) + dt R
              div((1/rho(phi*)) grad P) = div(u~2)/dt           (eq. poisson2)
              u^{k+1} = 1/2 (u~2 - dt (1/rho(phi*)) grad P)     (eq. runge2)

R (convection, gravity, viscosity, ...) and the advected volume fraction phi*
are inputs: their operators are not part of the projection.  Velocities live
on faces (the x-, y-, z-face layouts of the grid).  The gradient term on a
face is beta_f (p+ - p-)/h_f with the coefficients of the operator: beta_f =
2/(rho_L + rho_R) inside, 1/rho_c and h = half width on a Dirichlet boundary
face (p = 0 beyond it); Neumann boundary faces and closed faces (zero open
area: cut off by the body or next to an inactive cell) keep their provisional
velocity.  The body moves with velocity v: the stage-2 provisional field is
a sum of two fields that each carry v on the body, so its body flux is 2v.
"""
from __future__ import annotations

import numpy as np

from . import solvers
from .operator import Operator


def conductance(op):
    """beta_f / h_f on every face (x-, y-, z-face layouts); 0 on Neumann
    boundary faces and on faces with zero open area."""
    g, rho = op.grid, op.rho
    out = []
    for axis, (h, open_) in enumerate(((g.ax.h, op.body.open_x), (g.ay.h, op.body.open_y),
                                       (g.az.h, op.body.open_z))):
        ax = 2 - axis                     # array axis of this direction (z, y, x order)
        n = rho.shape[ax]
        shape = list(rho.shape)
        shape[ax] = n + 1
        gf = np.zeros(shape)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        inner = [slice(None)] * 3
        lo[ax], hi[ax], inner[ax] = slice(0, n - 1), slice(1, n), slice(1, n)
        hb = h.reshape([-1 if a == ax else 1 for a in range(3)])
        gf[tuple(inner)] = (2.0 / (rho[tuple(lo)] + rho[tuple(hi)])) / hb[tuple(inner)]
        for side, face, cell in ((0, 0, 0), (1, n, n - 1)):
            if g.bc[2 * axis + side]:
                fsl = [slice(None)] * 3
                csl = [slice(None)] * 3
                fsl[ax], csl[ax] = face, cell
                gf[tuple(fsl)] = (1.0 / rho[tuple(csl)]) / h[face]
        gf[open_ == 0] = 0.0
        out.append(gf)
    return out


def update_velocity(op, ut, p, dt, scale=1.0):
    """scale * (u~ - dt beta (p+ - p-)/h) on every face, p expanded over the
    merge groups and 0 beyond the domain."""
    p = op.expand(p)
    pp = np.pad(p, 1)
    gx, gy, gz = conductance(op)
    ux = ut[0] - dt * (gx * (pp[1:-1, 1:-1, 1:] - pp[1:-1, 1:-1, :-1]))
    uy = ut[1] - dt * (gy * (pp[1:-1, 1:, 1:-1] - pp[1:-1, :-1, 1:-1]))
    uz = ut[2] - dt * (gz * (pp[1:, 1:-1, 1:-1] - pp[:-1, 1:-1, 1:-1]))
    if scale != 1.0:
        ux, uy, uz = scale * ux, scale * uy, scale * uz
    return ux, uy, uz


def _solve(op, b, tol):
    res = solvers.pcg(op, b, tol=tol)
    return solvers.gauge_fixed(op, res.x), res


def cycle(grid, body, phi_k, phi_s, uk, R, dt, body_vel=(0.0, 0.0, 0.0), rho_l=1000.0,
          rho_g=1.2, smooth=True, tol=1e-10):
    """Both stages; returns a dict with the provisional fields, the pressures
    and the velocities of each stage."""
    vel = tuple(float(v) for v in body_vel)
    op1 = Operator(grid, body, phi_k, rho_l, rho_g, smooth)
    ut1 = tuple(u + dt * r for u, r in zip(uk, R))
    b1 = op1.rhs(*ut1, dt, vel)
    p1, res1 = _solve(op1, b1, tol)
    us = update_velocity(op1, ut1, p1, dt)
    op2 = Operator(grid, body, phi_s, rho_l, rho_g, smooth)
    ut2 = tuple((a + u) + dt * r for a, u, r in zip(us, uk, R))
    vel2 = tuple(2.0 * v for v in vel)
    b2 = op2.rhs(*ut2, dt, vel2)
    p2, res2 = _solve(op2, b2, tol)
    un = update_velocity(op2, ut2, p2, dt, 0.5)
    return dict(op1=op1, op2=op2, ut1=ut1, b1=b1, p1=p1, us=us, ut2=ut2, b2=b2, p2=p2, un=un,
                res1=res1, res2=res2, vel2=vel2)
