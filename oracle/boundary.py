"""Inhomogeneous Neumann data of the projection (oracle, FP64).

Test infrastructure: plain CPU statements of the two boundary fluxes the
paper feeds into the finite-volume equations of the pressure:

* the body flux of eq. integral2, the integral of v* . n over the body
  surface S_b in a cell, for a body velocity that varies from cell to cell
  (rotation, deformation): B_c = v_c . S_c, with S_c the area vector of the
  body surface in the cell (Enforcement of Body Boundary Conditions);
* the exit condition (Radiation Conditions, eqs. orlanski and exit): the
  x-velocity on the outflow face follows du/dt + u_c du/dx = 0.  Its upwind
  update of the face velocity, u_e - (u_c dt / dx)(u_e - u_i) with u_i the
  x-face one cell inward and dx that cell's width, is the provisional
  velocity of the exit face, so the prescribed flux enters the right-hand
  side through D F~ like any face flux and the exit face stays a Neumann
  face of the pressure.
"""
from __future__ import annotations

import numpy as np


def body_flux_cells(op, vb):
    """B_c = (vx_c Sx_c + vy_c Sy_c) + vz_c Sz_c with S_c = -(sum of the
    cell's signed open areas), the body surface's area vector in the cell."""
    b = op.body
    sx = -(b.open_x[:, :, 1:] - b.open_x[:, :, :-1])
    sy = -(b.open_y[:, 1:, :] - b.open_y[:, :-1, :])
    sz = -(b.open_z[1:] - b.open_z[:-1])
    return (vb[0] * sx + vb[1] * sy) + vb[2] * sz


def rhs_cells(op, u, v, w, dt, vb):
    """b' = P^T b, b = -((D F~) + B)/dt with the per-cell body flux; zero mean
    over the reduced unknowns when every boundary is Neumann."""
    fx, fy, fz = op.open_flux(u, v, w)
    b = -(op.divergence(fx, fy, fz) + body_flux_cells(op, vb)) / dt
    b = b * (op.body.active > 0)
    return op.compatible(op.gather(b))


def exit_velocity(uk_x, ut_x, uc, dt, dx_last):
    """ut_x with its +x boundary plane replaced by the upwind update of uk_x
    there: u_e - ((uc dt) / dx) (u_e - u_i)."""
    out = np.array(ut_x, dtype=np.float64, copy=True)
    c = (uc * dt) / dx_last
    ue, ui = uk_x[:, :, -1], uk_x[:, :, -2]
    out[:, :, -1] = ue - c * (ue - ui)
    return out
