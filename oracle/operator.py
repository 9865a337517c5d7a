"""Two-fluid cut-cell pressure operator (oracle).

Follows the Formulation section (eqs. density, pois), Numerical Time
Integration (eqs. poisson1, runge1), Enforcement of Body Boundary Conditions
(eqs. integral1, bc2, integral2), the face-flux definition and eq. diverge
of the interface section, and Density Smoothing.

The library solves the positive semidefinite form  A p = b  with
    (A p)_c = sum over the faces f of c of  T_f (p_c - p_nb(f))
           = -(cell integral of div((1/rho) grad p))                (eq. integral2, LHS)
    T_f     = (open area_f * beta_f) / h_f
    b_c     = -((D F~)_c + B_c) / dt                                 (eq. integral2, RHS)
    F~_f    = open area_f * u~_f          (u~ = u^k + dt R, eq. poisson1)
    B_c     = v . S_c,  S_c = -sum_f s_f open area_f e_d(f)          (body flux term)
The merged system is A' = P^T A P and b' = P^T b, where P copies a group's
root value to its slaves (merging of small cells).

Readings where the paper is silent:
  * H(phi) = clip(phi, 0, 1): phi is already a smeared volume fraction, so
    rho = rho_g + (rho_l - rho_g) H(phi) is the cell-average density.
  * rho_l and rho_g are passed as dimensional values (1000, 1.2); scaling rho
    scales A and p only.
  * smoothing (1/4, 1/2, 1/4) along x, then y, then z, evaluated as
    (0.25*a + 0.5*b) + 0.25*c, with mirrored ends (rho_-1 = rho_0).
  * interior face: beta_f = 2/(rho_L + rho_R) (harmonic mean of 1/rho);
    boundary face: beta = 1/rho_c.
  * Dirichlet p = 0 sits on the boundary face (h = half the cell width);
    Neumann faces carry no coefficient.
  * operator sum order x-, x+, y-, y+, z-, z+; merge gathers add the slaves
    (ascending index) to the root's value.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


# --------------------------------------------------------------------------
# density and face coefficients
# --------------------------------------------------------------------------
def density(phi, rho_l, rho_g, smooth):
    """Cell density from the volume fraction (eq. density), optionally
    smoothed by (1/4, 1/2, 1/4) consecutively along x, y, z (Density Smoothing)."""
    H = np.clip(np.asarray(phi, dtype=np.float64), 0.0, 1.0)
    rho = rho_g + (rho_l - rho_g) * H
    if smooth:
        for axis in (2, 1, 0):
            lo = np.concatenate([np.take(rho, [0], axis=axis),
                                 np.take(rho, range(0, rho.shape[axis] - 1), axis=axis)], axis=axis)
            hi = np.concatenate([np.take(rho, range(1, rho.shape[axis]), axis=axis),
                                 np.take(rho, [rho.shape[axis] - 1], axis=axis)], axis=axis)
            rho = (0.25 * lo + 0.5 * rho) + 0.25 * hi
    return rho


def face_beta(rho):
    """1/rho on the three face sets: 2/(rho_L + rho_R) inside, 1/rho_c on the boundary."""
    nz, ny, nx = rho.shape
    bx = np.empty((nz, ny, nx + 1))
    bx[:, :, 1:-1] = 2.0 / (rho[:, :, :-1] + rho[:, :, 1:])
    bx[:, :, 0] = 1.0 / rho[:, :, 0]
    bx[:, :, -1] = 1.0 / rho[:, :, -1]
    by = np.empty((nz, ny + 1, nx))
    by[:, 1:-1, :] = 2.0 / (rho[:, :-1, :] + rho[:, 1:, :])
    by[:, 0, :] = 1.0 / rho[:, 0, :]
    by[:, -1, :] = 1.0 / rho[:, -1, :]
    bz = np.empty((nz + 1, ny, nx))
    bz[1:-1] = 2.0 / (rho[:-1] + rho[1:])
    bz[0] = 1.0 / rho[0]
    bz[-1] = 1.0 / rho[-1]
    return bx, by, bz


class Operator:
    """Assembled operator for one projection: T on the three face sets and
    the Jacobi inverse diagonal of the merged operator."""

    def __init__(self, grid, body, phi, rho_l=1000.0, rho_g=1.2, smooth=True):
        g = grid
        self.grid, self.body = g, body
        self.rho = density(phi, rho_l, rho_g, smooth)
        bx, by, bz = face_beta(self.rho)
        hx = g.ax.h[None, None, :]
        hy = g.ay.h[None, :, None]
        hz = g.az.h[:, None, None]
        tx = (body.open_x * bx) / hx
        ty = (body.open_y * by) / hy
        tz = (body.open_z * bz) / hz
        bc = g.bc
        if not bc[0]:
            tx[:, :, 0] = 0.0
        if not bc[1]:
            tx[:, :, -1] = 0.0
        if not bc[2]:
            ty[:, 0, :] = 0.0
        if not bc[3]:
            ty[:, -1, :] = 0.0
        if not bc[4]:
            tz[0] = 0.0
        if not bc[5]:
            tz[-1] = 0.0
        self.tx, self.ty, self.tz = tx, ty, tz
        self.dinv = self._jacobi()

    # ---------------------------------------------------------------- apply
    def stencil(self, p):
        """(A p)_c = sum_f T_f (p_c - p_nb), order x-, x+, y-, y+, z-, z+;
        p_nb = 0 beyond the domain boundary."""
        p = np.asarray(p, dtype=np.float64).reshape(self.grid.shape)
        pp = np.pad(p, 1)
        c = pp[1:-1, 1:-1, 1:-1]
        s = self.tx[:, :, :-1] * (c - pp[1:-1, 1:-1, :-2])
        s = s + self.tx[:, :, 1:] * (c - pp[1:-1, 1:-1, 2:])
        s = s + self.ty[:, :-1, :] * (c - pp[1:-1, :-2, 1:-1])
        s = s + self.ty[:, 1:, :] * (c - pp[1:-1, 2:, 1:-1])
        s = s + self.tz[:-1] * (c - pp[:-2, 1:-1, 1:-1])
        s = s + self.tz[1:] * (c - pp[2:, 1:-1, 1:-1])
        return s

    def expand(self, x):
        """P x: slaves take their root's value (cell array in, cell array out)."""
        x = np.array(x, dtype=np.float64).reshape(-1)
        b = self.body
        x[b.slaves] = x[b.slave_root]
        return x.reshape(self.grid.shape)

    def gather(self, y):
        """P^T y on the cell array: each root adds its slaves (ascending), slaves -> 0."""
        y = np.array(y, dtype=np.float64).reshape(-1)
        for r, members in self.body.groups.items():
            acc = y[r]
            for s in members[1:]:
                acc = acc + y[s]
            y[r] = acc
        y[self.body.slaves] = 0.0
        return y.reshape(self.grid.shape)

    def apply(self, x):
        """A' x = P^T A P x, on cell arrays (slaves and inactive cells -> 0)."""
        return self.gather(self.stencil(self.expand(x)))

    # ------------------------------------------------------------- jacobi
    def _jacobi(self):
        """1 / diag(A'), 0 on slaves and inactive cells.  A group's diagonal is
        the sum of T over the faces of its members whose neighbour lies outside
        the group (members: root, then slaves ascending; faces x-, x+, y-, y+,
        z-, z+)."""
        g = self.grid
        nz, ny, nx = g.shape
        tx, ty, tz = self.tx, self.ty, self.tz
        d = (((((tx[:, :, :-1] + tx[:, :, 1:]) + ty[:, :-1, :]) + ty[:, 1:, :]) + tz[:-1]) + tz[1:])
        d = d.reshape(-1).copy()
        for r, members in self.body.groups.items():
            mset = set(members)
            acc = 0.0
            first = True
            for m in members:
                k, rem = divmod(m, nx * ny)
                j, i = divmod(rem, nx)
                faces = ((tx[k, j, i], m - 1 if i > 0 else -1),
                         (tx[k, j, i + 1], m + 1 if i < nx - 1 else -1),
                         (ty[k, j, i], m - nx if j > 0 else -1),
                         (ty[k, j + 1, i], m + nx if j < ny - 1 else -1),
                         (tz[k, j, i], m - nx * ny if k > 0 else -1),
                         (tz[k + 1, j, i], m + nx * ny if k < nz - 1 else -1))
                for t, nb in faces:
                    if nb in mset:
                        continue
                    acc = t if first else acc + t
                    first = False
            d[r] = acc
        d[self.body.slaves] = 0.0
        d = d.reshape(g.shape) * (self.body.active > 0)
        dinv = np.zeros_like(d)
        nzm = d > 0
        dinv[nzm] = 1.0 / d[nzm]
        return dinv

    # --------------------------------------------------------------- sparse
    def csr(self, coeffs=None):
        """A' as a scipy CSR matrix over the cell index (rows/cols of slaves and
        inactive cells are empty), assembled from the face list; `coeffs`
        (tx, ty, tz) replaces the operator's face coefficients."""
        g = self.grid
        nz, ny, nx = g.shape
        idx = np.arange(g.n).reshape(g.shape)
        tx, ty, tz = (self.tx, self.ty, self.tz) if coeffs is None else coeffs
        rows, cols, vals = [], [], []

        def couple(t, a, b):
            m = t != 0
            t, a, b = t[m], a[m], b[m]
            rows.extend([a, b, a, b])
            cols.extend([a, b, b, a])
            vals.extend([t, t, -t, -t])

        couple(tx[:, :, 1:-1].ravel(), idx[:, :, :-1].ravel(), idx[:, :, 1:].ravel())
        couple(ty[:, 1:-1, :].ravel(), idx[:, :-1, :].ravel(), idx[:, 1:, :].ravel())
        couple(tz[1:-1].ravel(), idx[:-1].ravel(), idx[1:].ravel())
        for t, cells in ((tx[:, :, 0], idx[:, :, 0]), (tx[:, :, -1], idx[:, :, -1]),
                         (ty[:, 0, :], idx[:, 0, :]), (ty[:, -1, :], idx[:, -1, :]),
                         (tz[0], idx[0]), (tz[-1], idx[-1])):
            t, cells = t.ravel(), cells.ravel()
            m = t != 0
            rows.append(cells[m])
            cols.append(cells[m])
            vals.append(t[m])
        A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(g.n, g.n))
        P = self.prolongation()
        return (P.T @ A @ P).tocsr()

    def prolongation(self):
        """P as an n x n 0/1 matrix: column r (a root) has ones on r and its slaves."""
        root = self.body.root.reshape(-1)
        act = root >= 0
        rows = np.nonzero(act)[0]
        return sp.csr_matrix((np.ones(rows.size), (rows, root[act])), shape=(self.grid.n, self.grid.n))

    # ------------------------------------------------------------ rhs etc.
    def divergence(self, fx, fy, fz):
        """(D F)_c = ((Fx+ - Fx-) + (Fy+ - Fy-)) + (Fz+ - Fz-)."""
        return ((fx[:, :, 1:] - fx[:, :, :-1]) + (fy[:, 1:, :] - fy[:, :-1, :])) + (fz[1:] - fz[:-1])

    def body_flux(self, vel):
        """B_c = v . S_c with S_c = -(sum of signed open areas): the area vector
        of the body surface inside the cell, pointing out of the fluid."""
        b = self.body
        sx = -(b.open_x[:, :, 1:] - b.open_x[:, :, :-1])
        sy = -(b.open_y[:, 1:, :] - b.open_y[:, :-1, :])
        sz = -(b.open_z[1:] - b.open_z[:-1])
        return (vel[0] * sx + vel[1] * sy) + vel[2] * sz

    def open_flux(self, u, v, w):
        b = self.body
        return b.open_x * u, b.open_y * v, b.open_z * w

    def rhs(self, u, v, w, dt, vel=(0.0, 0.0, 0.0)):
        """b' = P^T b with b = -((D F~) + B)/dt (eq. integral2); zero mean over
        the reduced unknowns when every boundary is Neumann."""
        fx, fy, fz = self.open_flux(u, v, w)
        b = -(self.divergence(fx, fy, fz) + self.body_flux(vel)) / dt
        b = b * (self.body.active > 0)
        b = self.gather(b)
        return self.compatible(b)

    def compatible(self, b):
        b = np.array(b, dtype=np.float64)
        if self.grid.all_neumann:
            m = self.body.reduced
            b[m] -= np.add.reduce(b[m].ravel()) / self.body.n_reduced
        return b

    def gauge(self, x):
        """All-Neumann: remove the mean over the reduced unknowns, expand to slaves."""
        x = np.array(x, dtype=np.float64).reshape(self.grid.shape)
        m = self.body.reduced
        if self.grid.all_neumann:
            x[m] -= np.add.reduce(x[m].ravel()) / self.body.n_reduced
        x[~m] = 0.0
        return self.expand(x)

    def project(self, u, v, w, p, dt):
        """Face flux after projection (eq. runge1 in flux form):
        F_f = F~_f - dt T_f (p_+ - p_-), p = 0 beyond a Dirichlet face."""
        p = self.expand(p)
        fx, fy, fz = self.open_flux(u, v, w)
        pp = np.pad(p, 1)
        fx = fx - dt * (self.tx * (pp[1:-1, 1:-1, 1:] - pp[1:-1, 1:-1, :-1]))
        fy = fy - dt * (self.ty * (pp[1:-1, 1:, 1:-1] - pp[1:-1, :-1, 1:-1]))
        fz = fz - dt * (self.tz * (pp[1:, 1:-1, 1:-1] - pp[:-1, 1:-1, 1:-1]))
        return fx, fy, fz

    def merged_divergence(self, fx, fy, fz, vel=(0.0, 0.0, 0.0)):
        """P^T (D F + B): discrete conservation of each merged cell (eq. diverge
        plus the body flux).  Zero for a solenoidal projected field."""
        d = (self.divergence(fx, fy, fz) + self.body_flux(vel)) * (self.body.active > 0)
        return self.gather(d)

    def reduced_mask(self):
        return self.body.reduced
