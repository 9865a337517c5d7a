"""Operator-split VOF advection (oracle, FP64).

Test infrastructure: a plain CPU statement of the volume-fraction update of
the Interface reconstruction and advection section (eqs. diverge and vof),
for checking the GPU path against.  It advances the water fraction phi by one
time step dt through a face-velocity field that is not exactly solenoidal and
is cut by the body:

1. Flux correction.  With the face fluxes F = A (u - v) (A the open face
   areas, u - v the velocity relative to the body, given), every active cell's
   imbalance E = (F1+ - F1-) + (F2+ - F2-) + (F3+ - F3-) is removed along the
   vertical: F3+ -= E A3+/(A3+ + A3-), F3- += E A3-/(A3+ + A3-) (when A3+ +
   A3- > 0).  Each cell then gets its own face velocities on uncut areas,
   uhat_i = dx_i F_i / V (continuous across x- and y-faces, per cell on
   z-faces).
2. Interface reconstruction (piecewise linear).  In each cell with
   EPS < phi < 1 - EPS the interface is the plane m . x = alpha with
   m = -grad phi from weighted central differences over the 3x3x3
   neighbourhood (weights 1/4, 1/2, 1/4 across the difference direction; a
   neighbour beyond the domain repeats the edge cell, one inside the body
   takes the cell's own fraction), and alpha such that the water below the
   plane fills phi of the cell.
3. Three one-directional sweeps, in the order x, y, z on even steps and z, y,
   x on odd ones.  In direction d each cell loses the water volume its faces
   pass in dt, F_d[uhat, phi, dt]: the water in the slab of thickness |uhat|
   dt of the upwind cell next to the face (full slab volume times phi in a
   cell without an interface plane), and gains the dilation term dt phi
   (uhat+ - uhat-)/dx_d that keeps 0 <= phi <= 1: with the sweep's input
   phi (explicit) in the first two sweeps, with its output (implicit) in the
   last.

Readings where the paper is silent or garbled (each taken identically by the
GPU path): the normal stencil and its boundary and body treatment; the plane
constant by 64 bisection steps on the cell's volume function; a fraction
within EPS = 1e-12 of 0 or 1 is an empty or full cell without a plane (the
rounding of the dilation term leaves full cells at 1 - 1e-16, whose planes
would be arbitrary); the first two sweeps explicit and the last implicit (the
text; the printed equations place the new value in the first and the old one
in the last, and name an undefined phi-hat in the last); a face on the domain
boundary draws from the cell inside it; cells inside the body keep their
fraction.
"""
from __future__ import annotations

import numpy as np

W = (0.25, 0.5, 0.25)
BISECT = 64
EPS = 1e-12        # fractions within EPS of 0 or 1 count as empty or full (no plane)


# --------------------------------------------------------------- geometry
def unit_fraction(n1, n2, n3, a):
    """Fraction of the unit cube with n1 x + n2 y + n3 z <= a, for
    0 <= n1 <= n2 <= n3, n1 + n2 + n3 = 1 (elementwise arrays)."""
    n1, n2, n3, a = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (n1, n2, n3, a)))
    out = np.zeros(a.shape)
    low = a <= 0.5
    s = np.where(low, a, 1.0 - a)                   # V(a) = 1 - V(1 - a)
    n12 = n1 + n2
    with np.errstate(divide="ignore", invalid="ignore"):
        vA = (s * s * s) / (6.0 * n1 * n2 * n3)
        vB = (s * (s - n1) + n1 * n1 / 3.0) / (2.0 * n2 * n3)
        vC = ((s * s * (3.0 * n12 - s) + n1 * n1 * (n1 - 3.0 * s)) + n2 * n2 * (n2 - 3.0 * s)) / (6.0 * n1 * n2 * n3)
        vD1 = (((s * s * (3.0 - 2.0 * s) + n1 * n1 * (n1 - 3.0 * s)) + n2 * n2 * (n2 - 3.0 * s))
               + n3 * n3 * (n3 - 3.0 * s)) / (6.0 * n1 * n2 * n3)
        vD2 = (2.0 * s - n12) / (2.0 * n3)
    v = np.where(s <= n1, vA,
                 np.where(s <= n2, vB,
                          np.where(s <= np.minimum(n12, n3), vC, np.where(n3 < n12, vD1, vD2))))
    v = np.where(s <= 0.0, 0.0, v)
    out = np.where(low, v, 1.0 - v)
    out = np.where(a <= 0.0, 0.0, np.where(a >= 1.0, 1.0, out))
    return out


def _sorted3(n):
    """n: (..., 3) -> ascending components."""
    return np.sort(n, axis=-1)


def box_fraction(n, lo, hi, t):
    """Water fraction of the sub-box [lo, hi] (scaled coordinates in the unit
    cube, (..., 3)) under sum_d n_d xi_d <= t, n >= 0."""
    ext = hi - lo
    nn = n * ext
    S = (nn[..., 0] + nn[..., 1]) + nn[..., 2]
    nl = n * lo
    tt = t - ((nl[..., 0] + nl[..., 1]) + nl[..., 2])
    with np.errstate(divide="ignore", invalid="ignore"):
        ns = _sorted3(nn / S[..., None])
        f = unit_fraction(ns[..., 0], ns[..., 1], ns[..., 2], tt / S)
    # a plane parallel to the box (S = 0 cannot occur for a real normal and
    # a slab of positive thickness) counts as empty/full by the sign of tt
    return np.where(S > 0, f, np.where(tt >= 0, 1.0, 0.0))


def plane(m, dims, phi):
    """Reflected, scaled plane of a cell: signs s (1 or -1 per axis: -1 where
    the axis is reflected so that the normal is non-negative), n >= 0 with
    sum 1, and t in [0, 1] such that the fraction of {n . xi <= t} is phi."""
    s = np.where(m < 0, -1.0, 1.0)
    nm = np.abs(m) * dims
    S = (nm[..., 0] + nm[..., 1]) + nm[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        n = nm / S[..., None]
    ns = _sorted3(n)
    lo = np.zeros(phi.shape)
    hi = np.ones(phi.shape)
    for _ in range(BISECT):
        mid = 0.5 * (lo + hi)
        f = unit_fraction(ns[..., 0], ns[..., 1], ns[..., 2], mid)
        below = f < phi
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    return s, n, 0.5 * (lo + hi)


def slab_water(s, n, t, phi, has_plane, d, upper, frac, vol):
    """Water volume in the slab of relative thickness frac (0..1) of a cell
    next to its upper (or lower) face in direction d; vol is the cell
    volume."""
    lo = np.zeros(n.shape)
    hi = np.ones(n.shape)
    if upper:
        lo[..., d] = 1.0 - frac
    else:
        hi[..., d] = frac
    # reflected axis: [l, h] -> [1 - h, 1 - l]
    refl = s[..., d] < 0
    l_d = np.where(refl, 1.0 - hi[..., d], lo[..., d])
    h_d = np.where(refl, 1.0 - lo[..., d], hi[..., d])
    lo[..., d], hi[..., d] = l_d, h_d
    f = box_fraction(n, lo, hi, t)
    slab = frac * vol
    return np.where(has_plane, slab * f, slab * phi)


# --------------------------------------------------------------- normals
def _shift(a, d, k, fill):
    """a shifted so that out[i] = a[i + k] along array axis d; `fill` where
    i + k leaves the domain."""
    out = np.empty_like(a)
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    n = a.shape[d]
    if k > 0:
        src[d], dst[d] = slice(k, n), slice(0, n - k)
        rest = [slice(None)] * 3
        rest[d] = slice(n - k, n)
    else:
        src[d], dst[d] = slice(0, n + k), slice(-k, n)
        rest = [slice(None)] * 3
        rest[d] = slice(0, -k)
    out[tuple(dst)] = a[tuple(src)]
    out[tuple(rest)] = fill[tuple(rest)]
    return out


def _clamp(a, d, k):
    """a shifted so that out[i] = a[i + k] along array axis d, with i + k
    clamped to the domain (the edge value repeats beyond it)."""
    idx = np.clip(np.arange(a.shape[d]) + k, 0, a.shape[d] - 1)
    return np.take(a, idx, axis=d)


def normals(grid, phi, active):
    """m = -grad phi (cells, (nz, ny, nx, 3) in x, y, z order) by weighted
    central differences; a neighbour beyond the domain repeats the edge cell
    (zero normal gradient at the boundary), one inside the body takes the
    centre cell's fraction."""
    ph = np.clip(phi, 0.0, 1.0)
    act = active > 0
    axes = (grid.ax, grid.ay, grid.az)
    arr_axis = (2, 1, 0)
    cache = {}

    def nb(dz, dy, dx):
        key = (dz, dy, dx)
        if key not in cache:
            v, a = ph, act
            for ax_, k in ((0, dz), (1, dy), (2, dx)):
                if k:
                    v = _clamp(v, ax_, k)
                    a = _clamp(a, ax_, k)
            cache[key] = np.where(a, v, ph)
        return cache[key]

    m = np.zeros(phi.shape + (3,))
    for d in range(3):
        ax = axes[d]
        c = ax.c
        # centre distances with mirrored ghosts across the boundary faces
        cg = np.concatenate([[2.0 * ax.f[0] - c[0]], c, [2.0 * ax.f[-1] - c[-1]]])
        den = cg[2:] - cg[:-2]
        shape = [1, 1, 1]
        shape[arr_axis[d]] = -1
        den = den.reshape(shape)
        others = [e for e in range(3) if e != d]
        acc = np.zeros(phi.shape)
        for i1, w1 in zip((-1, 0, 1), W):
            for i2, w2 in zip((-1, 0, 1), W):
                off_p = [0, 0, 0]
                off_m = [0, 0, 0]
                off_p[others[0]] = off_m[others[0]] = i1
                off_p[others[1]] = off_m[others[1]] = i2
                off_p[d], off_m[d] = 1, -1
                # offsets are in x, y, z order; nb takes (dz, dy, dx)
                vp = nb(off_p[2], off_p[1], off_p[0])
                vm = nb(off_m[2], off_m[1], off_m[0])
                acc = acc + (w1 * w2) * (vp - vm)
        m[..., d] = -(acc / den)
    return m


# --------------------------------------------------------------- fluxes
def corrected_velocities(grid, body, u, v, w):
    """uhat on the six faces of every cell: dict with keys ('x', 0|1) ...
    (0 = lower face, 1 = upper face), cell arrays; zero on inactive cells."""
    ox, oy, oz = body.open_x, body.open_y, body.open_z
    fx, fy, fz = ox * u, oy * v, oz * w
    Fxm, Fxp = fx[:, :, :-1], fx[:, :, 1:]
    Fym, Fyp = fy[:, :-1, :], fy[:, 1:, :]
    Fzm, Fzp = fz[:-1], fz[1:]
    E = ((Fxp - Fxm) + (Fyp - Fym)) + (Fzp - Fzm)
    Azm, Azp = oz[:-1], oz[1:]
    den = Azp + Azm
    with np.errstate(divide="ignore", invalid="ignore"):
        Fzp = np.where(den > 0, Fzp - (E * Azp) / den, Fzp)
        Fzm = np.where(den > 0, Fzm + (E * Azm) / den, Fzm)
    dx = grid.ax.d[None, None, :]
    dy = grid.ay.d[None, :, None]
    dz = grid.az.d[:, None, None]
    V = grid.volumes()
    act = body.active > 0
    out = {}
    for key, val in ((("x", 0), dx * Fxm / V), (("x", 1), dx * Fxp / V), (("y", 0), dy * Fym / V),
                     (("y", 1), dy * Fyp / V), (("z", 0), dz * Fzm / V), (("z", 1), dz * Fzp / V)):
        out[key] = np.where(act, val, 0.0)
    return out


def sweep(grid, body, phi, uhat, d, dt, implicit):
    """One directional sweep (d = 0, 1, 2 for x, y, z) of phi."""
    name = "xyz"[d]
    arr = (2, 1, 0)[d]
    act = body.active > 0
    dims_all = np.stack(np.broadcast_arrays(grid.ax.d[None, None, :], grid.ay.d[None, :, None],
                                            grid.az.d[:, None, None]), axis=-1)
    V = grid.volumes()
    m = normals(grid, phi, body.active)
    interface = (phi > EPS) & (phi < 1.0 - EPS) & (np.sum(np.abs(m), axis=-1) > 0)
    s, n, t = plane(m, dims_all, np.clip(phi, 0.0, 1.0))
    width = dims_all[..., d]

    def water(donor_shift, upper, speed):
        """Water volume passed by a face of speed `speed` (>= 0) from the donor
        cell `donor_shift` away along d (its upper or lower slab)."""
        fields = [s, n, t, phi, interface, width, V]
        if donor_shift:
            fields = [_shift(f, arr, donor_shift, f) for f in fields]
        ds, dn, dt_, dphi, dint, dw, dV = fields
        frac_d = np.minimum(speed * dt, dw) / dw
        return slab_water(ds, dn, dt_, np.clip(dphi, 0.0, 1.0), dint, d, upper, frac_d, dV)

    up = uhat[(name, 1)]
    lo = uhat[(name, 0)]
    # upper face: outflow from this cell's upper slab, inflow from the next
    # cell's lower slab (a boundary face draws from this cell)
    f_up = np.where(up > 0, water(0, True, up), -water(1, False, -up))
    # lower face: inflow from the previous cell's upper slab, outflow from
    # this cell's lower slab
    f_lo = np.where(lo > 0, water(-1, True, lo), -water(0, False, -lo))
    div = (up - lo) / width
    rest = phi - (f_up - f_lo) / V
    new = rest / (1.0 - dt * div) if implicit else rest + dt * phi * div
    return np.where(act, new, phi)


def advect(grid, body, phi, u, v, w, dt, step=0):
    """One time step of the split advection; returns the new fractions."""
    uhat = corrected_velocities(grid, body, u, v, w)
    order = (0, 1, 2) if step % 2 == 0 else (2, 1, 0)
    out = np.array(phi, dtype=np.float64, copy=True)
    for i, d in enumerate(order):
        out = sweep(grid, body, out, uhat, d, dt, implicit=(i == 2))
    return out
