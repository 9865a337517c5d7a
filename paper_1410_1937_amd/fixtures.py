"""Seeded synthetic inputs for the pressure projection (data only).

This module generates the *inputs* of one projection: stretched face
coordinates, nodal signed distance of the immersed body, the VOF volume
fraction, the provisional face velocity and the heave law of the body.  It
holds none of the projection's arithmetic (no metrics, apertures, densities,
face coefficients, operator or solver): both the CPU oracle and the HIP path
receive the arrays built here and compute everything else themselves.

Array conventions (all float64, C order, x fastest):
    cells      (nz, ny, nx)
    nodes      (nz+1, ny+1, nx+1)
    x-faces    (nz, ny, nx+1)
    y-faces    (nz, ny+1, nx)
    z-faces    (nz+1, ny, nx)

Workloads (stand-ins for the paper's towing-tank hulls and heaving sphere,
whose panelisations and measurements are not available):
    c1  32^3 unit cube, flat two-fluid interface at z = 0.5, Dirichlet top
    c2  256x128x96 stretched grid, wavy free surface, Wigley-like ellipsoid
    c3  512x256x192 stretched grid, free surface + 200 droplets/bubbles,
        immersed sphere
    c4  c2 geometry with the free surface advected over 200 time steps
    c5  768x384x256, c3 rules, heaving sphere, 50 consecutive projections
Domain proportions follow the paper's computational box (length, width,
depth, height = 3, 1, 1, 0.5 ship lengths; Results section) with ship length
0.5 and the mean free surface at z = 0.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BC_NEUMANN = 0
BC_DIRICHLET = 1

# Kelvin transverse wavelength 2*pi*Fr^2*L sets the free-surface wavenumber.
FROUDE = 0.4316
SHIP_LENGTH = 0.5
DOMAIN = ((-0.75, 0.75), (-0.25, 0.25), (-0.5, 0.25))


# --------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------
def uniform_faces(a: float, b: float, n: int) -> np.ndarray:
    return a + (b - a) * np.arange(n + 1, dtype=np.float64) / n


def stretched_faces(a: float, b: float, n: int, centers, delta: float = 0.05,
                    ratio: float = 8.0, samples: int = 400001) -> np.ndarray:
    """Face coordinates clustered toward `centers`.

    Target spacing h(s) ~ 1 + (ratio-1)*tanh(d(s)/delta), d = distance to the
    nearest centre.  Nodes equidistribute the weight w = 1/h, i.e. w(x) dx/dxi
    is constant: the exact first integral of the one-dimensional elliptic
    stretching equation (Gridding section, eq. grid).
    """
    s = np.linspace(a, b, samples)
    d = np.min(np.abs(s[:, None] - np.asarray(centers, dtype=np.float64)[None, :]), axis=1)
    h = 1.0 + (ratio - 1.0) * np.tanh(d / delta)
    w = 1.0 / h
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (w[1:] + w[:-1]) * np.diff(s))])
    cum /= cum[-1]
    xi = np.arange(n + 1, dtype=np.float64) / n
    x = np.interp(xi, cum, s)
    x[0], x[-1] = a, b
    return x


def centres(f: np.ndarray) -> np.ndarray:
    return 0.5 * (f[1:] + f[:-1])


# --------------------------------------------------------------------------
# free surface, VOF, droplets
# --------------------------------------------------------------------------
def surface_modes(seed: int, m: int = 16, amp: float = 0.002):
    rng = np.random.default_rng(seed)
    k0 = 1.0 / (FROUDE ** 2 * SHIP_LENGTH)
    kmag = rng.uniform(k0, 4.0 * k0, m)
    ang = rng.uniform(0.0, 2.0 * math.pi, m)
    a = amp * rng.standard_normal(m)
    th = rng.uniform(0.0, 2.0 * math.pi, m)
    return k0, kmag * np.cos(ang), kmag * np.sin(ang), a, th


def eta(x: np.ndarray, y: np.ndarray, modes, shift: float = 0.0) -> np.ndarray:
    """Free-surface elevation on the (y, x) plane of centres (shape (ny, nx))."""
    k0, kx, ky, a, th = modes
    X = (x - shift)[None, :]
    Y = y[:, None]
    e = 0.02 * np.sin(k0 * X) * np.exp(-(Y ** 2) / 0.1 ** 2)
    for i in range(len(a)):
        e = e + a[i] * np.cos(kx[i] * X + ky[i] * Y + th[i])
    return e


def vof_from_surface(xf, yf, zf, eta_yx, zshift: float = 0.0) -> np.ndarray:
    """phi = clip(0.5 - (z_c - eta)/(1.5 dz), 0, 1): a surface smeared over 1.5 cells."""
    zc = centres(zf) + zshift
    dz = np.diff(zf)
    phi = 0.5 - (zc[:, None, None] - eta_yx[None, :, :]) / (1.5 * dz[:, None, None])
    return np.clip(phi, 0.0, 1.0)


def add_droplets(phi, xf, yf, zf, eta_fn, seed: int, n_drop: int = 100,
                 n_bub: int = 100, body=None, shift=(0.0, 0.0, 0.0)):
    """Spherical droplets above and bubbles below the surface (breaking-wave
    stand-in).  Radius 1-4 local cells, smeared over 1.5 local cells."""
    rng = np.random.default_rng(seed)
    xc, yc, zc = centres(xf), centres(yf), centres(zf)
    dx, dy, dz = np.diff(xf), np.diff(yf), np.diff(zf)
    spheres = []
    for kind, count in (("drop", n_drop), ("bub", n_bub)):
        made = 0
        while made < count:
            cx = rng.uniform(-0.6, 0.6)
            cy = rng.uniform(-0.2, 0.2)
            off = rng.uniform(0.005, 0.05)
            e0 = float(eta_fn(np.array([cx]), np.array([cy]))[0, 0])
            cz = e0 + off if kind == "drop" else e0 - off
            i = int(np.clip(np.searchsorted(xf, cx) - 1, 0, len(xc) - 1))
            j = int(np.clip(np.searchsorted(yf, cy) - 1, 0, len(yc) - 1))
            k = int(np.clip(np.searchsorted(zf, cz) - 1, 0, len(zc) - 1))
            hloc = min(dx[i], dy[j], dz[k])
            r = rng.uniform(1.0, 4.0) * hloc
            if body is not None:
                bc, br = body
                if math.dist((cx, cy, cz), bc) < br + r + 3.0 * hloc:
                    continue
            spheres.append((kind, cx + shift[0], cy + shift[1], cz + shift[2], r, hloc))
            made += 1
    for kind, cx, cy, cz, r, hloc in spheres:
        reach = r + 2.0 * hloc
        i0, i1 = np.searchsorted(xc, cx - reach), np.searchsorted(xc, cx + reach)
        j0, j1 = np.searchsorted(yc, cy - reach), np.searchsorted(yc, cy + reach)
        k0, k1 = np.searchsorted(zc, cz - reach), np.searchsorted(zc, cz + reach)
        if i0 >= i1 or j0 >= j1 or k0 >= k1:
            continue
        dist = np.sqrt((xc[None, None, i0:i1] - cx) ** 2 + (yc[None, j0:j1, None] - cy) ** 2
                       + (zc[k0:k1, None, None] - cz) ** 2)
        f = np.clip(0.5 - (dist - r) / (1.5 * hloc), 0.0, 1.0)
        blk = phi[k0:k1, j0:j1, i0:i1]
        if kind == "drop":
            np.maximum(blk, f, out=blk)
        else:
            np.minimum(blk, 1.0 - f, out=blk)
    return phi


# --------------------------------------------------------------------------
# bodies: signed distance at nodes, positive in the fluid
# --------------------------------------------------------------------------
def psi_ellipsoid(xf, yf, zf, axes=(0.25, 0.025, 0.03125), centre=(0.0, 0.0, 0.0)):
    """Wigley-like ellipsoid (L:B:T = 1:0.1:0.0625, L = 0.5), centred on the
    mean waterline so that it pierces the free surface.  Only the sign and the
    direction of the gradient are used, so a scaled level function stands in
    for the true distance."""
    X = (xf - centre[0])[None, None, :] / axes[0]
    Y = (yf - centre[1])[None, :, None] / axes[1]
    Z = (zf - centre[2])[:, None, None] / axes[2]
    return 0.025 * (np.sqrt(X * X + Y * Y + Z * Z) - 1.0)


def psi_sphere(xf, yf, zf, radius=0.1, centre=(0.0, 0.0, -0.15)):
    return np.sqrt((xf[None, None, :] - centre[0]) ** 2 + (yf[None, :, None] - centre[1]) ** 2
                   + (zf[:, None, None] - centre[2]) ** 2) - radius


def psi_plane_z(xf, yf, zf, z0):
    """Half-space body below z = z0 (a flat sea bed); exact for tests."""
    return np.broadcast_to((zf - z0)[:, None, None], (len(zf), len(yf), len(xf))).copy()


# --------------------------------------------------------------------------
# provisional face velocity (u~ = u^k + dt R), zero normal flow on the walls
# --------------------------------------------------------------------------
def face_velocity(xf, yf, zf, seed: int, modes: int = 8, phase: float = 0.0):
    rng = np.random.default_rng(seed)
    def norm(f):
        return (f - f[0]) / (f[-1] - f[0])
    xs, ys, zs = norm(xf), norm(yf), norm(zf)           # at faces
    xc, yc, zc = centres(xs), centres(ys), centres(zs)  # at centres
    nx, ny, nz = len(xc), len(yc), len(zc)
    u = np.zeros((nz, ny, nx + 1))
    v = np.zeros((nz, ny + 1, nx))
    w = np.zeros((nz + 1, ny, nx))
    for comp, out in ((0, u), (1, v), (2, w)):
        c = rng.standard_normal(modes)
        p = rng.integers(1, 5, size=(modes, 3))
        for m in range(modes):
            ax = [xc, yc, zc]
            ax[comp] = [xs, ys, zs][comp]
            fx = (np.sin if comp == 0 else np.cos)(math.pi * p[m, 0] * ax[0] + (phase if comp == 0 else 0.0))
            fy = (np.sin if comp == 1 else np.cos)(math.pi * p[m, 1] * ax[1] + (phase if comp == 1 else 0.0))
            fz = (np.sin if comp == 2 else np.cos)(math.pi * p[m, 2] * ax[2] + (phase if comp == 2 else 0.0))
            out += c[m] * fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
    # keep the normal component zero on the walls even with a phase shift
    u[:, :, 0] = u[:, :, -1] = 0.0
    v[:, 0, :] = v[:, -1, :] = 0.0
    w[0, :, :] = w[-1, :, :] = 0.0
    return u, v, w


def fourier_rhs(xf, yf, zf, seed: int, kmax: int = 4) -> np.ndarray:
    """Smooth random Fourier modes (|k_i| <= kmax) times the cell volume, mean removed."""
    rng = np.random.default_rng(seed)
    xc, yc, zc = centres(xf), centres(yf), centres(zf)
    vol = np.diff(zf)[:, None, None] * np.diff(yf)[None, :, None] * np.diff(xf)[None, None, :]
    b = np.zeros(vol.shape)
    for kz in range(kmax + 1):
        for ky in range(kmax + 1):
            for kx in range(kmax + 1):
                if kx == ky == kz == 0:
                    continue
                a = rng.standard_normal() / (1.0 + kx * kx + ky * ky + kz * kz)
                th = rng.uniform(0.0, 2.0 * math.pi)
                b += a * np.cos(2 * math.pi * (kx * xc[None, None, :] + ky * yc[None, :, None]
                                                 + kz * zc[:, None, None]) + th)
    b *= vol
    return b - b.mean()


# --------------------------------------------------------------------------
# heave law (Initial Transients section, eq. heave)
# --------------------------------------------------------------------------
def ramp(t, T0=0.5):
    return 1.0 - math.exp(-(t / T0) ** 2), 2.0 * t / T0 ** 2 * math.exp(-(t / T0) ** 2)


def heave(t, A=0.05, omega=2 * math.pi, T0=0.5):
    f, fp = ramp(t, T0)
    z = A * math.sin(omega * t) * f
    v3 = A * omega * math.cos(omega * t) * f + A * math.sin(omega * t) * fp
    return z, v3


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    xf: np.ndarray
    yf: np.ndarray
    zf: np.ndarray
    bc: tuple
    phi: np.ndarray
    psi: np.ndarray | None
    theta: float
    smooth: bool
    rho_l: float = 1000.0
    rho_g: float = 1.2
    b: np.ndarray | None = None          # given directly (c1) ...
    u: np.ndarray | None = None          # ... or from the face velocity
    v: np.ndarray | None = None
    w: np.ndarray | None = None
    dt: float = 1.0
    body_vel: tuple = (0.0, 0.0, 0.0)
    tol: float = 1e-8
    samples: int = 8

    @property
    def shape(self):
        return (len(self.zf) - 1, len(self.yf) - 1, len(self.xf) - 1)

    @property
    def ncells(self):
        nz, ny, nx = self.shape
        return nx * ny * nz


ALL_NEUMANN = (BC_NEUMANN,) * 6


def c1(seed: int = 0) -> Workload:
    n = 32
    xf = yf = zf = uniform_faces(0.0, 1.0, n)
    zc = centres(zf)
    phi = np.broadcast_to((zc < 0.5).astype(np.float64)[:, None, None], (n, n, n)).copy()
    b = fourier_rhs(xf, yf, zf, seed)
    bc = (BC_NEUMANN, BC_NEUMANN, BC_NEUMANN, BC_NEUMANN, BC_NEUMANN, BC_DIRICHLET)
    return Workload("c1", xf, yf, zf.copy(), bc, phi, None, 0.25, False, b=b, tol=1e-10)


def _grid(nx, ny, nz, cx, cy, cz):
    (x0, x1), (y0, y1), (z0, z1) = DOMAIN
    return (stretched_faces(x0, x1, nx, cx), stretched_faces(y0, y1, ny, cy),
            stretched_faces(z0, z1, nz, cz))


def c2(seed: int = 0, nx=256, ny=128, nz=96, t: float = 0.0, rhs_seed=None) -> Workload:
    xf, yf, zf = _grid(nx, ny, nz, [-0.25, 0.25], [0.0], [0.0])
    modes = surface_modes(seed)
    e = eta(centres(xf), centres(yf), modes, shift=t)
    phi = vof_from_surface(xf, yf, zf, e)
    psi = psi_ellipsoid(xf, yf, zf)
    u, v, w = face_velocity(xf, yf, zf, seed if rhs_seed is None else rhs_seed)
    return Workload("c2", xf, yf, zf, ALL_NEUMANN, phi, psi, 0.1, True, u=u, v=v, w=w)


def c3(seed: int = 1, nx=512, ny=256, nz=192, t: float = 0.0) -> Workload:
    """Breaking-wave workload; t > 0 moves the surface and the droplets by t in
    x (the advected volume fraction of a later time)."""
    xf, yf, zf = _grid(nx, ny, nz, [-0.1, 0.1], [0.0], [0.0, -0.15])
    modes = surface_modes(seed)
    e = eta(centres(xf), centres(yf), modes, shift=t)
    phi = vof_from_surface(xf, yf, zf, e)
    phi = add_droplets(phi, xf, yf, zf, lambda x, y: eta(x, y, modes), seed,
                       body=((0.0, 0.0, -0.15), 0.1), shift=(t, 0.0, 0.0))
    psi = psi_sphere(xf, yf, zf)
    u, v, w = face_velocity(xf, yf, zf, seed)
    return Workload("c3", xf, yf, zf, ALL_NEUMANN, phi, psi, 0.25, True, u=u, v=v, w=w)


def c4_step(n: int, nx=256, ny=128, nz=96) -> Workload:
    """Time step n of the advected free surface (t_n = 0.005 n, unit speed)."""
    wl = c2(0, nx, ny, nz, t=0.005 * n, rhs_seed=1000 + n)
    wl.name = f"c4_{n}"
    return wl


class C4Sequence:
    """The 200-step advected free surface on the c2 geometry: the grid, the
    hull and the surface modes are built once; step n moves the surface by
    t_n = 0.005 n (unit speed) and draws the face velocity with seed 1000 + n."""

    def __init__(self, nx=256, ny=128, nz=96, seed=0):
        self.xf, self.yf, self.zf = _grid(nx, ny, nz, [-0.25, 0.25], [0.0], [0.0])
        self.modes = surface_modes(seed)
        self.psi = psi_ellipsoid(self.xf, self.yf, self.zf)
        self.xc, self.yc = centres(self.xf), centres(self.yf)
        self.bc = ALL_NEUMANN
        self.theta = 0.1
        self.shape = (nz, ny, nx)

    def step(self, n: int):
        e = eta(self.xc, self.yc, self.modes, shift=0.005 * n)
        phi = vof_from_surface(self.xf, self.yf, self.zf, e)
        return phi, face_velocity(self.xf, self.yf, self.zf, 1000 + n)

    def smooth_field(self, seed: int, modes: int = 6):
        """A smooth random cell field (low Fourier modes) used as a synthetic error."""
        rng = np.random.default_rng(seed)
        xs = (self.xc - self.xf[0]) / (self.xf[-1] - self.xf[0])
        ys = (self.yc - self.yf[0]) / (self.yf[-1] - self.yf[0])
        zc = centres(self.zf)
        zs = (zc - self.zf[0]) / (self.zf[-1] - self.zf[0])
        out = np.zeros(self.shape)
        for _ in range(modes):
            k = rng.integers(1, 7, size=3)
            ph = rng.uniform(0, 2 * math.pi, size=3)
            out += rng.standard_normal() * (np.cos(math.pi * k[2] * zs + ph[2])[:, None, None]
                                            * np.cos(math.pi * k[1] * ys + ph[1])[None, :, None]
                                            * np.cos(math.pi * k[0] * xs + ph[0])[None, None, :])
        return out


def c5_step(n: int, nx=768, ny=384, nz=256, seed: int = 1) -> Workload:
    """Projection n of the heaving-sphere sequence, body-fixed frame: the body
    is static; surface and droplets move by -z_h(t) in z and +t in x."""
    t = 0.5 + 0.01 * n
    zh, v3 = heave(t)
    xf, yf, zf = _grid(nx, ny, nz, [-0.1, 0.1], [0.0], [0.0, -0.15])
    modes = surface_modes(seed)
    e = eta(centres(xf), centres(yf), modes, shift=t) - zh
    phi = vof_from_surface(xf, yf, zf, e)
    phi = add_droplets(phi, xf, yf, zf, lambda x, y: eta(x, y, modes), seed,
                       body=((0.0, 0.0, -0.15), 0.1), shift=(t, 0.0, -zh))
    psi = psi_sphere(xf, yf, zf)
    u, v, w = face_velocity(xf, yf, zf, seed, phase=t)
    return Workload(f"c5_{n}", xf, yf, zf, ALL_NEUMANN, phi, psi, 0.25, True,
                    u=u, v=v, w=w, body_vel=(0.0, 0.0, v3))


# --------------------------------------------------------------------------
# triangulated body surfaces (panels (m, 3, 3), outward-oriented)
# --------------------------------------------------------------------------
def box_panels(lo, hi) -> np.ndarray:
    """The 12 triangles of an axis-aligned box, outward normals."""
    lo, hi = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
    corner = lambda i, j, k: np.array([(lo, hi)[i][0], (lo, hi)[j][1], (lo, hi)[k][2]])
    quads = [((0, 0, 0), (0, 1, 0), (1, 1, 0), (1, 0, 0)),    # z = lo (normal -z)
             ((0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)),    # z = hi
             ((0, 0, 0), (1, 0, 0), (1, 0, 1), (0, 0, 1)),    # y = lo
             ((0, 1, 0), (0, 1, 1), (1, 1, 1), (1, 1, 0)),    # y = hi
             ((0, 0, 0), (0, 0, 1), (0, 1, 1), (0, 1, 0)),    # x = lo
             ((1, 0, 0), (1, 1, 0), (1, 1, 1), (1, 0, 1))]    # x = hi
    tris = []
    for q in quads:
        v = [corner(*c) for c in q]
        tris += [(v[0], v[1], v[2]), (v[0], v[2], v[3])]
    return np.array(tris)


def icosphere_panels(radius=0.1, centre=(0.0, 0.0, -0.15), levels=3) -> np.ndarray:
    """A sphere triangulated by `levels` midpoint subdivisions of an
    icosahedron (20 * 4**levels triangles), vertices on the sphere."""
    t = (1.0 + 5 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6),
         (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
         (8, 6, 7), (9, 8, 1)]
    tris = np.array([[v[a], v[b], v[c]] for a, b, c in f], dtype=np.float64)
    tris /= np.linalg.norm(tris, axis=-1, keepdims=True)
    for _ in range(levels):
        a, b, c = tris[:, 0], tris[:, 1], tris[:, 2]
        ab, bc, ca = ((x + y) for x, y in ((a, b), (b, c), (c, a)))
        ab, bc, ca = (m / np.linalg.norm(m, axis=-1, keepdims=True) for m in (ab, bc, ca))
        tris = np.concatenate([np.stack(q, axis=1) for q in ((a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca))])
    if np.mean(np.sum(np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0]) * tris[:, 0], axis=-1)) < 0:
        tris = tris[:, ::-1]
    return tris * radius + np.asarray(centre, dtype=np.float64)


def wigley_panels(length=0.5, beam=0.05, draft=0.03125, freeboard=0.02, nx=40, nz=10) -> np.ndarray:
    """A closed Wigley-type hull: half-breadth y = (B/2)(1 - (2x/L)^2)(1 - (z/T)^2)
    below the waterline z = 0, vertical sides up to a flat deck at z = freeboard;
    the two sides meet on the keel and at bow and stern.  Outward normals."""
    xs = np.linspace(-length / 2, length / 2, nx + 1)
    zs = np.concatenate([np.linspace(-draft, 0.0, nz + 1), [freeboard]])
    def half(x, z):
        return 0.5 * beam * (1 - (2 * x / length) ** 2) * (1 - (min(z, 0.0) / draft) ** 2)
    tris = []
    for side in (1.0, -1.0):
        P = [[np.array([x, side * half(x, z), z]) for z in zs] for x in xs]
        for i in range(nx):
            for k in range(len(zs) - 1):
                a, b, c, d = P[i][k], P[i + 1][k], P[i + 1][k + 1], P[i][k + 1]
                tris += [(a, b, c), (a, c, d)] if side < 0 else [(a, c, b), (a, d, c)]
    top = freeboard
    for i in range(nx):
        x0, x1 = xs[i], xs[i + 1]
        a, b = np.array([x0, -half(x0, top), top]), np.array([x1, -half(x1, top), top])
        c, d = np.array([x1, half(x1, top), top]), np.array([x0, half(x0, top), top])
        tris += [(a, b, c), (a, c, d)]
    tris = np.array(tris)
    area = np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0])
    keep = np.linalg.norm(area, axis=-1) > 1e-14 * length ** 2      # drop the degenerate panels at bow and stern
    return tris[keep]


def vof_time_step(wl: Workload, courant: float = 0.45) -> float:
    """A VOF time step for the workload's face velocities: the velocity a
    face can carry after the flux correction is bounded by twice the sum of
    the three components' maxima, each over the smallest width along its
    axis, so this step keeps every Courant number below `courant`."""
    rate = 2.0 * (np.max(np.abs(wl.u)) / np.min(np.diff(wl.xf)) + np.max(np.abs(wl.v)) / np.min(np.diff(wl.yf))
                  + np.max(np.abs(wl.w)) / np.min(np.diff(wl.zf)))
    return courant / rate


def small(seed: int, nx: int, ny: int, nz: int, body: str = "sphere", bc=ALL_NEUMANN,
          stretch: bool = True, theta: float = 0.25, smooth: bool = True) -> Workload:
    """Reduced-size ship-wave-shaped workload for parity tests."""
    (x0, x1), (y0, y1), (z0, z1) = DOMAIN
    if stretch:
        xf, yf, zf = _grid(nx, ny, nz, [-0.1, 0.1], [0.0], [0.0, -0.15])
    else:
        xf, yf, zf = uniform_faces(x0, x1, nx), uniform_faces(y0, y1, ny), uniform_faces(z0, z1, nz)
    modes = surface_modes(seed)
    e = eta(centres(xf), centres(yf), modes)
    phi = vof_from_surface(xf, yf, zf, e)
    if body == "sphere":
        psi = psi_sphere(xf, yf, zf, radius=0.12, centre=(0.013, -0.007, -0.11))
    elif body == "ellipsoid":
        psi = psi_ellipsoid(xf, yf, zf, axes=(0.3, 0.08, 0.09))
    else:
        psi = None
    u, v, w = face_velocity(xf, yf, zf, seed)
    return Workload(f"small{nx}x{ny}x{nz}", xf, yf, zf, tuple(bc), phi, psi, theta, smooth,
                    u=u, v=v, w=w, body_vel=(0.0, 0.0, 0.3))
