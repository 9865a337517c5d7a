"""The split VOF advection on the GPU against the oracle (needs an MI355X):
each directional sweep and whole time steps bitwise on stretched grids cut
by a body, with droplets and bubbles, ragged sizes and one-cell-thin grids;
zero velocity is the identity; bad arguments are refused; at the full
512 x 256 x 192 breaking-wave size, sampled windows are recomputed by the
oracle."""
import numpy as np
import pytest

from oracle import vof
from oracle.geometry import Body
from oracle.grid import Grid
from paper_1410_1937_amd import fixtures as fx
from tests.gpu_helpers import host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SPHERE = ((0.013, -0.007, -0.11), 0.12)


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def courant_dt(og, ob, u, v, w, c=0.45):
    """The time step at which the largest corrected face velocity crosses
    the fraction c of its cell's width."""
    uh = vof.corrected_velocities(og, ob, u, v, w)
    width = {"x": og.ax.d[None, None, :], "y": og.ay.d[None, :, None], "z": og.az.d[:, None, None]}
    return c / max(float(np.max(np.abs(uh[k]) / width[k[0]])) for k in uh)


def _case(seed, nx, ny, nz, body="sphere", drops=6):
    wl = fx.small(seed, nx, ny, nz, body=body)
    if drops:
        modes = fx.surface_modes(seed)
        wl.phi = fx.add_droplets(wl.phi.copy(), wl.xf, wl.yf, wl.zf, lambda x, y: fx.eta(x, y, modes), seed,
                                 n_drop=drops, n_bub=drops, body=SPHERE if body == "sphere" else None)
    og = Grid(wl.xf, wl.yf, wl.zf, wl.bc)
    ob = Body(og, wl.psi, wl.theta, wl.samples)
    return wl, og, ob, courant_dt(og, ob, wl.u, wl.v, wl.w)


def _gpu_vof(wl):
    from paper_1410_1937_amd import nfa
    g = nfa.Grid(wl.xf, wl.yf, wl.zf, wl.bc)
    if wl.psi is not None:
        g.set_body(_t(wl.psi), wl.theta, wl.samples)
    return nfa.Vof(g)


SHAPES = [(37, 21, 17), (70, 9, 12), (6, 33, 25)]


@pytest.mark.parametrize("shape", SHAPES)
def test_every_sweep_bitwise(shape):
    wl, og, ob, dt = _case(1, *shape)
    g = _gpu_vof(wl)
    uh = vof.corrected_velocities(og, ob, wl.u, wl.v, wl.w)
    args = tuple(_t(a) for a in (wl.phi, wl.u, wl.v, wl.w))
    assert np.count_nonzero((wl.phi > 0) & (wl.phi < 1)) > 50
    for d in range(3):
        for implicit in (False, True):
            ref = vof.sweep(og, ob, wl.phi, uh, d, dt, implicit)
            got = host(g.sweep(*args, dt, d, implicit))
            assert np.array_equal(got, ref), (d, implicit, np.max(np.abs(got - ref)))


@pytest.mark.parametrize("shape,body", [((37, 21, 17), "sphere"), ((48, 16, 20), "ellipsoid"),
                                        ((29, 13, 11), None)])
def test_two_time_steps_bitwise(shape, body):
    wl, og, ob, dt = _case(2, *shape, body=body)
    g = _gpu_vof(wl)
    phi = wl.phi
    gphi = _t(phi)
    vel = tuple(_t(a) for a in (wl.u, wl.v, wl.w))
    for step in (0, 1):
        phi = vof.advect(og, ob, phi, wl.u, wl.v, wl.w, dt, step)
        gphi = g.advect(gphi, *vel, dt, step)
        got = host(gphi)
        assert np.array_equal(got, phi), (step, np.max(np.abs(got - phi)))
    act = ob.active > 0
    assert np.array_equal(host(gphi)[~act], wl.phi[~act])          # inactive cells keep their fraction


@pytest.mark.parametrize("shape", [(1, 1, 24), (1, 19, 1), (23, 1, 1), (2, 2, 2)])
def test_one_cell_thin_grids_bitwise(shape):
    nx, ny, nz = shape
    rng = np.random.default_rng(5)
    xf, yf, zf = (np.cumsum(np.r_[0.0, rng.uniform(0.5, 1.5, n)]) for n in (nx, ny, nz))
    u, v, w = fx.face_velocity(xf, yf, zf, 9)
    phi = np.clip(rng.uniform(-0.5, 1.5, (nz, ny, nx)), 0.0, 1.0)
    og = Grid(xf, yf, zf, (0,) * 6)
    ob = Body(og, None, 0.25, 8)
    dt = courant_dt(og, ob, u, v, w)
    from paper_1410_1937_amd import nfa
    g = nfa.Vof(nfa.Grid(xf, yf, zf, (0,) * 6))
    for step in (0, 1):
        ref = vof.advect(og, ob, phi, u, v, w, dt, step)
        got = host(g.advect(_t(phi), _t(u), _t(v), _t(w), dt, step))
        assert np.array_equal(got, ref)


def test_zero_velocity_is_the_identity_and_a_full_domain_stays_full():
    wl, og, ob, dt = _case(3, 33, 17, 15)
    g = _gpu_vof(wl)
    z = tuple(torch.zeros(s, dtype=torch.float64, device="cuda") for s in (wl.u.shape, wl.v.shape, wl.w.shape))
    assert np.array_equal(host(g.advect(_t(wl.phi), *z, dt, 0)), wl.phi)
    ones = np.ones(og.shape)
    got = host(g.advect(_t(ones), _t(wl.u), _t(wl.v), _t(wl.w), dt, 1))
    assert np.max(np.abs(got - 1.0)) <= 1e-14


def test_bad_arguments_are_refused():
    from paper_1410_1937_amd import nfa
    wl, og, ob, dt = _case(4, 16, 8, 8, drops=0)
    g = _gpu_vof(wl)
    phi, u, v, w = (_t(a) for a in (wl.phi, wl.u, wl.v, wl.w))
    with pytest.raises(nfa.NFAError, match="dt"):
        g.advect(phi, u, v, w, 0.0, 0)
    with pytest.raises(nfa.NFAError, match="dt"):
        g.sweep(phi, u, v, w, float("nan"), 0, False)
    with pytest.raises(nfa.NFAError, match="dir"):
        g.sweep(phi, u, v, w, dt, 3, False)
    with pytest.raises(nfa.NFAError, match="overlap"):
        g.advect(phi, u, v, w, dt, 0, out=phi)
    with pytest.raises(nfa.NFAError, match="overlap"):
        g.sweep(phi, u, v, w, dt, 1, True, out=phi)
    with pytest.raises(ValueError):
        g.advect(phi, v, u, w, dt, 0)


def _window(wl, centre, r):
    """The sub-grid of cells within r of centre (clipped to the grid) and the
    matching slices of every input."""
    k, j, i = centre
    nz, ny, nx = wl.phi.shape
    k0, k1 = max(k - r, 0), min(k + r + 1, nz)
    j0, j1 = max(j - r, 0), min(j + r + 1, ny)
    i0, i1 = max(i - r, 0), min(i + r + 1, nx)
    sub = dict(xf=wl.xf[i0:i1 + 1], yf=wl.yf[j0:j1 + 1], zf=wl.zf[k0:k1 + 1],
               psi=wl.psi[k0:k1 + 1, j0:j1 + 1, i0:i1 + 1], phi=wl.phi[k0:k1, j0:j1, i0:i1],
               u=wl.u[k0:k1, j0:j1, i0:i1 + 1], v=wl.v[k0:k1, j0:j1 + 1, i0:i1],
               w=wl.w[k0:k1 + 1, j0:j1, i0:i1])
    return sub, (k0, j0, i0), (k1, j1, i1)


def test_full_size_breaking_wave_step_on_sampled_windows():
    """512 x 256 x 192 (the breaking-wave grid: surface, 200 droplets and
    bubbles, the sphere), one step of each order on the GPU.  A cell's new
    fraction depends on the inputs within 4 cells (2 along a sweep's own
    direction, 1 across, summed over the three sweeps), so the oracle run on
    a 17-cell window reproduces the centre 7^3 cells of the full-size result
    exactly; windows are centred on interface cells of the input, on cells
    the sphere cuts and at the domain's corners and faces."""
    from paper_1410_1937_amd import nfa
    wl = fx.c3()
    nz, ny, nx = wl.phi.shape
    og_full = Grid(wl.xf, wl.yf, wl.zf, wl.bc)
    dt = courant_dt(og_full, Body(og_full, wl.psi, wl.theta, wl.samples), wl.u, wl.v, wl.w)
    del og_full
    g = _gpu_vof(wl)
    phi0 = _t(wl.phi)
    vel = tuple(_t(a) for a in (wl.u, wl.v, wl.w))
    out = [host(g.advect(phi0, *vel, dt, step)) for step in (0, 1)]
    del phi0, vel
    for o in out:
        assert np.all(np.isfinite(o))
    rng = np.random.default_rng(7)
    iface = np.argwhere((wl.phi > 0) & (wl.phi < 1))
    centres = [tuple(c) for c in iface[rng.choice(len(iface), 6, replace=False)]]
    # cells cut by the sphere (centre (0, 0, -0.15), radius 0.1): along the x axis through its centre
    kc = int(np.searchsorted(wl.zf, -0.15)) - 1
    jc = int(np.searchsorted(wl.yf, 0.0)) - 1
    for xb in (-0.1, 0.1):
        centres.append((kc, jc, int(np.searchsorted(wl.xf, xb)) - 1))
    centres += [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (nz // 2, 0, nx - 1)]
    r, inner = 8, 3
    for c in centres:
        sub, lo, hi = _window(wl, c, r)
        og = Grid(sub["xf"], sub["yf"], sub["zf"], wl.bc)
        ob = Body(og, sub["psi"], wl.theta, wl.samples)
        # compared: within `inner` of the centre and either 5 cells inside the
        # window or on the real domain's boundary
        sl = []
        for ax, (a0, a1, cc, n) in enumerate(zip(lo, hi, c, (nz, ny, nx))):
            s0 = max(cc - inner, a0 + (r - inner) if a0 > 0 else 0)
            s1 = min(cc + inner + 1, a1 - (r - inner) if a1 < n else n)
            sl.append(slice(s0, s1))
        assert all(s.stop > s.start for s in sl), c
        for step in (0, 1):
            ref = vof.advect(og, ob, sub["phi"], sub["u"], sub["v"], sub["w"], dt, step)
            local = tuple(slice(s.start - a0, s.stop - a0) for s, a0 in zip(sl, lo))
            got = out[step][tuple(sl)]
            assert np.array_equal(got, ref[local]), (c, step, np.max(np.abs(got - ref[local])))
