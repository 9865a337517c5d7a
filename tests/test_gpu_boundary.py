"""Inhomogeneous Neumann data on the GPU against the oracle (needs an
MI355X): the right-hand side with a per-cell body velocity (bitwise, up to the
removed mean when every boundary is Neumann), and the exit-face update of the
radiation condition (bitwise)."""
import numpy as np
import pytest

from oracle import boundary
from paper_1410_1937_amd import fixtures as fx
from tests.gpu_helpers import gpu_for, host, oracle_for

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("bc", [(0,) * 6, (0, 1, 0, 0, 0, 1)])
def test_rhs_with_a_per_cell_body_velocity_bitwise(bc):
    wl = fx.small(4, 40, 18, 14, body="sphere", bc=bc)
    og, ob, oop, _ = oracle_for(wl)
    gg, gop = gpu_for(wl)
    # a rotation about an axis through (0.01, 0, -0.1) plus a translation
    zc, yc, xc = np.meshgrid(fx.centres(wl.zf), fx.centres(wl.yf), fx.centres(wl.xf), indexing="ij")
    r = np.stack([xc - 0.01, yc, zc + 0.1])
    omega = np.array([0.2, -0.6, 0.4])
    vb = np.cross(omega, r, axis=0) + np.array([0.1, 0.0, 0.3])[:, None, None, None]
    ref = boundary.rhs_cells(oop, wl.u, wl.v, wl.w, 0.7, tuple(vb))
    got = host(gop.rhs_cells(_t(wl.u), _t(wl.v), _t(wl.w), 0.7, tuple(_t(a) for a in vb)))
    if any(bc):
        assert np.array_equal(got, ref)
    else:
        # identical up to the rounding of the removed mean (a reduction)
        assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_exit_face_update_bitwise_and_checked():
    from paper_1410_1937_amd.nfa import NFAError
    wl = fx.small(5, 36, 12, 10, body=None)
    gg, gop = gpu_for(wl)
    rng = np.random.default_rng(9)
    uk = rng.standard_normal(gg.face_shape(0))
    ut = rng.standard_normal(gg.face_shape(0))
    dx = wl.xf[-1] - wl.xf[-2]
    dt = 0.6 * dx / 1.3
    ref = boundary.exit_velocity(uk, ut, 1.3, dt, dx)
    got = gg.exit_velocity(_t(uk), 1.3, dt, ut_x=_t(ut))
    assert np.array_equal(host(got), ref)
    with pytest.raises(NFAError, match="width of the last cell"):
        gg.exit_velocity(_t(uk), 1.3, 2.0 * dx / 1.3)
