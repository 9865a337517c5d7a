"""Pins of the oracle's learned preconditioner (no GPU): convolution against
scipy's correlate, adjoint identities of every layer, finite-difference
gradients of the whole network, the step-loss closed forms, BF16 rounding
and the first Adam step."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import unet


def test_bf16_round_to_nearest_even():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 3.14159265, 1e-3])
    r = unet.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1 + 2 ** -6 and r[3] == -2.5
    assert abs(r[4] - 3.140625) == 0.0
    assert abs(r[5] - 1e-3) <= 2 ** -9 * 1e-3
    # every result is representable with 8 significant bits
    m, e = np.frexp(r[r != 0])
    assert np.all(m * 2 ** 8 == np.round(m * 2 ** 8))


def test_conv3d_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((5, 6, 7, 3))
    w = rng.standard_normal((27, 3, 4))
    b = rng.standard_normal(4)
    out = unet.conv3d(x, w, b)
    for co in range(4):
        ref = np.full(x.shape[:3], b[co])
        for ci in range(3):
            ref += ndimage.correlate(x[..., ci], w[:, ci, co].reshape(3, 3, 3), mode="constant", cval=0.0)
        assert np.max(np.abs(out[..., co] - ref)) <= 1e-12


def test_layer_adjoints():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 6, 8, 3))
    w = rng.standard_normal((27, 3, 5))
    y = rng.standard_normal((4, 6, 8, 5))
    lhs = np.sum(unet.conv3d(x, w) * y)
    assert abs(lhs - np.sum(x * unet.conv3d_dgrad(y, w))) <= 1e-10 * abs(lhs)
    dw, db = unet.conv3d_wgrad(x, y)
    assert abs(lhs - np.sum(w * dw)) <= 1e-10 * abs(lhs)
    assert np.allclose(db, y.reshape(-1, 5).sum(0))
    p = rng.standard_normal((2, 3, 4, 3))
    assert abs(np.sum(unet.pool(x) * p) - np.sum(x * unet.pool_T(p))) <= 1e-12
    q = rng.standard_normal((8, 12, 16, 3))
    assert abs(np.sum(unet.up(x) * q) - np.sum(x * unet.up_T(q))) <= 1e-10
    assert np.allclose(unet.pool(unet.up(x)), x)


def test_layer_shapes_for_three_and_five_levels():
    assert unet.shapes(3) == [(2, 16), (16, 32), (32, 64), (64, 32), (32, 16), (16, 16), (16, 1)]
    assert unet.shapes(5) == [(2, 16), (16, 32), (32, 64), (64, 64), (64, 64), (64, 64), (64, 64),
                              (64, 32), (32, 16), (16, 16), (16, 1)]
    assert unet.taps(3) == [27] * 6 + [1]


def test_untrained_network_is_the_jacobi_step():
    rng = np.random.default_rng(2)
    params = unet.init_params(0, zero_last=True)
    x0 = rng.standard_normal((8, 8, 8, 2))
    y, _ = unet.forward(params, x0, quant=False)
    assert np.array_equal(y, x0[..., 0])


@pytest.mark.parametrize("levels", [3, 4])
def test_network_gradient_matches_finite_differences(levels):
    rng = np.random.default_rng(3)
    params = unet.init_params(1, zero_last=False, levels=levels)
    params = [(w, rng.standard_normal(b.shape) * 0.1) for w, b in params]
    x0 = rng.standard_normal((16, 8, 8, 2))
    g = rng.standard_normal((16, 8, 8))

    def loss(ps):
        y, _ = unet.forward(ps, x0, quant=False)
        return float(np.sum(y * g))

    _, cache = unet.forward(params, x0, quant=False)
    grads = unet.backward(cache, g, quant=False)
    h = 1e-6
    for layer in range(len(params)):
        w, b = params[layer]
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in w.shape)
            wp, wm = w.copy(), w.copy()
            wp[idx] += h
            wm[idx] -= h
            pp = list(params)
            pp[layer] = (wp, b)
            pm = list(params)
            pm[layer] = (wm, b)
            fd = (loss(pp) - loss(pm)) / (2 * h)
            an = grads[layer][0][idx]
            assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (layer, idx, fd, an)
        k = rng.integers(0, b.shape[0])
        bp, bm = b.copy(), b.copy()
        bp[k] += h
        bm[k] -= h
        pp = list(params)
        pp[layer] = (w, bp)
        pm = list(params)
        pm[layer] = (w, bm)
        fd = (loss(pp) - loss(pm)) / (2 * h)
        assert abs(fd - grads[layer][1][k]) <= 1e-5 * max(1.0, abs(fd))


def test_step_loss_closed_forms_and_gradient():
    rng = np.random.default_rng(4)
    n = 12
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    r = rng.standard_normal(n)
    e = np.linalg.solve(A, r)
    eAe = float(e @ r)
    L, _ = unet.step_loss(e, r, A @ e, eAe)
    assert abs(L) <= 1e-12                       # the exact error direction
    L2, _ = unet.step_loss(3.7 * e, r, A @ (3.7 * e), eAe)
    assert abs(L2) <= 1e-12                      # scale invariant
    z = rng.standard_normal(n)
    L, dz = unet.step_loss(z, r, A @ z, eAe)
    # L equals the A-norm error left by the optimal step along z
    alpha = (z @ r) / (z @ A @ z)
    ee = e - alpha * z
    assert abs(L - (ee @ A @ ee) / eAe) <= 1e-12
    h = 1e-6
    for i in range(n):
        zp, zm = z.copy(), z.copy()
        zp[i] += h
        zm[i] -= h
        fd = (unet.step_loss(zp, r, A @ zp, eAe)[0] - unet.step_loss(zm, r, A @ zm, eAe)[0]) / (2 * h)
        assert abs(fd - dz[i]) <= 1e-6


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([0.3, -2.0, 1e-3])
    w = np.array([1.0, 2.0, 3.0])
    w1, m, v = unet.adam(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_head_is_the_centre_tap_of_a_three_by_three_convolution():
    """C4's 1x1x1 head on the finest decoder output d0 = relu(conv(up(d1) +
    a0)) equals a 3x3x3 convolution (pinned against scipy above) whose only
    non-zero tap is the centre one; d0 itself is that convolution of the
    skip sum."""
    rng = np.random.default_rng(7)
    params = unet.init_params(2, zero_last=False, levels=3)
    params = [(w, rng.standard_normal(b.shape) * 0.1) for w, b in params]
    assert params[-1][0].shape == (1, 16, 1)
    x0 = rng.standard_normal((8, 12, 16, 2))
    y, cache = unet.forward(params, x0, quant=False)
    w5, b5 = params[-1]
    w27 = np.zeros((27, 16, 1))
    w27[13] = w5[0]
    s0 = unet.up(cache["d"][1]) + cache["a"][0]
    d0 = unet.relu(unet.conv3d(s0, *params[-2]))
    assert np.max(np.abs(d0 - cache["d"][0])) <= 1e-12 * np.max(np.abs(d0))
    ref = x0[..., 0] + unet.conv3d(d0, w27, b5)[..., 0]
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))
