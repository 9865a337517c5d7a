"""Learned preconditioner of flexible CG (oracle, FP64).

The network is a small 3-D U-Net (3 levels, 16/32/64 channels, 3x3x3
convolutions, 2x2x2 average pooling, nearest-neighbour upsampling, additive
skip connections) that maps the scaled residual and the log of the inverse
density to a correction of the Jacobi step:

    x0 = [r / s, l]                 s = RMS of r over the unknowns,
                                    l = (log(1/rho) - L0) / L1
    a0 = relu(conv0(x0))            full resolution, 2 -> 16
    a1 = relu(conv1(pool(a0)))      1/2,  16 -> 32
    a2 = relu(conv2(pool(a1)))      1/4,  32 -> 64
    b2 = relu(conv3(a2))            1/4,  64 -> 32
    d1 = relu(conv4(up(b2) + a1))   1/2,  32 -> 16
    y  = r / s + conv5(up(d1) + a0) full,  16 -> 1
    z  = D^-1 y                     (Jacobi inverse diagonal of the operator)

so the untrained network with conv5 = 0 is exactly the Jacobi preconditioner.

Training loss per (residual r, error e = A'^-1 r) pair: the share of the
A-norm error that one flexible-CG step along z leaves,

    L = 1 - (z.r)^2 / ((z.A'z) (e.A'e)),    e.A'e = e.r,

which is scale invariant in z and needs only one operator apply.

GPU storage points are emulated: parameters, inputs and every stored
activation are rounded to BF16 (round to nearest even, from FP32), sums are
exact (FP64) here.  `quant=False` gives the pure FP64 network (used by the
gradient checks).  Convolutions are cross-correlations with zero 'same'
padding; tap t = 9 (dz+1) + 3 (dy+1) + (dx+1).  Arrays are channels-last
(D, H, W, C).
"""
from __future__ import annotations

import numpy as np

CH = (16, 32, 64)
SHAPES = [(2, 16), (16, 32), (32, 64), (64, 32), (32, 16), (16, 1)]   # conv0..conv5 (Cin, Cout)
TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
L0, L1 = -3.5, 3.4            # log(1/rho) normalisation: [-6.9, -0.18] -> about [-1, 1]


def bf16(x):
    """Round to the nearest BF16 (ties to even) via FP32; returns float64."""
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _q(x, quant):
    return bf16(x) if quant else np.asarray(x, dtype=np.float64)


# --------------------------------------------------------------- layers
def conv3d(x, w, b=None):
    """out[m, co] = b[co] + sum_t sum_ci x[m + off_t, ci] w[t, ci, co]."""
    D, H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((D, H, W, w.shape[2]))
    if b is not None:
        out += b
    for t, (dz, dy, dx) in enumerate(TAPS):
        out += xp[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :] @ w[t]
    return out


def conv3d_dgrad(dout, w):
    """d x[m, ci] = sum_t sum_co dout[m - off_t, co] w[t, ci, co]."""
    D, H, W, _ = dout.shape
    dp = np.pad(dout, ((1, 1), (1, 1), (1, 1), (0, 0)))
    dx = np.zeros((D, H, W, w.shape[1]))
    for t, (dz, dy, dx_) in enumerate(TAPS):
        dx += dp[1 - dz:1 - dz + D, 1 - dy:1 - dy + H, 1 - dx_:1 - dx_ + W, :] @ w[t].T
    return dx


def conv3d_wgrad(x, dout):
    """d w[t, ci, co] = sum_m x[m + off_t, ci] dout[m, co];  d b = sum_m dout."""
    D, H, W, Ci = x.shape
    Co = dout.shape[3]
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    dw = np.zeros((27, Ci, Co))
    g = dout.reshape(-1, Co)
    for t, (dz, dy, dx) in enumerate(TAPS):
        dw[t] = xp[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :].reshape(-1, Ci).T @ g
    return dw, g.sum(axis=0)


def pool(x):
    D, H, W, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5)) / 8.0


def pool_T(d):
    return up(d) / 8.0


def up(x):
    return x.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def up_T(d):
    D, H, W, C = d.shape
    return d.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


def relu(x):
    return np.maximum(x, 0.0)


# --------------------------------------------------------------- network
def init_params(seed=0, zero_last=True):
    """He-normal weights (FP32 master copies), zero biases; conv5 zero so that
    the untrained preconditioner is Jacobi."""
    rng = np.random.default_rng(seed)
    params = []
    for i, (ci, co) in enumerate(SHAPES):
        std = np.sqrt(2.0 / (27 * ci))
        w = rng.standard_normal((27, ci, co)) * std
        if zero_last and i == len(SHAPES) - 1:
            w[:] = 0.0
        params.append((w.astype(np.float32).astype(np.float64), np.zeros(co)))
    return params


def features(r, inv_rho, mask):
    """x0 = [r/s, (log(1/rho) - L0)/L1] on the cell grid (nz, ny, nx) -> (D,H,W,2)."""
    s = np.sqrt(np.add.reduce((r[mask > 0] ** 2).ravel()) / max(1, int(np.sum(mask > 0))))
    s = s if s > 0 else 1.0
    l = (np.log(inv_rho) - L0) / L1
    return np.stack([r / s, l], axis=-1), s


def forward(params, x0, quant=True):
    """Returns (y, cache); y = x0[..., 0] + conv5(...) on (D, H, W)."""
    P = [(_q(w, quant), _q(b, False)) for w, b in params]
    x0 = _q(x0, quant)
    a0 = _q(relu(conv3d(x0, *P[0])), quant)
    p0 = _q(pool(a0), quant)
    a1 = _q(relu(conv3d(p0, *P[1])), quant)
    p1 = _q(pool(a1), quant)
    a2 = _q(relu(conv3d(p1, *P[2])), quant)
    b2 = _q(relu(conv3d(a2, *P[3])), quant)
    s1 = _q(up(b2) + a1, quant)
    d1 = _q(relu(conv3d(s1, *P[4])), quant)
    s0 = _q(up(d1) + a0, quant)
    u = conv3d(s0, *P[5])[..., 0]
    y = x0[..., 0] + u
    cache = dict(P=P, x0=x0, a0=a0, p0=p0, a1=a1, p1=p1, a2=a2, b2=b2, s1=s1, d1=d1, s0=s0)
    return y, cache


def backward(cache, dy, quant=True):
    """Gradients (dw, db) of every conv for an upstream dL/dy on (D, H, W).
    Stored gradient tensors are BF16 when quant (as on the GPU)."""
    P = cache["P"]
    g = []
    dy4 = dy[..., None]
    dw5, db5 = conv3d_wgrad(cache["s0"], dy4)
    ds0 = _q(conv3d_dgrad(dy4, P[5][0]), quant)
    dd1 = up_T(ds0) * (cache["d1"] > 0)
    dd1 = _q(dd1, quant)
    dw4, db4 = conv3d_wgrad(cache["s1"], dd1)
    ds1 = _q(conv3d_dgrad(dd1, P[4][0]), quant)
    db2_ = _q(up_T(ds1) * (cache["b2"] > 0), quant)
    dw3, db3 = conv3d_wgrad(cache["a2"], db2_)
    da2 = _q(conv3d_dgrad(db2_, P[3][0]) * (cache["a2"] > 0), quant)
    dw2, db2 = conv3d_wgrad(cache["p1"], da2)
    dp1 = _q(conv3d_dgrad(da2, P[2][0]), quant)
    da1 = _q((ds1 + pool_T(dp1)) * (cache["a1"] > 0), quant)
    dw1, db1 = conv3d_wgrad(cache["p0"], da1)
    dp0 = _q(conv3d_dgrad(da1, P[1][0]), quant)
    da0 = _q((ds0 + pool_T(dp0)) * (cache["a0"] > 0), quant)
    dw0, db0 = conv3d_wgrad(cache["x0"], da0)
    return [(dw0, db0), (dw1, db1), (dw2, db2), (dw3, db3), (dw4, db4), (dw5, db5)]


# --------------------------------------------------------------- loss
def step_loss(z, r, Az, eAe):
    """L = 1 - (z.r)^2/((z.Az) e.A e) and dL/dz (z primal, r and Az gathered)."""
    a = float(np.add.reduce((z * r).ravel()))
    c = float(np.add.reduce((z * Az).ravel()))
    L = 1.0 - a * a / (c * eAe)
    dz = -(2.0 * a / (c * eAe)) * (r - (a / c) * Az)
    return L, dz


# --------------------------------------------------------------- Adam
def adam(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
