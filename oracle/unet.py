"""Learned preconditioner of flexible CG (oracle, FP64).

The network is a small 3-D U-Net (3 levels, 16/32/64 channels, 3x3x3
convolutions, 2x2x2 average pooling, nearest-neighbour upsampling, additive
skip connections) that maps the scaled residual and the log of the inverse
density to a correction of the Jacobi step (deeper variants add levels of
64 channels with the same pattern, see `shapes`):

    x0 = [r / s, l]                 s = RMS of r over the unknowns,
                                    l = (log(1/rho) - L0) / L1
    a0 = relu(conv0(x0))            full resolution, 2 -> 16
    a1 = relu(conv1(pool(a0)))      1/2,  16 -> 32
    a2 = relu(conv2(pool(a1)))      1/4,  32 -> 64
    b2 = relu(conv3(a2))            1/4,  64 -> 32
    d1 = relu(conv4(up(b2) + a1))   1/2,  32 -> 16
    d0 = relu(conv5(up(d1) + a0))   full, 16 -> 16
    y  = r / s + head(d0)           full, 16 -> 1, a 1x1x1 convolution
    z  = D^-1 y                     (Jacobi inverse diagonal of the operator)

so the untrained network with a zero head is exactly the Jacobi
preconditioner.  Every level decodes with a 3x3x3 convolution, the finest
too, before the 1x1x1 head (C4).

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

L0, L1 = -3.5, 3.4            # log(1/rho) normalisation: [-6.9, -0.18] -> about [-1, 1]
TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def channels(levels):
    """Channels per level: 16, 32, 64, then 64 for deeper levels."""
    return [16, 32, 64][:levels] + [64] * max(0, levels - 3)


def shapes(levels=3):
    """(Cin, Cout) of the convolutions in parameter order: encoder e0..e_{L-1},
    bottleneck b, decoder d_{L-2}..d_0, head.  Every convolution is 3x3x3
    except the head, 1x1x1 (C4's head); `taps` gives the count."""
    c = channels(levels)
    out = [(2, c[0])] + [(c[l - 1], c[l]) for l in range(1, levels)]
    out.append((c[levels - 1], c[levels - 2]))
    out += [(c[l], c[l - 1]) for l in range(levels - 2, 0, -1)]
    out.append((c[0], c[0]))
    out.append((c[0], 1))
    return out


SHAPES = shapes(3)


def bf16(x):
    """Round to the nearest BF16 (ties to even) via FP32; returns float64."""
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def taps(levels=3):
    """Taps of each convolution in parameter order: 27, ..., 27, 1 (head)."""
    return [27] * (len(shapes(levels)) - 1) + [1]


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
def init_params(seed=0, zero_last=True, levels=3):
    """He-normal weights (FP32 master copies), zero biases; the head zero so
    that the untrained preconditioner is Jacobi."""
    rng = np.random.default_rng(seed)
    params = []
    sh = shapes(levels)
    for i, ((ci, co), nt) in enumerate(zip(sh, taps(levels))):
        std = np.sqrt(2.0 / (nt * ci))
        w = rng.standard_normal((nt, ci, co)) * std
        if zero_last and i == len(sh) - 1:
            w[:] = 0.0
        params.append((w.astype(np.float32).astype(np.float64), np.zeros(co)))
    return params


def features(r, inv_rho, mask):
    """x0 = [r/s, (log(1/rho) - L0)/L1] on the cell grid (nz, ny, nx) -> (D,H,W,2)."""
    s = np.sqrt(np.add.reduce((r[mask > 0] ** 2).ravel()) / max(1, int(np.sum(mask > 0))))
    s = s if s > 0 else 1.0
    l = (np.log(inv_rho) - L0) / L1
    return np.stack([r / s, l], axis=-1), s


def _levels(params):
    return (len(params) - 1) // 2


def forward(params, x0, quant=True):
    """Returns (y, cache); y = x0[..., 0] + head(up(d1) + a0) on (D, H, W)."""
    L = _levels(params)
    P = [(_q(w, quant), _q(b, False)) for w, b in params]
    E, B, Dd, Hd = P[:L], P[L], P[L + 1:2 * L], P[2 * L]
    x0 = _q(x0, quant)
    a = [_q(relu(conv3d(x0, *E[0])), quant)]
    p = []
    for l in range(1, L):
        p.append(_q(pool(a[l - 1]), quant))
        a.append(_q(relu(conv3d(p[l - 1], *E[l])), quant))
    d = {L - 1: _q(relu(conv3d(a[L - 1], *B)), quant)}
    s = {}
    for i, l in enumerate(range(L - 2, -1, -1)):
        s[l] = _q(up(d[l + 1]) + a[l], quant)
        d[l] = _q(relu(conv3d(s[l], *Dd[i])), quant)
    wh, bh = Hd
    u = bh[0] + d[0] @ wh[0][:, 0]
    y = x0[..., 0] + u
    return y, dict(P=P, L=L, x0=x0, a=a, p=p, d=d, s=s)


def backward(cache, dy, quant=True):
    """Gradients (dw, db) of every conv, in parameter order, for dL/dy on
    (D, H, W).  Stored gradient tensors are BF16 when quant (as on the GPU)."""
    L, P, a, p, d, s = cache["L"], cache["P"], cache["a"], cache["p"], cache["d"], cache["s"]
    E, B, Dd, Hd = P[:L], P[L], P[L + 1:2 * L], P[2 * L]
    gE, gD = [None] * L, [None] * (L - 1)
    wh = Hd[0]
    gH = ((d[0].reshape(-1, d[0].shape[-1]).T @ dy.reshape(-1))[None, :, None], np.array([np.sum(dy)]))
    dd0 = _q(dy[..., None] * wh[0][:, 0] * (d[0] > 0), quant)
    gD[L - 2] = conv3d_wgrad(s[0], dd0)
    skip = {0: _q(conv3d_dgrad(dd0, Dd[L - 2][0]), quant)}
    for i, l in enumerate(range(1, L - 1)):
        di = L - 2 - l                      # index of d_l in decoder parameter order
        dd = _q(up_T(skip[l - 1]) * (d[l] > 0), quant)
        gD[di] = conv3d_wgrad(s[l], dd)
        skip[l] = _q(conv3d_dgrad(dd, Dd[di][0]), quant)
    ddb = _q(up_T(skip[L - 2]) * (d[L - 1] > 0), quant)
    gB = conv3d_wgrad(a[L - 1], ddb)
    da = _q(conv3d_dgrad(ddb, B[0]) * (a[L - 1] > 0), quant)
    for l in range(L - 1, 0, -1):
        gE[l] = conv3d_wgrad(p[l - 1], da)
        dp = _q(conv3d_dgrad(da, E[l][0]), quant)
        da = _q((skip[l - 1] + pool_T(dp)) * (a[l - 1] > 0), quant)
    gE[0] = conv3d_wgrad(cache["x0"], da)
    return gE + [gB] + gD + [gH]


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
