"""The learned preconditioner on the GPU against the FP64 oracle (needs an
MI355X).  Layers of the forward pass and stages of the backward pass are
checked one at a time, each fed with the GPU's own BF16 operands, to within
one BF16 rounding step of the oracle (FP32 against FP64 accumulation can move
a value across a rounding boundary), and each layer's weight gradient against
the FP64 sum over its own operands; the whole forward pass, the loss, the
end-to-end parameter gradients and the Adam update within the tolerances
stated below."""
import numpy as np
import pytest

from oracle import solvers, unet as ou
from paper_1410_1937_amd import fixtures as fx
from tests.gpu_helpers import gpu_for, host, oracle_for

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _bf(t):
    return t.float().cpu().numpy().astype(np.float64)


def _ulp_ok(gpu, ref, frac=1e-3):
    """|gpu - ref| within one BF16 step of |ref| (2^-7 relative) everywhere but
    a small fraction of entries, which may differ by two steps."""
    tol = np.maximum(np.abs(ref), 1e-30) * 2.0 ** -7 * 1.0001
    bad = np.abs(gpu - ref) > tol
    assert np.mean(bad) <= frac, np.mean(bad)
    assert np.all(np.abs(gpu - ref)[bad] <= 2 * tol[bad] + 1e-6 * np.max(np.abs(ref)))


@pytest.fixture(scope="module")
def setup():
    from paper_1410_1937_amd import nfa
    wl = fx.small(7, 32, 16, 12, body="sphere")
    og, ob, oop, ob_rhs = oracle_for(wl)
    gg, gop = gpu_for(wl)
    net = nfa.UNet(32, 16, 12, seed=3)
    rng = np.random.default_rng(5)
    params = ou.init_params(9, zero_last=False)
    params = [(w.astype(np.float32), (rng.standard_normal(b.shape) * 0.05).astype(np.float32)) for w, b in params]
    net.set_params(nfa.UNet.flatten(params))
    r = (ob_rhs * ob.reduced).astype(np.float32)
    rt = torch.as_tensor(r, device="cuda")
    z = host(net.forward(gop, rt, keep=True)).astype(np.float64)
    return wl, (og, ob, oop, ob_rhs), (gg, gop), net, [(w.astype(np.float64), b.astype(np.float64)) for w, b in params], r, rt, z


def test_forward_layers_within_one_bf16_step(setup):
    wl, (og, ob, oop, _), (gg, gop), net, params, r, rt, z = setup
    P = [(ou.bf16(w), b) for w, b in params]
    x0 = _bf(net.export("x0"))
    x0_ref, s = ou.features(r.astype(np.float64), 1.0 / oop.rho, ob.reduced)
    _ulp_ok(x0, ou.bf16(x0_ref))
    a0 = _bf(net.export("a0"))
    _ulp_ok(a0, ou.bf16(ou.relu(ou.conv3d(x0, *P[0]))))
    p0 = _bf(net.export("p0"))
    _ulp_ok(p0, ou.bf16(ou.pool(a0)))
    a1 = _bf(net.export("a1"))
    _ulp_ok(a1, ou.bf16(ou.relu(ou.conv3d(p0, *P[1]))))
    p1 = _bf(net.export("p1"))
    _ulp_ok(p1, ou.bf16(ou.pool(a1)))
    a2 = _bf(net.export("a2"))
    _ulp_ok(a2, ou.bf16(ou.relu(ou.conv3d(p1, *P[2]))))
    b2 = _bf(net.export("d2"))
    _ulp_ok(b2, ou.bf16(ou.relu(ou.conv3d(a2, *P[3]))))
    d1 = _bf(net.export("d1"))
    _ulp_ok(d1, ou.bf16(ou.relu(ou.conv3d(ou.bf16(ou.up(b2) + a1), *P[4]))))
    d0 = _bf(net.export("d0"))
    _ulp_ok(d0, ou.bf16(ou.relu(ou.conv3d(ou.bf16(ou.up(d1) + a0), *P[5]))))
    # the 1x1x1 head on d0
    w6, b6 = P[6]
    y = x0[..., 0] + (b6[0] + d0 @ w6[0][:, 0])
    zref = oop.dinv * y
    assert np.max(np.abs(z - zref)) <= 1e-5 * np.max(np.abs(zref))


def test_pipelined_encoder_over_many_bricks_per_workgroup():
    """The persistent 16 -> 32 encoder walks several bricks per workgroup when
    the level has more bricks than resident workgroups: on 264 x 136 x 76
    cells its level-1 grid, 132 x 68 x 38, has 9 x 17 x 10 bricks, ragged in
    every direction.  Fed the GPU's own pooled input, its output and its
    pooled output are within one BF16 step of the oracle's layer."""
    from paper_1410_1937_amd import nfa
    wl = fx.small(12, 264, 136, 76, body="sphere")
    gg, gop = gpu_for(wl)
    net = nfa.UNet(264, 136, 76, seed=5)
    rng = np.random.default_rng(21)
    params = ou.init_params(23, zero_last=False)
    params = [(w.astype(np.float32), (rng.standard_normal(b.shape) * 0.05).astype(np.float32)) for w, b in params]
    net.set_params(nfa.UNet.flatten(params))
    r = torch.as_tensor(rng.standard_normal((76, 136, 264)).astype(np.float32), device="cuda")
    net.forward(gop, r, keep=True)
    p0 = _bf(net.export("p0"))
    a1 = _bf(net.export("a1"))
    w1 = ou.bf16(params[1][0].astype(np.float64))
    ref = ou.bf16(ou.relu(ou.conv3d(p0, w1, params[1][1].astype(np.float64))))
    _ulp_ok(a1, ref)
    _ulp_ok(_bf(net.export("p1")), ou.bf16(ou.pool(a1)))


def test_decoders_over_runs_of_bricks_in_z():
    """The 16- and 32-channel decoders walk runs of up to 16 and 8 bricks up
    each column, moving the two halo planes that consecutive bricks share
    inside LDS: on 40 x 20 x 76 cells a finest-level column holds 19 bricks
    (runs of 16 and 3), a level-1 column 10 (8 and 2, the last brick half
    outside the grid), and the bricks are ragged in x.  Fed the GPU's own skip and
    coarser decoder output, each output is within one BF16 step of the
    oracle's layer and the head's z follows from the finest one."""
    from paper_1410_1937_amd import nfa
    wl = fx.small(13, 40, 20, 76, body="sphere")
    og, ob, oop, ob_rhs = oracle_for(wl)
    gg, gop = gpu_for(wl)
    net = nfa.UNet(40, 20, 76, seed=6)
    rng = np.random.default_rng(31)
    params = ou.init_params(29, zero_last=False)
    params = [(w.astype(np.float32), (rng.standard_normal(b.shape) * 0.05).astype(np.float32)) for w, b in params]
    net.set_params(nfa.UNet.flatten(params))
    P = [(ou.bf16(w.astype(np.float64)), b.astype(np.float64)) for w, b in params]
    r = (ob_rhs * ob.reduced).astype(np.float32)
    z = host(net.forward(gop, torch.as_tensor(r, device="cuda"), keep=True)).astype(np.float64)
    a0 = _bf(net.export("a0"))
    a1 = _bf(net.export("a1"))
    d2 = _bf(net.export("d2"))
    d1 = _bf(net.export("d1"))
    d0 = _bf(net.export("d0"))
    _ulp_ok(d1, ou.bf16(ou.relu(ou.conv3d(ou.bf16(ou.up(d2) + a1), *P[4]))))
    _ulp_ok(d0, ou.bf16(ou.relu(ou.conv3d(ou.bf16(ou.up(d1) + a0), *P[5]))))
    x0 = _bf(net.export("x0"))
    w6, b6 = P[6]
    zref = oop.dinv * (x0[..., 0] + (b6[0] + d0 @ w6[0][:, 0]))
    assert np.max(np.abs(z - zref)) <= 1e-5 * np.max(np.abs(zref))


def test_whole_forward_matches_oracle(setup):
    wl, (og, ob, oop, _), (gg, gop), net, params, r, rt, z = setup
    x0, s = ou.features(r.astype(np.float64), 1.0 / oop.rho, ob.reduced)
    y, _ = ou.forward(params, x0, quant=True)
    zref = oop.dinv * y
    err = np.linalg.norm(z - zref) / np.linalg.norm(zref)
    print(f"forward rel L2 vs oracle: {err:.2e}")
    assert err <= 2e-2


def test_untrained_network_is_jacobi_on_the_bf16_residual():
    from paper_1410_1937_amd import nfa
    wl = fx.small(8, 16, 16, 8, body="sphere")
    og, ob, oop, ob_rhs = oracle_for(wl)
    gg, gop = gpu_for(wl)
    net = nfa.UNet(16, 16, 8, seed=0)
    r = (ob_rhs * ob.reduced).astype(np.float32)
    z = host(net.forward(gop, torch.as_tensor(r, device="cuda"), keep=True))
    x0 = _bf(net.export("x0"))
    assert np.array_equal(z, (gop.export("dinv32").cpu().numpy() * x0[..., 0].astype(np.float32)))


def test_gradients_loss_and_adam_match_oracle(setup):
    from paper_1410_1937_amd import nfa
    wl, (og, ob, oop, ob_rhs), (gg, gop), net, params, r, rt, z = setup
    e = solvers.pcg(oop, r.astype(np.float64), tol=1e-12).x
    eAe = float(np.sum(e * r))
    loss = net.grad(gop, rt, eAe)
    x0, s = ou.features(r.astype(np.float64), 1.0 / oop.rho, ob.reduced)
    y, cache = ou.forward(params, x0, quant=True)
    zz = oop.dinv * y
    Lref, dz = ou.step_loss(zz, r.astype(np.float64), oop.apply(zz), eAe)
    print(f"loss gpu {loss:.6f} oracle {Lref:.6f}")
    assert abs(loss - Lref) <= 2e-2 * max(abs(Lref), 1e-3)
    grads = ou.backward(cache, oop.dinv * dz, quant=True)
    g = net.unflatten(net.get_grads())
    for layer, ((gw, gb), (rw, rb)) in enumerate(zip(g, grads)):
        ew = np.linalg.norm(gw - rw) / max(np.linalg.norm(rw), 1e-30)
        eb = np.linalg.norm(gb - rb) / max(np.linalg.norm(rb), 1e-30)
        print(f"layer {layer}: weight grad rel err {ew:.2e}, bias {eb:.2e}")
        assert ew <= 5e-2 and eb <= 5e-2
    # one Adam step on these gradients
    p_before = net.get_params().astype(np.float64)
    g_flat = net.get_grads().astype(np.float64)
    net.train_step(gop, rt, eAe, 1e-3, 1)
    g_flat = net.get_grads().astype(np.float64)     # same inputs -> same gradients
    expect, _, _ = ou.adam(p_before, g_flat, np.zeros_like(p_before), np.zeros_like(p_before), 1, lr=1e-3)
    assert np.max(np.abs(net.get_params() - expect)) <= 1e-6


@pytest.mark.parametrize("shape", [(32, 16, 12), (20, 12, 8)])
def test_backward_stages_and_weight_gradients_one_layer_at_a_time(shape):
    """Every stage of the GPU backward pass, fed with the GPU's own BF16
    operands (activations of the forward, gradients of the stage before),
    against the oracle's same stage: data gradients within one BF16 step,
    weight and bias gradients (FP32 sums of exact BF16 products) within 1e-4
    of the FP64 sums, and dL/dz against the closed form of the step loss.
    On 20 x 12 x 8 the rows (20, 10 and 5 cells on the three levels) are not
    multiples of the weight gradients' 8-position runs, which then cross rows."""
    from paper_1410_1937_amd import nfa
    nx, ny, nz = shape
    wl = fx.small(7, nx, ny, nz, body="sphere")
    og, ob, oop, ob_rhs = oracle_for(wl)
    gg, gop = gpu_for(wl)
    net = nfa.UNet(nx, ny, nz, seed=3)
    rng = np.random.default_rng(15)
    params = ou.init_params(13, zero_last=False)
    params = [(w.astype(np.float32), (rng.standard_normal(b.shape) * 0.05).astype(np.float32)) for w, b in params]
    net.set_params(nfa.UNet.flatten(params))
    W = [ou.bf16(w.astype(np.float64)) for w, _ in params]
    r = (ob_rhs * ob.reduced).astype(np.float32)
    rt = torch.as_tensor(r, device="cuda")
    e = solvers.pcg(oop, r.astype(np.float64), tol=1e-12).x
    eAe = float(np.sum(e * r))
    net.grad(gop, rt, eAe)
    z = host(net.forward(gop, rt, keep=True)).astype(np.float64)   # same parameters: same activations
    X = {k: _bf(net.export(k)) for k in ("x0", "a0", "a1", "a2", "p0", "p1", "d0", "d1", "d2",
                                         "dd0", "dd1", "dd2", "skip0", "skip1", "da0", "da1", "da2",
                                         "dp0", "dp1")}
    dz = host(net.export("dz")).astype(np.float64)
    _, dz_ref = ou.step_loss(z, r.astype(np.float64), oop.apply(z), eAe)
    assert np.linalg.norm(dz - dz_ref) <= 1e-4 * np.linalg.norm(dz_ref)
    dy = oop.dinv * dz
    q = ou.bf16
    _ulp_ok(X["dd0"], q(dy[..., None] * W[6][0][:, 0] * (X["d0"] > 0)))
    _ulp_ok(X["skip0"], q(ou.conv3d_dgrad(X["dd0"], W[5])))
    _ulp_ok(X["dd1"], q(ou.up_T(X["skip0"]) * (X["d1"] > 0)))
    _ulp_ok(X["skip1"], q(ou.conv3d_dgrad(X["dd1"], W[4])))
    _ulp_ok(X["dd2"], q(ou.up_T(X["skip1"]) * (X["d2"] > 0)))
    _ulp_ok(X["da2"], q(ou.conv3d_dgrad(X["dd2"], W[3]) * (X["a2"] > 0)))
    _ulp_ok(X["dp1"], q(ou.conv3d_dgrad(X["da2"], W[2])))
    _ulp_ok(X["da1"], q((X["skip1"] + ou.pool_T(X["dp1"])) * (X["a1"] > 0)))
    _ulp_ok(X["dp0"], q(ou.conv3d_dgrad(X["da1"], W[1])))
    _ulp_ok(X["da0"], q((X["skip0"] + ou.pool_T(X["dp0"])) * (X["a0"] > 0)))
    # weight and bias gradients of each layer from its own operands
    s0 = q(ou.up(X["d1"]) + X["a0"])
    s1 = q(ou.up(X["d2"]) + X["a1"])
    operands = [(X["x0"], X["da0"]), (X["p0"], X["da1"]), (X["p1"], X["da2"]), (X["a2"], X["dd2"]),
                (s1, X["dd1"]), (s0, X["dd0"])]
    g = net.unflatten(net.get_grads())
    for layer, (xin, dout) in enumerate(operands):
        rw, rb = ou.conv3d_wgrad(xin, dout)
        gw, gb = (a.astype(np.float64) for a in g[layer])
        assert np.linalg.norm(gw - rw) <= 1e-4 * np.linalg.norm(rw), layer
        assert np.linalg.norm(gb - rb) <= 1e-4 * np.linalg.norm(rb) + 1e-30, layer
    gw, gb = (a.astype(np.float64) for a in g[6])
    rw = (X["d0"].reshape(-1, 16).T @ dy.reshape(-1))[None, :, None]
    assert np.linalg.norm(gw - rw) <= 1e-4 * np.linalg.norm(rw)
    assert abs(gb[0] - dy.sum()) <= 1e-4 * np.abs(dy).sum()


def test_backward_and_adam_step_compose_to_the_training_step():
    """nfa_unet_backward on the step loss's dL/dz after a forward with keep
    gives nfa_unet_grad's gradients bit for bit, and nfa_unet_adam_step after
    it nfa_unet_train_step's parameters; backward is refused after a forward
    without keep; for a loss of the caller's, L = |z|^2 / 2 (dL/dz = z), the
    head bias gradient is sum D^-1 z (z = D^-1 (x0 + b + w . d0))."""
    from paper_1410_1937_amd import nfa
    wl = fx.small(7, 32, 16, 12, body="sphere")
    og, ob, oop, ob_rhs = oracle_for(wl)
    gg, gop = gpu_for(wl)
    rng = np.random.default_rng(17)
    params = ou.init_params(19, zero_last=False)
    flat = nfa.UNet.flatten([(w.astype(np.float32), (rng.standard_normal(b.shape) * 0.05).astype(np.float32))
                             for w, b in params])
    r = (ob_rhs * ob.reduced).astype(np.float32)
    rt = torch.as_tensor(r, device="cuda")
    e = solvers.pcg(oop, r.astype(np.float64), tol=1e-12).x
    eAe = float(np.sum(e * r))
    a, b = nfa.UNet(32, 16, 12, seed=3), nfa.UNet(32, 16, 12, seed=3)
    a.set_params(flat)
    b.set_params(flat)
    a.grad(gop, rt, eAe)
    g1 = a.get_grads()
    dz = a.export("dz").clone()
    b.forward(gop, rt, keep=True)
    b.backward(gop, dz)
    assert np.array_equal(b.get_grads(), g1)
    b.forward(gop, rt)
    with pytest.raises(nfa.NFAError):
        b.backward(gop, dz)
    a.train_step(gop, rt, eAe, 1e-3, 1)
    b.grad(gop, rt, eAe)
    b.adam_step(1e-3, 1)
    assert np.array_equal(b.get_params(), a.get_params())
    z = b.forward(gop, rt, keep=True)
    b.backward(gop, z.contiguous())
    gb = b.unflatten(b.get_grads())[-1][1]
    zz = host(z).astype(np.float64)
    dinv = host(gop.export("dinv32")).astype(np.float64)
    ref = float(np.sum(dinv * zz))
    assert abs(float(gb[0]) - ref) <= 1e-4 * float(np.sum(np.abs(dinv * zz)))


@pytest.mark.parametrize("levels", [4, 5])
def test_deeper_network_forward_and_gradients(levels):
    from paper_1410_1937_amd import nfa
    wl = fx.small(10, 32, 16, 16, body="sphere")
    og, ob, oop, ob_rhs = oracle_for(wl)
    gg, gop = gpu_for(wl)
    net = nfa.UNet(32, 16, 16, seed=2, levels=levels)
    rng = np.random.default_rng(6)
    params = ou.init_params(11, zero_last=False, levels=levels)
    params = [(w.astype(np.float32), (rng.standard_normal(b.shape) * 0.05).astype(np.float32)) for w, b in params]
    net.set_params(nfa.UNet.flatten(params))
    params = [(w.astype(np.float64), b.astype(np.float64)) for w, b in params]
    r = (ob_rhs * ob.reduced).astype(np.float32)
    rt = torch.as_tensor(r, device="cuda")
    z = host(net.forward(gop, rt)).astype(np.float64)
    x0, s = ou.features(r.astype(np.float64), 1.0 / oop.rho, ob.reduced)
    y, cache = ou.forward(params, x0, quant=True)
    zref = oop.dinv * y
    assert np.linalg.norm(z - zref) / np.linalg.norm(zref) <= 2e-2
    e = solvers.pcg(oop, r.astype(np.float64), tol=1e-12).x
    eAe = float(np.sum(e * r))
    net.grad(gop, rt, eAe)
    Lref, dz = ou.step_loss(zref, r.astype(np.float64), oop.apply(zref), eAe)
    grads = ou.backward(cache, oop.dinv * dz, quant=True)
    for layer, ((gw, gb), (rw, rb)) in enumerate(zip(net.unflatten(net.get_grads()), grads)):
        ew = np.linalg.norm(gw - rw) / max(np.linalg.norm(rw), 1e-30)
        assert ew <= 5e-2, (layer, ew)


def test_flexible_cg_with_the_network_meets_the_fp64_tolerance():
    from paper_1410_1937_amd import nfa
    wl = fx.small(9, 32, 24, 16, body="sphere")
    og, ob, oop, ob_rhs = oracle_for(wl)
    gg, gop = gpu_for(wl)
    net = nfa.UNet(32, 24, 16, seed=1)
    b = torch.as_tensor(ob_rhs, device="cuda")
    x, res = gop.solve(b, tol=1e-8, precision="mixed", precond="unet", unet=net, fallback_ratio=2.0)
    assert res.status == 0 and res.relres <= 1e-8
    assert solvers.true_relres(oop, ob_rhs, host(x)) <= 1.01e-8


def test_trained_network_gains_over_the_untrained_one_on_a_held_out_step():
    """What the committed weights (3 levels, trained on steps 0-159 of the
    advected-surface sequence) gain on held-out step 160 of that sequence
    (256x128x96): the share of the A-norm error one step along z leaves, for
    residual/error pairs of the plain solver after k = 0, 16 and 64 iterations,
    trained against untrained (the Jacobi step), and the full mixed FCG solve
    with the stagnation monitor meeting the FP64 tolerance (the network does
    not carry the solve to 1e-8 by itself: the monitor hands it to Jacobi-PCG,
    see the evaluation record beside the weights)."""
    import os
    from paper_1410_1937_amd import nfa
    wl = fx.c4_step(160)
    wl.phi = wl.phi.astype(np.float32).astype(np.float64)   # held in FP32 on both sides
    og, ob, oop, ob_rhs = oracle_for(wl)
    gg, gop = gpu_for(wl, phi_dtype=torch.float32)
    b = torch.as_tensor(ob_rhs, device="cuda")
    wpath = os.path.join(os.path.dirname(nfa.__file__), "weights", "unet_l3_c4.npy")
    trained = nfa.UNet(256, 128, 96, levels=3)
    trained.set_params(np.load(wpath))
    untrained = nfa.UNet(256, 128, 96, levels=3)
    xs, _ = gop.solve(b, tol=1e-10, precision="f64")
    x = torch.zeros_like(b)
    done = 0
    loss = {"trained": [], "untrained": []}
    for k in (0, 16, 64):
        if k > done:
            x, _ = gop.solve(b, x=x, tol=1e-30, precision="f64", max_iters=k - done, warm_start=True)
            done = k
        r, _ = gop.residual(b, x)
        eAe = float(torch.dot((xs - x).ravel(), r.ravel()))
        for tag, net in (("trained", trained), ("untrained", untrained)):
            loss[tag].append(net.grad(gop, r.float().contiguous(), eAe))
    print(f"[learned] step loss trained {loss['trained']} untrained {loss['untrained']}", flush=True)
    assert all(t <= 0.75 * u for t, u in zip(loss["trained"], loss["untrained"])), loss
    x, res = gop.solve(b, tol=1e-8, precision="mixed", precond="unet", unet=trained)
    print(f"[learned] full solve: {res.iterations} its, fallback {res.fallback}, relres {res.relres:.3e}", flush=True)
    assert res.status == 0 and res.relres <= 1e-8
    assert solvers.true_relres(oop, ob_rhs, host(x)) <= 1.01e-8
