"""The Runge-Kutta projection cycle on the GPU against the oracle (needs an
MI355X): the face-array combination and the velocity update bitwise, the
whole cycle to the solve tolerances, and a full-size cycle checked by the
oracle's own operators."""
import numpy as np
import pytest

from oracle import rk2, solvers
from oracle.operator import Operator
from paper_1410_1937_amd import fixtures as fx
from tests.gpu_helpers import gpu_for, host, oracle_for, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _forcing(wl, seed):
    return tuple(0.1 * a for a in fx.face_velocity(wl.xf, wl.yf, wl.zf, seed))


def _open(body):
    return body.open_x, body.open_y, body.open_z


def test_faces_combine_bitwise():
    from paper_1410_1937_amd import nfa
    rng = np.random.default_rng(0)
    a, b, c = (rng.standard_normal(1001) for _ in range(3))
    out = host(nfa.faces_combine(_t(a), _t(b), 0.37, _t(c)))
    assert np.array_equal(out, (a + b) + 0.37 * c)
    out = host(nfa.faces_combine(_t(a), None, 0.37, _t(c)))
    assert np.array_equal(out, a + 0.37 * c)


@pytest.mark.parametrize("bc", [(0,) * 6, (1, 0, 0, 1, 0, 1)])
def test_velocity_update_bitwise(bc):
    wl = fx.small(2, 40, 18, 14, body="sphere", bc=bc)
    og, ob, oop, _ = oracle_for(wl)
    gg, gop = gpu_for(wl)
    p = np.random.default_rng(4).standard_normal(og.shape)
    ut = (wl.u, wl.v, wl.w)
    for scale in (1.0, 0.5):
        ref = rk2.update_velocity(oop, ut, p, 0.3, scale)
        got = gop.velocity(tuple(_t(a) for a in ut), _t(p), 0.3, scale)
        for r, g in zip(ref, got):
            assert np.array_equal(host(g), r)


@pytest.mark.parametrize("precision,precond", [("f64", "jacobi"), ("mixed", "mg")])
def test_cycle_matches_oracle(precision, precond):
    wl = fx.small(3, 36, 20, 16, body="sphere")       # all-Neumann, moving sphere
    og, ob, _, _ = oracle_for(wl)
    phi_s = np.roll(wl.phi, 1, axis=2)
    R = _forcing(wl, 11)
    uk = (wl.u, wl.v, wl.w)
    dt = 0.01
    ref = rk2.cycle(og, ob, wl.phi, phi_s, uk, R, dt, wl.body_vel, tol=1e-12)
    gg, gop = gpu_for(wl)
    out = gop.rk2_cycle(_t(wl.phi), _t(phi_s), tuple(_t(a) for a in uk), tuple(_t(a) for a in R), dt,
                        wl.body_vel, tol=1e-10, precision=precision, precond=precond)
    assert out["status"] == 0 and out["stage1"].relres <= 1e-10 and out["stage2"].relres <= 1e-10
    assert not out["stage1"].fallback and not out["stage2"].fallback
    assert rel_l2(host(out["pstar"]), ref["p1"]) <= 1e-8
    assert rel_l2(host(out["p"]), ref["p2"]) <= 1e-8
    for name, rname in (("ustar", "us"), ("unext", "un")):
        for g, r, o in zip(out[name], ref[rname], _open(ob)):
            m = o > 0
            assert rel_l2(host(g)[m], r[m]) <= 1e-8, name
    # the new velocity is discretely solenoidal with the body moving at v
    F = [o * host(a) for o, a in zip(_open(ob), out["unext"])]
    d = ref["op2"].merged_divergence(*F, wl.body_vel)
    d0 = ref["op2"].merged_divergence(*[o * a for o, a in zip(_open(ob), ref["ut2"])], ref["vel2"])
    assert np.linalg.norm(d) <= 1e-8 * np.linalg.norm(d0)


def test_full_size_cycle_on_the_hull_sequence():
    """Steps 40 -> 41 of the advected-surface sequence (256 x 128 x 96), mixed
    precision, checked step by step from the seeded inputs: stage 1 meets the
    FP64 tolerance under the oracle's operator; u* is the velocity update of that P*;
    u~2 is (u* + u^k) + dt R; P meets it for that u~2 and u^{k+1} is its
    halved update, discretely solenoidal."""
    seq = fx.C4Sequence()
    wl = fx.c4_step(40)
    wl.phi = wl.phi.astype(np.float32).astype(np.float64)
    phi_s = seq.step(41)[0].astype(np.float32).astype(np.float64)
    R = _forcing(wl, 77)
    uk = (wl.u, wl.v, wl.w)
    dt = 0.005
    og, ob, _, _ = oracle_for(wl)
    gg, gop = gpu_for(wl, phi_dtype=torch.float32)
    out = gop.rk2_cycle(_t(wl.phi).float(), _t(phi_s).float(), tuple(_t(a) for a in uk),
                        tuple(_t(a) for a in R), dt, tol=1e-8, precision="mixed")
    print(f"[rk2] stage 1: {out['stage1'].iterations} its {out['stage1'].ms:.0f} ms; "
          f"stage 2: {out['stage2'].iterations} its {out['stage2'].ms:.0f} ms", flush=True)
    assert out["status"] == 0
    op1 = Operator(og, ob, wl.phi, wl.rho_l, wl.rho_g, wl.smooth)
    op2 = Operator(og, ob, phi_s, wl.rho_l, wl.rho_g, wl.smooth)
    ut1 = tuple(u + dt * r for u, r in zip(uk, R))
    pstar = host(out["pstar"])
    assert solvers.true_relres(op1, op1.rhs(*ut1, dt), pstar) <= 1.01e-8
    ustar = tuple(host(a) for a in out["ustar"])
    for g, r in zip(ustar, rk2.update_velocity(op1, ut1, pstar, dt)):
        assert np.array_equal(g, r)
    ut2 = tuple(host(a) for a in out["ut2"])
    for g, a, u, r in zip(ut2, ustar, uk, R):
        assert np.array_equal(g, (a + u) + dt * r)
    p = host(out["p"])
    assert solvers.true_relres(op2, op2.rhs(*ut2, dt), p) <= 1.01e-8
    unext = tuple(host(a) for a in out["unext"])
    for g, r in zip(unext, rk2.update_velocity(op2, ut2, p, dt, 0.5)):
        assert np.array_equal(g, r)
    d = op2.merged_divergence(*[o * a for o, a in zip(_open(ob), unext)])
    d0 = op2.merged_divergence(*[o * a for o, a in zip(_open(ob), ut2)])
    assert np.linalg.norm(d) <= 2e-8 * np.linalg.norm(d0)
