"""Full-size workloads (3.1M and 25M cells) in the configuration the
benchmark times: geometry and coefficients compared bitwise with the oracle
over the whole grid, and every solve checked by the oracle's own FP64 apply
on the returned pressure (true relative residual <= 1e-8)."""
import numpy as np
import pytest

from paper_1410_1937_amd import fixtures as fx
from oracle import solvers
from tests.gpu_helpers import gpu_for, host, oracle_for

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("name,phi_dtype", [("c2", "float64"), ("c3", "float32")])
def test_full_size_projection(name, phi_dtype):
    """The 25M-cell case holds phi in FP32, as the benchmark does; the oracle
    gets the same FP32-representable values."""
    wl = getattr(fx, name)()
    if phi_dtype == "float32":
        wl.phi = wl.phi.astype(np.float32).astype(np.float64)
    print(f"[{name}] building oracle", flush=True)
    og, ob, oop, ob_rhs = oracle_for(wl)
    print(f"[{name}] building GPU operator", flush=True)
    gg, gop = gpu_for(wl, phi_dtype=getattr(torch, phi_dtype))
    for item, ref in (("frac_x", ob.frac_x), ("vfrac", ob.vfrac), ("open_y", ob.open_y),
                      ("open_z", ob.open_z)):
        assert np.array_equal(host(gg.export(item)), ref), item
    assert np.array_equal(host(gg.export("root")), ob.root.astype(np.int32))
    for item, ref in (("tx", oop.tx), ("ty", oop.ty), ("tz", oop.tz), ("dinv", oop.dinv)):
        assert np.array_equal(host(gop.export(item)), ref), item
    u, v, w = (torch.as_tensor(a, device="cuda") for a in (wl.u, wl.v, wl.w))
    b = gop.rhs(u, v, w, wl.dt, wl.body_vel)
    bh = host(b)
    assert np.max(np.abs(bh - ob_rhs)) <= 1e-14 * np.max(np.abs(ob_rhs))
    # sampled apply parity on a random vector
    x = torch.randn(gop.shape, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(0))
    y = host(gop.apply(x))
    assert np.array_equal(y, oop.apply(host(x)))
    for precision in ("f64", "mixed"):
        print(f"[{name}] solve {precision}", flush=True)
        p, res = gop.solve(b, tol=1e-8, precision=precision)
        print(f"[{name}] {precision}: {res.iterations} its, outer {res.outer}, relres {res.relres:.3e}, "
              f"{res.ms:.1f} ms", flush=True)
        assert res.status == 0 and res.relres <= 1e-8
        tr = solvers.true_relres(oop, ob_rhs, host(p))
        assert tr <= 1.01e-8, tr


def test_heaving_sphere_sequence_warm_started():
    """Three consecutive projections of the 768x384x256 heaving-sphere sequence
    (75.5M cells) in the chosen form: mixed precision, the first one with the
    learned preconditioner behind the stagnation monitor (it runs at any grid
    size divisible by 16), each later one warm-started from the previous
    pressure and each checked by the oracle's own FP64 apply."""
    import os
    from oracle.operator import Operator
    from paper_1410_1937_amd import nfa
    # phi is held in FP32 (as the benchmark does); both sides get the same
    # FP32-representable values
    wl = fx.c5_step(0)
    wl.phi = wl.phi.astype(np.float32).astype(np.float64)
    print("[c5] building oracle geometry", flush=True)
    og, ob, oop, ob_rhs = oracle_for(wl)
    gg, gop = gpu_for(wl, phi_dtype=torch.float32)
    net = nfa.UNet(*gop.shape[::-1], levels=3)
    wpath = os.path.join(os.path.dirname(nfa.__file__), "weights", "unet_l3_c4.npy")
    net.set_params(np.load(wpath))
    x = torch.zeros(gop.shape, dtype=torch.float64, device="cuda")
    for n in range(3):
        if n > 0:
            wl = fx.c5_step(n)
            wl.phi = wl.phi.astype(np.float32).astype(np.float64)
            oop = Operator(og, ob, wl.phi, wl.rho_l, wl.rho_g, wl.smooth)
            ob_rhs = oop.rhs(wl.u, wl.v, wl.w, wl.dt, wl.body_vel)
            gop.assemble(torch.as_tensor(wl.phi, device="cuda").float().contiguous(), wl.rho_l, wl.rho_g, wl.smooth)
        u, v, w = (torch.as_tensor(a, device="cuda") for a in (wl.u, wl.v, wl.w))
        b = gop.rhs(u, v, w, wl.dt, wl.body_vel)
        kw = dict(precond="unet", unet=net) if n == 0 else {}
        x, res = gop.solve(b, x=x, tol=1e-8, precision="mixed", warm_start=n > 0, **kw)
        print(f"[c5] projection {n}: {res.iterations} its, outer {res.outer}, fallback {res.fallback}, "
              f"relres {res.relres:.3e}, {res.ms:.0f} ms", flush=True)
        assert res.status == 0 and res.relres <= 1e-8
        assert solvers.true_relres(oop, ob_rhs, host(x)) <= 1.01e-8
