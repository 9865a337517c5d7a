"""HIP path vs the CPU oracle, through the C ABI (needs an MI355X).

Geometry, assembly and the FP64 operator are compared bitwise (same
expressions, same order, FP contraction off on both sides); reductions and
solves within the tolerances stated per test.  Sizes span several 64 x 4 x 16
tiles with ragged tails in every direction.
"""
import math

import numpy as np
import pytest

from paper_1410_1937_amd import fixtures as fx
from oracle import solvers
from tests.gpu_helpers import gpu_for, host, oracle_for, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cases():
    return {
        "sphere_neumann": fx.small(0, 70, 36, 30, body="sphere"),
        "ellipsoid_dirichlet": fx.small(1, 64, 20, 17, body="ellipsoid", bc=(0, 1, 0, 0, 1, 0), theta=0.4),
        "nobody_uniform_all_dirichlet": fx.small(2, 33, 7, 5, body=None, bc=(1,) * 6, stretch=False,
                                                 smooth=False),
        "c1": fx.c1(),
        # three FP32 column tiles across x (the last 8 cells wide), five FP64
        # ones, and a partial 16-row tile in y
        "wide_ragged": fx.small(6, 520, 18, 9, body="sphere"),
        # the FP64 sweep-A tile widths of the full-size grids: rows of 512
        # cells (4 wavefronts across, 4 rows per tile; 10 rows leave a 2-row
        # tile) and of 256 cells (2 across, 8 rows; 13 rows leave 5), both with
        # merged cells
        "wx4_sphere_neumann": fx.small(3, 512, 10, 6, body="sphere", theta=0.5),
        "wx2_sphere_dirichlet_top": fx.small(4, 256, 13, 7, body="sphere", bc=(0, 0, 0, 0, 0, 1), theta=0.5),
    }


CASES = _cases()


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    wl = CASES[request.param]
    og, ob, oop, ob_rhs = oracle_for(wl)
    gg, gop = gpu_for(wl)
    return request.param, wl, (og, ob, oop, ob_rhs), (gg, gop)


def test_geometry_bitwise(case):
    name, wl, (og, ob, oop, _), (gg, gop) = case
    assert np.array_equal(host(gg.export("frac_x")), ob.frac_x)
    assert np.array_equal(host(gg.export("frac_y")), ob.frac_y)
    assert np.array_equal(host(gg.export("frac_z")), ob.frac_z)
    assert np.array_equal(host(gg.export("vfrac")), ob.vfrac)
    assert np.array_equal(host(gg.export("active")), ob.active.astype(np.uint8))
    assert np.array_equal(host(gg.export("open_x")), ob.open_x)
    assert np.array_equal(host(gg.export("open_y")), ob.open_y)
    assert np.array_equal(host(gg.export("open_z")), ob.open_z)
    assert np.array_equal(host(gg.export("root")), ob.root.astype(np.int32))
    assert np.array_equal(host(gg.export("reduced")), ob.reduced.astype(np.uint8))
    info = gg.info()
    assert info["slaves"] == len(ob.slaves) and info["reduced"] == ob.n_reduced


def test_assembly_bitwise(case):
    name, wl, (og, ob, oop, _), (gg, gop) = case
    assert np.array_equal(host(gop.export("rho")), oop.rho)
    assert np.array_equal(host(gop.export("tx")), oop.tx)
    assert np.array_equal(host(gop.export("ty")), oop.ty)
    assert np.array_equal(host(gop.export("tz")), oop.tz)
    assert np.array_equal(host(gop.export("dinv")), oop.dinv)
    # FP32 copies are the round-to-nearest FP32 values of the FP64 ones
    assert np.array_equal(host(gop.export("tx32")), oop.tx.astype(np.float32))
    assert np.array_equal(host(gop.export("dinv32")), oop.dinv.astype(np.float32))


def test_apply_fp64_bitwise_and_fp32_within_rounding_bound(case):
    name, wl, (og, ob, oop, _), (gg, gop) = case
    rng = np.random.default_rng(11)
    x = rng.standard_normal(og.shape)
    y_or = oop.apply(x)
    y = host(gop.apply(torch.as_tensor(x, device="cuda")))
    assert np.array_equal(y, y_or)
    x32 = x.astype(np.float32)
    y32 = host(gop.apply(torch.as_tensor(x32, device="cuda"))).astype(np.float64)
    ref = oop.apply(x32.astype(np.float64))
    # |error| <= c u sum_f |T_f (p_c - p_nb)| with u = 2^-24 (flux form)
    xe = oop.expand(x32.astype(np.float64))
    pp = np.pad(xe, 1)
    c = pp[1:-1, 1:-1, 1:-1]
    mag = (np.abs(oop.tx[:, :, :-1] * (c - pp[1:-1, 1:-1, :-2])) + np.abs(oop.tx[:, :, 1:] * (c - pp[1:-1, 1:-1, 2:]))
           + np.abs(oop.ty[:, :-1] * (c - pp[1:-1, :-2, 1:-1])) + np.abs(oop.ty[:, 1:] * (c - pp[1:-1, 2:, 1:-1]))
           + np.abs(oop.tz[:-1] * (c - pp[:-2, 1:-1, 1:-1])) + np.abs(oop.tz[1:] * (c - pp[2:, 1:-1, 1:-1])))
    mag = oop.gather(mag)
    assert np.all(np.abs(y32 - ref) <= 10 * 2.0 ** -24 * mag + 1e-300)


def test_rhs_matches_oracle(case):
    name, wl, (og, ob, oop, ob_rhs), (gg, gop) = case
    if wl.u is None:
        pytest.skip("right-hand side given directly")
    b = host(gop.rhs(torch.as_tensor(wl.u, device="cuda"), torch.as_tensor(wl.v, device="cuda"),
                     torch.as_tensor(wl.w, device="cuda"), wl.dt, wl.body_vel))
    scale = np.max(np.abs(ob_rhs))
    # identical up to the rounding of the removed mean (a reduction)
    assert np.max(np.abs(b - ob_rhs)) <= 1e-14 * scale
    assert np.array_equal(b == 0, ob_rhs == 0) or np.max(np.abs(b[(b == 0) != (ob_rhs == 0)])) <= 1e-14 * scale


def _gpu_b(wl, gop):
    if wl.b is not None:
        return torch.as_tensor(wl.b, device="cuda").contiguous()
    return gop.rhs(torch.as_tensor(wl.u, device="cuda"), torch.as_tensor(wl.v, device="cuda"),
                   torch.as_tensor(wl.w, device="cuda"), wl.dt, wl.body_vel)


def test_fp64_solve_matches_oracle_at_relres_1e10(case):
    """rel L2 <= 1e-9 against the oracle solved tightly (to 1e-13)."""
    name, wl, (og, ob, oop, ob_rhs), (gg, gop) = case
    ref = solvers.pcg(oop, ob_rhs, tol=1e-13)
    xr = oop.gauge(ref.x)
    b = _gpu_b(wl, gop)
    x, res = gop.solve(b, tol=1e-10, precision="f64")
    assert res.status == 0 and res.relres <= 1e-10
    xg = host(x)
    assert rel_l2(xg, xr) <= 1e-9
    # the reported residual is the true one (oracle apply on the GPU result)
    assert solvers.true_relres(oop, ob_rhs, xg) <= 1.01e-10
    # PCG in the same order of operations needs about the oracle's iteration count
    it_or = solvers.pcg(oop, ob_rhs, tol=1e-10).iterations
    assert abs(res.iterations - it_or) <= max(3, 0.05 * it_or)


def test_mixed_solve_meets_fp64_tolerance(case):
    name, wl, (og, ob, oop, ob_rhs), (gg, gop) = case
    b = _gpu_b(wl, gop)
    x, res = gop.solve(b, tol=1e-8, precision="mixed")
    assert res.status == 0 and res.relres <= 1e-8 and not res.fallback
    xg = host(x)
    assert solvers.true_relres(oop, ob_rhs, xg) <= 1.01e-8
    xr = oop.gauge(solvers.pcg(oop, ob_rhs, tol=1e-13).x)
    err = rel_l2(xg, xr)
    x64, r64 = gop.solve(b, tol=1e-8, precision="f64")
    err64 = rel_l2(host(x64), xr)
    print(f"[{name}] mixed: {res.iterations} its ({r64.iterations} FP64), {res.outer} FP64 residuals, "
          f"rel L2 err {err:.2e} (FP64 at the same tol: {err64:.2e})")
    # the FP32 recursion with its residual replaced every 10x continues as CG
    # (the next direction keeps the recursion's beta with the replaced r.z on
    # top), so it needs about FP64's iterations; 1.3-1.6x when beta was taken
    # against the last r.z instead
    assert res.iterations <= 1.15 * r64.iterations + 10
    assert err <= 1e-5


def test_flexible_cg_with_jacobi_tracks_pcg(case):
    name, wl, (og, ob, oop, ob_rhs), (gg, gop) = case
    b = _gpu_b(wl, gop)
    _, r1 = gop.solve(b, tol=1e-8, precision="mixed", precond="jacobi")
    # monitor off: plain Jacobi converges at ~0.99 per iteration on these grids
    _, r2 = gop.solve(b, tol=1e-8, precision="mixed", precond="jacobi_fcg", fallback_ratio=2.0)
    assert r2.status == 0 and r2.relres <= 1e-8 and not r2.fallback
    # equal in exact arithmetic (the oracle pins that in FP64); in FP32 the
    # explicit orthogonalisation of FCG(1) drifts differently from PCG's
    assert r2.iterations <= 2.0 * r1.iterations + 10


def test_projection_and_divergence(case):
    name, wl, (og, ob, oop, ob_rhs), (gg, gop) = case
    if wl.u is None:
        pytest.skip("right-hand side given directly")
    u, v, w = (torch.as_tensor(a, device="cuda") for a in (wl.u, wl.v, wl.w))
    b = gop.rhs(u, v, w, wl.dt, wl.body_vel)
    p, res = gop.solve(b, tol=1e-10, precision="f64")
    F = gop.project(u, v, w, p, wl.dt)
    Fo = oop.project(wl.u, wl.v, wl.w, host(p), wl.dt)
    for a, bo in zip(F, Fo):
        assert np.array_equal(host(a), bo)
    div = host(gop.divergence(*F, wl.body_vel))
    assert np.array_equal(div, oop.merged_divergence(*Fo, wl.body_vel))
    # post-projection discrete divergence is at the solver tolerance (eq. diverge)
    assert np.linalg.norm(div) <= wl.dt * 1.01e-10 * np.linalg.norm(ob_rhs) + 1e-13 * np.linalg.norm(
        oop.merged_divergence(*oop.open_flux(wl.u, wl.v, wl.w), wl.body_vel))


def test_failure_paths():
    wl = fx.small(3, 40, 24, 20, body="sphere")
    og, ob, oop, ob_rhs = oracle_for(wl)
    gg, gop = gpu_for(wl)
    b = _gpu_b(wl, gop)
    # sabotaged preconditioner: the stagnation monitor falls back to Jacobi-PCG
    x, res = gop.solve(b, tol=1e-8, precision="mixed", precond="sabotage")
    assert res.status == 0 and res.fallback and res.relres <= 1e-8
    assert solvers.true_relres(oop, ob_rhs, host(x)) <= 1.01e-8
    # iteration cap: a warning with the state filled in
    x, res = gop.solve(b, tol=1e-8, precision="f64", max_iters=3)
    assert res.status == 1 and res.iterations == 3 and res.relres > 1e-8
    # NaN in b
    bad = b.clone()
    bad[3, 4, 5] = float("nan")
    from paper_1410_1937_amd.nfa import NFAError
    with pytest.raises(NFAError, match="NaN"):
        gop.solve(bad, tol=1e-8)
    # warm start from the solution: nothing to do
    x, res = gop.solve(b, tol=1e-8, precision="f64")
    x2, res2 = gop.solve(b, x=x.clone(), tol=1e-8, precision="f64", warm_start=True)
    assert res2.iterations == 0 and res2.relres <= 1e-8


@pytest.mark.parametrize("name", ["wx4_sphere_neumann", "wx2_sphere_dirichlet_top"])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 8])
def test_solve_cut_off_after_n_iterations_returns_the_oracle_iterate(name, n):
    """Jacobi-PCG defers its x update over two iterations (every other sweep
    leaves x alone and the next applies both owed steps); a solve stopped
    after n iterations, n odd or even, must return PCG's n-th iterate.
    Compared through the residual b' - A'x of the oracle's operator, which
    does not depend on the gauge."""
    wl = CASES[name]
    og, ob, oop, ob_rhs = oracle_for(wl)
    gg, gop = gpu_for(wl)
    b = _gpu_b(wl, gop)
    ref = solvers.pcg(oop, ob_rhs, tol=1e-30, maxit=n)
    assert ref.iterations == n
    r_ref = ob_rhs - oop.apply(ref.x)
    x, res = gop.solve(b, tol=1e-30, precision="f64", max_iters=n)
    assert res.status == 1 and res.iterations == n
    assert rel_l2(ob_rhs - oop.apply(host(x)), r_ref) <= 1e-11
    # the FP32 recursion folds its increment (the owed steps applied) into
    # the FP64 solution when it stops: the same iterate to FP32 rounding
    xm, resm = gop.solve(b, tol=1e-30, precision="mixed", max_iters=n)
    assert resm.status == 1 and resm.iterations == n
    assert rel_l2(ob_rhs - oop.apply(host(xm)), r_ref) <= 1e-4


def test_solves_are_bitwise_reproducible():
    wl = fx.small(4, 50, 30, 22, body="sphere")
    gg, gop = gpu_for(wl)
    b = _gpu_b(wl, gop)
    x1, r1 = gop.solve(b, tol=1e-9, precision="f64")
    x2, r2 = gop.solve(b, tol=1e-9, precision="f64")
    x3, r3 = gop.solve(b, tol=1e-9, precision="mixed")
    x4, r4 = gop.solve(b, tol=1e-9, precision="mixed")
    assert r1.iterations == r2.iterations and torch.equal(x1, x2)
    assert r3.iterations == r4.iterations and torch.equal(x3, x4)


def test_float32_phi_input():
    wl = fx.small(5, 48, 16, 12, body="sphere")
    wl.phi = wl.phi.astype(np.float32).astype(np.float64)
    og, ob, oop, _ = oracle_for(wl)
    gg, gop = gpu_for(wl, phi_dtype=torch.float32)
    assert np.array_equal(host(gop.export("tz")), oop.tz)


def test_zero_rhs_and_a_single_column():
    """Degenerate inputs: a zero right-hand side returns x = 0 at once; a
    1 x 1 x 64 column (one lane live in every sweep) with the 1000 : 1.2 jump,
    Neumann bottom and Dirichlet top, solved against a banded direct solve of
    the oracle's own matrix."""
    from scipy.linalg import solve_banded
    from oracle.geometry import Body
    from oracle.grid import Grid
    from oracle.operator import Operator
    from paper_1410_1937_amd import nfa
    nz = 64
    xf = yf = np.array([0.0, 1.0])
    zf = fx.stretched_faces(0.0, 1.0, nz, [0.5])
    phi = (fx.centres(zf) < 0.5).astype(np.float64).reshape(nz, 1, 1)
    bc = (0, 0, 0, 0, 0, 1)
    g = nfa.Grid(xf, yf, zf, bc)
    g.set_body(None)
    op = nfa.Poisson(g)
    op.assemble(torch.as_tensor(phi, device="cuda"), 1000.0, 1.2, False)
    for precision in ("f64", "mixed"):
        x, res = op.solve(torch.zeros((nz, 1, 1), dtype=torch.float64, device="cuda"), precision=precision)
        assert res.status == 0 and res.iterations == 0 and res.relres == 0.0
        assert not torch.any(x)
    og = Grid(xf, yf, zf, bc)
    oop = Operator(og, Body(og, None, 0.25, 8), phi, 1000.0, 1.2, False)
    A = oop.csr().toarray()
    ab = np.zeros((3, nz))
    ab[0, 1:] = np.diag(A, 1)
    ab[1] = np.diag(A)
    ab[2, :-1] = np.diag(A, -1)
    b = np.random.default_rng(8).standard_normal(nz)
    ref = solve_banded((1, 1), ab, b)
    x, res = op.solve(torch.as_tensor(b.reshape(nz, 1, 1), device="cuda"), tol=1e-12, precision="f64")
    assert res.status == 0 and res.relres <= 1e-12
    assert rel_l2(host(x).ravel(), ref) <= 1e-9


def test_a_new_body_leaves_the_operator_stale_until_it_is_assembled_again():
    """nfa_grid_set_body after an assembly changes the apertures, the active
    set and the merge groups the coefficients were formed from: the
    operator's calls refuse until it is assembled again, then match the
    oracle of the new body."""
    import dataclasses
    from paper_1410_1937_amd import nfa
    wl = fx.small(5, 40, 14, 12, body="sphere", theta=0.5)
    gg, gop = gpu_for(wl)
    x = torch.as_tensor(np.random.default_rng(2).standard_normal(gg.shape), device="cuda")
    gop.apply(x)
    b = _gpu_b(wl, gop)
    wl2 = dataclasses.replace(wl, psi=fx.psi_sphere(wl.xf, wl.yf, wl.zf, radius=0.09, centre=(0.05, 0.02, -0.2)))
    gg.set_body(torch.as_tensor(wl2.psi, device="cuda").contiguous(), wl2.theta, wl2.samples)
    for call in (lambda: gop.apply(x), lambda: gop.solve(b, tol=1e-8), lambda: gop.residual(b, x),
                 lambda: gop.project(*(torch.as_tensor(a, device="cuda") for a in (wl.u, wl.v, wl.w)), x)):
        with pytest.raises(nfa.NFAError, match="assemble again"):
            call()
    gop.assemble(torch.as_tensor(wl2.phi, device="cuda").contiguous(), wl2.rho_l, wl2.rho_g, wl2.smooth)
    og, ob, oop, _ = oracle_for(wl2)
    assert np.array_equal(host(gop.apply(x)), oop.apply(host(x)))
    assert np.array_equal(host(gop.export("dinv")), oop.dinv)


def test_apply_on_unaligned_views_takes_the_scalar_sweep():
    """Inputs and outputs that are not 16-byte aligned run the one-cell-per-lane
    form of the operator sweep; it is bitwise the vector form's result."""
    wl = CASES["wx4_sphere_neumann"]
    og, ob, oop, _ = oracle_for(wl)
    gg, gop = gpu_for(wl)
    rng = np.random.default_rng(12)
    x = rng.standard_normal(og.shape)
    n = x.size
    buf = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    buf[1:] = torch.as_tensor(x.reshape(-1), device="cuda")
    xv = buf[1:].view(og.shape)
    assert xv.data_ptr() % 16 != 0
    out = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    yv = out[1:].view(og.shape)
    gop.apply(xv, out=yv)
    assert np.array_equal(host(yv), oop.apply(x))
    assert np.array_equal(host(yv), host(gop.apply(torch.as_tensor(x, device="cuda"))))
