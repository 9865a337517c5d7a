"""The multigrid preconditioner on the GPU against the oracle (needs an
MI355X): every coarse level's stencil equals the oracle's Galerkin product
(and a rebuild is bitwise the same), one V-cycle equals the oracle's to FP32
accuracy, multigrid-preconditioned mixed solves meet their tolerance and the
oracle's solution in a handful of the Jacobi iterations, and the 25M-cell
breaking-wave projection converges, checked by the oracle's FP64
operator."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import multigrid, solvers
from paper_1410_1937_amd import fixtures as fx
from tests.gpu_helpers import gpu_for, host, oracle_for, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _stencil_to_sparse(st):
    """(27, nz, ny, nx) stencil -> n x n sparse matrix."""
    _, nz, ny, nx = st.shape
    n = nz * ny * nx
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rows, cols, vals = [], [], []
    for o in range(27):
        dz, dy, dx = o // 9 - 1, (o // 3) % 3 - 1, o % 3 - 1
        kn, jn, inn = k + dz, j + dy, i + dx
        ok = (kn >= 0) & (kn < nz) & (jn >= 0) & (jn < ny) & (inn >= 0) & (inn < nx) & (st[o] != 0)
        rows.append(((k * ny + j) * nx + i)[ok])
        cols.append(((kn * ny + jn) * nx + inn)[ok])
        vals.append(st[o][ok])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


CASES = [("sphere", (0,) * 6, (37, 21, 17)), ("sphere", (0, 0, 0, 0, 0, 1), (40, 24, 20)),
         ("ellipsoid", (0,) * 6, (48, 16, 20))]


@pytest.mark.parametrize("body,bc,shape", CASES)
def test_every_level_matches_the_oracle_and_rebuilds_bitwise(body, bc, shape):
    wl = fx.small(5, *shape, body=body, bc=bc)
    og, ob, oop, b = oracle_for(wl)
    H = multigrid.Hierarchy(oop)
    g, op = gpu_for(wl)
    mg = op.multigrid()
    mg.setup()
    levels = mg.levels()
    assert [tuple(s) for s in levels] == [tuple(s) for s in H.shapes]
    first = []
    for l in range(1, len(levels)):
        st = host(mg.export(l))
        first.append(st)
        A = _stencil_to_sparse(st)
        ref = H.A[l]
        scale = np.max(np.abs(ref.diagonal()))
        assert abs(A - ref).max() <= 1e-12 * scale, l
        if l < len(levels) - 1:
            # rows coupled beyond the 7 points, as the cycle's side list holds them
            far = np.zeros(st.shape[1:], dtype=bool)
            for o in set(range(27)) - {4, 10, 12, 13, 14, 16, 22}:
                far |= st[o] != 0
            assert mg.side_rows(l) == int(far.sum()), l
    mg.setup()
    for l in range(1, len(levels)):
        assert np.array_equal(host(mg.export(l)), first[l - 1])


@pytest.mark.parametrize("tail", [-1, 0])
@pytest.mark.parametrize("body,bc,shape", CASES + [("sphere", (0,) * 6, (64, 48, 40)), ("sphere", (0,) * 6, (300, 20, 10))])
def test_one_vcycle_matches_the_oracle(body, bc, shape, tail):
    """tail -1: every coarse level in the one-workgroup kernel; 0: the
    grid-wide level kernels down to the coarsest.  The 300 x 20 x 10 grid
    spans several level-0 tiles in x and y, each with a ragged last one."""
    wl = fx.small(6, *shape, body=body, bc=bc)
    og, ob, oop, b = oracle_for(wl)
    H = multigrid.Hierarchy(oop)
    g, op = gpu_for(wl)
    mg = op.multigrid()
    mg.set_tail(tail)
    mg.setup()
    assert mg.side_rows(1) > 0   # merges couple level 1 beyond the 7 points
    red = oop.reduced_mask() > 0
    r = np.where(red, np.random.default_rng(0).standard_normal(og.shape), 0.0).astype(np.float32)
    z = host(mg.apply(torch.as_tensor(r, device="cuda")))
    ref = oop.expand(H.precond(r.astype(np.float64)))
    assert rel_l2(z[red | (ob.root.reshape(og.shape) >= 0)], ref[red | (ob.root.reshape(og.shape) >= 0)]) <= 1e-4


@pytest.mark.parametrize("tail", [-1, 0])
def test_vcycle_with_merges_at_a_dirichlet_wall(tail):
    """A sphere cut by the bottom wall, which holds p = 0: slaves and roots
    lie on the wall, so the merged rows' corrections meet boundary faces with
    nonzero coefficients."""
    import dataclasses
    wl = fx.small(11, 60, 28, 24, body="sphere", bc=(0, 0, 0, 0, 1, 0))
    wl = dataclasses.replace(wl, psi=fx.psi_sphere(wl.xf, wl.yf, wl.zf, radius=0.15, centre=(0.02, 0.01, -0.47)))
    og, ob, oop, b = oracle_for(wl)
    root = ob.root.reshape(og.shape)
    slave = (root >= 0) & (root != np.arange(root.size).reshape(og.shape))
    assert slave[0].sum() > 0   # slaves on the wall layer
    H = multigrid.Hierarchy(oop)
    g, op = gpu_for(wl)
    mg = op.multigrid()
    mg.set_tail(tail)
    mg.setup()
    red = oop.reduced_mask() > 0
    r = np.where(red, np.random.default_rng(3).standard_normal(og.shape), 0.0).astype(np.float32)
    z = host(mg.apply(torch.as_tensor(r, device="cuda")))
    ref = oop.expand(H.precond(r.astype(np.float64)))
    act = red | (root >= 0)
    assert rel_l2(z[act], ref[act]) <= 1e-4


@pytest.mark.parametrize("tail", [-1, 0])
def test_vcycle_with_other_damping_and_coarse_scale(tail):
    wl = fx.small(8, 64, 48, 40, body="sphere")
    og, ob, oop, b = oracle_for(wl)
    H = multigrid.Hierarchy(oop, omega=0.85, alpha=1.6)
    g, op = gpu_for(wl)
    mg = op.multigrid()
    mg.set_tail(tail)
    mg.set_params(0.85, 1.6)
    mg.setup()
    red = oop.reduced_mask() > 0
    r = np.where(red, np.random.default_rng(1).standard_normal(og.shape), 0.0).astype(np.float32)
    z = host(mg.apply(torch.as_tensor(r, device="cuda")))
    ref = oop.expand(H.precond(r.astype(np.float64)))
    keep = red | (ob.root.reshape(og.shape) >= 0)
    assert rel_l2(z[keep], ref[keep]) <= 1e-4
    with pytest.raises(Exception):
        mg.set_params(1.0, 1.0)
    with pytest.raises(Exception):
        mg.set_params(0.7, 2.0)


@pytest.mark.parametrize("name,tail", [("c1", -1), ("sphere", -1), ("sphere", 0)])
def test_mg_solve_meets_tolerance_and_the_oracle(name, tail):
    wl = fx.c1() if name == "c1" else fx.small(7, 37, 21, 17, body="sphere")
    og, ob, oop, b = oracle_for(wl)
    ref = solvers.pcg(oop, b, tol=1e-11)
    H = multigrid.Hierarchy(oop)
    ref_mg = solvers.fcg(oop, b, H.precond, tol=1e-10, fallback=False)
    g, op = gpu_for(wl)
    op.multigrid().set_tail(tail)
    bt = torch.as_tensor(b, device="cuda")
    x, res = op.solve(bt, tol=1e-10, precision="mixed", precond="mg")
    assert res.status == 0 and res.relres <= 1e-10 and not res.fallback
    xs = host(x)
    if og.all_neumann:
        xs = oop.gauge(xs)
        xr = oop.gauge(ref.x)
    else:
        xr = ref.x
    assert rel_l2(xs, xr) <= 1e-7
    assert res.iterations <= 1.5 * ref_mg.iterations + 5, (res.iterations, ref_mg.iterations)
    assert res.iterations * 5 <= ref.iterations


def test_full_size_breaking_wave_projection_with_multigrid():
    """512 x 256 x 192 with phi held in FP32 (as the benchmark does): mixed
    precision with the multigrid preconditioner to FP64 true relres 1e-8,
    the residual recomputed by the oracle's operator."""
    wl = fx.c3()
    wl.phi = wl.phi.astype(np.float32).astype(np.float64)
    print("[c3] building oracle", flush=True)
    og, ob, oop, ob_rhs = oracle_for(wl)
    g, op = gpu_for(wl, phi_dtype=torch.float32)
    u, v, w = (torch.as_tensor(a, device="cuda") for a in (wl.u, wl.v, wl.w))
    bt = op.rhs(u, v, w, wl.dt, wl.body_vel)
    print("[c3] multigrid solve", flush=True)
    x, res = op.solve(bt, tol=1e-8, precision="mixed", precond="mg")
    print(f"[c3] mg: {res.iterations} its, outer {res.outer}, relres {res.relres:.3e}, {res.ms:.1f} ms", flush=True)
    assert res.status == 0 and res.relres <= 1e-8 and not res.fallback
    assert res.iterations < 400, res.iterations
    assert solvers.true_relres(oop, ob_rhs, host(x)) <= 1.01e-8


@pytest.mark.parametrize("shape,body,bc", [((3, 2, 2), "none", (0, 0, 0, 0, 0, 1)), ((5, 4, 3), "none", (0,) * 6),
                                           ((9, 7, 6), "sphere", (0,) * 6), ((12, 8, 8), "sphere", (0, 0, 0, 0, 0, 1))])
def test_tiny_grids_solve_with_one_coarsening(shape, body, bc):
    """Grids small enough that level 1 is already the coarsest (dense) level,
    odd sizes and the one-cell-per-lane level-0 sweeps: the multigrid solve
    meets its tolerance and the oracle's solution."""
    wl = fx.small(9, *shape, body=body, bc=bc)
    og, ob, oop, b = oracle_for(wl)
    H = multigrid.Hierarchy(oop)
    g, op = gpu_for(wl)
    mg = op.multigrid()
    assert [tuple(s) for s in mg.levels()] == [tuple(s) for s in H.shapes]
    x, res = op.solve(torch.as_tensor(b, device="cuda"), tol=1e-10, precision="mixed", precond="mg")
    assert res.status == 0 and res.relres <= 1e-10
    ref = solvers.pcg(oop, b, tol=1e-12)
    xs, xr = host(x), ref.x
    if og.all_neumann:
        xs, xr = oop.gauge(xs), oop.gauge(xr)
    assert rel_l2(xs, xr) <= 1e-7


@pytest.mark.parametrize("tail", [-1, 0])
@pytest.mark.parametrize("body,bc,shape", [CASES[0], CASES[1], ("sphere", (0,) * 6, (64, 48, 40))])
def test_vcycle_with_bf16_coefficients_matches_the_oracle(body, bc, shape, tail):
    """Level 0 of the cycle reading its coefficients and D^-1 in BF16: equal
    to the oracle's cycle with the same roundings."""
    wl = fx.small(6, *shape, body=body, bc=bc)
    og, ob, oop, b = oracle_for(wl)
    H = multigrid.Hierarchy(oop, coef="bf16")
    g, op = gpu_for(wl)
    mg = op.multigrid()
    mg.set_tail(tail)
    mg.set_coef("bf16")
    mg.setup()
    red = oop.reduced_mask() > 0
    r = np.where(red, np.random.default_rng(2).standard_normal(og.shape), 0.0).astype(np.float32)
    z = host(mg.apply(torch.as_tensor(r, device="cuda")))
    ref = oop.expand(H.precond(r.astype(np.float64)))
    keep = red | (ob.root.reshape(og.shape) >= 0)
    assert rel_l2(z[keep], ref[keep]) <= 1e-4


@pytest.mark.parametrize("coef", ["f32", "bf16"])
def test_mg_solve_with_either_coefficient_precision(coef):
    wl = fx.small(7, 64, 48, 40, body="sphere")
    og, ob, oop, b = oracle_for(wl)
    ref = solvers.pcg(oop, b, tol=1e-11)
    g, op = gpu_for(wl)
    op.multigrid().set_coef(coef)
    x, res = op.solve(torch.as_tensor(b, device="cuda"), tol=1e-10, precision="mixed", precond="mg")
    assert res.status == 0 and res.relres <= 1e-10 and not res.fallback
    assert rel_l2(oop.gauge(host(x)), oop.gauge(ref.x)) <= 1e-7
