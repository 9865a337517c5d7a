"""Pins of the oracle's aggregation multigrid (no GPU): the level-1 operator
of a uniform problem is the 7-point operator with four fine faces per coarse
face; Galerkin levels keep the constants in the null space when every
boundary is Neumann; the V-cycle is a symmetric positive definite operator
(dense check, with a body and merges); the coarsest level is solved
exactly; and multigrid-preconditioned CG converges in a small fraction of
the Jacobi iterations to the dense solution."""
import numpy as np
import pytest

from oracle import multigrid, solvers
from oracle.geometry import Body
from oracle.grid import Grid
from oracle.operator import Operator
from paper_1410_1937_amd import fixtures as fx
from tests.gpu_helpers import oracle_for


def _uniform_op(n, bc=(0,) * 6):
    f = fx.uniform_faces(0.0, 1.0, n)
    g = Grid(f, f, f, bc)
    return Operator(g, Body(g, None, 0.25, 8), np.ones(g.shape), 1.0, 1.0, smooth=False)


def test_level_one_of_a_uniform_problem_is_the_coarse_seven_point_operator():
    op = _uniform_op(8)
    H = multigrid.Hierarchy(op, min_coarse=1)
    T = op.tx[0, 0, 1]
    A1 = H.A[1].toarray()
    assert H.shapes[1] == (4, 4, 4)
    c = (1 * 4 + 2) * 4 + 1                    # an interior block
    nbrs = {c - 1, c + 1, c - 4, c + 4, c - 16, c + 16}
    assert A1[c, c] == pytest.approx(24 * T, rel=1e-14)
    for m in nbrs:
        assert A1[c, m] == pytest.approx(-4 * T, rel=1e-14)
    assert np.count_nonzero(A1[c]) == 7


def test_constants_stay_in_the_null_space_of_every_level():
    wl = fx.small(1, 24, 16, 12, body="sphere")
    og, ob, op, b = oracle_for(wl)
    H = multigrid.Hierarchy(op, min_coarse=10)
    assert len(H.A) >= 3
    for l, A in enumerate(H.A[1:], start=1):
        rows = np.abs(A @ np.ones(A.shape[0]))
        assert np.max(rows) <= 1e-12 * np.max(np.abs(A.diagonal())), l


@pytest.mark.parametrize("alpha,coef", [(1.0, "f64"), (0.5, "f64"), (1.9, "f64"), (1.0, "bf16")])
@pytest.mark.parametrize("bc", [(0,) * 6, (0, 0, 0, 0, 0, 1)])
def test_vcycle_is_symmetric_positive_definite(bc, alpha, coef):
    wl = fx.small(2, 12, 10, 8, body="sphere", bc=bc)
    og, ob, op, b = oracle_for(wl)
    H = multigrid.Hierarchy(op, min_coarse=20, alpha=alpha, coef=coef)
    red = np.nonzero(op.reduced_mask().reshape(-1))[0]
    n = op.grid.n
    M = np.zeros((len(red), len(red)))
    for col, c in enumerate(red):
        e = np.zeros(n)
        e[c] = 1.0
        M[:, col] = H.vcycle(e)[red]
    assert np.max(np.abs(M - M.T)) <= 1e-12 * np.max(np.abs(M))
    assert np.min(np.linalg.eigvalsh(0.5 * (M + M.T))) > 0


@pytest.mark.parametrize("bc", [(0,) * 6, (0, 0, 0, 0, 0, 1)])
def test_coarsest_level_is_solved_exactly(bc):
    wl = fx.small(3, 8, 6, 6, body="sphere", bc=bc)
    og, ob, op, b = oracle_for(wl)
    H = multigrid.Hierarchy(op, min_coarse=10 ** 6)
    assert len(H.A) == 2                     # one coarsening, always
    rc = H.maps[0].T @ b.reshape(-1)         # a compatible coarse right-hand side
    xc = H.coarse_inv @ rc
    assert np.linalg.norm(H.A[1] @ xc - rc) <= 1e-10 * np.linalg.norm(rc)


def test_multigrid_cg_converges_fast_to_the_dense_solution():
    wl = fx.c1()
    og, ob, op, b = oracle_for(wl)
    H = multigrid.Hierarchy(op)
    res = solvers.fcg(op, b, H.precond, tol=1e-10, fallback=False)
    jac = solvers.pcg(op, b, tol=1e-10)
    assert res.relres <= 1e-10
    assert res.iterations * 5 <= jac.iterations, (res.iterations, jac.iterations)
    assert np.linalg.norm(res.x - jac.x) <= 1e-8 * np.linalg.norm(jac.x)


@pytest.mark.parametrize("alpha", [0.6, 1.0, 1.7])
def test_two_level_cycle_follows_its_error_propagation(alpha):
    """With an exact coarse solve, e -> S (I - alpha P A_c^-1 P^T A) S e for
    the error e = x - V(A x), S = I - omega D^-1 A: the pre-smoothing, the
    scaled coarse correction and the post-smoothing in that order, built
    here from dense matrices."""
    wl = fx.small(3, 10, 8, 8, body="sphere", bc=(0, 0, 0, 0, 0, 1))
    og, ob, op, b = oracle_for(wl)
    omega = 0.8
    H = multigrid.Hierarchy(op, min_coarse=10 ** 6, omega=omega, alpha=alpha)
    assert len(H.A) == 2
    red = np.nonzero(op.reduced_mask().reshape(-1))[0]
    A = H.A[0][red][:, red].toarray()
    P = H.maps[0][red].toarray()
    ne = np.nonzero(P.sum(axis=0) > 0)[0]
    P = P[:, ne]
    Ac = H.A[1][ne][:, ne].toarray()
    I = np.eye(len(red))
    S = I - omega * (A / np.diag(A)[:, None])
    E = S @ (I - alpha * P @ np.linalg.solve(Ac, P.T @ A)) @ S
    x = np.random.default_rng(0).standard_normal(len(red))
    r = np.zeros(op.grid.n)
    r[red] = A @ x
    got = H.vcycle(r)[red]
    assert np.linalg.norm(got - (x - E @ x)) <= 1e-10 * np.linalg.norm(x)


def test_bf16_rounding_is_nearest_even_after_fp32():
    """Worked values: ties go to the even mantissa, magnitudes below a half
    unit round down, signs and zero pass through, and an FP64 value takes
    its FP32 rounding first."""
    one = 1.0
    u = 2.0 ** -7                      # BF16 spacing at 1
    vals = np.array([one + u / 2, one + 3 * u / 2, one + u / 2 + 2.0 ** -20, one + u / 4, -(one + 3 * u / 2), 0.0,
                     3.0e-30])
    got = multigrid.bf16(vals)
    want = [one, one + 2 * u, one + u, one, -(one + 2 * u), 0.0]
    assert np.array_equal(got[:6], want)
    # the last value: FP32 first, then 8 significant bits
    x32 = np.float32(3.0e-30)
    m, e = np.frexp(np.float64(x32))
    assert abs(got[6] - np.ldexp(np.round(m * 256) / 256, e)) <= np.ldexp(1.0, e - 9)


def test_bf16_cycle_stays_close_to_the_exact_one():
    """Rounding the level-0 coefficients to BF16 (relative error <= 2^-9)
    moves one V-cycle's output by a comparable relative amount."""
    wl = fx.small(5, 20, 14, 12, body="sphere")
    og, ob, op, b = oracle_for(wl)
    Hf = multigrid.Hierarchy(op)
    Hb = multigrid.Hierarchy(op, coef="bf16")
    r = np.where(op.reduced_mask() > 0, np.random.default_rng(3).standard_normal(og.shape), 0.0)
    zf, zb = Hf.precond(r), Hb.precond(r)
    d = np.linalg.norm(zb - zf) / np.linalg.norm(zf)
    assert 1e-6 < d < 3e-2
