"""The panel signed distance on the GPU against the oracle (needs an
MI355X): psi at every node of small stretched grids for a box, an icosphere
and a Wigley hull (to 1e-13, signs equal), one open triangle, the chain
panels -> psi -> body fractions against the oracle's chain, and sampled
nodes of the 512 x 256 x 192 breaking-wave grid around a 5120-panel
sphere."""
import numpy as np
import pytest

from oracle import panels as opanels
from oracle.geometry import Body
from oracle.grid import Grid
from paper_1410_1937_amd import fixtures as fx
from tests.gpu_helpers import host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _grid(n=(29, 17, 13), lo=(-0.75, -0.25, -0.5), hi=(0.75, 0.25, 0.25), seed=0):
    rng = np.random.default_rng(seed)
    faces = []
    for m, a, b in zip(n, lo, hi):
        w = rng.uniform(0.5, 1.5, m)
        faces.append(a + (b - a) * np.concatenate([[0.0], np.cumsum(w)]) / np.sum(w))
    return faces


MESHES = {
    "box": lambda: fx.box_panels((-0.31, -0.083, -0.27), (0.22, 0.121, 0.093)),
    "sphere": lambda: fx.icosphere_panels(0.17, (0.013, -0.007, -0.11), levels=2),
    "wigley": lambda: fx.wigley_panels(length=0.9, beam=0.2, draft=0.15, freeboard=0.1, nx=24, nz=6),
}


@pytest.mark.parametrize("mesh", sorted(MESHES))
def test_psi_at_every_node_matches_the_oracle(mesh):
    from paper_1410_1937_amd import nfa
    tri = MESHES[mesh]()
    xf, yf, zf = _grid()
    g = nfa.Grid(xf, yf, zf, (0,) * 6)
    got = host(g.panels_psi(_t(tri)))
    ref = opanels.nodes_psi(xf, yf, zf, tri)
    assert np.max(np.abs(got - ref)) <= 1e-13
    assert np.array_equal(np.sign(got), np.sign(ref))
    assert np.count_nonzero(ref < 0) > 20


def test_one_open_triangle_is_a_plain_distance():
    from paper_1410_1937_amd import nfa
    tri = np.array([[[-0.2, -0.1, -0.3], [0.4, 0.05, -0.1], [0.0, 0.2, 0.1]]])
    xf, yf, zf = _grid(seed=1)
    g = nfa.Grid(xf, yf, zf, (0,) * 6)
    got = host(g.panels_psi(_t(tri)))
    ref = opanels.nodes_psi(xf, yf, zf, tri)
    assert np.all(got >= 0) and np.max(np.abs(got - ref)) <= 1e-13


def test_panels_to_body_fractions_match_the_oracle_chain():
    from paper_1410_1937_amd import nfa
    tri = MESHES["wigley"]()
    xf, yf, zf = _grid((40, 24, 18), seed=2)
    g = nfa.Grid(xf, yf, zf, (0,) * 6)
    psi = g.panels_psi(_t(tri))
    g.set_body(psi, 0.25, 8)
    og = Grid(xf, yf, zf, (0,) * 6)
    ob = Body(og, opanels.nodes_psi(xf, yf, zf, tri), 0.25, 8)
    assert np.array_equal(host(g.export("active")).astype(bool), ob.active > 0)
    for name, ref in (("open_x", ob.open_x), ("open_y", ob.open_y), ("open_z", ob.open_z)):
        assert np.max(np.abs(host(g.export(name)) - ref)) <= 1e-15
    assert 0.005 < np.mean(ob.active == 0) < 0.5


def test_bad_arguments_are_refused():
    from paper_1410_1937_amd import nfa
    g = nfa.Grid(*_grid(), (0,) * 6)
    with pytest.raises(ValueError):
        g.panels_psi(_t(np.zeros((4, 9))))
    with pytest.raises(nfa.NFAError, match="panels"):
        g.panels_psi(torch.zeros((0, 3, 3), dtype=torch.float64, device="cuda"))


def test_full_size_grid_sampled_nodes_around_a_sphere():
    """The breaking-wave grid (513 x 257 x 193 nodes) and a sphere of 5120
    panels at its immersed body's place: 4000 nodes drawn at random plus the
    nodes nearest the surface, recomputed by the oracle."""
    from paper_1410_1937_amd import nfa
    wl = fx.c3()
    tri = fx.icosphere_panels(0.1, (0.0, 0.0, -0.15), levels=4)
    g = nfa.Grid(wl.xf, wl.yf, wl.zf, wl.bc)
    got = host(g.panels_psi(_t(tri)))
    assert got.shape == (len(wl.zf), len(wl.yf), len(wl.xf))
    rng = np.random.default_rng(4)
    idx = [tuple(rng.integers(0, s, 4000)) for s in got.shape]
    k, j, i = (np.asarray(v) for v in idx)
    zc, yc, xc = np.meshgrid(wl.zf, wl.yf, wl.xf, indexing="ij")
    near = np.argwhere(np.abs(np.sqrt(xc ** 2 + yc ** 2 + (zc + 0.15) ** 2) - 0.1) < 0.004)
    del zc, yc, xc
    pick = near[rng.choice(len(near), min(2000, len(near)), replace=False)]
    k, j, i = np.concatenate([k, pick[:, 0]]), np.concatenate([j, pick[:, 1]]), np.concatenate([i, pick[:, 2]])
    pts = np.stack([wl.xf[i], wl.yf[j], wl.zf[k]], axis=1)
    ref = opanels.signed_distance(pts, tri)
    assert np.max(np.abs(got[k, j, i] - ref)) <= 1e-13
    assert np.array_equal(np.sign(got[k, j, i]), np.sign(ref))
    exact = np.linalg.norm(pts - np.array([0.0, 0.0, -0.15]), axis=1) - 0.1
    assert np.max(np.abs(ref - exact)) < 1e-3
