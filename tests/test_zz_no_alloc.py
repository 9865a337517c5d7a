"""nfa_panels_psi_noalloc, the entry point that allocates no device memory,
against nfa_panels_psi (needs an MI355X): the same signed distance bit for
bit on two calls in a row, the second with fewer panels (its static work
memory keeps the first call's contents), no change in free device memory
across the calls, and more panels than its work memory holds refused before
any device work."""
import ctypes

import numpy as np
import pytest

from paper_1410_1937_amd import fixtures as fx
from tests.gpu_helpers import host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _faces(n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    out = []
    for m, a, b in zip(n, lo, hi):
        w = rng.uniform(0.5, 1.5, m)
        out.append(a + (b - a) * np.concatenate([[0.0], np.cumsum(w)]) / np.sum(w))
    return out


def test_noalloc_signed_distance_equals_the_allocating_one_on_two_calls():
    from paper_1410_1937_amd import nfa
    print("no-alloc signed distance: 5120 then 320 panels on a 48x28x22 grid", flush=True)
    xf, yf, zf = _faces((48, 28, 22), (-0.75, -0.25, -0.5), (0.75, 0.25, 0.25), seed=3)
    g = nfa.Grid(xf, yf, zf, (0,) * 6)
    shape = (len(zf), len(yf), len(xf))
    meshes = [fx.icosphere_panels(0.21, (0.013, -0.007, -0.11), levels=4),
              fx.icosphere_panels(0.12, (-0.05, 0.03, -0.2), levels=2)]
    assert meshes[0].shape[0] == 5120 and meshes[1].shape[0] == 320
    tris = [torch.as_tensor(np.ascontiguousarray(t), device="cuda") for t in meshes]
    refs = [host(g.panels_psi(t)) for t in tris]
    outs = [torch.full(shape, np.nan, dtype=torch.float64, device="cuda") for _ in tris]
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for t, out in zip(tris, outs):
        g.panels_psi(t, out=out, noalloc=True)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    for out, ref in zip(outs, refs):
        got = host(out)
        assert np.array_equal(got, ref)
        assert np.count_nonzero(ref < 0) > 20
    # the two bodies differ, so a stale work memory would have shown
    assert not np.array_equal(refs[0], refs[1])


def test_noalloc_signed_distance_refuses_more_panels_than_its_work_memory():
    from paper_1410_1937_amd import nfa
    xf, yf, zf = _faces((8, 6, 5), (-0.75, -0.25, -0.5), (0.75, 0.25, 0.25), seed=4)
    g = nfa.Grid(xf, yf, zf, (0,) * 6)
    tri = torch.as_tensor(np.ascontiguousarray(fx.box_panels((-0.3, -0.1, -0.3), (0.2, 0.1, 0.1))), device="cuda")
    psi = torch.zeros((6, 7, 9), dtype=torch.float64, device="cuda")
    f = nfa.lib.nfa_panels_psi_noalloc
    st = f(g.h, ctypes.c_void_p(tri.data_ptr()), 65537, ctypes.c_void_p(psi.data_ptr()), None)
    assert st == -1
    assert b"at most 65536 panels" in nfa.lib.nfa_last_error()
    assert torch.count_nonzero(psi).item() == 0
    # within the limit it runs
    assert f(g.h, ctypes.c_void_p(tri.data_ptr()), tri.shape[0], ctypes.c_void_p(psi.data_ptr()), None) == 0
