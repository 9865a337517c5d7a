"""The boundary's memory contract on the GPU (needs an MI355X): the
operator's and the network's device memory are caller-owned workspaces
(torch tensors here), solves with every preconditioner and re-assemblies
allocate no device memory, a workspace shorter than the library asks for is
refused with NFA_ERR_NOMEM before anything is created, and the network's
parameter state lives in caller arrays from which training resumes exactly."""
import ctypes

import numpy as np
import pytest

from paper_1410_1937_amd import fixtures as fx
from tests.gpu_helpers import host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NFA_ERR_INVALID, NFA_ERR_NOMEM = -1, -2


def _problem():
    from paper_1410_1937_amd import nfa
    wl = fx.small(3, 64, 32, 24, body="sphere")
    g, op, b = nfa.from_workload(wl, device_phi_dtype=torch.float32)
    phi = torch.as_tensor(wl.phi, device="cuda").float().contiguous()
    return nfa, wl, g, op, b, phi


def test_solves_and_assemblies_allocate_no_device_memory():
    nfa, wl, g, op, b, phi = _problem()
    print("memory contract: 64x32x24 sphere, four solver forms", flush=True)
    assert op.workspace.numel() == nfa.lib.nfa_poisson_workspace_bytes(g.h)
    net = nfa.UNet(64, 32, 24, levels=3)
    op.multigrid()
    x = torch.zeros_like(b)
    forms = [dict(precision="f64"), dict(precision="mixed"), dict(precision="mixed", precond="mg"),
             dict(precision="mixed", precond="unet", unet=net)]

    def sweep():
        for kw in forms:
            op.assemble(phi, wl.rho_l, wl.rho_g, wl.smooth)        # the multigrid set-up reruns in the solve
            _, res = op.solve(b, x=x, tol=1e-8, **kw)
            assert res.status == 0 and res.relres <= 1e-8, (kw, res)
    sweep()                       # first use: torch's allocator cache settles
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(10):
        sweep()
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, (free0, free1)


def test_short_or_misaligned_workspace_is_refused_before_anything_is_created():
    from paper_1410_1937_amd import nfa
    wl = fx.small(4, 32, 16, 12, body="sphere")
    g = nfa.Grid(wl.xf, wl.yf, wl.zf, wl.bc)
    need = int(nfa.lib.nfa_poisson_workspace_bytes(g.h))
    assert need > 100 * 32 * 16 * 12
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    st = nfa.lib.nfa_poisson_create(g.h, ctypes.c_void_p(ws.data_ptr()), need - 1, ctypes.byref(h))
    assert st == NFA_ERR_NOMEM and h.value is None
    assert b"needs" in nfa.lib.nfa_last_error()
    st = nfa.lib.nfa_poisson_create(g.h, ctypes.c_void_p(ws.data_ptr() + 16), need, ctypes.byref(h))
    assert st == NFA_ERR_INVALID and h.value is None
    st = nfa.lib.nfa_poisson_create(g.h, ctypes.c_void_p(ws.data_ptr()), need, ctypes.byref(h))
    assert st == 0 and h.value is not None
    nfa.lib.nfa_poisson_destroy(h)
    un = int(nfa.lib.nfa_unet_workspace_bytes(32, 16, 12, 3))
    assert un > 0 and nfa.lib.nfa_unet_workspace_bytes(30, 16, 12, 3) == 0
    wsu = torch.empty(un, dtype=torch.uint8, device="cuda")
    hu = ctypes.c_void_p()
    st = nfa.lib.nfa_unet_create(32, 16, 12, 3, 0, ctypes.c_void_p(wsu.data_ptr()), un - 256, ctypes.byref(hu))
    assert st == NFA_ERR_NOMEM and hu.value is None


def test_training_resumes_exactly_from_the_caller_owned_state():
    """Three Adam steps, a checkpoint of (params, m, v), then the fourth step
    taken by the same network and by a new one loaded from the checkpoint:
    the parameters agree bit for bit (the gradients are fixed-order sums)."""
    from paper_1410_1937_amd import nfa
    from oracle import solvers
    from tests.gpu_helpers import oracle_for
    wl = fx.small(5, 32, 16, 12, body="sphere")
    og, ob, oop, ob_rhs = oracle_for(wl)
    g, op, b = nfa.from_workload(wl)
    r = torch.as_tensor((ob_rhs * ob.reduced).astype(np.float32), device="cuda")
    e = solvers.pcg(oop, r.cpu().numpy().astype(np.float64), tol=1e-12).x
    eAe = float(np.sum(e * r.cpu().numpy()))
    a = nfa.UNet(32, 16, 12, seed=1)
    p0 = host(a.params).copy()
    for t in range(1, 4):
        a.train_step(op, r, eAe, 1e-3, t)
    assert not np.array_equal(host(a.params), p0)          # the bound tensor is what training updates
    ckpt = a.state()
    bnet = nfa.UNet(32, 16, 12, seed=7)
    bnet.load_state(ckpt)
    la = a.train_step(op, r, eAe, 1e-3, 4)
    lb = bnet.train_step(op, r, eAe, 1e-3, 4)
    assert la == lb
    assert np.array_equal(host(a.params), host(bnet.params))
    assert np.array_equal(host(a.adam_v), host(bnet.adam_v))
