"""Shared set-up of the GPU parity tests: the same seeded workload handed to
the oracle (NumPy) and to the HIP library (through the C ABI binding)."""
import numpy as np

from oracle.geometry import Body
from oracle.grid import Grid
from oracle.operator import Operator


def oracle_for(wl):
    g = Grid(wl.xf, wl.yf, wl.zf, wl.bc)
    body = Body(g, wl.psi, wl.theta, wl.samples)
    op = Operator(g, body, wl.phi, wl.rho_l, wl.rho_g, wl.smooth)
    if wl.b is not None:
        b = op.compatible(op.gather(np.asarray(wl.b) * (body.active > 0)))
    else:
        b = op.rhs(wl.u, wl.v, wl.w, wl.dt, wl.body_vel)
    return g, body, op, b


def gpu_for(wl, phi_dtype=None):
    import torch
    from paper_1410_1937_amd import nfa
    g = nfa.Grid(wl.xf, wl.yf, wl.zf, wl.bc)
    if wl.psi is not None:
        g.set_body(torch.as_tensor(wl.psi, device="cuda").contiguous(), wl.theta, wl.samples)
    op = nfa.Poisson(g)
    phi = torch.as_tensor(wl.phi, device="cuda").contiguous()
    if phi_dtype is not None:
        phi = phi.to(phi_dtype)
    op.assemble(phi, wl.rho_l, wl.rho_g, wl.smooth)
    return g, op


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
