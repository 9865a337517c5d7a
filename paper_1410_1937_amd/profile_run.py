"""A short, fixed workload for hardware-counter runs of the CG sweeps.

Sets up the 512 x 256 x 192 breaking-wave projection problem
(fixtures.c3), then runs a fixed number of mixed-precision and FP64
Jacobi-PCG iterations (tolerance unreachable, so every iteration runs both
sweeps), and finally three plain device-to-device copies of known size (the library's
k_stream_copy, 1 GiB each by default) whose counter readings calibrate the
FETCH_SIZE / WRITE_SIZE counters to bytes; with --fill, three plain writes of
the same size after them (the library's k_stream_fill).
With --mg N it runs N mixed-precision iterations preconditioned by the
multigrid V-cycle (hierarchy set-up included).  With --unet L it also runs --unet-reps forward passes of an L-level learned
preconditioner on the same grid (the committed weights for L = 3), then
--unet-train training steps of it.  With
--vof N it runs N split VOF advection steps (alternating sweep order) of the
FP64 volume fraction through the workload's face velocities.  With --psi L
it computes the signed distance of an L-times subdivided icosphere (the
workload's sphere) at the grid nodes three times.  Each phase prints a line
when it ends.

    rocprofv3 --pmc FETCH_SIZE -d F -o run -- python3 -m paper_1410_1937_amd.profile_run --iters 8
    rocprofv3 --pmc WRITE_SIZE -d W -o run -- python3 -m paper_1410_1937_amd.profile_run --iters 8
    python3 -m paper_1410_1937_amd.profile_summary traffic F/run_results.db W/run_results.db
    rocprofv3 --kernel-trace --stats -d OUT -- python3 -m paper_1410_1937_amd.profile_run --iters 0 --unet 5
    rocprofv3 --kernel-trace --stats -d OUT -- python3 -m paper_1410_1937_amd.profile_run --iters 0 --vof 6
"""
from __future__ import annotations

import argparse
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=8, help="iterations per precision")
    ap.add_argument("--copy-mib", type=int, default=1024, help="size of the calibration copy (4x the 256 MiB Infinity Cache by default)")
    ap.add_argument("--mg", type=int, default=0, help="mixed-precision multigrid-preconditioned iterations")
    ap.add_argument("--unet", type=int, default=0, help="levels of the learned preconditioner to run (0: none)")
    ap.add_argument("--unet-reps", type=int, default=5)
    ap.add_argument("--unet-train", type=int, default=0,
                    help="after the forward passes, this many training steps of the same network (nfa_unet_train_step)")
    ap.add_argument("--vof", type=int, default=0, help="VOF advection steps to run")
    ap.add_argument("--psi", type=int, default=-1, help="icosphere subdivision levels for the signed distance")
    ap.add_argument("--fill", action="store_true", help="after the copies, three plain writes of the same size (k_stream_fill)")
    args = ap.parse_args(argv)
    import torch
    from paper_1410_1937_amd import fixtures as fx
    from paper_1410_1937_amd import nfa

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = fx.c3()
    g = nfa.Grid(wl.xf, wl.yf, wl.zf, wl.bc)
    g.set_body(torch.as_tensor(wl.psi, device=dev), wl.theta, wl.samples)
    op = nfa.Poisson(g)
    op.assemble(torch.as_tensor(wl.phi, device=dev).float().contiguous(), wl.rho_l, wl.rho_g, wl.smooth)
    b = op.rhs(*(torch.as_tensor(a, device=dev) for a in (wl.u, wl.v, wl.w)), wl.dt, wl.body_vel)
    torch.cuda.synchronize()
    print(f"[profile_run] set up {g.nx * g.ny * g.nz} cells", flush=True)
    for prec in ("mixed", "f64") if args.iters > 0 else ():
        _, res = op.solve(b, tol=1e-30, precision=prec, max_iters=args.iters)
        torch.cuda.synchronize()
        print(f"[profile_run] {prec}: {res.iterations} iterations", flush=True)
    if args.mg:
        _, res = op.solve(b, tol=1e-30, precision="mixed", precond="mg", max_iters=args.mg)
        torch.cuda.synchronize()
        print(f"[profile_run] mixed+mg: {res.iterations} iterations", flush=True)
    if args.unet:
        import os
        import numpy as np
        net = nfa.UNet(g.nx, g.ny, g.nz, levels=args.unet)
        wpath = os.path.join(os.path.dirname(nfa.__file__), "weights", f"unet_l{args.unet}_c4.npy")
        if os.path.exists(wpath):
            net.set_params(np.load(wpath))
        r = (b / torch.linalg.vector_norm(b)).float().contiguous()
        for _ in range(args.unet_reps):
            net.forward(op, r)
        torch.cuda.synchronize()
        print(f"[profile_run] unet L{args.unet}: {args.unet_reps} forward passes", flush=True)
        # training steps on the same residual: forward with the activations
        # kept, the A-norm step loss and its gradient, the backward pass and
        # Adam (eAe only scales the loss, so any positive value runs the
        # same kernels)
        for t in range(1, args.unet_train + 1):
            net.train_step(op, r, 1.0, 1e-5, t)
        torch.cuda.synchronize()
        if args.unet_train:
            print(f"[profile_run] unet L{args.unet}: {args.unet_train} training steps", flush=True)
    if args.vof:
        vf = nfa.Vof(g)
        phi = torch.as_tensor(wl.phi, device=dev)
        out = torch.empty_like(phi)
        vel = tuple(torch.as_tensor(a, device=dev) for a in (wl.u, wl.v, wl.w))
        dt = fx.vof_time_step(wl)
        for step in range(args.vof):
            vf.advect(phi, *vel, dt, step, out=out)
        torch.cuda.synchronize()
        print(f"[profile_run] vof: {args.vof} steps", flush=True)
    if args.psi >= 0:
        tri = torch.as_tensor(fx.icosphere_panels(0.1, (0.0, 0.0, -0.15), levels=args.psi), device=dev)
        psi = g.panels_psi(tri)
        for _ in range(2):
            g.panels_psi(tri, out=psi)
        torch.cuda.synchronize()
        print(f"[profile_run] psi: 3 x {tri.shape[0]} panels", flush=True)
    n = args.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        nfa.stream_copy(dst, src)     # k_stream_copy, one dispatch of known size
    torch.cuda.synchronize()
    print(f"[profile_run] copy: 3 x {args.copy_mib} MiB read + written (k_stream_copy)", flush=True)
    if args.fill:
        for _ in range(3):
            nfa.stream_fill(dst, 0)   # k_stream_fill, writes only
        torch.cuda.synchronize()
        print(f"[profile_run] write: 3 x {args.copy_mib} MiB written (k_stream_fill)", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
