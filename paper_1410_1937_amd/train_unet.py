"""Train the learned preconditioner on the GPU with the library's own kernels.

Data: the 200-step advected free surface on the 256 x 128 x 96 hull grid
(fixtures.C4Sequence).  For every time step the plain FP64 Jacobi-PCG solver
gives x* (relative residual 1e-10); residual/error pairs (r_k, e_k = x* - x_k)
are taken along its iteration after k = 0, 4, 16, 64, 256 steps, plus two
smooth synthetic errors e with r = A'e.  Steps 0-159 train, 160-199 test.

Each training step runs nfa_unet_train_step: forward, the A-norm step loss
1 - (z.r)^2/((z.A'z)(e.A'e)), backward and one Adam step.  The weights are
written as a raw float32 .npy (no pickling) with a JSON record of the run.

    python -m paper_1410_1937_amd.train_unet --minutes 3 --out paper_1410_1937_amd/weights/unet_c4
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from paper_1410_1937_amd import fixtures as fx
from paper_1410_1937_amd import nfa

KS = (0, 4, 16, 64, 256)


def log(*a):
    print(*a, flush=True)


def make_operator(seq):
    g = nfa.Grid(seq.xf, seq.yf, seq.zf, seq.bc)
    g.set_body(torch.as_tensor(seq.psi, device="cuda"), seq.theta, 8)
    return g, nfa.Poisson(g)


def generate(seq, op, steps, synth=2):
    """Per time step: phi (FP32, device) and a list of (r FP32 device, e.A'e)."""
    data = []
    nz, ny, nx = seq.shape
    red = None
    for n in steps:
        phi, (u, v, w) = seq.step(n)
        phi_t = torch.as_tensor(phi, device="cuda").float().contiguous()
        op.assemble(phi_t)
        b = op.rhs(*(torch.as_tensor(a, device="cuda") for a in (u, v, w)))
        xs, res = op.solve(b, tol=1e-10, precision="f64")
        if red is None:
            red = op.grid.export("reduced").double()
        samples = []
        x = torch.zeros_like(b)
        done = 0
        for k in KS:
            if k > done:
                x, _ = op.solve(b, x=x, tol=1e-30, precision="f64", max_iters=k - done, warm_start=True)
                done = k
            r, _ = op.residual(b, x)
            e = xs - x
            eAe = float(torch.dot(e.ravel(), r.ravel()))
            if eAe > 0:
                samples.append((r.float().contiguous(), eAe))
        for q in range(synth):
            e = torch.as_tensor(seq.smooth_field(7919 * n + q), device="cuda") * red
            r = op.apply(e)
            eAe = float(torch.dot(e.ravel(), r.ravel()))
            if eAe > 0:
                samples.append((r.float().contiguous(), eAe))
        data.append((n, phi_t, samples))
        log(f"[train] data step {n}: {res.iterations} its to 1e-10, {len(samples)} pairs")
    return data


def evaluate(op, net, seq, steps, tol=1e-8):
    rows = []
    for n in steps:
        phi, (u, v, w) = seq.step(n)
        op.assemble(torch.as_tensor(phi, device="cuda").float().contiguous())
        b = op.rhs(*(torch.as_tensor(a, device="cuda") for a in (u, v, w)))
        row = {"step": n}
        for name, kw in (("fp64_jacobi", dict(precision="f64")),
                         ("mixed_jacobi", dict(precision="mixed")),
                         ("mixed_unet", dict(precision="mixed", precond="unet", unet=net))):
            op.solve(b, tol=tol, **kw)   # warm caches
            _, r = op.solve(b, tol=tol, **kw)
            row[name] = {"iterations": r.iterations, "ms": r.ms, "relres": r.relres, "fallback": r.fallback}
        rows.append(row)
        log(f"[train] eval step {n}: " + ", ".join(f"{k} {v['iterations']} its {v['ms']:.1f} ms"
                                                 for k, v in row.items() if k != "step"))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--minutes", type=float, default=3.0, help="training time budget")
    ap.add_argument("--train-steps", type=int, default=160)
    ap.add_argument("--test-steps", type=int, default=40)
    ap.add_argument("--stride", type=int, default=1, help="use every stride-th time step")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--ny", type=int, default=128)
    ap.add_argument("--nz", type=int, default=96)
    ap.add_argument("--eval", type=int, default=4, help="test steps to evaluate")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "weights", "unet_c4"))
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    seq = fx.C4Sequence(args.nx, args.ny, args.nz)
    g, op = make_operator(seq)
    train_ids = list(range(0, args.train_steps, args.stride))
    test_ids = list(range(args.train_steps, args.train_steps + args.test_steps, args.stride))
    t0 = time.time()
    data = generate(seq, op, train_ids)
    t_data = time.time() - t0
    net = nfa.UNet(args.nx, args.ny, args.nz, seed=args.seed)
    rng = np.random.default_rng(args.seed)
    budget = args.minutes * 60.0
    t1 = time.time()
    step, epoch, hist = 0, 0, []
    total_est = None
    while time.time() - t1 < budget:
        order = rng.permutation(len(data))
        losses = []
        for idx in order:
            n, phi_t, samples = data[idx]
            op.assemble(phi_t)
            for r, eAe in samples:
                step += 1
                frac = min(1.0, (time.time() - t1) / budget)
                lr = args.lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * frac)))
                losses.append(net.train_step(op, r, eAe, lr, step))
            if time.time() - t1 >= budget:
                break
        epoch += 1
        hist.append(float(np.mean(losses)))
        log(f"[train] epoch {epoch}: {step} steps, mean loss {hist[-1]:.4f}, "
            f"{(time.time() - t1) / step * 1e3:.1f} ms/step")
    t_train = time.time() - t1
    params = net.get_params()
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.save(args.out + ".npy", params)
    evals = evaluate(op, net, seq, test_ids[:args.eval]) if args.eval > 0 else []
    untrained = nfa.UNet(args.nx, args.ny, args.nz, seed=args.seed)
    ev_un = evaluate(op, untrained, seq, test_ids[:1]) if args.eval > 0 else []
    rec = {"grid": [args.nx, args.ny, args.nz], "train_steps": train_ids, "test_steps": test_ids[:args.eval],
           "pairs": sum(len(s) for _, _, s in data), "optimizer_steps": step, "epochs": epoch,
           "lr": args.lr, "minutes_budget": args.minutes, "data_seconds": t_data, "train_seconds": t_train,
           "epoch_loss": hist, "eval": evals, "eval_untrained": ev_un, "param_count": int(params.size)}
    with open(args.out + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    log(f"[train] wrote {args.out}.npy and .json")
    return 0


if __name__ == "__main__":
    sys.exit(main())
