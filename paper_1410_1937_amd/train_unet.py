"""Train the learned preconditioner on the GPU with the library's own kernels,
and evaluate it on the held-out steps of the advected-surface sequence.

Data (the 3.1M-cell advected-surface sequence, 256 x 128 x 96 around the
Wigley-like hull, fixtures.C4Sequence): for every training step n in
0..159 (every --stride-th) the plain FP64 Jacobi-PCG solver gives x* to
relative residual 1e-10; the residual/error pairs (r_k, e_k = x* - x_k) are
taken along its iteration after k = 0, 4, 16, 64, 256 steps, plus four smooth
synthetic errors e with r = A'e.  Optionally (--breaking) snapshots of the
breaking-wave geometry at the same size, and (--rounds > 1) pairs met by
flexible CG with the current network, are added.

Each training step runs nfa_unet_train_step: forward, the A-norm step loss
1 - (z.r)^2/((z.A'z)(e.A'e)), backward and one Adam step, with a cosine
learning-rate decay over the step budget.  The weights are written as a raw
float32 .npy (no pickling) with a JSON record of the run and of the held-out
evaluation: on every step 160..199, iterations and milliseconds to the FP64
relative residual 1e-8 for FP64 Jacobi-PCG, mixed Jacobi-PCG, mixed FCG with
the trained network and with the untrained one (the Jacobi step), the
stagnation monitor on; the relative residual after 100 FCG iterations with
the monitor off; and the one-step A-norm loss on the held-out step's own
pairs (k = 0, 16, 64, 256), trained against untrained.

    python -m paper_1410_1937_amd.train_unet --levels 3 --max-steps 3000 \
        --out paper_1410_1937_amd/weights/unet_l3_c4

Besides the weights it writes <out>.state.npz (parameters, Adam moments and the
step count, arrays only), from which --resume continues training.
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
ONPOLICY_KS = (8, 32, 96)
SYNTH = 4
EVAL_KS = (0, 16, 64, 256)


def log(*a):
    print(*a, flush=True)


class Problem:
    """One projection problem on the GPU: operator, rhs, reference solution
    and its training pairs."""

    def __init__(self, name, op, phi_t, b, xs, red):
        self.name, self.op, self.phi_t, self.b, self.xs, self.red = name, op, phi_t, b, xs, red
        self.samples = []

    def activate(self):
        self.op.assemble(self.phi_t)

    def add_pair(self, x):
        r, _ = self.op.residual(self.b, x)
        e = self.xs - x
        eAe = float(torch.dot(e.ravel(), r.ravel()))
        if eAe > 0:
            self.samples.append((r.float().contiguous(), eAe))


def operator_for(xf, yf, zf, bc, psi, theta):
    g = nfa.Grid(xf, yf, zf, bc)
    g.set_body(torch.as_tensor(psi, device="cuda"), theta, 8)
    return g, nfa.Poisson(g)


def build_problem(name, op, phi, uvw, smooth_src=None, synth=SYNTH, seed=0):
    phi_t = torch.as_tensor(phi, device="cuda").float().contiguous()
    op.assemble(phi_t)
    b = op.rhs(*(torch.as_tensor(a, device="cuda") for a in uvw))
    xs, res = op.solve(b, tol=1e-10, precision="f64")
    red = op.grid.export("reduced").double()
    p = Problem(name, op, phi_t, b, xs, red)
    x = torch.zeros_like(b)
    done = 0
    for k in KS:
        if k > done:
            x, _ = op.solve(b, x=x, tol=1e-30, precision="f64", max_iters=k - done, warm_start=True)
            done = k
        p.add_pair(x)
    if smooth_src is not None:
        for q in range(synth):
            e = torch.as_tensor(smooth_src(seed * 7919 + q), device="cuda") * red
            r = op.apply(e)
            eAe = float(torch.dot(e.ravel(), r.ravel()))
            if eAe > 0:
                p.samples.append((r.float().contiguous(), eAe))
    log(f"[train] problem {name}: {res.iterations} its to 1e-10, {len(p.samples)} pairs")
    return p


def add_onpolicy(problems, net):
    for p in problems:
        p.activate()
        for k in ONPOLICY_KS:
            x, _ = p.op.solve(p.b, tol=1e-30, precision="mixed", precond="unet", unet=net, max_iters=k,
                              fallback_ratio=2.0)
            p.add_pair(x)


def train(problems, net, minutes, lr0, step0, rng, max_steps=0):
    """Adam over shuffled problems for `minutes` or, when max_steps > 0, for
    that many optimizer steps; cosine learning-rate decay over the budget."""
    budget = minutes * 60.0
    t1 = time.time()
    step, hist = step0, []

    def progress():
        if max_steps > 0:
            return (step - step0) / max_steps
        return (time.time() - t1) / budget

    while progress() < 1.0:
        losses = []
        for idx in rng.permutation(len(problems)):
            p = problems[idx]
            p.activate()
            for r, eAe in p.samples:
                if progress() >= 1.0:
                    break
                step += 1
                frac = min(1.0, progress())
                lr = lr0 * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * frac)))
                losses.append(net.train_step(p.op, r, eAe, lr, step))
            if progress() >= 1.0:
                break
        if not losses:
            break
        hist.append(float(np.mean(losses)))
        log(f"[train] epoch {len(hist)}: {step} steps, mean loss {hist[-1]:.4f}, "
            f"{(time.time() - t1) / max(1, step - step0) * 1e3:.1f} ms/step")
    return step, hist


SOLVERS = (("fp64_jacobi", dict(precision="f64")),
           ("mixed_jacobi", dict(precision="mixed")),
           ("mixed_unet", dict(precision="mixed", precond="unet")),
           ("mixed_unet_untrained", dict(precision="mixed", precond="unet")))


def evaluate(seq, op, net, untrained, steps, tol=1e-8):
    """Every held-out step: each solver to the FP64 tolerance (second of two
    runs timed), and the relative residual after 100 FCG iterations with the
    monitor off for the trained and the untrained network."""
    rows = []
    for n in steps:
        phi, uvw = seq.step(n)
        op.assemble(torch.as_tensor(phi, device="cuda").float().contiguous())
        b = op.rhs(*(torch.as_tensor(a, device="cuda") for a in uvw))
        row = {"step": n}
        for name, kw in SOLVERS:
            kw = dict(kw)
            if name == "mixed_unet":
                kw["unet"] = net
            elif name == "mixed_unet_untrained":
                kw["unet"] = untrained
            op.solve(b, tol=tol, **kw)
            _, r = op.solve(b, tol=tol, **kw)
            row[name] = {"iterations": r.iterations, "ms": r.ms, "relres": r.relres, "fallback": r.fallback,
                         "status": r.status}
        for name, nn in (("trained", net), ("untrained", untrained)):
            _, r = op.solve(b, tol=1e-30, precision="mixed", precond="unet", unet=nn, fallback_ratio=2.0,
                            max_iters=100, history=256)
            row[f"relres_after_100_{name}"] = float(r.history[-1])
        # one-step A-norm loss on this held-out step's pairs (r_k, e_k) of the
        # plain solver: the share of the error one step along z leaves
        xs, _ = op.solve(b, tol=1e-10, precision="f64")
        x = torch.zeros_like(b)
        done = 0
        losses = {"trained": [], "untrained": []}
        for k in EVAL_KS:
            if k > done:
                x, _ = op.solve(b, x=x, tol=1e-30, precision="f64", max_iters=k - done, warm_start=True)
                done = k
            rk, _ = op.residual(b, x)
            eAe = float(torch.dot((xs - x).ravel(), rk.ravel()))
            r32 = rk.float().contiguous()
            for name, nn in (("trained", net), ("untrained", untrained)):
                losses[name].append(nn.grad(op, r32, eAe))
        row["step_loss_trained"] = losses["trained"]
        row["step_loss_untrained"] = losses["untrained"]
        rows.append(row)
        log(f"[eval] step {n}: " + ", ".join(
            f"{k} {v['iterations']} its {v['ms']:.1f} ms{' (fallback)' if v['fallback'] else ''}"
            for k, v in row.items() if isinstance(v, dict))
            + f"; after 100 its trained {row['relres_after_100_trained']:.2e} "
              f"untrained {row['relres_after_100_untrained']:.2e}; step loss trained "
              f"{np.mean(row['step_loss_trained']):.3f} untrained {np.mean(row['step_loss_untrained']):.3f}")
    return rows


def summarize(rows):
    out = {}
    for name, _ in SOLVERS:
        its = np.array([r[name]["iterations"] for r in rows], dtype=float)
        ms = np.array([r[name]["ms"] for r in rows], dtype=float)
        out[name] = {"iterations_mean": float(its.mean()), "iterations_median": float(np.median(its)),
                     "ms_mean": float(ms.mean()), "ms_median": float(np.median(ms)),
                     "fallbacks": int(sum(r[name]["fallback"] for r in rows)),
                     "max_relres": float(max(r[name]["relres"] for r in rows)),
                     "all_converged": bool(all(r[name]["status"] == 0 for r in rows))}
    for tag in ("trained", "untrained"):
        v = np.array([r[f"relres_after_100_{tag}"] for r in rows])
        out[f"relres_after_100_{tag}"] = {"geomean": float(np.exp(np.mean(np.log(v)))),
                                          "median": float(np.median(v))}
        sl = np.array([r[f"step_loss_{tag}"] for r in rows])
        out[f"step_loss_{tag}"] = {"mean": float(sl.mean()),
                                   "mean_per_k": {str(k): float(v) for k, v in zip(EVAL_KS, sl.mean(axis=0))}}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--minutes", type=float, default=6.0, help="total training time budget")
    ap.add_argument("--max-steps", type=int, default=0,
                    help="total optimizer steps (replaces the time budget when > 0)")
    ap.add_argument("--rounds", type=int, default=1, help="training phases (the first without on-policy pairs)")
    ap.add_argument("--hull-steps", type=int, default=160)
    ap.add_argument("--stride", type=int, default=1, help="use every stride-th hull time step")
    ap.add_argument("--breaking", type=int, default=0, help="breaking-wave geometry snapshots")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--levels", type=int, default=3)
    ap.add_argument("--eval-steps", default="160-199", help="held-out steps to evaluate (a-b, or empty)")
    ap.add_argument("--init", default=None, help="start from these weights (.npy)")
    ap.add_argument("--resume", default=None,
                    help="continue from a checkpoint written by an earlier run (<out>.state.npz: parameters, Adam "
                         "moments and step count; the learning-rate schedule restarts over the new budget)")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "weights", "unet"))
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    nx, ny, nz = 256, 128, 96
    t0 = time.time()
    seq = fx.C4Sequence(nx, ny, nz)
    _, op_hull = operator_for(seq.xf, seq.yf, seq.zf, seq.bc, seq.psi, seq.theta)
    problems = []
    for n in range(0, args.hull_steps, args.stride):
        phi, uvw = seq.step(n)
        problems.append(build_problem(f"hull_{n}", op_hull, phi, uvw, seq.smooth_field, seed=n))
    if args.breaking > 0:
        wl0 = fx.c3(seed=100, nx=nx, ny=ny, nz=nz)
        _, op_brk = operator_for(wl0.xf, wl0.yf, wl0.zf, wl0.bc, wl0.psi, wl0.theta)
    for q in range(args.breaking):
        wl = fx.c3(seed=100 + q, nx=nx, ny=ny, nz=nz)
        problems.append(build_problem(f"breaking_{100 + q}", op_brk, wl.phi, (wl.u, wl.v, wl.w),
                                      seq.smooth_field, seed=100 + q))
    t_data = time.time() - t0
    net = nfa.UNet(nx, ny, nz, seed=args.seed, levels=args.levels)
    step, hist = 0, []
    if args.init:
        net.set_params(np.load(args.init))
    if args.resume:
        with np.load(args.resume) as ck:       # plain arrays, no pickled objects
            net.load_state({k: ck[k] for k in ("params", "adam_m", "adam_v")})
            step = int(ck["step"])
        log(f"[train] resumed from {args.resume} at step {step}")
    rng = np.random.default_rng(args.seed)
    t1 = time.time()
    per_round = args.minutes / max(1, args.rounds)
    for rnd in range(args.rounds):
        if rnd > 0:
            add_onpolicy(problems, net)
            log(f"[train] round {rnd}: {sum(len(p.samples) for p in problems)} pairs")
        step, h = train(problems, net, per_round, args.lr if rnd == 0 else args.lr * 0.5, step, rng,
                        args.max_steps // max(1, args.rounds))
        hist += h
    t_train = time.time() - t1
    n_pairs = sum(len(p.samples) for p in problems)
    params = net.get_params()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out + ".npy", params)
    np.savez(args.out + ".state.npz", step=np.int64(step), **net.state())
    steps = []
    if args.eval_steps:
        a_, b_ = (int(v) for v in args.eval_steps.split("-"))
        steps = list(range(a_, b_ + 1))
    untrained = nfa.UNet(nx, ny, nz, seed=args.seed, levels=args.levels)
    del problems
    torch.cuda.empty_cache()
    t2 = time.time()
    evals = evaluate(seq, op_hull, net, untrained, steps) if steps else []
    rec = {"levels": args.levels, "grid": [nx, ny, nz], "train_steps": list(range(0, args.hull_steps, args.stride)),
           "pairs_per_step": len(KS) + SYNTH, "pairs": n_pairs,
           "optimizer_steps": step, "rounds": args.rounds, "lr": args.lr, "minutes_budget": args.minutes,
           "max_steps": args.max_steps, "stride": args.stride, "hull_steps": args.hull_steps,
           "breaking": args.breaking, "data_seconds": t_data, "train_seconds": t_train,
           "eval_seconds": time.time() - t2, "epoch_loss": hist, "param_count": int(params.size),
           "eval_summary": summarize(evals) if evals else {}, "eval": evals}
    with open(args.out + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    log(f"[train] wrote {args.out}.npy and .json")
    return 0


if __name__ == "__main__":
    sys.exit(main())
