"""Learned interface correction: training-set construction, training and
evaluation drivers around the library's C ABI (lic_* entry points).

Every numerical step runs in the library's kernels (problem setup, global
ILU0 targets, corrected and adjoint applies, MLP forward/backward, Adam);
this module only generates the seeded inputs, moves them to the device and
sequences the calls.

Training set: 48^3 log-normal problems (sigma ~ U[1,3]), seeds 1000..,
explicit 16^3 subdomains, 16 N(0,1) probes each; regression target: the
global ILU0 apply of the probes.

usage:
    python -m paper_2508_04917_amd.lic train [--problems 256] [--epochs E] [--out FILE]
    python -m paper_2508_04917_amd.lic eval  [--params FILE] [--n 128] [--seeds 2000 2001 ...]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import ddilu as dd
from .solver import DDSolver

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PARAMS = os.path.join(HERE, "lic_params.npz")


def _log(msg):
    print(f"[lic] {msg}", file=sys.stderr, flush=True)


def _cuda(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda").to(dtype)


def prepare_problem(p, sub, nq, probe_seed):
    """Set up one training problem: DD factors, faces, global ILU0, probes and
    their regression targets (all on the device)."""
    from problems import probe_vectors
    s = DDSolver.from_problem(p, sub=sub)
    dd.lic_setup(s.h)
    dd.dd_global_factor(s.h)
    R = _cuda(probe_vectors(probe_seed, nq, p.n * 3), torch.float64)
    Zs, den = dd.lic_targets(s.h, R)
    return s, R, Zs, den


def train(nprob=256, epochs=10, nq=16, n=48, sub=(16, 16, 16), lr=1e-3, init_seed=0, order_seed=1,
          first_seed=1000, nval=4, first_val_seed=1900, out=None, lr_final=None):
    """Adam over the training problems, one step per problem, epochs in a
    seeded order; the learning rate decays geometrically from lr to lr_final
    over the epochs (constant when lr_final is None)."""
    from problems import lic_init_params, training_order, training_problem
    probs = []
    t0 = time.time()
    for k in range(nprob):
        seed = first_seed + k
        p = training_problem(seed, n)
        probs.append(prepare_problem(p, sub, nq, seed))
        if (k + 1) % 16 == 0 or k + 1 == nprob:
            _log(f"prepared {k + 1}/{nprob} problems ({time.time() - t0:.1f}s)")
    vals = [prepare_problem(training_problem(first_val_seed + k, n), sub, nq, first_val_seed + k)
            for k in range(nval)]

    def val_loss(params):
        if not vals:
            return float("nan")
        return float(np.mean([dd.lic_loss_grad(q[0].h, params, q[1], q[2], q[3])[0].item() for q in vals]))

    params = _cuda(lic_init_params(init_seed), torch.float32)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    order = training_order(order_seed, epochs, nprob)
    hist, vhist, meta = [], [], {}
    t1 = time.time()
    for ep in range(epochs):
        lr_ep = lr if lr_final is None or epochs == 1 else lr * (lr_final / lr) ** (ep / (epochs - 1))
        h = dd.lic_train([q[0].h for q in probs], [q[1] for q in probs], [q[2] for q in probs],
                         [q[3] for q in probs], params, m, v, 1, order[ep:ep + 1], lr=lr_ep, step0=ep * nprob)
        hist.append(float(h[0]))
        vhist.append(val_loss(params))
        _log(f"epoch {ep + 1}/{epochs}: mean loss {hist[-1]:.4f}, held-out {vhist[-1]:.4f} "
             f"({time.time() - t1:.1f}s)")
        meta = {"nprob": nprob, "epochs": ep + 1, "nq": nq, "grid": n, "subdomain": list(sub), "lr": lr,
                "lr_final": lr_final,
                "init_seed": init_seed, "order_seed": order_seed, "first_seed": first_seed,
                "loss_history": hist, "val_seeds": [first_val_seed, first_val_seed + nval - 1],
                "val_loss_history": vhist, "train_seconds": time.time() - t1}
        if out:  # checkpoint after every epoch
            save_params(out, params.cpu().numpy(), meta)
    for q in probs + vals:
        q[0].close()
    return params.cpu().numpy(), meta


def save_params(path, params, meta):
    np.savez(path, params=params.astype(np.float32), meta=json.dumps(meta))


def load_params(path=DEFAULT_PARAMS):
    with np.load(path, allow_pickle=False) as f:
        return f["params"].astype(np.float32), json.loads(str(f["meta"]))


def heldout_loss(params, p, sub, nq=8, probe_seed=99):
    """Mean loss of the correction on probes of an unseen problem."""
    s, R, Zs, den = prepare_problem(p, sub, nq, probe_seed)
    loss, _ = dd.lic_loss_grad(s.h, _cuda(params, torch.float32), R, Zs, den)
    out = float(loss.item())
    s.close()
    return out


def evaluate(params, p, sub=(0, 0, 0), rtol=1e-8, maxit=5000, with_global=True):
    """BiCGSTAB iterations and solve times: plain DD-ILU0 (FP64 and mixed),
    learned correction (FP64 and mixed), and global ILU0 (FP64)."""
    s = DDSolver.from_problem(p, sub=sub)
    dd.lic_setup(s.h)
    b = _cuda(p.b, torch.float64)
    out = {"subdomain": [s.info["sx"], s.info["sy"], s.info["sz"]]}
    P = _cuda(params, torch.float32)
    for name, prec, learned in (("plain_fp64", dd.DD_FP64, False), ("plain_mixed", dd.DD_MIXED, False),
                                ("learned_fp64", dd.DD_FP64, True), ("learned_mixed", dd.DD_MIXED, True)):
        s.set_precision(prec)
        dd.lic_set_params(s.h, P if learned else None)
        # a learned solve that fails is repeated with plain DD-ILU0 by the
        # library itself (dd_set_lic_fallback, on by default)
        x, info = s.solve(b, rtol=rtol, maxit=maxit)
        out[name] = {k: info[k] for k in ("iters", "status", "solve_seconds", "rel_res_true")}
        out[name]["fallback"] = bool(info["fallback"])
    dd.lic_set_params(s.h, None)
    s.set_precision(dd.DD_FP64)
    if with_global:
        dd.dd_global_factor(s.h)
        dd.dd_set_preconditioner(s.h, 1)
        x, info = s.solve(b, rtol=rtol, maxit=maxit)
        dd.dd_set_preconditioner(s.h, 0)
        out["global_fp64"] = {k: info[k] for k in ("iters", "status", "solve_seconds", "rel_res_true")}
    s.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sp = ap.add_subparsers(dest="cmd", required=True)
    t = sp.add_parser("train")
    t.add_argument("--problems", type=int, default=256)
    t.add_argument("--epochs", type=int, default=10)
    t.add_argument("--probes", type=int, default=16)
    t.add_argument("--grid", type=int, default=48)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--lr-final", type=float, default=None)
    t.add_argument("--val", type=int, default=4)
    t.add_argument("--out", default=DEFAULT_PARAMS)
    e = sp.add_parser("eval")
    e.add_argument("--params", default=DEFAULT_PARAMS)
    e.add_argument("--n", type=int, default=128)
    e.add_argument("--seeds", type=int, nargs="+", default=[2000, 2001, 2002, 2003])
    e.add_argument("--sigma", type=float, default=2.0)
    e.add_argument("--no-global", action="store_true")
    e.add_argument("--workload", default=None, help="a named workload (problems.WORKLOADS) instead of --n/--seeds")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    if args.cmd == "train":
        params, meta = train(nprob=args.problems, epochs=args.epochs, nq=args.probes, n=args.grid, lr=args.lr,
                             nval=args.val, out=args.out, lr_final=args.lr_final)
        print(json.dumps(meta))
    else:
        from problems import lognormal_problem, make_workload
        params, meta = load_params(args.params)
        if args.workload:
            res = evaluate(params, make_workload(args.workload), with_global=not args.no_global)
            res["workload"] = args.workload
            print(json.dumps(res), flush=True)
            return
        for seed in args.seeds:
            p = lognormal_problem(args.n, args.n, args.n, seed=seed, sigma=args.sigma)
            res = evaluate(params, p, with_global=not args.no_global)
            res["seed"] = seed
            print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
