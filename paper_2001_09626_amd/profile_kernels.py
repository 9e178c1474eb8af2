"""Run one operator of the hot path repeatedly on a workload, for profilers.

    python -m paper_2001_09626_amd.profile_kernels --workload c2 --op stiffness --reps 5

After the operator launches it copies a buffer of --copy-bytes with a plain
device copy, whose hardware byte counters give the scale of the counters
read for the operator's kernels.
"""
from __future__ import annotations

import argparse
import sys

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--op", default="stiffness")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--fd", default="fp64")
    ap.add_argument("--precond", default="fd", help="local solvers: fd (parametric) or geo (geometry inclusion)")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    args = ap.parse_args()
    import torch
    import workloads as W
    from paper_2001_09626_amd import Solver
    make = {"c1": W.make_c1, "c2": W.make_c2, "c3": W.make_c3, "c4": W.make_c4, "c5": W.make_c5}[args.workload]
    prob = make(seed=0)
    s = Solver(prob, fd_precision=args.fd, precond=args.precond)
    n_in = s.n_dof + s.n_c if args.op in ("prec", "saddle") else (s.n_c if args.op in ("P_chi", "P_S", "Bt") else s.n_dof)
    x = torch.from_numpy(np.random.default_rng(0).standard_normal(n_in)).cuda()
    for i in range(args.reps):
        if args.op == "fd":
            s.apply_fd(x)
        elif args.op == "solve":
            s.solve()
        else:
            s.apply(args.op, x)
        torch.cuda.synchronize()
        print(f"[profile] {args.op} launch {i} done", file=sys.stderr, flush=True)
    n = args.copy_bytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for i in range(args.reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"[profile] copied {args.reps} x {args.copy_bytes} bytes", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
