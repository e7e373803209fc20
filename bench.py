#!/usr/bin/env python
"""Throughput benchmark: Newton-solved pairs per second at 512^2 to residual 1e-6.

One step solves a batch of blob-density pairs (8 periodic Gaussian blobs on a 0.1
floor, seeded) of size 512 x 512 with the damped Newton / Strain-GMRES method to
an rms residual of 1e-6, all pairs in one batched call.  The inputs are resident
in device memory before the timed region.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--batch B] [--gpus 1]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "Newton-solved pairs/sec at 512^2 to residual 1e-6; learned-init vs plain"


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--gmres-tol", type=float, default=0.1)
    ap.add_argument("--damping-policy", default="backtrack")
    ap.add_argument("--symbol", default="spectral", help="spectral (the paper) or fd4 (option)")
    ap.add_argument("--profile-class", default="row_c",
                    help="kernel class timed for the roofline: residual, row_a, column, row_c")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB mebibytes (scales HBM byte counters)")
    return ap.parse_args()


def copy_probe(mib):
    """A plain copy kernel of known size: reads and writes mib MiB once."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4}), flush=True)


def cpu_baseline(f, g, args):
    """The FP64 oracle on one pair of the same workload, pinned to one thread."""
    from threadpoolctl import threadpool_limits
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from oracle import ma
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        psi, _, rep = ma.solve(f, g, tau=1.0, tol=args.tol, damping_policy=args.damping_policy,
                               gmres_tol=args.gmres_tol, max_newton=300, symbol=args.symbol)
        dt = time.perf_counter() - t0
    return psi, rep, dt


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this solver build runs on a single device "
              "(batches of pairs would shard across GPUs without communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1009_6039_amd import maot
    from paper_1009_6039_amd import workloads as W

    N, B = args.n, args.batch
    seeds = [W.seed_for(1, q) for q in range(B)]
    host_pairs = [W.blobs(N, s) for s in seeds]
    fs = [torch.from_numpy(f).cuda() for f, _ in host_pairs]
    gs = [torch.from_numpy(g).cuda() for _, g in host_pairs]
    plan = maot.Plan(n_max=N, batch_capacity=B, damping_policy=args.damping_policy,
                     gmres_tol=args.gmres_tol, max_newton=300, symbol=args.symbol)

    def step():
        psis, _, reps = plan.solve_batched(fs, gs, damping=1.0, tol=args.tol)
        bad = [r for r in reps if r["status"] != 0 or r["res_rms"] > args.tol]
        if bad:
            raise RuntimeError("unsolved pairs: %d (first: %s)" % (len(bad), bad[0]))
        return psis, reps

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.profile(args.profile_class)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        psis, reps = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile("none")

    pairs = B * args.steps
    value = pairs / elapsed
    achieved = prof["bytes"] / (prof["ms"] * 1e-3) / 1e9 if prof["ms"] > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": "blob-density pairs %dx%d (8 periodic Gaussian blobs, 0.1 floor), "
                               "batch %d per step, rms residual %.0e, plain zero init" % (N, N, B, args.tol),
                   "n": N, "batch": B, "tol": args.tol, "damping_policy": args.damping_policy,
                   "gmres_tol": args.gmres_tol, "gmres_m": 10, "init": "zero", "symbol": args.symbol},
        "newton_iters_mean": float(np.mean([r["newton_iters"] for r in reps])),
        "gmres_iters_mean": float(np.mean([r["gmres_iters"] for r in reps])),
        "backtracks_mean": float(np.mean([r["backtracks"] for r in reps])),
        "res_rms_max": float(max(r["res_rms"] for r in reps)),
        "roofline": {"bound": "hbm", "kernel": args.profile_class, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "launches": prof["launches"],
                     "avg_launch_us": round(1e3 * prof["ms"] / max(prof["launches"], 1), 3),
                     "bytes_per_launch": round(prof["bytes"] / max(prof["launches"], 1)),
                     "algorithmic_bytes_total": prof["bytes"]},
    }
    if not args.no_cpu_baseline:
        f0, g0 = host_pairs[0]
        psi_ref, rep_ref, dt = cpu_baseline(f0, g0, args)
        err = float(np.max(np.abs(psis[0].cpu().numpy() - psi_ref)) / np.max(np.abs(psi_ref)))
        out["cpu_baseline"] = {"value": round(1.0 / dt, 5), "unit": "pairs/s", "cores": 1, "kind": "oracle",
                               "sample": "1 pair (seed %d) of the same workload, FP64 NumPy oracle, "
                                         "one thread, %.1f s" % (seeds[0], dt)}
        out["err_vs_oracle_pair0"] = err
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
