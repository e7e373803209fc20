#!/usr/bin/env python
"""Throughput benchmark: Newton-solved pairs per second at 512^2 to residual 1e-6.

One step solves a batch of blob-density pairs (8 periodic Gaussian blobs on a 0.1
floor, seeded) of size 512 x 512 with the damped Newton / Strain-GMRES method to
an rms residual of 1e-6, all pairs in one batched call.  Arms: the plain method
(Newton from zero) and the learned start (the warm-start network's guess for every
pair, computed inside the timed region, then Newton from it), each with two ways of
solving the linear equation:
  fast   symbols of the fourth-order differences (the Jacobian of the discrete
         residual) and GMRES on the system scaled by the relative trace of the
         coefficients, GMRES tolerance 2e-1 tightened after hard steps: the same
         fixed point in fewer iterations;
  paper  the paper's spectral symbols, unscaled, GMRES tolerance 1e-2.
`value` is the first method's learned-start throughput; every arm is reported
beside it.  The inputs are resident in device memory before the timed region.
Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--batch B] [--gpus 1] [--init both|zero|learned]
                  [--methods fast,paper]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = "row_c_%d_batch%d_hbm_traffic.md"  # written by paper_1009_6039_amd.rocprof_summary traffic
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "Newton-solved pairs/sec at 512^2 to residual 1e-6; learned-init vs plain"
# linear-solve method -> plan options (symbols of the derivatives, left scaling)
# and GMRES tolerance.  The paper's method runs at its 1e-2 (Section 5.2): at 1e-1 its
# iteration count on some blob pairs depends on FP32 summation order (35 to 330
# Newton steps on one benchmark pair), at 1e-2 it does not.  The fast method runs at
# 2e-1 with adaptive forcing (the direction after a step, other than the first, that
# was halved twice or more is solved 4x tighter): fewer passes in total than at 1e-1,
# and no held-out pair drifts into the boundary of convexity from the zero start
# (with a fixed 2e-1 some do).
METHODS = {"fast": {"symbol": "fd4", "precond": "diag", "gmres_tol": 0.2, "forcing": "adaptive"},
           "fd4": {"symbol": "fd4", "precond": "none", "gmres_tol": 0.1},
           "paper": {"symbol": "spectral", "precond": "none", "gmres_tol": 0.01},
           "spectral-diag": {"symbol": "spectral", "precond": "diag", "gmres_tol": 0.1}}
MAX_NEWTON = 500


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="blobs", choices=("blobs", "mixed"),
                    help="blobs: B pairs of side n (the metric's workload); mixed: B pairs with sides drawn "
                         "from {128, 256, 384, 512} (zero init only)")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=256,
                    help="pairs per batched solve (one step); a larger batch spreads the last, nearly "
                         "empty ticks of the slowest pairs over more pairs")
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--max-active", type=int, default=0,
                    help="continuous batching: at most this many pairs in flight per call, finished "
                         "slots refilled with the batch's pending pairs (0: every pair at once)")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--gmres-tol", type=float, default=None, help="overrides every method's GMRES tolerance")
    ap.add_argument("--damping-policy", default="backtrack")
    ap.add_argument("--methods", default="fast,paper",
                    help="comma list of linear-solve methods (%s); the first is the headline"
                         % ", ".join(sorted(METHODS)))
    ap.add_argument("--profile-class", default="row_c",
                    help="kernel class timed for the roofline: residual, row_a, column, row_c")
    ap.add_argument("--profile-every", type=int, default=1,
                    help="time every k-th launch of that class with HIP events (events add a few "
                         "microseconds of queue time per timed launch; launch durations vary tenfold "
                         "over a solve, so a sampled average can be off by 20%%)")
    ap.add_argument("--init", default="both", choices=("both", "zero", "learned"),
                    help="arms to time; value is the learned arm unless only zero is run")
    ap.add_argument("--weights", default=os.path.join(HERE, "paper_1009_6039_amd", "warmstart_256.npz"))
    ap.add_argument("--tune-cache", default=os.path.join(HERE, "paper_1009_6039_amd", "tune_cache.json"),
                    help="autotuner cache (JSON); 'none' skips the autotuner (default geometries)")
    ap.add_argument("--cpu-pairs", type=int, default=0,
                    help="pairs in the oracle's timed sample (0: one per worker)")
    ap.add_argument("--cpu-workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="single-threaded oracle processes (the host cores used)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the configurations reported beside the headline (single pairs, mixed-size batch, "
                         "2048^2 pair, finite differences, 3-D)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fd-only", action="store_true",
                    help="run only the finite-difference configurations (fd_bicg_256, table1_e1_256) and print them")
    ap.add_argument("--only-3d", action="store_true", help="run only the three-dimensional configuration and print it")
    ap.add_argument("--only-single", action="store_true",
                    help="run only the single-pair configurations (64^2 manufactured, 512^2 blob pair) and print them")
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


def copy_rate(mib=1024, reps=10):
    """GB/s (bytes read + written) of a plain device-to-device copy of mib MiB, timed
    with events over reps copies after one untimed: what a streaming copy reaches on
    this part, a practical ceiling next to the published HBM peak."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    del src, dst
    return 2.0 * n * 4 * reps / (ms * 1e-3) / 1e9


def method_options(name, args):
    o = dict(METHODS[name])
    if args.gmres_tol is not None:
        o["gmres_tol"] = args.gmres_tol
    return o


def load_weights(path):
    """Trained warm-start parameters and their shape (layers, channels, n_net)."""
    d = np.load(path, allow_pickle=False)
    meta = json.loads(str(d["meta"]))
    return d["params"].astype(np.float32), meta


def _oracle_worker(job):
    """One pair in a worker process pinned to one thread: (seconds, psi)."""
    f, g, opts, params, meta = job
    from threadpoolctl import threadpool_limits
    sys.path.insert(0, HERE)
    from oracle import cnn, ma
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        psi0 = None
        if params is not None:
            shaped = cnn.unflatten_params(params, meta["layers"], meta["channels"])
            psi0 = cnn.warm_start(f, g, shaped, meta["n_net"], dilations=meta.get("dilations"))
        psi, _, _ = ma.solve(f, g, psi0=psi0, **opts)
        return os.getpid(), time.perf_counter() - t0, psi


def cpu_baseline(pairs, args, params=None, meta=None):
    """The FP64 oracle on a sample of pairs of the same workload, one single-threaded
    process per host core (the network's start, BF16-emulated, when params are given,
    then the solve).  Returns (psis, pairs/s summed over the workers, workers, CPU seconds)."""
    import multiprocessing as mp
    opts = dict(tau=1.0, tol=args.tol, damping_policy=args.damping_policy, max_newton=MAX_NEWTON,
                **method_options(args.method0, args))
    jobs = [(f, g, opts, params, meta) for f, g in pairs]
    workers = min(len(jobs), args.cpu_workers)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    with mp.get_context("spawn").Pool(workers) as pool:
        out = pool.map(_oracle_worker, jobs, chunksize=1)
    # each process solves its pairs one after another: its rate is pairs / its busy time
    per = {}
    for pid, dt, _ in out:
        per.setdefault(pid, []).append(dt)
    rate = sum(len(v) / sum(v) for v in per.values())
    return [psi for _, _, psi in out], rate, workers, sum(dt for _, dt, _ in out)


def single_pair_configs(args, maot, W, method, cache):
    """The single-pair configurations, each potential compared with the oracle's stored
    solution (tests/golden/c0_c1_reference.npz): the manufactured 64^2 pair with the
    paper's method (spectral symbols, fixed tau = 1, GMRES tolerance 1e-4) to rms
    residual 1e-8, and one 512^2 blob pair to the headline's residual with the paper's
    linear solve and with the headline's (step halving, zero start).  Median of five
    solves after a warm-up."""
    import torch
    ref_path = os.path.join(HERE, "tests", "golden", "c0_c1_reference.npz")
    ref = np.load(ref_path, allow_pickle=False) if os.path.exists(ref_path) else None
    res = {}

    def timed(plan, fd, gd, tol):
        plan.solve(fd, gd, damping=1.0, tol=tol)  # warm-up
        t = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            psi, _, rep = plan.solve(fd, gd, damping=1.0, tol=tol)
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
        return psi.cpu().numpy(), rep, 1e3 * float(np.median(t))

    f, g, _ = W.manufactured(64)
    plan = maot.Plan(n_max=64, batch_capacity=1, damping_policy="fixed", symbol="spectral", gmres_tol=1e-4,
                     max_newton=MAX_NEWTON)
    psi, rep, ms = timed(plan, torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda(), 1e-8)
    plan.close()
    err = None if ref is None else float(np.max(np.abs(psi - ref["c0_psi"])) / np.max(np.abs(ref["c0_psi"])))
    res["c0_manufactured_64"] = {
        "workload": "manufactured 64 x 64 pair (psi* = 0.01 sin sin, g = 1), paper linear solve, fixed tau = 1, "
                    "rms residual 1e-08", "ms_per_solve": round(ms, 3), "status": rep["status"],
        "newton_iters": rep["newton_iters"], "gmres_iters": rep["gmres_iters"], "res_rms": rep["res_rms"],
        "err_vs_oracle": err}
    f, g = W.blobs(512, W.seed_for(1, 0))
    fd, gd = torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda()
    for name in ("paper", method):
        plan = maot.Plan(n_max=512, batch_capacity=1, damping_policy=args.damping_policy, max_newton=MAX_NEWTON,
                         **method_options(name, args))
        if cache:
            plan.autotune(512, 1, cache)
        psi, rep, ms = timed(plan, fd, gd, args.tol)
        plan.close()
        err = None
        if ref is not None:
            st = int(ref["c1_stride"])
            err = float(np.max(np.abs(psi[::st, ::st] - ref["c1_psi"])) / float(ref["c1_psi_absmax"]))
        res["c1_single_512_" + name] = {
            "workload": "one 512 x 512 blob pair, %s linear solve, step halving, zero start, rms residual %.0e"
                        % (name, args.tol), "ms_per_solve": round(ms, 3), "status": rep["status"],
            "newton_iters": rep["newton_iters"], "gmres_iters": rep["gmres_iters"], "res_rms": rep["res_rms"],
            "err_vs_oracle_sampled": err}
    return res


def extra_configs(args, maot, W, method, tuning_cache):
    """The other full-size configurations, timed beside the headline (not part of
    `value`): the single-pair configurations (single_pair_configs), a batch of 256 blob
    pairs with sides drawn from {128, 256, 384, 512} (zero start, the headline's linear
    solve, one batched call), and one 2048^2 smooth-noise pair with the paper's method
    (spectral symbols, fixed tau = 1, GMRES tolerance 1e-2) and with the headline's, its
    potential compared with the oracle's stored solution at every 16th node
    (tests/golden/c2_noise_2048_reference.npz)."""
    import torch
    cache = None if tuning_cache == "none" else tuning_cache
    res = single_pair_configs(args, maot, W, method, cache)
    # mixed-size batch
    sizes = W.mixed_sizes(256, W.seed_for(3, 0))
    pairs = [W.blobs(n, W.seed_for(3, q)) for q, n in enumerate(sizes)]
    fs = [torch.from_numpy(f).cuda() for f, _ in pairs]
    gs = [torch.from_numpy(g).cuda() for _, g in pairs]
    plan = maot.Plan(n_max=512, batch_capacity=256, damping_policy=args.damping_policy, max_newton=MAX_NEWTON,
                     **method_options(method, args))
    for n in sorted(set(sizes)):
        plan.autotune(n, sizes.count(n), cache)
    plan.solve_batched(fs, gs, damping=1.0, tol=args.tol, want_map=True)  # warm-up
    reps_all, t = [], []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, reps = plan.solve_batched(fs, gs, damping=1.0, tol=args.tol, want_map=True)
        torch.cuda.synchronize()
        t.append(time.perf_counter() - t0)
        reps_all += reps
    plan.close()
    bad = sum(r["status"] != 0 or r["res_rms"] > args.tol for r in reps_all)
    res["mixed_256"] = {"workload": "256 blob pairs, sides %s, zero start, %s linear solve, rms residual %.0e"
                                    % (", ".join("%d x %d" % (n, sizes.count(n)) for n in sorted(set(sizes))),
                                       method, args.tol),
                        "value": round((len(reps_all) - bad) / sum(t), 3), "unit": "pairs/s", "unsolved": bad,
                        "ms_per_batch": round(1e3 * sum(t) / len(t), 3), **summary(reps_all)}
    del fs, gs
    # one 2048^2 pair
    N = 2048
    f, g = W.smooth_noise(N, W.seed_for(2, 0))
    fd, gd = torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda()
    ref_path = os.path.join(HERE, "tests", "golden", "c2_noise_2048_reference.npz")
    ref = np.load(ref_path, allow_pickle=False) if os.path.exists(ref_path) else None
    for name, opts in (("paper", dict(damping_policy="fixed", symbol="spectral", gmres_tol=1e-2)),
                       (method, dict(damping_policy=args.damping_policy, **method_options(method, args)))):
        plan = maot.Plan(n_max=N, batch_capacity=1, max_newton=MAX_NEWTON, **opts)
        if cache:
            plan.autotune(N, 1, cache)
        plan.solve(fd, gd, damping=1.0, tol=args.tol)  # warm-up
        t = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            psi, _, rep = plan.solve(fd, gd, damping=1.0, tol=args.tol)
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
        plan.close()
        err = None
        if ref is not None:
            st = int(ref["stride"])
            err = float(np.max(np.abs(psi.cpu().numpy()[::st, ::st] - ref["psi"])) / float(ref["psi_absmax"]))
        res["noise_2048_" + name] = {
            "workload": "one 2048 x 2048 smooth-noise pair (exp(z/2), z filtered white noise, 4 px), %s linear "
                        "solve, rms residual %.0e" % (name, args.tol),
            "ms_per_solve": round(1e3 * float(np.median(t)), 3), "status": rep["status"],
            "newton_iters": rep["newton_iters"], "gmres_iters": rep["gmres_iters"], "res_rms": rep["res_rms"],
            "err_vs_oracle_sampled": err}
    del fd, gd
    res.update(fd_bicg_configs(args, maot, W))
    res.update(configs_3d(args, maot, W))
    return res


def configs_3d(args, maot, W):
    """The method in three dimensions: one 128^3 pair of the Section 5.1 construction
    (u* = cos sin cos / k, g = 1 + 0.3 cos cos cos), fixed tau = 1, GMRES(10) at
    tolerance 1e-4, solved to the headline's residual (median of five solves after a
    warm-up), with the GMRES iterations and the time per iteration."""
    import torch
    N = 128
    f, g, _ = W.e1_example3(N)
    fd, gd = torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda()
    plan = maot.Plan3(n_max=N, damping_policy="fixed", gmres_tol=1e-4)
    plan.solve(fd, gd, damping=1.0, tol=args.tol)  # warm-up
    t = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, rep = plan.solve(fd, gd, damping=1.0, tol=args.tol)
        torch.cuda.synchronize()
        t.append(time.perf_counter() - t0)
    plan.close()
    ms = 1e3 * float(np.median(t))
    return {"e1_3d_128": {
        "workload": "one 128^3 pair of the Section 5.1 construction in 3-D (u* = cos sin cos / 100, g = 1 + 0.3 "
                    "cos cos cos), tau = 1, GMRES(10) tolerance 1e-4, rms residual %.0e" % args.tol,
        "ms_per_solve": round(ms, 3), "status": rep["status"], "newton_iters": rep["newton_iters"],
        "gmres_iters": rep["gmres_iters"], "res_rms": rep["res_rms"],
        "us_per_gmres_iteration": round(1e3 * ms / max(rep["gmres_iters"], 1), 2)}}


def fd_bicg_configs(args, maot, W):
    """The finite-difference linear step of Section 4.1 (nine-point system, BiCG at
    tolerance 1e-1, fixed tau = 1 as in Section 5.1) on the workload the paper runs it on:
    a batch of 64 members of the Section 5.1 example family at 256^2 (seeded parameters),
    solved to the headline's residual, with the event-timed bandwidth of the BiCG matvec
    kernel; and Table 1's row N = 256 on the example itself (20 Newton steps at tolerance
    1e-1, tau = 1) with both linear steps."""
    import torch
    res = {}
    B, N = 64, 256
    pairs = [W.e1_family(N, W.seed_for(6, q))[:2] for q in range(B)]
    fs = [torch.from_numpy(f).cuda() for f, _ in pairs]
    gs = [torch.from_numpy(g).cuda() for _, g in pairs]
    plan = maot.Plan(n_max=N, batch_capacity=B, damping_policy="fixed", max_newton=MAX_NEWTON,
                     linear_solver="fd_bicg", gmres_tol=0.1)
    plan.solve_batched(fs, gs, damping=1.0, tol=args.tol)  # warm-up
    torch.cuda.synchronize()
    plan.profile("bicg_matvec", 4)  # every 4th matvec launch timed with events
    t0 = time.perf_counter()
    _, _, reps = plan.solve_batched(fs, gs, damping=1.0, tol=args.tol)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile("none")
    plan.close()
    bad = sum(r["status"] != 0 or r["res_rms"] > args.tol for r in reps)
    ach = prof["bytes"] / (prof["ms"] * 1e-3) / 1e9 if prof["ms"] > 0 else 0.0
    res["fd_bicg_256"] = {
        "workload": "64 pairs 256 x 256 of the Section 5.1 example family (u* = cos sin / k, k in [80, 200]; "
                    "g = 1 + alpha cos cos, alpha in [0.1, 0.5], rho in {1, 2, 3}), zero start, tau = 1, "
                    "finite-difference step with BiCG (tolerance 1e-1), rms residual %.0e" % args.tol,
        "value": round((B - bad) / el, 3), "unit": "pairs/s", "unsolved": bad, "ms_per_batch": round(1e3 * el, 3),
        "bicg_iters_per_newton": round(float(np.sum([r["gmres_iters"] for r in reps]) /
                                             max(1, np.sum([r["newton_iters"] for r in reps]))), 2),
        **summary(reps),
        "roofline_matvec": {"bound": "hbm", "kernel": "k_bicg_matvec<64>", "achieved": round(ach, 1),
                            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                            "launches": prof["launches"], "timed_every": 4,
                            "avg_launch_us": round(1e3 * prof["ms"] / max(prof["launches"], 1), 3),
                            "bytes_per_launch": round(prof["bytes"] / max(prof["launches"], 1))}}
    del fs, gs
    # Table 1, row N = 256: 20 Newton steps at tolerance 1e-1 on the Section 5.1 example
    f, g, _ = W.e1_example(N)
    fd, gd = torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda()
    row = {"workload": "Section 5.1 example 256 x 256 (u* = 0.01 cos sin, g = 1 + 0.3 cos cos), 20 Newton "
                       "steps, tau = 1, linear tolerance 1e-1 (Table 1's setting)"}
    for ls in ("strain_gmres", "fd_bicg"):
        plan = maot.Plan(n_max=N, batch_capacity=1, linear_solver=ls, gmres_tol=0.1, max_newton=20)
        plan.solve(fd, gd, damping=1.0, tol=1e-14)  # warm-up
        t = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, rep = plan.solve(fd, gd, damping=1.0, tol=1e-14)
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
        plan.close()
        row[ls] = {"ms_20_newton": round(1e3 * float(np.median(t)), 3), "newton_iters": rep["newton_iters"],
                   "inner_iters_per_newton": round(rep["gmres_iters"] / max(rep["newton_iters"], 1), 2),
                   "res_rms": rep["res_rms"]}
    res["table1_e1_256"] = row
    return res


def summary(reps):
    return {"newton_iters_mean": float(np.mean([r["newton_iters"] for r in reps])),
            "gmres_iters_mean": float(np.mean([r["gmres_iters"] for r in reps])),
            "backtracks_mean": float(np.mean([r["backtracks"] for r in reps])),
            "warm_accepted": int(sum(r["warm_steps"] for r in reps)),
            "res_rms_max": float(max(r["res_rms"] for r in reps))}


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this solver build runs on a single device "
              "(batches of pairs would shard across GPUs without communication)",
              file=sys.stderr)
        sys.exit(2)
    if args.fd_only or args.only_3d or args.only_single:
        from paper_1009_6039_amd import maot
        from paper_1009_6039_amd import workloads as W
        if args.fd_only:
            out = fd_bicg_configs(args, maot, W)
        elif args.only_3d:
            out = configs_3d(args, maot, W)
        else:
            out = single_pair_configs(args, maot, W, args.methods.split(",")[0],
                                      args.tune_cache if args.tune_cache != "none" else None)
        print(json.dumps(out), flush=True)
        return
    import torch
    from paper_1009_6039_amd import maot
    from paper_1009_6039_amd.rocprof_summary import read_traffic_record
    from paper_1009_6039_amd import workloads as W

    B = args.batch
    if args.workload == "mixed":
        if args.init != "zero":
            args.init = "zero"  # the network takes sides 256 and 512 only
        sizes = W.mixed_sizes(B, W.seed_for(3, 0))
        seeds = [W.seed_for(3, q) for q in range(B)]
    else:
        sizes = [args.n] * B
        seeds = [W.seed_for(1, q) for q in range(B)]
    N = max(sizes)
    host_pairs = [W.blobs(n, s) for n, s in zip(sizes, seeds)]
    fs = [torch.from_numpy(f).cuda() for f, _ in host_pairs]
    gs = [torch.from_numpy(g).cuda() for _, g in host_pairs]
    symbols = args.methods.split(",")
    for sym in symbols:
        if sym not in METHODS:
            raise SystemExit("unknown method %r" % sym)
    args.method0 = symbols[0]
    plans = {sym: maot.Plan(n_max=N, batch_capacity=args.max_active or B, damping_policy=args.damping_policy,
                            max_newton=MAX_NEWTON, max_active=args.max_active, **method_options(sym, args))
             for sym in symbols}

    tuning = None
    if args.tune_cache != "none":  # launch geometry chosen before the timed region, per size class
        for sym in symbols:
            for n in sorted(set(sizes)):
                t = plans[sym].autotune(n, sizes.count(n), args.tune_cache)
                tuning = t if n == N else tuning
        print("tuning %s" % json.dumps(tuning), file=sys.stderr, flush=True)

    net, params, meta = None, None, None
    if args.init != "zero":
        params, meta = load_weights(args.weights)
        net = maot.WarmStartNet(layers=meta["layers"], channels=meta["channels"], n_net=meta["n_net"],
                                max_batch=B, dilations=meta.get("dilations"))
        net.set_params(params)

    def step(plan, learned, strict):
        """One batched solve; an unsolved pair aborts the headline arm (strict) and is
        counted, not credited, in the others."""
        psi0 = net.warm_start(fs, gs) if learned else None
        psis, _, reps = plan.solve_batched(fs, gs, damping=1.0, tol=args.tol, psi0s=psi0, want_map=True)
        bad = [r for r in reps if r["status"] != 0 or r["res_rms"] > args.tol]
        if bad and strict:
            raise RuntimeError("unsolved pairs: %d (first: %s)" % (len(bad), bad[0]))
        return psis, reps, len(bad)

    def timed(plan, learned, profile, strict):
        for _ in range(args.warmup):
            step(plan, learned, strict)
        torch.cuda.synchronize()
        if profile:
            plan.profile(args.profile_class, args.profile_every)
        unsolved = 0
        t0 = time.perf_counter()
        for _ in range(args.steps):
            psis, reps, nbad = step(plan, learned, strict)
            unsolved += nbad
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        prof = plan.profile_read() if profile else None
        plan.profile("none")
        return elapsed, psis, reps, prof, unsolved

    inits = {"both": ("zero", "learned"), "zero": ("zero",), "learned": ("learned",)}[args.init]
    head = (symbols[0], inits[-1])
    arms = {}
    for sym in reversed(symbols):  # the headline arm runs last: its launches end the kernel trace
        for init in inits:
            arms[(sym, init)] = timed(plans[sym], init == "learned", (sym, init) == head, (sym, init) == head)
            el, _, _, _, nbad = arms[(sym, init)]
            print("arm %s/%s: %.3f pairs/s%s" % (sym, init, (B * args.steps - nbad) / el,
                                                 " (%d unsolved)" % nbad if nbad else ""), file=sys.stderr, flush=True)
    elapsed, psis, reps, prof, _ = arms[head]

    pairs = B * args.steps
    value = pairs / elapsed
    achieved = prof["bytes"] / (prof["ms"] * 1e-3) / 1e9 if prof["ms"] > 0 else 0.0
    init_txt = ("learned start (8-layer 32-channel %s3x3 network at 256^2, checked)"
                % ("dilated " if meta and any(d > 1 for d in meta.get("dilations", [1])) else "")
                if head[1] == "learned" else "zero init")
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
        "config": {"workload": ("blob-density pairs %dx%d (8 periodic Gaussian blobs, 0.1 floor), "
                                "batch %d per step, rms residual %.0e, %s, %s linear solve"
                                % (N, N, B, args.tol, init_txt, head[0])) if args.workload == "blobs" else
                               ("mixed-size blob-density pairs, sides drawn from {128, 256, 384, 512} "
                                "(%s), batch %d per step, rms residual %.0e, %s, %s linear solve"
                                % (", ".join("%d x %d" % (n, sizes.count(n)) for n in sorted(set(sizes))), B,
                                   args.tol, init_txt, head[0])),
                   "n": N if args.workload == "blobs" else sorted(set(sizes)), "batch": B, "tol": args.tol, "damping_policy": args.damping_policy,
                   "gmres_m": 10, "init": head[1], "method": head[0], "max_active": args.max_active,
                   **method_options(head[0], args)},
    }
    out.update(summary(reps))
    if tuning is not None:
        out["tuning"] = {"n": N, "variant_row_a_column_row_c_residual": tuning["variant"],
                         "from_cache": tuning["from_cache"],
                         "us_per_launch": [round(x, 2) for x in tuning["us"]],
                         "us_per_launch_default": [round(x, 2) for x in tuning["us_default"]]}
    out["arms"] = {}
    for (sym, init), (el, _, rp, _, nbad) in arms.items():
        out["arms"]["%s/%s" % (sym, init)] = dict(value=round((pairs - nbad) / el, 3), unsolved=nbad,
                                                  ms_per_step=round(1e3 * el / args.steps, 3), **summary(rp))
    for sym in symbols:
        if (sym, "zero") in arms and (sym, "learned") in arms:
            out["learned_vs_plain_" + sym] = round(out["arms"][sym + "/learned"]["value"] /
                                                   out["arms"][sym + "/zero"]["value"], 4)
    cls = {"row_a": 0, "column": 1, "row_c": 2, "residual": 3}[args.profile_class]
    var = plans[head[0]].get_tuning(N)[cls]
    # the kernel as rocprofv3 names it
    kname = maot.pass_kernel_name(args.profile_class, N, var) if args.workload == "blobs" else None
    rec = read_traffic_record(os.path.join(HERE, "profiles", TRAFFIC_FILE % (N, B)), kname) if kname else None
    if rec and rec.get("variant") != var:
        rec = None  # counters taken with another launch geometry
    bpl = prof["all_bytes"] / max(prof["all_launches"], 1)  # over every launch, as the counters are
    if rec and abs(rec.get("algorithmic_bytes_per_launch", 0.0) - bpl) > 1e-3 * bpl:
        rec = None  # counters taken on another launch mix (workload, start or iteration path)
    out["roofline"] = {"bound": "hbm", "kernel": args.profile_class, "achieved": round(achieved, 1),
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                       "traffic": round(rec["traffic_bytes_per_launch"]) if rec else None,
                       "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled; null unless the "
                                       "kernel sources, geometry and launch mix are the profiled ones)",
                       "launches": prof["launches"], "timed_every": args.profile_every,
                       "launches_all": prof["all_launches"],
                       "avg_launch_us": round(1e3 * prof["ms"] / max(prof["launches"], 1), 3),
                       "bytes_per_launch": round(prof["bytes"] / max(prof["launches"], 1)),
                       "bytes_per_launch_all": round(bpl),
                       "algorithmic_bytes_timed": prof["bytes"]}
    cr = copy_rate()  # after the timed region
    out["roofline"]["copy_achieved"] = round(cr, 1)
    out["roofline"]["frac_of_copy"] = round(achieved / cr, 4)
    if not args.no_configs and args.workload == "blobs":
        out["configs"] = extra_configs(args, maot, W, head[0], tuning_cache=args.tune_cache)
    if not args.no_cpu_baseline:
        idx = list(range(min(args.cpu_pairs or args.cpu_workers, B)))  # the front of the batch
        k = len(idx)
        refs, rate, workers, busy = cpu_baseline([host_pairs[q] for q in idx], args,
                                                 params if head[1] == "learned" else None, meta)
        err = max(float(np.max(np.abs(psis[q].cpu().numpy() - refs[i])) / np.max(np.abs(refs[i])))
                  for i, q in enumerate(idx))
        out["cpu_baseline"] = {"value": round(rate, 5), "unit": "pairs/s", "cores": workers, "kind": "oracle",
                               "sample": "%d pairs (seeds %s..%s, sides %s) of the same workload (%s, %s linear "
                                         "solve), FP64 NumPy oracle, %d single-threaded processes, %.1f s of "
                                         "CPU time in all" % (k, seeds[idx[0]], seeds[idx[-1]],
                                                              ",".join(sorted({str(sizes[q]) for q in idx})),
                                                              init_txt, head[0], workers, busy)}
        out["err_vs_oracle_max"] = err
        out["err_vs_oracle_pairs"] = k
    print(json.dumps(out), flush=True)
    if net is not None:
        net.close()
    for plan in plans.values():
        plan.close()


if __name__ == "__main__":
    main()
