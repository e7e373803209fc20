"""Trains the warm-start network on pairs the GPU solver produces.

Pipeline (every numerical step runs in libmaot.so kernels; torch only holds device
memory and gathers minibatches):
  1. blob-density pairs at n_net x n_net (seeds workloads.seed_for(4, q), disjoint
     from the held-out pairs seed_for(5, q) and the benchmark's seed_for(1, q)), drawn
     on the host by the shared input generator;
  2. solved on the GPU to rms residual 1e-8 (step-halving damping, fourth-order
     symbols and the diagonally scaled GMRES system: the same fixed point, fewer
     iterations);
  3. network input (log f, log g of the mean-one densities) in BF16 and target = the fourth-order
     difference Laplacian of the solution minus log f + log g (what the linearised
     equation misses), both kept on the device;
  4. Adam on the MSE loss (cosine learning-rate decay), seeded shuffles, a held-out
     split for the validation loss;
  5. an evaluation: Newton iterations from zero and from the learned start on
     held-out pairs.

  python -m paper_1009_6039_amd.train_warmstart --pairs 20000 \
      --out paper_1009_6039_amd/warmstart_256.npz
"""

import argparse
import json
import math
import multiprocessing as mp
import time

import numpy as np

from . import workloads as W

TRAIN_CONFIG = 4  # seed_for(4, q): training pairs; the benchmark uses seed_for(1, q)


def init_params(layers, channels, seed):
    """He-normal weights (the output layer scaled by 0.1), zero biases; flat FP32."""
    rng = np.random.default_rng(seed)
    chans = [2] + [channels] * (layers - 1) + [1]
    out = []
    for l in range(layers):
        ci, co = chans[l], chans[l + 1]
        w = rng.standard_normal((co, ci, 3, 3)) * math.sqrt(2.0 / (9 * ci))
        if l == layers - 1:
            w *= 0.1
        out += [w.ravel(), np.zeros(co)]
    return np.concatenate(out).astype(np.float32)


def _gen_chunk(args):
    q0, b, n = args
    return np.stack([np.stack(W.blobs(n, W.seed_for(TRAIN_CONFIG, q0 + k))) for k in range(b)])


def generate(maot, net, npairs, n, chunk=128, workers=16, tol=1e-8, log=print):
    import torch
    X = torch.empty((npairs, n, n, 8), dtype=torch.bfloat16, device="cuda")
    T = torch.empty((npairs, n, n), dtype=torch.float32, device="cuda")
    plan = maot.Plan(n_max=n, batch_capacity=chunk, damping_policy="backtrack", gmres_tol=0.1,
                     max_newton=300, symbol="fd4", precond="diag")
    t0 = time.time()
    newton = []
    ok = np.zeros(npairs, dtype=bool)
    jobs = [(q0, min(chunk, npairs - q0), n) for q0 in range(0, npairs, chunk)]
    with mp.get_context("spawn").Pool(workers) as pool:
        for (q0, b, _), arr in zip(jobs, pool.imap(_gen_chunk, jobs)):
            fg = torch.from_numpy(arr).cuda()
            f, g = fg[:, 0].contiguous(), fg[:, 1].contiguous()
            psis, _, reps = plan.solve_batched(list(f.unbind(0)), list(g.unbind(0)), damping=1.0, tol=tol)
            ok[q0:q0 + b] = [r["status"] == 0 for r in reps]
            newton += [r["newton_iters"] for r in reps]
            X[q0:q0 + b] = net.prepare_input(f, g)
            T[q0:q0 + b] = net.target(torch.stack(psis), f, g)
            if (q0 // chunk) % 20 == 0:
                log("generate: %d/%d pairs, %.1f s" % (q0 + b, npairs, time.time() - t0))
    plan.close()
    torch.cuda.synchronize()
    return X, T, ok, {"pairs": npairs, "unsolved": int(np.sum(~ok)), "newton_mean": float(np.mean(newton)),
                      "seconds": time.time() - t0}


def train(net, X, T, ok, epochs, batch, lr0, val_frac=0.05, seed=0, log=print):
    """Pairs the solver did not solve (ok False) are left out."""
    import torch
    g = torch.Generator().manual_seed(seed)
    valid = torch.from_numpy(np.flatnonzero(ok))
    npairs = len(valid)
    perm = valid[torch.randperm(npairs, generator=g)]
    n_val = max(batch, int(npairs * val_frac)) // batch * batch
    val_idx, tr_idx = perm[:n_val].cuda(), perm[n_val:]
    steps_per_epoch = len(tr_idx) // batch
    total = epochs * steps_per_epoch
    step = 0
    hist = []
    t0 = time.time()

    def val_loss():
        return float(np.mean([net.gradients(X[val_idx[s:s + batch]], T[val_idx[s:s + batch]])[1]
                              for s in range(0, n_val, batch)]))

    log("epoch 0: val %.4e" % val_loss())
    for ep in range(epochs):
        order = tr_idx[torch.randperm(len(tr_idx), generator=g)].cuda()
        for s in range(steps_per_epoch):
            idx = order[s * batch:(s + 1) * batch]
            lr = 1e-5 + 0.5 * (lr0 - 1e-5) * (1 + math.cos(math.pi * step / total))
            net.train_step(X[idx], T[idx], lr)
            step += 1
        tl = net.gradients(X[order[:batch]], T[order[:batch]])[1]
        hist.append({"epoch": ep + 1, "train_loss": tl, "val_loss": val_loss(), "seconds": time.time() - t0})
        log("epoch %d: train %.4e  val %.4e  (%.1f s)" % (ep + 1, tl, hist[-1]["val_loss"], time.time() - t0))
    return hist


# the two ways of solving the linear equation that bench.py times
METHODS = (("paper", {"symbol": "spectral", "gmres_tol": 0.01}),
           ("fast", {"symbol": "fd4", "precond": "diag", "gmres_tol": 0.2, "forcing": "adaptive"}))


def evaluate(maot, net, n, count=64, log=print):
    """Newton iterations and wall time on held-out pairs from zero, from the linearised
    start (the network's output set to zero) and from the learned start, for the
    paper's linear solve and the fast one."""
    import torch
    pairs = [W.blobs(n, W.seed_for(TRAIN_CONFIG + 1, q)) for q in range(count)]
    f = [torch.from_numpy(a).cuda() for a, _ in pairs]
    g = [torch.from_numpy(b).cuda() for _, b in pairs]
    lin = maot.WarmStartNet(layers=net.layers, channels=net.channels, n_net=net.n_net, max_batch=net.max_batch,
                            dilations=net.dilations)
    lin.set_params(np.zeros(lin.count, dtype=np.float32))
    out = {}
    for method, opts in METHODS:
        plan = maot.Plan(n_max=n, batch_capacity=count, damping_policy="backtrack", max_newton=500, **opts)
        plan.autotune(n, count)
        for arm, start in (("zero", None), ("linearised", lin), ("learned", net)):
            for rep_i in range(2):  # the first run of an arm warms up
                torch.cuda.synchronize()
                t0 = time.time()
                psi0 = start.warm_start(f, g) if start is not None else None
                _, _, reps = plan.solve_batched(f, g, damping=1.0, tol=1e-6, psi0s=psi0)
                torch.cuda.synchronize()
            key = "%s/%s" % (method, arm)
            out[key] = {"seconds": time.time() - t0,
                        "newton_mean": float(np.mean([r["newton_iters"] for r in reps])),
                        "gmres_mean": float(np.mean([r["gmres_iters"] for r in reps])),
                        "warm_accepted": int(sum(r["warm_steps"] for r in reps)),
                        "unsolved": int(sum(r["status"] != 0 for r in reps)),
                        "unsolved_pairs": [[q, int(r["status"]), int(r["newton_iters"]), float(r["res_rms"])]
                                           for q, r in enumerate(reps) if r["status"] != 0]}
            log("eval n=%d pairs=%d %s: %s" % (n, count, key, json.dumps(out[key])))
        plan.close()
    lin.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=32)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--layers", type=int, default=8)
    ap.add_argument("--channels", type=int, default=32)
    ap.add_argument("--dilations", default="1,2,4,8,16,16,16,1",
                    help="per-layer dilation of the 3x3 taps (comma list, one per layer)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", help="where to save the trained parameters (npz)")
    ap.add_argument("--eval-only", metavar="NPZ", help="evaluate saved parameters instead of training")
    ap.add_argument("--eval-pairs", default="256,64", help="held-out pairs at n_net and at 2 n_net")
    args = ap.parse_args()
    import torch
    from . import maot
    log = lambda s: print(s, flush=True)  # noqa: E731
    cnt = [int(v) for v in args.eval_pairs.split(",")]
    if args.eval_only:
        d = np.load(args.eval_only, allow_pickle=False)
        meta = json.loads(str(d["meta"]))
        net = maot.WarmStartNet(layers=meta["layers"], channels=meta["channels"], n_net=meta["n_net"],
                                max_batch=max(cnt), dilations=meta.get("dilations"))
        net.set_params(d["params"].astype(np.float32))
        res = {"n_net": evaluate(maot, net, meta["n_net"], cnt[0], log=log),
               "2n_net": evaluate(maot, net, 2 * meta["n_net"], cnt[1], log=log)}
        log("evaluation: " + json.dumps(res))
        net.close()
        return
    if not args.out:
        ap.error("--out is required for training")
    dil = [int(v) for v in args.dilations.split(",")]
    net = maot.WarmStartNet(layers=args.layers, channels=args.channels, n_net=args.n, max_batch=args.batch,
                            dilations=dil)
    net.set_params(init_params(args.layers, args.channels, args.seed))
    X, T, ok, gen = generate(maot, net, args.pairs, args.n, workers=args.workers, log=log)
    log("dataset: %s" % json.dumps(gen))
    tq = T[torch.from_numpy(ok).cuda()]
    log("target: mean square %.4e, max |t| %.4e" % (float((tq * tq).mean()), float(tq.abs().max())))
    del tq
    hist = train(net, X, T, ok, args.epochs, args.batch, args.lr, seed=args.seed, log=log)
    del X, T
    ev = evaluate(maot, net, args.n, cnt[0], log=log)
    ev512 = evaluate(maot, net, 2 * args.n, cnt[1], log=log)
    meta = {"layers": args.layers, "channels": args.channels, "dilations": dil, "n_net": args.n, "pairs": args.pairs,
            "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "seed": args.seed,
            "dataset": gen, "history": hist, "eval_n_net": ev, "eval_2n_net": ev512}
    np.savez(args.out, params=net.get_params(), meta=np.array(json.dumps(meta)))
    log("saved %s" % args.out)
    net.close()


if __name__ == "__main__":
    main()
