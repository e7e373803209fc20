"""GPU parity of the warm-start network kernels against the FP64 oracle with BF16 emulation.

The GPU stores inputs, weights, activations and inter-layer gradients in BF16 and
accumulates in FP32; the oracle rounds the same tensors to BF16 and accumulates in
FP64.  FP32-vs-FP64 accumulation order can flip a rare BF16 rounding of an
intermediate value, so tensors are compared by relative L2 error, to 1e-3 per
tensor (measured on MI355X: forward at most 6.6e-4, weight and bias gradients at
most 9.0e-4; the kernels are deterministic, so these do not vary between runs) and
1e-4 for the warm start, whose FP64 head dilutes the network's share (measured at
most 4.1e-5).
"""

import numpy as np
import pytest

from oracle import cnn
from paper_1009_6039_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def maot():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1009_6039_amd import maot as m
    m.load()
    return m


def flat(params):
    return np.concatenate([np.concatenate([Wl.ravel(), bl.ravel()]) for Wl, bl in params]).astype(np.float32)


def f32_params(seed, layers=8):
    rng = np.random.default_rng(seed + 100)
    p = cnn.init_params(channels=32, layers=layers, seed=seed)
    p = [(Wl.astype(np.float32).astype(np.float64), (0.05 * rng.standard_normal(bl.shape)).astype(np.float32)
          .astype(np.float64)) for Wl, bl in p]
    return p


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def inputs(n, batch, seed):
    pairs = [W.blobs(n, W.seed_for(4, seed + k)) for k in range(batch)]
    f = np.stack([a for a, _ in pairs])
    g = np.stack([b for _, b in pairs])
    return f, g


DILATED = [(32, None), (64, (1, 2, 4, 2, 1, 4, 2, 1)), (48, (1, 3, 1, 1, 3, 1, 1, 1))]


@pytest.mark.parametrize("n,dil", DILATED)
def test_forward_matches_oracle(maot, n, dil):
    B = 2
    params = f32_params(1)
    net = maot.WarmStartNet(layers=8, channels=32, n_net=n, max_batch=B, dilations=dil)
    try:
        net.set_params(flat(params))
        f, g = inputs(n, B, 0)
        x = net.prepare_input(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda())
        c = net.forward(x)
        torch.cuda.synchronize()
        c = c.cpu().numpy().astype(np.float64)
        for k in range(B):
            ref, _ = cnn.forward(cnn.network_input(f[k], g[k]), params, bf16=True, dilations=dil)
            print("forward n=%d dil=%s sample %d: rel L2 %.3e" % (n, dil, k, rel_l2(c[k], ref[0])))
            assert rel_l2(c[k], ref[0]) < 1e-3, k
        # the prepared input is the BF16 rounding of (log(f/mean), log(g/mean)); the device
        # logarithm may differ from NumPy's in the last FP32 bit, which moves rare roundings
        xin = x.float().cpu().numpy()
        ref_in = cnn.bf16_round(np.log(f[0] / f[0].mean())).astype(np.float32)
        assert np.mean(xin[0, :, :, 0] == ref_in) > 0.99
        assert np.max(np.abs(xin[0, :, :, 0] - ref_in)) <= 2.0 ** -7 * np.max(np.abs(ref_in))
        assert np.all(xin[..., 2:] == 0)
    finally:
        net.close()


@pytest.mark.parametrize("n,dil", DILATED)
def test_gradients_match_oracle(maot, n, dil):
    B = 2
    params = f32_params(2)
    net = maot.WarmStartNet(layers=8, channels=32, n_net=n, max_batch=B, dilations=dil)
    try:
        net.set_params(flat(params))
        f, g = inputs(n, B, 10)
        t = np.stack([0.3 * (a / a.mean() - b / b.mean()) for a, b in zip(f, g)]).astype(np.float32)
        x = net.prepare_input(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda())
        grads, loss = net.gradients(x, torch.from_numpy(t).cuda())
        torch.cuda.synchronize()
        grads = grads.cpu().numpy().astype(np.float64)
        tot, lref = None, 0.0
        for k in range(B):
            c, cache = cnn.forward(cnn.network_input(f[k], g[k]), params, bf16=True, dilations=dil)
            gk = cnn.backward(c, t[k:k + 1].astype(np.float64), cache, params, bf16=True, count=B * n * n,
                              dilations=dil)
            lref += np.sum((c - t[k]) ** 2) / (B * n * n)
            tot = gk if tot is None else [(a[0] + b[0], a[1] + b[1]) for a, b in zip(tot, gk)]
        assert loss == pytest.approx(lref, rel=1e-3)
        ref = flat(tot).astype(np.float64)
        off = 0
        errs = []
        for l, (Wl, bl) in enumerate(params):
            nw, nb = Wl.size, bl.size
            errs.append((rel_l2(grads[off:off + nw], ref[off:off + nw]),
                         rel_l2(grads[off + nw:off + nw + nb], ref[off + nw:off + nw + nb])))
            off += nw + nb
        print("gradients n=%d dil=%s: rel L2 per layer (W, b): %s" % (
            n, dil, " ".join("%.2e/%.2e" % e for e in errs)))
        off = 0
        for l, (Wl, bl) in enumerate(params):
            nw, nb = Wl.size, bl.size
            assert rel_l2(grads[off:off + nw], ref[off:off + nw]) < 1e-3, ("W", l)
            assert rel_l2(grads[off + nw:off + nw + nb], ref[off + nw:off + nw + nb]) < 1e-3, ("b", l)
            off += nw + nb
    finally:
        net.close()


def test_adam_steps_reduce_the_loss(maot):
    n, B = 32, 4
    net = maot.WarmStartNet(layers=8, channels=32, n_net=n, max_batch=B)
    try:
        net.set_params(flat(f32_params(3)))
        f, g = inputs(n, B, 20)
        t = np.stack([0.5 * (a / a.mean() - b / b.mean()) for a, b in zip(f, g)]).astype(np.float32)
        x = net.prepare_input(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda())
        tt = torch.from_numpy(t).cuda()
        _, l0 = net.gradients(x, tt)
        for _ in range(40):
            net.train_step(x, tt, 2e-3)
        _, l1 = net.gradients(x, tt)
        assert l1 < 0.5 * l0, (l0, l1)
    finally:
        net.close()


def test_training_target_matches_oracle(maot):
    net = maot.WarmStartNet(layers=2, channels=32, n_net=32, max_batch=1)
    try:
        with pytest.raises(maot.MAError):  # a dilation the grid cannot tile
            maot.WarmStartNet(layers=2, channels=32, n_net=32, max_batch=1, dilations=(1, 4))
        rng = np.random.default_rng(4)
        u = rng.standard_normal((2, 48, 48)) * 1e-3
        f = 0.2 + rng.random((2, 48, 48))
        g = 0.5 + rng.random((2, 48, 48))
        dev = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
        plain = net.target(dev(u)).cpu().numpy()
        full = net.target(dev(u), dev(f), dev(g)).cpu().numpy()
        for k in range(2):
            assert rel_l2(plain[k], cnn.training_target(u[k])) < 1e-6
            assert rel_l2(full[k], cnn.training_target(u[k], f[k], g[k])) < 1e-6
    finally:
        net.close()


@pytest.mark.parametrize("n,dil", [(32, None), (64, None), (64, (1, 2, 1, 2, 1, 2, 1, 1))])
def test_warm_start_matches_oracle(maot, n, dil):
    n_net = 32
    params = f32_params(5)
    net = maot.WarmStartNet(layers=8, channels=32, n_net=n_net, max_batch=2, dilations=dil)
    try:
        net.set_params(flat(params))
        f, g = inputs(n, 3, 30)
        psis = net.warm_start([torch.from_numpy(a).cuda() for a in f], [torch.from_numpy(b).cuda() for b in g])
        torch.cuda.synchronize()
        for k in range(3):
            ref = cnn.warm_start(f[k], g[k], params, n_net, dilations=dil)
            got = psis[k].cpu().numpy()
            print("warm start n=%d dil=%s sample %d: rel L2 %.3e" % (n, dil, k, rel_l2(got, ref)))
            assert rel_l2(got, ref) < 1e-4, k
            assert abs(got.mean()) < 1e-6 * np.max(np.abs(ref))
    finally:
        net.close()


def test_benchmark_configuration_learned_start_matches_oracle(maot):
    # the configuration bench.py times: 256 blob pairs at 512^2 in one batched call,
    # learned start from the committed network, the fast linear solve (fd4 symbols,
    # scaled system, tolerance 0.2 with adaptive forcing), residual 1e-6.  Every pair
    # must converge; two sampled pairs are compared with the oracle, solved from the
    # oracle's own network start (BF16 emulation) to 1e-10.
    import json
    import os
    from oracle import ma
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    d = np.load(os.path.join(root, "paper_1009_6039_amd", "warmstart_256.npz"), allow_pickle=False)
    meta = json.loads(str(d["meta"]))
    B, N = 256, 512
    pairs = [W.blobs(N, W.seed_for(1, q)) for q in range(B)]
    opts = dict(damping_policy="backtrack", symbol="fd4", precond="diag", gmres_tol=0.2, forcing="adaptive")
    net = maot.WarmStartNet(layers=meta["layers"], channels=meta["channels"], n_net=meta["n_net"], max_batch=B,
                            dilations=meta["dilations"])
    p = maot.Plan(n_max=N, batch_capacity=B, max_newton=500, **opts)
    try:
        net.set_params(d["params"].astype(np.float32))
        fs = [torch.from_numpy(a).cuda() for a, _ in pairs]
        gs = [torch.from_numpy(b).cuda() for _, b in pairs]
        psi0 = net.warm_start(fs, gs)
        psis, _, reps = p.solve_batched(fs, gs, damping=1.0, tol=1e-6, psi0s=psi0)
        assert all(r["status"] == 0 and r["res_rms"] <= 1e-6 for r in reps)
        assert sum(r["warm_steps"] for r in reps) == B
        shaped = cnn.unflatten_params(d["params"], meta["layers"], meta["channels"])
        for q in (0, 137):
            print("benchmark configuration: sample pair %d" % q, flush=True)
            f, g = pairs[q]
            start = cnn.warm_start(f, g, shaped, meta["n_net"], dilations=meta["dilations"])
            ref, _, rr = ma.solve(f, g, tau=1.0, tol=1e-10, max_newton=500, psi0=start, **opts)
            assert rr.status == ma.OK
            err = np.max(np.abs(psis[q].cpu().numpy() - ref)) / np.max(np.abs(ref))
            print("pair %d: newton %d, max|psi - psi_oracle| / max|psi| = %.2e" % (q, reps[q]["newton_iters"], err))
            assert err <= 1e-6
    finally:
        p.close()
        net.close()


def test_learned_start_saves_newton_steps_and_wall_time_on_held_out_pairs(maot):
    # What the trained network gains over the method without it: 128 held-out blob pairs
    # at 256^2 (seeds seed_for(5, q), disjoint from the training pairs seed_for(4, q)),
    # the fast linear solve at residual 1e-6, one batched call per arm.  Every pair must
    # be solved from both starts; the learned start (network inference and head inside
    # the timing) must need fewer Newton steps on average and less wall time than the
    # zero start.  Each arm is timed three times after a warm-up; the fastest counts.
    import json
    import os
    import time
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    d = np.load(os.path.join(root, "paper_1009_6039_amd", "warmstart_256.npz"), allow_pickle=False)
    meta = json.loads(str(d["meta"]))
    B, N = 128, 256
    pairs = [W.blobs(N, W.seed_for(5, 300 + q)) for q in range(B)]
    opts = dict(damping_policy="backtrack", symbol="fd4", precond="diag", gmres_tol=0.2, forcing="adaptive")
    net = maot.WarmStartNet(layers=meta["layers"], channels=meta["channels"], n_net=meta["n_net"], max_batch=B,
                            dilations=meta["dilations"])
    p = maot.Plan(n_max=N, batch_capacity=B, max_newton=500, **opts)
    try:
        net.set_params(d["params"].astype(np.float32))
        p.autotune(N, B)
        fs = [torch.from_numpy(a).cuda() for a, _ in pairs]
        gs = [torch.from_numpy(b).cuda() for _, b in pairs]

        def run(arm):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            psi0 = net.warm_start(fs, gs) if arm == "learned" else None
            _, _, reps = p.solve_batched(fs, gs, damping=1.0, tol=1e-6, psi0s=psi0)
            torch.cuda.synchronize()
            return time.perf_counter() - t0, reps

        for arm in ("zero", "learned"):  # warm-up
            run(arm)
        times, last = {"zero": [], "learned": []}, {}
        for _ in range(3):  # interleaved, so that clock drift hits both arms alike
            for arm in ("zero", "learned"):
                dt, last[arm] = run(arm)
                times[arm].append(dt)
        res = {}
        for arm, reps in last.items():
            assert all(r["status"] == 0 and r["res_rms"] <= 1e-6 for r in reps), arm
            res[arm] = (float(np.mean([r["newton_iters"] for r in reps])), min(times[arm]),
                        float(np.mean([r["gmres_iters"] for r in reps])))
        print("held-out 256^2 x %d: zero start newton %.2f gmres %.1f %.2f ms; learned start newton %.2f "
              "gmres %.1f %.2f ms (x%.3f)" % (B, res["zero"][0], res["zero"][2], 1e3 * res["zero"][1],
                                              res["learned"][0], res["learned"][2], 1e3 * res["learned"][1],
                                              res["zero"][1] / res["learned"][1]))
        assert res["learned"][0] < res["zero"][0]
        assert res["learned"][1] < res["zero"][1]
    finally:
        p.close()
        net.close()
