"""GPU: the three-dimensional solver (ma3_*) against the 3-D oracle (oracle.ma3d).

Tolerances as in 2-D (derived in the design notes): the residual kernel is FP64 with
FP32-stored fields (r and the coefficients within 1e-6 of their max norm; the b
coefficients also carry the FP32 gradient of g), its FP64 scalars within 1e-10
relative; the operator and Lbar^{-1} run FP32 transforms (within 1e-4 of the output's
max norm); converged potentials and maps within 1e-6 of the oracle's.
"""

import numpy as np
import pytest

from oracle import ma3d
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


@pytest.fixture(scope="module")
def plan(maot):
    p = maot.Plan3(n_max=64)
    yield p
    p.close()


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def fields(N, seed=0):
    f, g, _ = W.e1_example3(N, k=60.0, alpha=0.4, rho=1)
    X1, X2, X3 = W.grid3(N)
    t = 2 * np.pi
    u = 0.003 * np.sin(t * X1 + 0.2) * np.cos(t * X2) * np.sin(t * X3 + 0.5) + 0.002 * np.cos(t * (X1 - X2))
    return f / f.mean(), g / g.mean(), u


@pytest.mark.parametrize("N", [16, 48, 64])
def test_residual_kernel_matches_oracle(plan, N):
    f, g, u = fields(N)
    r, coef, sc = plan.step_residual(dev(u), dev(f), dev(g))
    prob = ma3d.Problem3(f, g)
    ev = ma3d.evaluate3(u, prob)
    ref = ma3d.coefficients3(ev)
    er = np.max(np.abs(host(r) - ev.r)) / np.max(np.abs(ev.r))
    print("N %d: r %.2e" % (N, er), flush=True)
    assert er <= 1e-6
    c = host(coef)
    for q in range(9):
        scale = np.max(np.abs(ref[q])) if q < 6 else np.max(np.abs(np.stack(ref[6:])))
        e = np.max(np.abs(c[q] - ref[q])) / scale
        assert e <= 1e-6, (q, e)
    abar = ma3d.averaged3(ref)
    assert sc[0] == pytest.approx(ev.res_rms, rel=1e-10)
    assert sc[1] == pytest.approx(ev.res_max, rel=1e-10)
    assert sc[2] == pytest.approx(ev.mass_defect, rel=1e-9, abs=1e-14)
    assert sc[3] == pytest.approx(ev.min_det, rel=1e-10)
    for q in range(6):
        assert sc[6 + q] == pytest.approx(abar[q], rel=1e-10, abs=1e-12)
    bscale = max(abs(a) for a in abar[6:]) + np.mean(np.abs(np.stack(ref[6:])))
    for q in range(6, 9):
        assert abs(sc[6 + q] - abar[q]) <= 1e-6 * bscale
    w2 = float(np.mean((ev.grad[0] ** 2 + ev.grad[1] ** 2 + ev.grad[2] ** 2) * prob.f))
    assert sc[15] == pytest.approx(w2, rel=1e-10)
    assert sc[16] == pytest.approx(float(np.mean(u)), abs=1e-15)


@pytest.mark.parametrize("N", [16, 48, 64])
def test_strain_operator_and_lbar_inverse_match_oracle(plan, N):
    f, g, u = fields(N)
    ev = ma3d.evaluate3(u, ma3d.Problem3(f, g))
    coef = np.stack(ma3d.coefficients3(ev)).astype(np.float32)
    c64 = tuple(c.astype(np.float64) for c in coef)
    abar = ma3d.averaged3(c64)
    rho = ma3d.symbol3(abar, N)
    rng = np.random.default_rng(N)
    v = rng.standard_normal((N, N, N)).astype(np.float32)
    w = host(plan.step_strain_apply(dev(v, torch.float32), dev(coef, torch.float32), abar))
    want = ma3d.strain_apply3(v.astype(np.float64), c64, rho)
    ew = np.max(np.abs(w - want)) / np.max(np.abs(want))
    th = host(plan.step_lbar_inverse(dev(v, torch.float32), abar))
    want_th = ma3d.lbar_inverse3(v.astype(np.float64), rho)
    et = np.max(np.abs(th - want_th)) / np.max(np.abs(want_th))
    print("N %d: operator %.2e, Lbar^-1 %.2e" % (N, ew, et), flush=True)
    assert ew <= 1e-4 and et <= 1e-4


@pytest.mark.parametrize("N,policy", [(16, "fixed"), (32, "fixed"), (48, "fixed"), (32, "backtrack")])
def test_solve_matches_oracle(maot, N, policy):
    f, g, _ = W.e1_example3(N)
    ref, mref, rr = ma3d.solve3(f, g, tau=1.0, tol=1e-11, gmres_tol=1e-4, damping_policy=policy)
    assert rr.status == ma3d.OK
    p = maot.Plan3(n_max=N, damping_policy=policy)
    try:
        psi, mp, rep = p.solve(dev(f), dev(g), damping=1.0, tol=1e-9)
        psi, mp = host(psi), host(mp)
    finally:
        p.close()
    err = np.max(np.abs(psi - ref)) / np.max(np.abs(ref))
    em = np.max(np.abs(mp - mref))
    print("3-D N %d %s: newton %d (oracle %d), gmres %d (oracle %d), err %.2e, map %.2e" % (
        N, policy, rep["newton_iters"], rr.newton_iters, rep["gmres_iters"], rr.gmres_iters, err, em), flush=True)
    assert rep["status"] == 0 and rep["res_rms"] <= 1e-9
    assert err <= 1e-6 and em <= 1e-6
    assert abs(rep["newton_iters"] - rr.newton_iters) <= max(3, 0.3 * rr.newton_iters)


def test_blob_pair_with_step_halving_matches_oracle(maot):
    N = 32
    f, g = W.blobs3(N, W.seed_for(7, 0))
    ref, _, rr = ma3d.solve3(f, g, tau=1.0, tol=1e-10, gmres_tol=1e-2, damping_policy="backtrack", max_newton=200)
    assert rr.status == ma3d.OK
    p = maot.Plan3(n_max=N, damping_policy="backtrack", gmres_tol=1e-2, max_newton=200)
    try:
        psi, _, rep = p.solve(dev(f), dev(g), damping=1.0, tol=1e-9)
        psi = host(psi)
    finally:
        p.close()
    err = np.max(np.abs(psi - ref)) / np.max(np.abs(ref))
    print("3-D blobs: newton %d (oracle %d), halvings %d (oracle %d), err %.2e" % (
        rep["newton_iters"], rr.newton_iters, rep["backtracks"], rr.backtracks, err), flush=True)
    assert rep["status"] == 0 and err <= 1e-6
    # the GPU's psi also solves the oracle's discrete equation
    ev = ma3d.evaluate3(psi, ma3d.Problem3(f, g))
    assert ev.res_rms <= 1.001e-9


def test_invalid_inputs_are_refused(maot, plan):
    with pytest.raises(maot.MAError):
        maot.Plan3(n_max=40)
    f = torch.ones((24, 24, 24), dtype=torch.float64, device="cuda")
    with pytest.raises(maot.MAError):
        plan.solve(f, f)  # N = 24 is not a supported grid
    f = torch.ones((16, 16, 16), dtype=torch.float64, device="cuda")
    g = f.clone()
    g[3, 4, 5] = -1.0
    with pytest.raises(maot.MAError):
        plan.solve(f, g)
    psi, _, rep = plan.solve(f, f.clone())
    assert rep["status"] == 0 and rep["newton_iters"] == 0 and not torch.any(psi)
