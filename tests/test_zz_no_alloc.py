"""GPU: the no-allocation entry point ma_solve_noalloc against ma_solve.

Both run the same kernels on the same pair with the same options (no autotuning):
the potentials, maps and reports must agree to the parity bar (in fact bitwise),
on two calls in a row, the second on a smaller grid; sizes beyond the static
array are refused.
"""

import numpy as np
import pytest

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_noalloc_solve_matches_plan_solve_on_two_calls(maot):
    opts = dict(damping_policy="backtrack", symbol="fd4", precond="diag", gmres_tol=0.2, forcing="adaptive",
                max_newton=300)
    for n, q in ((512, 0), (128, 1)):  # the second call on a smaller grid
        f, g = W.blobs(n, W.seed_for(1, q))
        print("noalloc: n = %d, pair seed %d" % (n, W.seed_for(1, q)), flush=True)
        fd, gd = dev(f), dev(g)
        psi_a, map_a, rep_a = maot.solve_noalloc(fd, gd, damping=1.0, tol=1e-8,
                                                 map=torch.empty((2, n, n), dtype=torch.float64, device="cuda"),
                                                 **opts)
        plan = maot.Plan(n_max=n, batch_capacity=1, **opts)
        try:
            psi_b, map_b, rep_b = plan.solve(fd, gd, damping=1.0, tol=1e-8)
        finally:
            plan.close()
        torch.cuda.synchronize()
        assert rep_a["status"] == 0 and rep_b["status"] == 0 and rep_a["res_rms"] <= 1e-8
        pa, pb = psi_a.cpu().numpy(), psi_b.cpu().numpy()
        assert np.max(np.abs(pa - pb)) <= 1e-6 * np.max(np.abs(pb))
        assert np.array_equal(pa, pb) and torch.equal(map_a, map_b)
        for k in ("newton_iters", "gmres_iters", "backtracks", "res_rms", "w2sq"):
            assert rep_a[k] == rep_b[k], k


def test_noalloc_fd_bicg_solve_matches_plan_solve_on_two_calls(maot):
    # the finite-difference BiCG step (its vectors carved from the same static array;
    # the host drains the stream every 16 BiCG iterations instead of polling a summary)
    opts = dict(linear_solver="fd_bicg", damping_policy="backtrack", gmres_tol=0.1, max_newton=300)
    for n, q in ((128, 2), (64, 3)):
        f, g = W.blobs(n, W.seed_for(1, q))
        print("noalloc fd-bicg: n = %d, pair seed %d" % (n, W.seed_for(1, q)), flush=True)
        fd, gd = dev(f), dev(g)
        psi_a, _, rep_a = maot.solve_noalloc(fd, gd, damping=1.0, tol=1e-8, **opts)
        plan = maot.Plan(n_max=n, batch_capacity=1, **opts)
        try:
            psi_b, _, rep_b = plan.solve(fd, gd, damping=1.0, tol=1e-8)
        finally:
            plan.close()
        torch.cuda.synchronize()
        assert rep_a["status"] == 0 and rep_b["status"] == 0 and rep_a["res_rms"] <= 1e-8
        assert torch.equal(psi_a, psi_b)
        for k in ("newton_iters", "gmres_iters", "backtracks", "res_rms"):
            assert rep_a[k] == rep_b[k], k


def test_noalloc_rejects_sizes_beyond_its_array(maot):
    f = torch.ones((768, 768), dtype=torch.float64, device="cuda")
    with pytest.raises(maot.MAError) as e:
        maot.solve_noalloc(f, f)
    assert e.value.code == maot.EINVAL
    g = torch.ones((512, 512), dtype=torch.float64, device="cuda")
    with pytest.raises(maot.MAError) as e:  # the Krylov basis of m = 30 does not fit at 512^2
        maot.solve_noalloc(g, g, gmres_m=30)
    assert e.value.code == maot.EINVAL
