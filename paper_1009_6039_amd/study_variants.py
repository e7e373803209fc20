"""The paper's variants of the method on the GPU (Section 5.1, Remarks of Section 3.3).

On the Section 5.1 example family (workloads.e1_example: u* = 0.01 cos sin,
g = 1 + 0.3 cos cos), for N = 32 .. 256: Newton iterations, GMRES iterations per Newton
step and solve time for the step sizes tau = 1, 2, 4, 8 (Figure error_diff_tau), the
GMRES tolerances 1e-1 and 1e-4 (Figures bigtol and smalltol, Table 1), and the full
and simplified (no b . grad theta) operators; each solve to rms residual 1e-9, with the
rms distance to the continuous u* (the interpolation of g bounds it at O(h^2)).
Prints one JSON object per line.

  python -m paper_1009_6039_amd.study_variants [--sizes 32,64,128,256]
"""

import argparse
import json
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="32,64,128,256")
    ap.add_argument("--taus", default="1,2,4,8")
    args = ap.parse_args()
    import torch
    from . import maot
    from . import workloads as W
    for N in [int(v) for v in args.sizes.split(",")]:
        f, g, us = W.e1_example(N)
        fd, gd = torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda()
        cases = [("full", t, gt) for gt in (1e-1, 1e-4) for t in [float(v) for v in args.taus.split(",")]]
        cases += [("no_drift", 1.0, gt) for gt in (1e-1, 1e-4)]
        for op, tau, gt in cases:
            p = maot.Plan(n_max=N, batch_capacity=1, gmres_tol=gt, max_newton=400, op_mode=op)
            p.solve(fd, gd, damping=tau, tol=1e-9)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            psi, _, rep = p.solve(fd, gd, damping=tau, tol=1e-9)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            p.close()
            e = psi.cpu().numpy() - (us - us.mean())
            print(json.dumps({"n": N, "operator": op, "tau": tau, "gmres_tol": gt, "status": rep["status"],
                              "newton": rep["newton_iters"],
                              "gmres_per_newton": round(rep["gmres_iters"] / max(rep["newton_iters"], 1), 2),
                              "ms": round(1e3 * dt, 3), "res_rms": rep["res_rms"],
                              "err_rms_vs_u_star": float(np.sqrt(np.mean(e * e)))}), flush=True)


if __name__ == "__main__":
    main()
