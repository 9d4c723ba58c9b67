"""Write the oracle's ridge CG solution of the full ridge workload (golden file).

Workload: m = 2000 drugs, q = 500 targets, Gaussian bases (sigma = 4) on 64-dim
N(0, 1) features, n = 200 000 training pairs (20% of the grid), rank-10
bilinear labels with N(0, 0.1^2) noise, lambda = 1e-2, tolerance 1e-6 on the
relative residual, at most 200 iterations: the ridge system of Section 3
eq. (1) solved by textbook conjugate gradients in FP64 (the oracle).

Only the seeded generator and ``oracle`` are called; nothing here comes from
the GPU library.  Run from the repository root (about 20 minutes on 8 threads):

    python tests/golden/make_ridge_cg_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2009_01054_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ridge_cg_m2000_q500_n200k.npz")


def main():
    p = W.config2()
    t0 = time.time()
    A, iters, rr, rt = oracle.krr_cg("kronecker", p["D"], p["T"], (p["c"], p["e"]), p["y"], [p["lam"]],
                                     max_iter=200, tol=1e-6)
    dt = time.time() - t0
    np.savez_compressed(OUT, a=A[:, 0], iters=iters, relres_recurrence=rr, relres_true=rt,
                        lam=np.array([p["lam"]]), tol=np.array([1e-6]), max_iter=np.array([200]))
    print(f"oracle CG: {int(iters[0])} iterations, recurrence {rr[0]:.3e}, true {rt[0]:.3e}, "
          f"{dt:.1f} s on {oracle.max_threads()} threads -> {OUT}")


if __name__ == "__main__":
    main()
