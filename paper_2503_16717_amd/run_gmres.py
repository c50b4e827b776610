"""One s-step GMRES solve of a named synthetic workload, for profiling runs.

    python -m paper_2503_16717_amd.run_gmres --workload convdiff3d --precision f64
    python -m paper_2503_16717_amd.run_gmres --workload laplace2d

Workloads (the recipes of the solver benchmarks):
  laplace2d   2-D 5-point Laplacian on a 100 x 100 grid, one-stage, s = 5, m = 30, Gaussian
              sketch k = 24, right-hand side uniform in [-1, 1] (seed 1);
  convdiff3d  3-D 7-point convection-diffusion on 192^3, wind (10, 20, 30), Jacobi, two-stage
              s = 10, s_hat = m = 60, sparse-sign sketch k = 128, right-hand side all ones.
Prints one line with the iteration count and the solve time.  Every step runs in libsko.
"""
from __future__ import annotations

import argparse
import sys


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", choices=("laplace2d", "convdiff3d"), required=True)
    ap.add_argument("--precision", choices=("f64", "mixed"), default="f64")
    ap.add_argument("--solves", type=int, default=1, help="solves in a row (the first sizes the workspace)")
    a = ap.parse_args(argv)

    import numpy as np
    import torch

    from . import binding as B
    from . import workloads as wl

    ctx = B.Context(0)
    if a.workload == "laplace2d":
        A = wl.laplacian_2d(100)
        b = wl.rhs_uniform(A.n, 1)
        th = B.colmajor_from_numpy(wl.gaussian_theta(A.n, 24, 0), "cuda")
        kw = dict(s=5, m=30, tol=1e-10, precision=a.precision, sketch=B.make_sketch("gaussian", theta=th))
    else:
        A = wl.convdiff_3d(192, (10.0, 20.0, 30.0))
        b = np.ones(A.n)
        kw = dict(s=10, m=60, shat=60, two_stage=True, precond=1, tol=1e-10, precision=a.precision,
                  sketch=B.make_sketch("sparse_sign", 128, 8, 0))
    Ad = B.csr_to_device(A)
    bt = torch.from_numpy(np.asarray(b, dtype=np.float64)).cuda()
    for i in range(a.solves):
        x, info, st = ctx.gmres(Ad, bt, **kw)
        torch.cuda.synchronize()
        print(f"{a.workload} {a.precision} solve {i}: status {st}, iterations {info['iters']}, "
              f"relres {info['relres']:.3e}, {info['t_total']:.4f} s", flush=True)
        if st != B.SKO_OK:
            return 1
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
