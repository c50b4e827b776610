"""One s-step GMRES solve of a named synthetic workload, for profiling runs.

    python -m paper_2503_16717_amd.run_gmres --workload convdiff3d --precision f64
    python -m paper_2503_16717_amd.run_gmres --workload laplace2d
    python -m paper_2503_16717_amd.run_gmres --workload batch256 --precision mixed

Workloads (the recipes of the solver benchmarks):
  laplace2d   2-D 5-point Laplacian on a 100 x 100 grid, one-stage, s = 5, m = 30, Gaussian
              sketch k = 24, right-hand side uniform in [-1, 1] (seed 1);
  convdiff3d  3-D 7-point convection-diffusion on 192^3, wind (10, 20, 30), Jacobi, two-stage
              s = 10, s_hat = m = 60, sparse-sign sketch k = 128, right-hand side all ones;
  batch256    256 independent 2-D convection-diffusion systems (2^12..2^18 rows, seeded winds and
              right-hand sides), solved in lock step by sko_gmres_batched: two-stage s = 5,
              s_hat = 20, m = 40, sparse-sign sketch k = 48.
Prints one line per solve with the iteration count and the time.  Every step runs in libsko.
"""
from __future__ import annotations

import argparse
import sys


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", choices=("laplace2d", "convdiff3d", "batch256"), required=True)
    ap.add_argument("--precision", choices=("f64", "mixed"), default="f64")
    ap.add_argument("--solves", type=int, default=1, help="solves in a row (the first sizes the workspace)")
    a = ap.parse_args(argv)

    import numpy as np
    import torch

    from . import binding as B
    from . import workloads as wl

    ctx = B.Context(0)
    if a.workload == "batch256":
        return run_batch(B, wl, ctx, torch, a)
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


def run_batch(B, wl, ctx, torch, a) -> int:
    import time
    As, keep, bs, xs = [], [], [], []
    for sp in wl.batched_convdiff_specs(256):
        A = wl.convdiff_2d(sp["N"], sp["bx"], sp["by"])
        Ad, k = B.csr_to_device(A)
        As.append(Ad)
        keep.append(k)
        bt = torch.from_numpy(wl.batched_rhs(A.n, sp["rhs_seed"])).cuda()
        bs.append(bt)
        xs.append(torch.zeros_like(bt))
    opts = B.gmres_opts(s=5, m=40, shat=20, two_stage=True, tol=1e-10, precision=a.precision,
                        sketch=B.make_sketch("sparse_sign", 48, 8, 0))
    for i in range(a.solves):
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, infos = ctx.sko_gmres_batched(As, [b.data_ptr() for b in bs], [x.data_ptr() for x in xs], opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(f"batch256 {a.precision} solve {i}: status {st}, {sum(f.converged for f in infos)} of {len(infos)} "
              f"converged, iterations {sum(f.iters for f in infos)}, {dt:.4f} s", flush=True)
        if st != B.SKO_OK:
            return 1
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
