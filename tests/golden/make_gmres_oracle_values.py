"""Writes oracle_gmres_fullsize.json: the oracle's s-step GMRES runs on full-size workloads
that take it minutes to hours, stored so that GPU tests can compare against them.

Test infrastructure: calls only the oracle and the seeded input generators.

    python tests/golden/make_gmres_oracle_values.py [--only config4|config5]

Workloads
  config4  systems of the 256-system batch (2-D convection-diffusion, sizes 2^12..2^18,
           two-stage s = 5, s_hat = 20, m = 40, sparse-sign k = 48, zeta = 8, the batch's
           sketch seed of system i is i), FP64, tol 1e-10.
  config5  3-D convection-diffusion 192^3, wind (10, 20, 30), right Jacobi, two-stage
           s = 10, s_hat = m = 60, sparse-sign k = 128, zeta = 8, seed 0, b = 1, tol 1e-10.
For each run: converged, iterations, restarts, final explicit relative residual, the
implicit residual at every check point, ||x||_2 and x at 256 seeded sample rows (plus the
first and last row).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import krylov  # noqa: E402
from oracle.sketch import Sketch  # noqa: E402
from paper_2503_16717_amd import workloads as wl  # noqa: E402

OUT = os.path.join(HERE, "oracle_gmres_fullsize.json")
CONFIG4_SYSTEMS = [29, 4, 16, 3, 23, 14, 1]   # n = 5929 ... 241081


def sample_rows(n: int) -> list[int]:
    rows = set(np.random.default_rng([9, n]).choice(n, 256, replace=False).tolist())
    rows.update((0, n - 1))
    return sorted(int(r) for r in rows)


def record(res, n: int, seconds: float) -> dict:
    rows = sample_rows(n)
    return {"converged": bool(res.converged), "iters": int(res.iters), "restarts": int(res.restarts),
            "relres": float(res.relres), "history": [[int(i), float(r)] for i, r in res.history],
            "x_norm2": float(np.linalg.norm(res.x)), "sample_rows": rows,
            "x_samples": [float(res.x[r]) for r in rows], "oracle_seconds": round(seconds, 1)}


def config4() -> dict:
    specs = wl.batched_convdiff_specs(256)
    out = {}
    for i in CONFIG4_SYSTEMS:
        sp = specs[i]
        A = wl.convdiff_2d(sp["N"], sp["bx"], sp["by"])
        b = wl.batched_rhs(A.n, sp["rhs_seed"])
        t0 = time.perf_counter()
        res = krylov.sstep_gmres(A, b, s=5, m=40, shat=20, two_stage=True, sk=Sketch.sparse_sign(48, 8, i),
                                 tol=1e-10)
        dt = time.perf_counter() - t0
        r = record(res, A.n, dt)
        r.update({"system": i, "N": sp["N"], "n": A.n, "bx": sp["bx"], "by": sp["by"], "sketch_seed": i})
        out[str(i)] = r
        print(f"config4 system {i}: n={A.n} iters={res.iters} converged={res.converged} {dt:.0f}s", flush=True)
    return out


def config5() -> dict:
    A = wl.convdiff_3d(192, (10.0, 20.0, 30.0))
    b = np.ones(A.n)
    t0 = time.perf_counter()
    res = krylov.sstep_gmres(A, b, s=10, m=60, shat=60, two_stage=True, jacobi=True,
                             sk=Sketch.sparse_sign(128, 8, 0), tol=1e-10)
    dt = time.perf_counter() - t0
    r = record(res, A.n, dt)
    r.update({"N": 192, "n": A.n, "nnz": A.nnz})
    print(f"config5: iters={res.iters} converged={res.converged} relres={res.relres:.3e} {dt:.0f}s", flush=True)
    return r


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", choices=["config4", "config5"])
    args = ap.parse_args()
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data["_about"] = ("Oracle s-step GMRES runs at full size, written by make_gmres_oracle_values.py "
                      "(oracle only).")
    if args.only in (None, "config4"):
        data["config4"] = config4()
        json.dump(data, open(OUT, "w"), indent=1)
    if args.only in (None, "config5"):
        data["config5"] = config5()
        json.dump(data, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main()
