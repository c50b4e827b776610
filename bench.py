#!/usr/bin/env python3
"""Benchmark of the sketched block-orthogonalisation hot path on one MI355X.

Workload (a step): orthogonalise a tall matrix of n = 2^24 rows made of 12 blocks of
s+1 = 6 columns, every block V_j = U_j diag(sigma) W_j^T with sigma log-spaced from 1 to
1e-12, by one-stage BCGS2 with the RandCholQR first intra-block step and a sparse-sign
sketch (k = 64 rows, zeta = 8 nonzeros per row of Theta), all in FP64.  V is resident in
HBM before timing starts; Q is written to a separate buffer so every step sees the
same input.

value = algorithmic HBM bytes of one step / time per step, in GB/s.  Algorithmic bytes
count each tall operand once per pass of the pass schedule (block j with p = 6j
previous columns: (4p + 10w) columns of 8 bytes per row; first block 6w).

Also reported: roofline of the dominant kernel (event-timed launches over the timed
region), the two-stage variant (s_hat = 30), the CPU oracle timed on a bounded sample of
the same workload, and under "gmres" the time to a 1e-10 relative residual of the
restarted s-step solver on the 100x100 Laplacian, the 192^3 convection-diffusion problem
(FP64 and mixed) and 256 independent convection-diffusion systems (FP64 and mixed).

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--no-cpu-baseline] [--skip-gmres]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_ROWS = 1 << 24
NB, W, LOG10_COND = 12, 6, 12.0
SK_K, SK_ZETA, SK_SEED = 64, 8, 0


def alg_bytes_one_stage(n: int, nb: int, w: int, eb: int = 8) -> float:
    cols = 0
    for j in range(nb):
        p = j * w
        cols += (4 * p + 10 * w) if p > 0 else 6 * w
    return float(cols) * n * eb


def alg_bytes_two_stage_method(n: int, nb: int, w: int, ppb: int, eb: int = 8) -> float:
    """Tall traffic the two-stage method needs (each operand once per pass, the big-panel
    close fused like the one-stage passes): per panel the projection and update + sketch
    against Q_old (p + w, p + 2w; a sketch of w without previous big panels) and the
    forward substitution ((i + 2) w for panel i); per big panel with previous columns the
    close Gram (W), solve + write + projection (2W + p), update + write + Gram (2W + p) and
    solve + write (2W); the first big panel's two CholQR passes pairs (6W).  193.3 GB at
    n = 2^24, 12 blocks of 6, s_hat = 30."""
    Wb = ppb * w
    cols = 0
    for big in range(nb // ppb):
        p = big * Wb
        for i in range(ppb):
            cols += (p + w) + (p + 2 * w) if p > 0 else w
            cols += (i + 2) * w
        cols += (Wb + (2 * Wb + p) + (2 * Wb + p) + 2 * Wb) if p > 0 else 6 * Wb
    return float(cols) * n * eb


def alg_bytes_two_stage(n: int, nb: int, w: int, ppb: int, eb: int = 8) -> float:
    """Pass schedule the library executes for the two-stage scheme (each tall operand once
    per pass).  In the big-panel close of panels up to 40 columns, the row solve by R_h also
    accumulates the reduction that follows it: the Gram matrix of the second CholQR (first
    big panel) or the projection on up to 48 previous columns; the row update and its Gram
    matrix stay two sweeps."""
    Wb = ppb * w
    fuse = Wb <= 40
    cols = 0
    for big in range(nb // ppb):
        p = big * Wb
        for i in range(ppb):
            if p > 0:
                cols += p + w          # C_i = Q_old^T V_i
                cols += p + 2 * w      # V_hat_i = V_i - Q_old C_i (written) + sketch
            else:
                cols += w              # sketch of V_i
            cols += (i * w + w) + w    # forward substitution, written
        cols += Wb + 2 * Wb            # Gram of Q_bar, Q_hat = Q_bar R^{-1} (+ fused reduction)
        if p > 0:
            if fuse and p <= 48:
                cols += p              # Q_old read by the fused C_2 = Q_old^T Q_hat
            else:
                cols += p + Wb         # C_2 = Q_old^T Q_hat
            cols += (p + 2 * Wb) + Wb  # V_bar = Q_hat - Q_old C_2, Gram of V_bar
        elif not fuse:
            cols += Wb                 # Gram of Q_hat
        cols += 2 * Wb                 # Q_P = V_bar R^{-1}
    return float(cols) * n * eb


def c3_suite(B, torch, wl, n: int, no_autotune: bool = False) -> dict:
    """Mixed precision at the config-2 shape with w = 11 (s = 10): the same blocks stored in
    FP32 and in FP64, one-stage RandCholQR-BCGS2, sparse-sign k = 64; errors of the FP32 run
    measured in FP64 on the device (||I - Q^T Q||_2 and ||V - QR||_F / ||V||_F, V the FP32
    input itself)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    w, nb = 11, 12
    N = w * nb
    out = {}
    ctx = B.Context(0)
    sk = B.make_sketch("sparse_sign", SK_K, SK_ZETA, SK_SEED)
    for e in (6.0, 10.0):
        V64 = torch.empty((N, n), dtype=torch.float64, device="cuda")

        def one(j):
            blk = wl.glued_block(n, w, e, j)
            V64[j * w:(j + 1) * w].copy_(torch.from_numpy(np.ascontiguousarray(blk.T)))

        with ThreadPoolExecutor(max_workers=12) as ex:
            list(ex.map(one, range(nb)))
        V32 = V64.float()
        res = {}
        for prec, V in (("f64", V64), ("mixed", V32)):
            Q = torch.empty_like(V)
            R = np.zeros((N, N), order="F")
            o = B.orth_opts(intra="randcholqr", precision=prec, sketch=sk)
            if not no_autotune:
                st = ctx.sko_autotune_orth(n, nb, w, o)
                if st != B.SKO_OK:
                    raise B.SkoError(st, "sko_autotune_orth")

            def step():
                st, col = ctx.sko_orth_blocks(n, nb, w, V.data_ptr(), n, Q.data_ptr(), n, R, N, o)
                if st != B.SKO_OK:
                    raise B.SkoError(st, "sko_orth_blocks", col)

            step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                step()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / 3 * 1e3
            ab = alg_bytes_one_stage(n, nb, w, 4 if prec == "mixed" else 8)
            top = None
            if e == 6.0:   # a profiled run for the kernel breakdown (its events slow short launches)
                ctx.sko_profile_enable(True)
                step()
                torch.cuda.synchronize()
                ctx.sko_profile_enable(False)
                top = [{"name": q["name"], "ms": round(q["total_ms"], 3), "launches": q["launches"],
                        "GBps": round(q["bytes"] / (q["total_ms"] * 1e-3) / 1e9, 1) if q["total_ms"] > 0
                        else None} for q in ctx.sko_profile_read()[:8]]
            Qd = Q.t().double()            # n x N
            G = (Qd.t() @ Qd).cpu().numpy()
            orth = float(np.linalg.norm(np.eye(N) - G, 2))
            Rt = torch.from_numpy(R).cuda()
            num = den = 0.0
            for r0 in range(0, n, 1 << 22):
                Vc = V.t()[r0:r0 + (1 << 22)].double()
                num += float(((Vc - Qd[r0:r0 + (1 << 22)] @ Rt) ** 2).sum())
                den += float((Vc ** 2).sum())
            res[prec] = {"ms_per_step": round(ms, 3), "GBps": round(ab / (ms * 1e-3) / 1e9, 1),
                         "orth_error": orth, "backward_error": (num / den) ** 0.5}
            if top:
                res[prec]["kernels_top_profiled_run"] = top
            del Q, Qd, Rt
            log(f"config3 kappa 1e{e:g} {prec}: {res[prec]}")
        out[f"kappa_1e{int(e)}"] = res
        del V64, V32
        torch.cuda.empty_cache()
    ctx.close()
    return out


def next_rows_suite(B, torch, wl, n: int) -> dict:
    """The rows beyond the core path, on the config-2 shape (n rows, 12 blocks of 6 columns):
    f1  BCGS-PIP pre-processing in the two-stage scheme (s_hat = 30), against the RandBCGS2
        pre-processing on the same blocks (kappa 1e6 per block: PIP needs the accumulated
        condition number below about u^{-1/2}), and recursive CholQR2 as the intra-block step
        of the one-stage scheme (kappa 1e12: the first Cholesky of every block breaks down
        and recurses);
    f2  the Count-Gaussian sketch (Count part: 2 s^2 = 50 rows, one nonzero per input row;
        Gaussian part 2 (s + 1) = 12 rows) in one-stage RandCholQR-BCGS2 (kappa 1e12), against
        the sparse-sign sketch;
    f3  the Newton basis in s-step GMRES on the config-1 Laplacian: s = 10 and 15 against the
        monomial basis (restart 30, Gaussian sketch of max(24, 2 (s + 1)) rows)."""
    import numpy as np
    out = {}
    ctx = B.Context(0)
    N = NB * W
    R = np.zeros((N, N), order="F")

    def timed(V, Q, o, steps=3):
        def step():
            st, col = ctx.sko_orth_blocks(n, NB, W, V.data_ptr(), n, Q.data_ptr(), n, R, N, o)
            return st, col
        st, col = step()
        torch.cuda.synchronize()
        if st != B.SKO_OK:
            return {"status": int(st), "breakdown_col": int(col)}
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        return {"status": 0, "ms_per_step": round(ms, 3)}

    Q = torch.empty((N, n), dtype=torch.float64, device="cuda").t()
    for e in (6.0, 12.0):
        V = build_inputs(n, torch, wl, e)
        if e == 6.0:
            sk = B.make_sketch("sparse_sign", SK_K, SK_ZETA, SK_SEED)
            r_pip = timed(V, Q, B.orth_opts(two_stage=True, panels_per_big=6, reorth=True, preproc="pip", sketch=sk))
            r_rb = timed(V, Q, B.orth_opts(two_stage=True, panels_per_big=6, reorth=True, sketch=sk))
            ab = alg_bytes_two_stage_method(n, NB, W, 6)
            for r in (r_pip, r_rb):
                if r.get("ms_per_step"):
                    r["GBps_on_method_bytes"] = round(ab / (r["ms_per_step"] * 1e-3) / 1e9, 1)
            out["f1_pip_two_stage_kappa1e6"] = {"pip": r_pip, "randbcgs2": r_rb}
            log(f"f1 PIP two-stage: {out['f1_pip_two_stage_kappa1e6']}")
        else:
            sk = B.make_sketch("sparse_sign", SK_K, SK_ZETA, SK_SEED)
            r_rec = timed(V, Q, B.orth_opts(intra="cholqr2_recursive", sketch=sk))
            r_c2 = timed(V, Q, B.orth_opts(intra="cholqr2", sketch=sk))
            out["f1_recursive_cholqr2_kappa1e12"] = {"recursive": r_rec, "cholqr2": r_c2}
            log(f"f1 recursive CholQR2: {out['f1_recursive_cholqr2_kappa1e12']}")
            tg = B.colmajor_from_numpy(wl.gaussian_theta(50, 12, 7), "cuda")
            r_cg = timed(V, Q, B.orth_opts(sketch=B.make_sketch("count_gauss", zeta=1, seed=SK_SEED, theta=tg)))
            r_ss = timed(V, Q, B.orth_opts(sketch=sk))
            ab = alg_bytes_one_stage(n, NB, W)
            for r in (r_cg, r_ss):
                if r.get("ms_per_step"):
                    r["GBps"] = round(ab / (r["ms_per_step"] * 1e-3) / 1e9, 1)
            out["f2_count_gauss_kappa1e12"] = {"count_gauss_50x12": r_cg, "sparse_sign_64": r_ss}
            log(f"f2 Count-Gauss: {out['f2_count_gauss_kappa1e12']}")
            del tg
        del V
        torch.cuda.empty_cache()
    del Q
    # f3: Newton basis, config-1 Laplacian
    A1 = wl.laplacian_2d(100)
    b1 = wl.rhs_uniform(A1.n, 1)
    Ad = B.csr_to_device(A1)
    bt = torch.from_numpy(b1).cuda()
    res = {}
    for s_, basis in ((5, "monomial"), (10, "monomial"), (10, "newton"), (15, "monomial"), (15, "newton")):
        k = max(24, 2 * (s_ + 1))
        th = B.colmajor_from_numpy(wl.gaussian_theta(A1.n, k, 0), "cuda")
        kw = dict(s=s_, m=30, tol=1e-10, basis=basis, sketch=B.make_sketch("gaussian", theta=th))
        ctx.gmres(Ad, bt, **kw)
        torch.cuda.synchronize()
        x, info, st = ctx.gmres(Ad, bt, **kw)
        torch.cuda.synchronize()
        res[f"s{s_}_{basis}"] = {"status": int(st), "converged": info["converged"], "iters": info["iters"],
                                 "relres": info["relres"], "time_s": round(info["t_total"], 5)}
    out["f3_newton_laplace2d_100"] = res
    log(f"f3 Newton basis: {res}")
    ctx.close()
    return out


def gmres_suite(B, torch, wl, args) -> dict:
    """Time to relative residual 1e-10 (explicit, FP64) for the solver configurations."""
    import numpy as np
    out = {}
    ctx = B.Context(0)

    def solve(A, b, profile=False, **kw):
        Ad = B.csr_to_device(A)
        bt = torch.from_numpy(np.asarray(b, dtype=np.float64)).cuda()
        # the first solve sizes the workspace; the second is the one reported; a third,
        # with the per-kernel profiler on (its events slow short launches), gives the breakdown
        x, info, st = ctx.gmres(Ad, bt, **kw)
        torch.cuda.synchronize()
        x, info, st = ctx.gmres(Ad, bt, **kw)
        torch.cuda.synchronize()
        r = {"status": st, "converged": info["converged"], "iters": info["iters"],
             "restarts": info["restarts"], "relres": info["relres"], "time_s": round(info["t_total"], 5)}
        if profile:
            ctx.sko_profile_enable(True)
            ctx.gmres(Ad, bt, **kw)
            torch.cuda.synchronize()
            ctx.sko_profile_enable(False)
            r["kernels_top"] = [{"name": q["name"], "ms": round(q["total_ms"], 3), "launches": q["launches"],
                                 "GBps": round(q["bytes"] / (q["total_ms"] * 1e-3) / 1e9, 1) if q["total_ms"] > 0
                                 else None} for q in ctx.sko_profile_read()[:8]]
        return r

    # config 1: 2-D Laplacian 100x100, one-stage RandCholQR-BCGS2, Gaussian k = 24, s = 5, m = 30
    A1 = wl.laplacian_2d(100)
    th = B.colmajor_from_numpy(wl.gaussian_theta(A1.n, 24, 0), "cuda")
    out["config1_fp64"] = solve(A1, wl.rhs_uniform(A1.n, 1), s=5, m=30, tol=1e-10,
                                sketch=B.make_sketch("gaussian", theta=th))
    log(f"config1: {out['config1_fp64']}")
    # config 5: 3-D convection-diffusion 192^3, wind (10,20,30), Jacobi, two-stage s=10, s_hat=m=60, k=128
    log("config5: assembling 192^3 convection-diffusion")
    A5 = wl.convdiff_3d(192, (10.0, 20.0, 30.0))
    b5 = np.ones(A5.n)
    sk5 = B.make_sketch("sparse_sign", 128, 8, 0)
    for prec in ("f64", "mixed"):
        out[f"config5_{prec}"] = solve(A5, b5, profile=True, s=10, m=60, shat=60, two_stage=True, precond=1,
                                       tol=1e-10, precision=prec, sketch=sk5)
        log(f"config5 {prec}: {out[f'config5_{prec}']}")
    del A5
    # config 4: 256 independent 2-D convection-diffusion systems, two-stage s=5, s_hat=20, m=40, k=48
    specs = wl.batched_convdiff_specs(256)
    As, bs, xs, keep = [], [], [], []
    for sp in specs:
        A = wl.convdiff_2d(sp["N"], sp["bx"], sp["by"])
        Ad, k = B.csr_to_device(A)
        As.append(Ad)
        keep.append(k)
        bt = torch.from_numpy(wl.batched_rhs(A.n, sp["rhs_seed"])).cuda()
        bs.append(bt)
        xs.append(torch.zeros_like(bt))
    for prec in ("f64", "mixed"):
        for x in xs:
            x.zero_()
        opts = B.gmres_opts(s=5, m=40, shat=20, two_stage=True, tol=1e-10, precision=prec,
                            sketch=B.make_sketch("sparse_sign", 48, 8, 0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, infos = ctx.sko_gmres_batched(As, [b.data_ptr() for b in bs], [x.data_ptr() for x in xs], opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof4 = None
        if prec == "f64":   # a second, profiled run for the kernel breakdown
            for x in xs:
                x.zero_()
            ctx.sko_profile_enable(True)
            ctx.sko_gmres_batched(As, [b.data_ptr() for b in bs], [x.data_ptr() for x in xs], opts)
            torch.cuda.synchronize()
            ctx.sko_profile_enable(False)
            prof4 = [{"name": q["name"], "ms": round(q["total_ms"], 2), "launches": q["launches"]}
                     for q in ctx.sko_profile_read()[:8]]
        out[f"config4_{prec}"] = {"status": st, "time_s": round(dt, 4),
                                  "converged": int(sum(i.converged for i in infos)),
                                  "iters_total": int(sum(i.iters for i in infos)),
                                  "iters_max": int(max(i.iters for i in infos)), "systems": len(infos)}
        if prof4:
            out[f"config4_{prec}"]["kernels_top_profiled_run"] = prof4
        log(f"config4 {prec}: {out[f'config4_{prec}']}")
    # the same 256 systems solved one by one (FP64), the plain path the batched form replaces
    for x in xs:
        x.zero_()
    opts = B.gmres_opts(s=5, m=40, shat=20, two_stage=True, tol=1e-10,
                        sketch=B.make_sketch("sparse_sign", 48, 8, 0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    conv = iters = 0
    for i, (Ad, b, x) in enumerate(zip(As, bs, xs)):
        oi = B.gmres_opts(s=5, m=40, shat=20, two_stage=True, tol=1e-10,
                          sketch=B.make_sketch("sparse_sign", 48, 8, i))
        st, inf = ctx.sko_gmres(Ad, b.data_ptr(), x.data_ptr(), oi)
        conv += inf.converged
        iters += inf.iters
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["config4_one_by_one_f64"] = {"time_s": round(dt, 4), "converged": int(conv), "iters_total": int(iters),
                                     "systems": len(As)}
    log(f"config4 one-by-one f64: {out['config4_one_by_one_f64']}")
    del opts
    ctx.close()
    return out


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_inputs(n: int, torch, wl, log10_cond: float = LOG10_COND):
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    N = NB * W
    Vd = torch.empty((N, n), dtype=torch.float64, device="cuda").t()

    def one(j):
        blk = wl.glued_block(n, W, log10_cond, j)
        Vd[:, j * W:(j + 1) * W].copy_(torch.from_numpy(np.ascontiguousarray(blk.T)).t())
        return j

    threads = max(1, min(NB, os.cpu_count() or 1, 12))
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for j in ex.map(one, range(NB)):
            pass
    torch.cuda.synchronize()
    return Vd


def copy_ceiling(torch, nbytes: int = 1 << 31, reps: int = 20) -> float:
    """Device-to-device copy bandwidth (read + write bytes / time) of a plain copy kernel."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_pass_kernels_blockorth_n2p24_w6.md")


def pass_source_digest() -> str:
    """Digest of the pass kernels' sources, as the traffic summary's rows carry it."""
    from paper_2503_16717_amd.rocprof_summary import source_digest
    return source_digest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when it is missing or was taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    digest = pass_source_digest()
    for line in open(TRAFFIC_FILE):
        if not line.startswith("|") or "kernel" in line or "---" in line:
            continue
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 5 and cells[0] == kernel and cells[4] == digest:
            return float(cells[3])
    return None


def cpu_baseline(n_sample: int):
    """The FP64 oracle, untuned, on the first n_sample rows' worth of the same recipe, with the
    host's BLAS thread pool and with one thread."""
    import numpy as np
    from oracle import orth
    from oracle.sketch import Sketch
    from paper_2503_16717_amd import workloads as wl
    V = wl.glued_blocks(n_sample, NB, W, LOG10_COND)
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    sk = Sketch.sparse_sign(SK_K, SK_ZETA, SK_SEED)
    t0 = time.perf_counter()
    r = orth.orth_blocks_one_stage(V, W, "randcholqr", sk)
    dt = time.perf_counter() - t0
    assert r.info == 0
    gbs = alg_bytes_one_stage(n_sample, NB, W) / dt / 1e9
    out = {"value": round(gbs, 4), "unit": "GB/s", "cores": int(cores), "kind": "oracle",
           "sample": f"one-stage RandCholQR-BCGS2, {n_sample} rows (1/{N_ROWS // n_sample} of n) x 12 blocks "
                     f"x 6 columns, same generator, {dt:.1f} s"}
    # the same oracle on one host thread (BLAS pool limited to 1), on an eighth of that sample
    try:
        from threadpoolctl import threadpool_limits
        n1 = max(4096, n_sample // 8)
        V1 = np.asfortranarray(V[:n1])
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            r1 = orth.orth_blocks_one_stage(V1, W, "randcholqr", sk)
            dt1 = time.perf_counter() - t0
        assert r1.info == 0
        out["one_thread"] = {"value": round(alg_bytes_one_stage(n1, NB, W) / dt1 / 1e9, 4), "unit": "GB/s",
                             "cores": 1, "sample": f"first {n1} rows of the same sample, {dt1:.1f} s"}
    except ImportError:
        pass
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=1 << 21)
    ap.add_argument("--n", type=int, default=N_ROWS, help="rows (default 2^24)")
    ap.add_argument("--skip-gmres", action="store_true", help="skip the GMRES time-to-solution runs")
    ap.add_argument("--skip-two-stage", action="store_true", help="skip the two-stage orthogonalisation run")
    ap.add_argument("--skip-c3", action="store_true", help="skip the mixed-precision block orthogonalisation run")
    ap.add_argument("--skip-next-rows", action="store_true",
                    help="skip the BCGS-PIP, recursive CholQR2, Count-Gauss and Newton-basis runs")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB five times (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read_per_launch": a.numel() * 8,
                          "copy_calibration_bytes_written_per_launch": a.numel() * 8, "launches": 5}))
        return 0
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU: the library has no multi-GPU path (row "
                                   "sharding with one all-reduce per reduction is a design, not code)",
                          "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    from paper_2503_16717_amd import binding as B
    from paper_2503_16717_amd import workloads as wl

    n = args.n
    N = NB * W
    log(f"generating {NB} blocks of {n} x {W} (kappa 1e{LOG10_COND:g}) and uploading")
    t0 = time.perf_counter()
    Vd = build_inputs(n, torch, wl)
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s")
    Qd = torch.empty((N, n), dtype=torch.float64, device="cuda").t()
    ctx = B.Context(0)
    opts = B.orth_opts(intra="randcholqr", sketch=B.make_sketch("sparse_sign", SK_K, SK_ZETA, SK_SEED))
    R = np.zeros((N, N), order="F")

    def step(o=opts):
        st, col = ctx.sko_orth_blocks(n, NB, W, Vd.data_ptr(), n, Qd.data_ptr(), n, R, N, o)
        if st != B.SKO_OK:
            raise B.SkoError(st, "sko_orth_blocks", col)

    # launch shapes tuned once per context and workload (before any timing)
    t_tune = time.perf_counter()
    opts2 = B.orth_opts(two_stage=True, panels_per_big=6, reorth=True,
                        sketch=B.make_sketch("sparse_sign", SK_K, SK_ZETA, SK_SEED))
    if not args.no_autotune:
        for o in (opts, opts2):
            st = ctx.sko_autotune_orth(n, NB, W, o)
            if st != B.SKO_OK:
                raise B.SkoError(st, "sko_autotune_orth")
        torch.cuda.synchronize()
    t_tune = time.perf_counter() - t_tune
    log(f"autotune: {t_tune:.2f} s")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    R_first = R.copy() if args.warmup > 0 else None
    log("warmup done; timing")
    # Region 1 (the reported throughput): K steps with one event per step only.
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for i in range(args.steps):
        step()
        evs[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps))
    ms = (t1 - t0) / args.steps * 1e3
    # Region 2 (the per-kernel durations of the roofline): the same K steps with the library's
    # event pair around every launch, on the stream the kernels run on.  The events add about
    # a millisecond of gaps per step, so the throughput above is taken without them.
    ctx.sko_profile_enable(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_profiled = (time.perf_counter() - t2) / args.steps * 1e3
    ctx.sko_profile_enable(False)
    stats = ctx.sko_profile_read()
    abytes = alg_bytes_one_stage(n, NB, W)
    value = abytes / (ms * 1e-3) / 1e9
    log(f"one-stage: {ms:.3f} ms/step, {value:.1f} GB/s algorithmic")

    dom = stats[0]
    avg_ms = dom["total_ms"] / dom["launches"]
    avg_bytes = dom["bytes"] / dom["launches"]
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom["name"])
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom["name"], "launches_per_step": dom["launches"] / args.steps,
                "avg_launch_ms": round(avg_ms, 4), "alg_bytes_per_launch": avg_bytes,
                "timing": "per-launch event pairs over a second timed region of the same steps"}
    kernels = [{"name": s["name"], "ms_per_step": round(s["total_ms"] / args.steps, 4),
                "launches_per_step": s["launches"] / args.steps,
                "GBps": round(s["bytes"] / (s["total_ms"] * 1e-3) / 1e9, 1) if s["total_ms"] > 0 else None}
               for s in stats[:8]]
    event_ms = sum(s["total_ms"] for s in stats) / args.steps

    # correctness guard on the benchmarked output: finite Q samples, a positive diagonal,
    # and the same R bit for bit as the first warm-up step
    Qs = Qd[:: max(1, n // 65536)]
    same = R_first is None or np.array_equal(R, R_first)
    if not (torch.isfinite(Qs).all().item() and np.all(np.diag(R) > 0) and same):
        log(f"R check failed: diag min {np.diag(R).min():.3e}, equal to first step: {same}")
        log("diag: " + " ".join(f"{v:.3e}" for v in np.diag(R)))
        return 3

    extra = {"kernels_top": kernels, "event_ms_per_step": round(event_ms, 3),
             "ms_per_step_with_launch_events": round(ms_profiled, 4),
             "step_ms_median": round(step_ms[len(step_ms) // 2], 4), "step_ms_min": round(step_ms[0], 4),
             "alg_bytes_per_step": abytes, "autotune_s": None if args.no_autotune else round(t_tune, 3)}

    if not args.skip_two_stage:
        # two-stage variant of the same workload (s_hat = 30: 6 blocks per big panel, W = 36)
        for _ in range(args.warmup):
            step(opts2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(opts2)
        torch.cuda.synchronize()
        ms2 = (time.perf_counter() - t0) / args.steps * 1e3
        # per-kernel breakdown from a second region with launch events
        ctx.sko_profile_enable(True)
        for _ in range(args.steps):
            step(opts2)
        torch.cuda.synchronize()
        ctx.sko_profile_enable(False)
        stats2 = ctx.sko_profile_read()
        ab2 = alg_bytes_two_stage_method(n, NB, W, 6)
        ex2 = alg_bytes_two_stage(n, NB, W, 6)
        extra["two_stage"] = {"ms_per_step": round(ms2, 4), "GBps": round(ab2 / (ms2 * 1e-3) / 1e9, 2),
                              "pct_hbm_peak": round(100 * ab2 / (ms2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 2),
                              "alg_bytes_per_step": ab2, "executed_schedule_bytes_per_step": ex2,
                              "s_hat": 30, "big_panel_width": 36,
                              "kernels_top": [{"name": q["name"], "ms_per_step": round(q["total_ms"] / args.steps, 4),
                                               "launches_per_step": q["launches"] / args.steps,
                                               "GBps": round(q["bytes"] / (q["total_ms"] * 1e-3) / 1e9, 1)
                                               if q["total_ms"] > 0 else None} for q in stats2[:10]]}
        log(f"two-stage: {ms2:.3f} ms/step")
    ceiling = copy_ceiling(torch)
    extra["copy_ceiling_GBps"] = round(ceiling, 1)
    extra["pct_of_copy_ceiling"] = round(100.0 * value / ceiling, 2)
    ctx.close()
    del Qd
    if not (args.skip_gmres and args.skip_c3):
        del Vd
        torch.cuda.empty_cache()
    if not args.skip_c3:
        extra["config3_mixed_blockorth"] = c3_suite(B, torch, wl, n, args.no_autotune)
    if not args.skip_gmres:
        extra["gmres"] = gmres_suite(B, torch, wl, args)
    if not args.skip_next_rows:
        extra["next_rows"] = next_rows_suite(B, torch, wl, n)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline on {args.cpu_sample_rows} rows")
        cpu = cpu_baseline(args.cpu_sample_rows)

    line = {
        "metric": "block-orth GB/s (% HBM peak); time to 1e-10 residual, mixed/batched vs FP64",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "standalone block orthogonalization: n=2^24 rows, 12 blocks x 6 columns "
                               "(s=5), kappa=1e12 per block, one-stage RandCholQR-BCGS2, sparse-sign "
                               "sketch k=64 zeta=8, FP64",
                   "n": n, "blocks": NB, "block_width": W, "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
