"""Summaries of rocprofv3 output for the pass kernels (markdown tables on stdout).

    python -m paper_2503_16717_amd.rocprof_summary stats KERNEL_STATS_CSV [--top N]
    python -m paper_2503_16717_amd.rocprof_summary traffic --fetch CSV --write CSV \\
        --copy-fetch CSV --copy-write CSV --copy-bytes BYTES [--all --source FILE --top N]
    python -m paper_2503_16717_amd.rocprof_summary last KERNEL_TRACE_CSV --kernel NAME --last N
    python -m paper_2503_16717_amd.rocprof_summary requests --reads CSV --writes CSV \\
        --copy-reads CSV --copy-writes CSV --copy-bytes BYTES [--since KERNEL:N]

`stats` lists the kernels of a `--kernel-trace --stats` run by total time.  `traffic`
turns two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs (KiB per dispatch) into HBM bytes
per launch of each pass kernel.  Each counter is scaled by the factor that makes it read
the known size of a plain device copy (`bench.py --copy-calibration`: read and written
bytes per launch given by --copy-bytes).  Pass kernels are named as the library's
profiler names them (sko_profile_read), and each row carries the digest of the pass-kernel
sources (pass_impl.h and uniform.h), so a reader can tell whether the counts still describe the current kernels.  With
--all every kernel is listed (others under their demangled names), with the digest of the
source file given by --source.  --since KERNEL:N keeps the dispatches from the N-th last
dispatch of KERNEL on.  `requests` gives the same bytes from the L2-to-memory request
counters by request size (TCC_EA0_RDREQ_32B/64B/128B, TCC_EA0_WRREQ and _64B), which need
no calibration factor: on this chip every read of a streamed operand is one 128-byte
request, which FETCH_SIZE's formula counts as 64 bytes (hence its factor of two on the copy).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import re
import sys
from collections import defaultdict

_REDS = ["none", "proj", "gram", "sketch_sparse", "sketch_dense"]
_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
# the pass kernels' source: the kernel bodies and the row-update helpers they include
PASS_SOURCES = (os.path.join(_CSRC, "pass_impl.h"), os.path.join(_CSRC, "uniform.h"))


def source_digest(paths=PASS_SOURCES) -> str:
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def profiler_name(kernel: str) -> str | None:
    """'void sko::passk::pass_kernel<6, double, 1, false, 0, false, 4>(...)' -> the name the
    library's profiler gives the same launch ('pass W=6 f64 red=proj/mt4 upd=0 trsm=0 write=0')."""
    m = re.search(r"pass_kernel(?:_batched)?<(\d+), (double|float), (\d), (true|false), (\d), (true|false)"
                  r"(?:, (\d+))?>", kernel)
    if not m:
        return None
    w, t, red, upd, ntrsm, write, mtx = m.groups()
    red = int(red)
    mt = ""
    if red == 1:
        mt = f"/mt{int(mtx)}" if mtx is not None and int(mtx) in (4, 6) else "/mt8"
    return (f"pass W={w} {'f32' if t == 'float' else 'f64'} red={_REDS[red]}{mt} upd={int(upd == 'true')} "
            f"trsm={ntrsm} write={int(write == 'true')}")


def short_name(kernel: str) -> str:
    p = profiler_name(kernel)
    if p:
        return p
    k = re.sub(r"\([^()]*\)$", "", kernel)
    return k[:80]


def counter_means(path: str, counter: str, since: str | None = None) -> dict[str, tuple[int, float]]:
    """Kernel name -> (dispatches, mean counter value).  With since = 'KERNEL:N' only the
    dispatches from the N-th last dispatch of KERNEL on are counted (the pipeline's steps,
    not the launch-shape tuner's candidate launches that precede them)."""
    rows = [r for r in csv.DictReader(open(path)) if r.get("Counter_Name") == counter]
    first = since_dispatch(rows, since)
    acc = defaultdict(list)
    for row in rows:
        if int(row["Dispatch_Id"]) >= first:
            acc[row["Kernel_Name"]].append(float(row["Counter_Value"]))
    return {k: (len(v), sum(v) / len(v)) for k, v in acc.items()}


def since_dispatch(rows, since: str | None) -> int:
    if not since:
        return 0
    kernel, n = since.rsplit(":", 1)
    ids = sorted(int(r["Dispatch_Id"]) for r in rows if short_name(r["Kernel_Name"]) == kernel)
    if len(ids) < int(n):
        raise SystemExit(f"{kernel}: {len(ids)} dispatches, fewer than {n}")
    return ids[-int(n)]


def cmd_stats(a) -> int:
    rows = list(csv.DictReader(open(a.csv)))
    print("| kernel | calls | average µs | total ms | % of kernel time |")
    print("|---|---:|---:|---:|---:|")
    for r in rows[: a.top]:
        print(f"| {short_name(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
              f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    return 0


def cmd_last(a) -> int:
    """Average duration of the last N dispatches of one kernel (by profiler name or a
    substring of the demangled name): the launches of the timed steps, after any tuning."""
    rows = [r for r in csv.DictReader(open(a.csv))
            if a.kernel == short_name(r["Kernel_Name"]) or a.kernel in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows][-a.last:]
    if not d:
        print("no dispatches of", a.kernel, file=sys.stderr)
        return 1
    print(f"{a.kernel}: {len(d)} dispatches, average {sum(d) / len(d):.1f} µs")
    return 0


def cmd_traffic(a) -> int:
    cf = counter_means(a.copy_fetch, "FETCH_SIZE")
    cw = counter_means(a.copy_write, "WRITE_SIZE")
    copy = [k for k in cf if "copyBuffer" in k]
    if not copy or copy[0] not in cw:
        print("no copy kernel in the calibration runs", file=sys.stderr)
        return 1
    fr = a.copy_bytes / (cf[copy[0]][1] * 1024.0)
    fw = a.copy_bytes / (cw[copy[0]][1] * 1024.0)
    pf = counter_means(a.fetch, "FETCH_SIZE", a.since)
    pw = counter_means(a.write, "WRITE_SIZE", a.since)
    dig = source_digest(a.source) if a.source else source_digest()
    print(f"Calibration (plain copy of {a.copy_bytes} bytes): FETCH_SIZE x {fr:.4f}, WRITE_SIZE x {fw:.4f}")
    print()
    print("| kernel | HBM read bytes / launch | HBM write bytes / launch | HBM bytes / launch | source digest |")
    print("|---|---:|---:|---:|---|")
    shown = 0
    for k in sorted(pf, key=lambda k: -pf[k][1] * pf[k][0]):
        name = short_name(k) if a.all else profiler_name(k)
        if not name or k not in pw or (a.top and shown >= a.top):
            continue
        shown += 1
        rb = pf[k][1] * 1024.0 * fr
        wb = pw[k][1] * 1024.0 * fw
        print(f"| {name} | {rb:.4g} | {wb:.4g} | {rb + wb:.6g} | {dig} |")
    return 0


_READ_REQS = (("TCC_EA0_RDREQ_32B_sum", 32), ("TCC_EA0_RDREQ_64B_sum", 64), ("TCC_EA0_RDREQ_128B_sum", 128))


def request_bytes(read_csv: str, write_csv: str, since: str | None):
    """Kernel name -> (read bytes, write bytes) per dispatch from the L2-to-memory request
    counters: read requests by size (32, 64 or 128 bytes) and write requests (64 bytes, the
    rest 32)."""
    rd = {c: counter_means(read_csv, c, since) for c, _ in _READ_REQS}
    wr = {c: counter_means(write_csv, c, since) for c in ("TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum")}
    out = {}
    for k in rd["TCC_EA0_RDREQ_128B_sum"]:
        if k not in wr["TCC_EA0_WRREQ_sum"]:
            continue
        rb = sum(rd[c].get(k, (0, 0.0))[1] * size for c, size in _READ_REQS)
        w64 = wr["TCC_EA0_WRREQ_64B_sum"].get(k, (0, 0.0))[1]
        wb = w64 * 64 + (wr["TCC_EA0_WRREQ_sum"][k][1] - w64) * 32
        out[k] = (rd["TCC_EA0_RDREQ_128B_sum"][k][0], rb, wb)
    return out


def cmd_requests(a) -> int:
    cp = request_bytes(a.copy_reads, a.copy_writes, None)
    copy = [k for k in cp if "copyBuffer" in k]
    if not copy:
        print("no copy kernel in the calibration runs", file=sys.stderr)
        return 1
    _, crb, cwb = cp[copy[0]]
    print(f"Plain copy of {a.copy_bytes:.0f} bytes: read requests give {crb:.6g} bytes "
          f"(x {crb / a.copy_bytes:.4f}), write requests {cwb:.6g} bytes (x {cwb / a.copy_bytes:.4f})")
    print()
    print("| kernel | dispatches | HBM read bytes / launch | HBM write bytes / launch | HBM bytes / launch |")
    print("|---|---:|---:|---:|---:|")
    pk = request_bytes(a.reads, a.writes, a.since)
    for k in sorted(pk, key=lambda k: -(pk[k][1] + pk[k][2]) * pk[k][0]):
        name = profiler_name(k)
        if name:
            d, rb, wb = pk[k]
            print(f"| {name} | {d} | {rb:.4g} | {wb:.4g} | {rb + wb:.6g} |")
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=15)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--all", action="store_true", help="list every kernel, not only the pass kernels")
    t.add_argument("--source", action="append", default=None,
                   help="source file whose digest the rows carry (repeat for several, hashed in order)")
    t.add_argument("--top", type=int, default=0, help="at most this many kernels (by total fetch)")
    t.add_argument("--since", default=None, help="KERNEL:N, count from the N-th last dispatch of KERNEL on")
    q = sub.add_parser("requests")
    for o in ("--reads", "--writes", "--copy-reads", "--copy-writes"):
        q.add_argument(o, required=True)
    q.add_argument("--copy-bytes", type=float, required=True)
    q.add_argument("--since", default=None, help="KERNEL:N, count from the N-th last dispatch of KERNEL on")
    la = sub.add_parser("last")
    la.add_argument("csv")
    la.add_argument("--kernel", required=True)
    la.add_argument("--last", type=int, required=True)
    a = ap.parse_args(argv)
    return {"stats": cmd_stats, "traffic": cmd_traffic, "last": cmd_last, "requests": cmd_requests}[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
