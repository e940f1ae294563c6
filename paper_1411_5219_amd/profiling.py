"""Summaries of rocprofv3 output databases (kernel traces and counters).

    python -m paper_1411_5219_amd.profiling stats  <results.db> [name-filter]
    python -m paper_1411_5219_amd.profiling counters <results.db> [name-filter]
    python -m paper_1411_5219_amd.profiling bursts <results.db> [--min-len N]
    python -m paper_1411_5219_amd.profiling traffic --fetch <db> --write <db> [--kernel K] [--copy-bytes N]

``stats`` lists calls, total and mean duration per kernel, and for each
kernel also the mean over dispatches that did work: solver kernels whose
control block says "converged" return at once (a few microseconds), and
those predicated no-op launches are counted separately.

``bursts`` picks out runs of at least N back-to-back dispatches of one
kernel with one grid (the Dslash bursts that bench.py times with HIP
events) and gives their mean duration per kernel.

``traffic`` turns FETCH_SIZE / WRITE_SIZE passes into bytes per dispatch of a
kernel, each scaled by what the same counter reads for the plain copy of
known size that the profiled program runs (rocclr's copyBuffer).

``kernel_source_digest()`` hashes the sources the Dslash kernel is built
from, so recorded counters can be matched to the kernel they were taken on.
"""

from __future__ import annotations

import argparse
import hashlib
import os
import sqlite3
import statistics
import sys
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/dslash_impl.h", "csrc/block_order.h", "csrc/dslash.hip", "csrc/lqcd_device.h", "csrc/lqcd_kernels.h"]


# sources of the pseudo-fermion force kernel
FORCE_SOURCES = ["csrc/force.hip", "csrc/dslash_impl.h", "csrc/block_order.h", "csrc/lqcd_device.h",
                 "csrc/lqcd_kernels.h"]


def kernel_source_digest(sources=None) -> str:
    h = hashlib.sha256()
    for rel in sources or KERNEL_SOURCES:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _rows(db, query):
    con = sqlite3.connect(db)
    try:
        return con.execute(query).fetchall()
    finally:
        con.close()


def kernel_stats(db, name_filter="", busy_us=10.0):
    d = defaultdict(list)
    for name, dur in _rows(db, "select name, duration from kernels"):
        if name_filter in name:
            d[name].append(dur / 1e3)
    out = []
    for name, du in d.items():
        busy = [x for x in du if x > busy_us]
        out.append({"name": name, "calls": len(du), "total_us": sum(du), "mean_us": sum(du) / len(du),
                    "busy_calls": len(busy), "busy_mean_us": (sum(busy) / len(busy)) if busy else 0.0,
                    "busy_median_us": statistics.median(busy) if busy else 0.0})
    out.sort(key=lambda r: -r["total_us"])
    return out


def bursts(db, min_len=20):
    rows = _rows(db, "select name, grid_x, grid_y, workgroup_x, duration from kernels order by start")
    runs, cur = [], []
    for r in rows:
        if cur and (r[0], r[1], r[2], r[3]) != cur[-1][:4]:
            runs.append(cur)
            cur = []
        cur.append(r)
    if cur:
        runs.append(cur)
    out = defaultdict(list)
    for run in runs:
        if len(run) >= min_len:
            out[(run[0][0], run[0][1] // run[0][3], run[0][2], run[0][3])].append([x[4] / 1e3 for x in run])
    res = []
    for (name, blocks, gy, wx), rs in out.items():
        du = [x for r in rs for x in r]
        res.append({"name": name, "blocks": blocks, "grid_y": gy, "block": wx, "bursts": len(rs), "calls": len(du),
                    "mean_us": sum(du) / len(du), "median_us": statistics.median(du)})
    return res


def counters(db, name_filter=""):
    d = defaultdict(lambda: defaultdict(list))
    q = "select dispatch_id, kernel_name, counter_name, value from counters_collection order by dispatch_id"
    for _, name, cn, v in _rows(db, q):
        if name_filter in name:
            d[name][cn].append(v)
    return d


def traffic(fetch_db, write_db, kernel, copy_bytes=1 << 30):
    f = counters(fetch_db)
    w = counters(write_db)
    copy_f = [v for n, c in f.items() if "copyBuffer" in n for v in c.get("FETCH_SIZE", [])]
    copy_w = [v for n, c in w.items() if "copyBuffer" in n for v in c.get("WRITE_SIZE", [])]
    kf = [v for n, c in f.items() if kernel in n for v in c.get("FETCH_SIZE", [])]
    kw = [v for n, c in w.items() if kernel in n for v in c.get("WRITE_SIZE", [])]
    if not (copy_f and copy_w and kf and kw):
        raise SystemExit("missing dispatches in the counter databases")
    ff = copy_bytes / (statistics.median(copy_f) * 1024)
    fw = copy_bytes / (statistics.median(copy_w) * 1024)
    return {"fetch_kib_median": statistics.median(kf), "write_kib_median": statistics.median(kw),
            "copy_fetch_kib": statistics.median(copy_f), "copy_write_kib": statistics.median(copy_w),
            "fetch_factor": ff, "write_factor": fw,
            "read_bytes": statistics.median(kf) * 1024 * ff, "write_bytes": statistics.median(kw) * 1024 * fw,
            "dispatches": (len(kf), len(kw))}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("filter", nargs="?", default="")
    c = sub.add_parser("counters")
    c.add_argument("db")
    c.add_argument("filter", nargs="?", default="")
    b = sub.add_parser("bursts")
    b.add_argument("db")
    b.add_argument("--min-len", type=int, default=20)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", default="k_dslash_eo<64, 18, false, 0, 1, true>")
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(f"{'calls':>6} {'total_us':>12} {'mean_us':>10} {'busy_calls':>10} {'busy_mean_us':>12}  kernel")
        for r in kernel_stats(a.db, a.filter):
            print(f"{r['calls']:>6} {r['total_us']:>12.1f} {r['mean_us']:>10.2f} {r['busy_calls']:>10} "
                  f"{r['busy_mean_us']:>12.2f}  {r['name']}")
    elif a.cmd == "bursts":
        print(f"{'bursts':>6} {'calls':>6} {'mean_us':>9} {'median_us':>9} {'blocks':>7} {'block':>5}  kernel")
        for r in bursts(a.db, a.min_len):
            print(f"{r['bursts']:>6} {r['calls']:>6} {r['mean_us']:>9.2f} {r['median_us']:>9.2f} {r['blocks']:>7} "
                  f"{r['block']:>5}  {r['name']}")
    elif a.cmd == "counters":
        for name, cs in counters(a.db, a.filter).items():
            for cn, vals in cs.items():
                print(f"{name}  {cn}  n={len(vals)} median={statistics.median(vals):.0f}")
    else:
        r = traffic(a.fetch, a.write, a.kernel, a.copy_bytes)
        for k, v in r.items():
            print(f"{k} = {v}")
        print(f"kernel_source_digest = {kernel_source_digest()}")


if __name__ == "__main__":
    sys.exit(main())
