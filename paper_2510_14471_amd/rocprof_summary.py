"""Text summaries of rocprofv3 result databases, and the copy kernel that
calibrates the HBM traffic counters.

    python -m paper_2510_14471_amd.rocprof_summary stats DB [--top N]
        per-kernel launches, total and average duration (kernel trace)
    python -m paper_2510_14471_amd.rocprof_summary pmc DB [--regex RE]
        per-kernel dispatch count and average counter value per dispatch
    python -m paper_2510_14471_amd.rocprof_summary copy [--mib N] [--reps R]
        launches R plain device-to-device copies of N MiB (the calibration
        kernel: it reads and writes exactly N MiB per dispatch)

DB is the `*_results.db` SQLite file rocprofv3 writes (rocpd format).
"""
from __future__ import annotations

import argparse
import glob
import os
import re
import sqlite3
import sys


def _db(path: str) -> sqlite3.Connection:
    if os.path.isdir(path):
        found = sorted(glob.glob(os.path.join(path, "**", "*.db"), recursive=True))
        if not found:
            raise SystemExit(f"no rocprofv3 database under {path}")
        path = found[0]
    return sqlite3.connect(path)


def stats(path: str, top: int = 15) -> str:
    c = _db(path)
    rows = c.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
        "from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1
    out = [f"{'kernel':<90} {'calls':>7} {'total_ms':>10} {'avg_us':>10} {'min_us':>9} "
           f"{'max_us':>9} {'pct':>6}"]
    for name, n, tot, avg, mn, mx in rows[:top]:
        out.append(f"{name[:90]:<90} {n:>7d} {tot / 1e6:>10.3f} {avg / 1e3:>10.2f} "
                   f"{mn / 1e3:>9.2f} {mx / 1e3:>9.2f} {100.0 * tot / total:>5.1f}%")
    out.append(f"all kernels: {sum(r[1] for r in rows)} launches, {total / 1e6:.3f} ms")
    return "\n".join(out)


def pmc(path: str, regex: str = ".") -> str:
    c = _db(path)
    pat = re.compile(regex)
    rows = c.execute(
        "select kernel_name, counter_name, count(*), avg(value), sum(value) "
        "from counters_collection group by kernel_name, counter_name "
        "order by kernel_name, counter_name").fetchall()
    out = [f"{'kernel':<90} {'counter':<14} {'dispatches':>10} {'avg/dispatch':>14} {'sum':>16}"]
    for name, ctr, n, avg, tot in rows:
        if pat.search(name):
            out.append(f"{name[:90]:<90} {ctr:<14} {n:>10d} {avg:>14.6g} {tot:>16.6g}")
    return "\n".join(out)


def copy(mib: int = 2048, reps: int = 5) -> str:
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    return f"copied {mib} MiB x {reps} (bytes read and written per dispatch: {mib * (1 << 20)})"


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2510_14471_amd.rocprof_summary")
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("db")
    a.add_argument("--top", type=int, default=15)
    b = sub.add_parser("pmc")
    b.add_argument("db")
    b.add_argument("--regex", default=".")
    d = sub.add_parser("copy")
    d.add_argument("--mib", type=int, default=2048)
    d.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print(stats(args.db, args.top))
    elif args.cmd == "pmc":
        print(pmc(args.db, args.regex))
    else:
        print(copy(args.mib, args.reps), flush=True)


if __name__ == "__main__":
    sys.exit(main())
