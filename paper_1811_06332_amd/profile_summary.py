"""Summarise a rocprofv3 result database (rocpd SQLite) as short text.

    python -m paper_1811_06332_amd.profile_summary stats   RESULTS.db
    python -m paper_1811_06332_amd.profile_summary counter RESULTS.db COUNTER [COPY_BYTES]
    python -m paper_1811_06332_amd.profile_summary tail    RESULTS.db PREFIX K

`stats`: per-kernel dispatch count, total and average duration.
`tail`: the last K dispatches (in start order) of the kernels whose name
starts with PREFIX, and their average duration: the timed steps of a run whose
earlier dispatches of the same kernel are warm-up and tuning launches.
`counter`: per-kernel average of one PMC counter (e.g. FETCH_SIZE, WRITE_SIZE,
in KiB per dispatch as rocprofv3 reports them).  With COPY_BYTES, the counter
of the largest plain copy kernel in the run (a device-to-device copy of known
size, `bench.py --copy-calibration`) gives the scale factor
bytes / (counter KiB * 1024) applied to every kernel, printed as scaled MB per
dispatch.
"""
from __future__ import annotations

import sqlite3
import sys


def _short(name: str, width: int = 70) -> str:
    name = name.replace("void ctfmm::", "").replace("ctfmm::", "")
    return name if len(name) <= width else name[: width - 3] + "..."


def stats(db: str) -> str:
    cur = sqlite3.connect(db).cursor()
    rows = cur.execute("select name, count(*), sum(duration), avg(duration) from kernels "
                       "group by name order by sum(duration) desc").fetchall()
    tot = sum(r[2] for r in rows) or 1
    out = [f"{'kernel':72s} {'calls':>6s} {'total_ms':>10s} {'avg_ms':>10s} {'%':>6s}"]
    for name, n, total, avg in rows:
        out.append(f"{_short(name):72s} {n:6d} {total / 1e6:10.3f} {avg / 1e6:10.4f} {100 * total / tot:6.2f}")
    return "\n".join(out)


def counter(db: str, cname: str, copy_bytes: float | None = None) -> str:
    cur = sqlite3.connect(db).cursor()
    rows = cur.execute("select name, count(*), avg(counter_value), avg(duration) from pmc_events "
                       "where counter_name = ? group by name order by avg(counter_value) desc", (cname,)).fetchall()
    scale = None
    if copy_bytes:
        # the single largest dispatch of a copy kernel is the known-size reference copy
        best = cur.execute("select max(counter_value) from pmc_events where counter_name = ? and "
                           "lower(name) like '%copy%'", (cname,)).fetchone()[0]
        if best:
            scale = copy_bytes / (best * 1024.0)
    out = [f"counter {cname}" + (f"; copy-kernel scale factor {scale:.4f} (bytes per counted byte)" if scale else "")]
    out.append(f"{'kernel':72s} {'calls':>6s} {'avg_KiB':>14s}" + (f" {'scaled_MB':>12s}" if scale else ""))
    for name, n, val, dur in rows:
        line = f"{_short(name):72s} {n:6d} {val:14.1f}"
        if scale:
            line += f" {val * 1024.0 * scale / 1e6:12.2f}"
        out.append(line)
    return "\n".join(out)


def tail(db: str, prefix: str, k: int) -> str:
    cur = sqlite3.connect(db).cursor()
    rows = [r for r in cur.execute("select name, start, duration from kernels order by start").fetchall()
            if _short(r[0]).startswith(prefix)]
    last = rows[-k:]
    if not last:
        return f"no dispatch of {prefix}"
    avg = sum(r[2] for r in last) / len(last)
    names = sorted({_short(r[0]) for r in last})
    return (f"last {len(last)} dispatches of {prefix}* (the timed steps): average {avg / 1e6:.4f} ms; "
            f"kernel {', '.join(names)}")


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        print(stats(argv[1]))
    elif len(argv) >= 4 and argv[0] == "tail":
        print(tail(argv[1], argv[2], int(argv[3])))
    elif len(argv) >= 3 and argv[0] == "counter":
        print(counter(argv[1], argv[2], float(argv[3]) if len(argv) > 3 else None))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
