"""Summarise a rocprofv3 result database (rocpd SQLite) as short text.

    python -m paper_1811_06332_amd.profile_summary stats   RESULTS.db
    python -m paper_1811_06332_amd.profile_summary counter RESULTS.db COUNTER [COPY_BYTES]
    python -m paper_1811_06332_amd.profile_summary tail    RESULTS.db PREFIX K
    python -m paper_1811_06332_amd.profile_summary record  TRACE.db PREFIX K [PMC.db ...] -- SOURCES... > X.json

`stats`: per-kernel dispatch count, total and average duration.
`tail`: the last K dispatches (in start order) of the kernels whose name
starts with PREFIX, and their average duration: the timed steps of a run whose
earlier dispatches of the same kernel are warm-up and tuning launches.
`record`: a JSON record of one kernel for bench.py: the average duration of
its last K dispatches in the kernel trace, the per-dispatch averages of the
PMC counters of its last K dispatches in each counter run (MFMA MOPS, MFMA
busy cycles, GRBM_GUI_ACTIVE ...), the MFMA utilisation and issued MFMA
flops derived from them, and a hash of the kernel's source files so that
the record is used only while it describes the built kernel.
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
    per = {}
    for name, c in _pmc_dispatches(db).values():
        if cname in c:
            per.setdefault(name, []).append(c[cname])
    rows = sorted(((name, len(v), sum(v) / len(v)) for name, v in per.items()), key=lambda r: -r[2])
    scale = None
    if copy_bytes:
        # the single largest dispatch of a copy kernel is the known-size reference copy
        best = max((max(v) for name, v in per.items() if "copy" in name.lower()), default=None)
        if best:
            scale = copy_bytes / (best * 1024.0)
    out = [f"counter {cname}" + (f"; copy-kernel scale factor {scale:.4f} (bytes per counted byte)" if scale else "")]
    out.append(f"{'kernel':72s} {'calls':>6s} {'avg_KiB':>14s}" + (f" {'scaled_MB':>12s}" if scale else ""))
    for name, n, val in rows:
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


def _pmc_dispatches(db: str):
    """{dispatch: (kernel name, {counter: value})} from a counter run: the
    rows of one dispatch (one per hardware instance of a counter) summed,
    GRBM counters (one clock per instance) reduced by max, as rocprofv3's
    derived metrics do."""
    cur = sqlite3.connect(db).cursor()
    cols = [r[1] for r in cur.execute("PRAGMA table_info(pmc_events)").fetchall()]
    key = "dispatch_id" if "dispatch_id" in cols else None
    order = next((c for c in ("start", "dispatch_id", "id") if c in cols), None)
    rows = cur.execute(f"select name, counter_name, counter_value, {key or 'NULL'} from pmc_events" +
                       (f" order by {order}" if order else "")).fetchall()
    disp = {}
    for i, (name, cname, val, did) in enumerate(rows):
        d = disp.setdefault(did if key else i, (name, {}))[1]
        if cname.startswith("GRBM_"):
            d[cname] = max(d.get(cname, 0.0), float(val))
        else:
            d[cname] = d.get(cname, 0.0) + float(val)
    return disp


def _pmc_last(db: str, prefix: str, k: int) -> dict:
    """Per-dispatch counter values averaged over the last k dispatches of
    the kernels starting with prefix."""
    sel = [c for name, c in _pmc_dispatches(db).values() if _short(name).startswith(prefix)][-k:]
    names = sorted({n for c in sel for n in c})
    return {n: sum(c.get(n, 0.0) for c in sel) / len(sel) for n in names} if sel else {}


def source_hash(root: str, sources) -> str:
    import hashlib
    import os
    h = hashlib.sha256()
    for src in sources:
        h.update(open(os.path.join(root, src), "rb").read())
    return h.hexdigest()[:16]


def record(trace_db: str, prefix: str, k: int, pmc_dbs, sources) -> dict:
    import os
    cur = sqlite3.connect(trace_db).cursor()
    rows = [r for r in cur.execute("select name, start, duration from kernels order by start").fetchall()
            if _short(r[0]).startswith(prefix)]
    last = rows[-k:]
    out = {"kernel_prefix": prefix, "kernels": sorted({_short(r[0]) for r in last}),
           "dispatches": len(last), "avg_launch_ms": sum(r[2] for r in last) / max(len(last), 1) / 1e6}
    counters = {}
    for db in pmc_dbs:
        counters.update(_pmc_last(db, prefix, k))
    out["counters_per_dispatch"] = counters
    simd = 256 * 4  # MI355X: 256 CUs of 4 SIMDs
    if "SQ_VALU_MFMA_BUSY_CYCLES" in counters and counters.get("GRBM_GUI_ACTIVE"):
        out["mfma_util"] = counters["SQ_VALU_MFMA_BUSY_CYCLES"] / (counters["GRBM_GUI_ACTIVE"] * simd)
    mops = sum(v for c, v in counters.items() if c.startswith("SQ_INSTS_VALU_MFMA_MOPS_"))
    if mops:
        out["issued_mfma_flops"] = mops * 512.0
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out["kernel_sources"] = list(sources)
    out["kernel_sources_sha256_16"] = source_hash(root, sources)
    return out


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        print(stats(argv[1]))
    elif len(argv) >= 4 and argv[0] == "tail":
        print(tail(argv[1], argv[2], int(argv[3])))
    elif len(argv) >= 4 and argv[0] == "record":
        import json
        sep = argv.index("--") if "--" in argv else len(argv)
        print(json.dumps(record(argv[1], argv[2], int(argv[3]), argv[4:sep], argv[sep + 1:]), indent=1))
    elif len(argv) >= 3 and argv[0] == "counter":
        print(counter(argv[1], argv[2], float(argv[3]) if len(argv) > 3 else None))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
