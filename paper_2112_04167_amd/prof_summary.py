"""Summarise rocprofv3 result databases (kernel trace + FETCH_SIZE / WRITE_SIZE
counter passes) into a short text report.

    python -m paper_2112_04167_amd.prof_summary --trace T.db --fetch F.db \
        --write W.db --kernel k_apply --calib __amd_rocclr_copyBuffer \
        --calib-bytes 1073741824 --algo-bytes 268435456 --cmd "..." > report.md

The counters of a plain copy kernel of known size give the factor between
what FETCH_SIZE / WRITE_SIZE read and the bytes actually moved; the apply
kernel's per-dispatch counters are scaled by those factors.
"""
import argparse
import hashlib
import json
import os
import sqlite3

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f)
                  for f in ("kernels.hip", "apply_core.h", "device_common.h", "gll_constexpr.h")]


def kernel_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def trace_stats(db, pattern):
    c = sqlite3.connect(db)
    rows = c.execute("select name, total_calls, total_duration, average, percentage "
                     "from top_kernels").fetchall()
    out = []
    for name, calls, tot, avg, pct in rows:
        out.append((name, calls, tot, avg, pct))
    sel = [r for r in out if pattern in r[0]]
    return out, sel


def trace_since(db, since, until=None, exclude=None):
    """Per-kernel totals over the dispatches from the first one whose name
    contains `since` onward (up to, not including, the first later one whose
    name contains `until`; leaving out names that contain `exclude`):
    [(name, calls, total_ns, avg_ns, pct)], and the wall span of the window
    in ns."""
    c = sqlite3.connect(db)
    rows = c.execute("select name, start, end, duration from kernels order by start").fetchall()
    t0 = next(r[1] for r in rows if since in r[0])
    sel = [r for r in rows if r[1] >= t0]
    if until:
        stop = next((i for i, r in enumerate(sel) if until in r[0]), len(sel))
        sel = sel[:stop]
    span = sel[-1][2] - sel[0][1]
    if exclude:
        sel = [r for r in sel if exclude not in r[0]]
    agg = {}
    for name, st, en, d in sel:
        a = agg.setdefault(name, [0, 0.0])
        a[0] += 1
        a[1] += d
    tot = sum(a[1] for a in agg.values())
    out = [(k, a[0], a[1], a[1] / a[0], 100.0 * a[1] / tot) for k, a in agg.items()]
    out.sort(key=lambda r: -r[2])
    return out, span


def range_stats(db, outer, skip=0, count=None):
    """Host-side marker ranges (rocprofv3 --marker-trace) inside the ranges
    named `outer`, taking those from the skip-th on (count of them, or all):
    [(name, calls, total_ns)] of the ranges on the same thread that lie
    within them, the outer ranges' total duration in ns, how many there were,
    and the kernel time of the dispatches that started within them."""
    c = sqlite3.connect(db)
    rows = []
    # a ROCTx range is recorded under its API call's name; its message is in
    # the record's extdata
    for name, ext, tid, st, en in c.execute("select name, extdata, tid, start, end from regions "
                                           "where category like '%MARKER%' order by start"):
        try:
            name = json.loads(ext).get("message", name) if ext else name
        except ValueError:
            pass
        rows.append((name, tid, st, en))
    outs = [r for r in rows if r[0] == outer][skip:]
    if count is not None:
        outs = outs[:count]
    agg = {}
    for name, tid, st, en in rows:
        if name == outer:
            continue
        if any(t == tid and st >= s0 and en <= e0 for _, t, s0, e0 in outs):
            a = agg.setdefault(name, [0, 0])
            a[0] += 1
            a[1] += en - st
    total = sum(e0 - s0 for _, _, s0, e0 in outs)
    kt = 0
    for st, en in c.execute("select start, end from kernels").fetchall():
        if any(s0 <= st <= e0 for _, _, s0, e0 in outs):
            kt += en - st
    out = sorted(((k, a[0], a[1]) for k, a in agg.items()), key=lambda r: -r[2])
    return out, total, len(outs), kt


def counter(db, name, pattern, grid=None):
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, grid_size, value from counters_collection "
                     "where counter_name=?", (name,)).fetchall()
    vals = [v for k, g, v in rows if pattern in k and (grid is None or g == grid)]
    return np.array(vals, dtype=np.float64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", help="FETCH_SIZE pass (omit for a trace-only summary)")
    ap.add_argument("--write", help="WRITE_SIZE pass (omit for a trace-only summary)")
    ap.add_argument("--kernel", help="the kernel the counter and trace summaries are about")
    ap.add_argument("--calib", default="__amd_rocclr_copyBuffer")
    ap.add_argument("--calib-grid", type=int, default=131072)
    ap.add_argument("--calib-bytes", type=float, default=float(1 << 30))
    ap.add_argument("--algo-bytes", type=float, default=0.0)
    ap.add_argument("--cmd", action="append", default=[])
    ap.add_argument("--title", default="rocprofv3 summary")
    ap.add_argument("--since", help="trace-only: dispatches from the first kernel containing this on")
    ap.add_argument("--until", help="trace-only with --since: stop before the first later kernel containing this")
    ap.add_argument("--exclude", help="trace-only with --since: leave out kernels whose names contain this")
    ap.add_argument("--per", type=float, default=0.0, help="trace-only with --since: also per-unit totals")
    ap.add_argument("--ranges", help="marker ranges nested in the ranges of this name (--marker-trace)")
    ap.add_argument("--range-skip", type=int, default=0, help="with --ranges: outer ranges to skip")
    ap.add_argument("--range-count", type=int, help="with --ranges: outer ranges to take")
    a = ap.parse_args()

    if a.ranges:
        rows, total, n, kt = range_stats(a.trace, a.ranges, a.range_skip, a.range_count)
        print("# %s" % a.title)
        print()
        print("Commands (from the repository root):")
        print()
        for c in a.cmd:
            print("    " + c)
        print()
        print("## Host ranges within `%s` (rocprofv3 --marker-trace), %d of them from the %d-th on"
              % (a.ranges, n, a.range_skip))
        print()
        print("`%s`: %.3f ms per call on the host; kernel time of the dispatches started within: "
              "%.3f ms per call" % (a.ranges, total / 1e6 / max(n, 1), kt / 1e6 / max(n, 1)))
        print()
        print("| range | calls per `%s` | ms per `%s` | %% of `%s` |" % ((a.ranges,) * 3))
        print("|---|---|---|---|")
        for name, calls, t in rows:
            print("| `%s` | %.2f | %.3f | %.1f |" % (name, calls / max(n, 1), t / 1e6 / max(n, 1),
                                                   100.0 * t / max(total, 1)))
        return

    if a.since:
        rows, span = trace_since(a.trace, a.since, a.until, a.exclude)
        tot = sum(r[2] for r in rows)
        print("# %s" % a.title)
        print()
        print("Commands (from the repository root):")
        print()
        for c in a.cmd:
            print("    " + c)
        print()
        print("## Kernel trace from the first `%s` dispatch on%s%s (rocprofv3 --kernel-trace --stats)"
              % (a.since, " up to the first `%s`" % a.until if a.until else "",
                 ", without `%s`" % a.exclude if a.exclude else ""))
        print()
        print("kernel time %.3f ms over a wall span of %.3f ms" % (tot / 1e6, span / 1e6), end="")
        print(" (per unit, %g units: %.3f ms)" % (a.per, tot / 1e6 / a.per) if a.per else "")
        print()
        print("| kernel | calls | total us | average us | % |")
        print("|---|---|---|---|---|")
        for name, calls, t, avg, pct in rows[:20]:
            short = name if len(name) < 90 else name[:87] + "..."
            print("| `%s` | %d | %.1f | %.2f | %.1f |" % (short, calls, t / 1e3, avg / 1e3, pct))
        return
    if not a.kernel:
        ap.error("--kernel is needed without --ranges or --since")
    allk, sel = trace_stats(a.trace, a.kernel)
    if not (a.fetch and a.write):
        print("# %s" % a.title)
        print()
        print("Commands (from the repository root):")
        print()
        for c in a.cmd:
            print("    " + c)
        print()
        print("## Kernel trace (rocprofv3 --kernel-trace --stats)")
        print()
        print("| kernel | calls | total us | average us | % |")
        print("|---|---|---|---|---|")
        for name, calls, tot, avg, pct in allk[:16]:
            short = name if len(name) < 90 else name[:87] + "..."
            print("| `%s` | %d | %.1f | %.2f | %.1f |" % (short, calls, tot, avg, pct))
        return
    fk = counter(a.fetch, "FETCH_SIZE", a.kernel) * 1024.0
    wk = counter(a.write, "WRITE_SIZE", a.kernel) * 1024.0
    fc = counter(a.fetch, "FETCH_SIZE", a.calib, a.calib_grid) * 1024.0
    wc = counter(a.write, "WRITE_SIZE", a.calib, a.calib_grid) * 1024.0
    ffac = a.calib_bytes / fc.mean()
    wfac = a.calib_bytes / wc.mean()
    fetch_b = fk.mean() * ffac
    write_b = wk.mean() * wfac
    print("# %s" % a.title)
    print()
    print("Commands (from the repository root):")
    print()
    for c in a.cmd:
        print("    " + c)
    print()
    print("## Kernel trace (rocprofv3 --kernel-trace --stats)")
    print()
    print("| kernel | calls | total us | average us | % |")
    print("|---|---|---|---|---|")
    for name, calls, tot, avg, pct in allk[:8]:
        short = name if len(name) < 70 else name[:67] + "..."
        print("| `%s` | %d | %.1f | %.2f | %.1f |" % (short, calls, tot, avg, pct))
    print()
    print("## HBM traffic per dispatch (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)")
    print()
    print("calibration kernel `%s` moving %.0f bytes each way: FETCH_SIZE reads %.0f B "
          "(factor %.3f), WRITE_SIZE reads %.0f B (factor %.3f)"
          % (a.calib, a.calib_bytes, fc.mean(), ffac, wc.mean(), wfac))
    print()
    print("| quantity | value |")
    print("|---|---|")
    print("| dispatches counted | %d / %d |" % (fk.size, wk.size))
    print("| raw FETCH_SIZE per dispatch | %.0f B |" % fk.mean())
    print("| raw WRITE_SIZE per dispatch | %.0f B |" % wk.mean())
    print("| scaled fetch per dispatch | %.0f B |" % fetch_b)
    print("| scaled write per dispatch | %.0f B |" % write_b)
    print("| algorithmic bytes per dispatch | %.0f B |" % a.algo_bytes)
    print("| traffic / algorithmic | %.3f |" % ((fetch_b + write_b) / a.algo_bytes))
    if sel:
        print("| kernel average duration (trace) | %.2f us |" % sel[0][3])
    print()
    print("machine-readable:")
    print()
    print("    traffic_bytes_per_launch: %.0f" % (fetch_b + write_b))
    print("    fetch_bytes_per_launch: %.0f" % fetch_b)
    print("    write_bytes_per_launch: %.0f" % write_b)
    if sel:
        print("    trace_avg_us: %.3f" % sel[0][3])
    print("    kernel_sha: %s" % kernel_sha())


if __name__ == "__main__":
    main()
