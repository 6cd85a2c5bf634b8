"""Summaries of rocprofv3 CSV output for the library's kernels.

    python -m paper_1909_00573_amd.profile_summary stats <kernel_stats.csv>
    python -m paper_1909_00573_amd.profile_summary counters <counter_collection.csv> <counter> [name regex]

`stats` prints the kernel statistics (calls, total and average duration)
sorted by total time; `counters` prints, per kernel name, the number of
dispatches and the average value of one counter per dispatch (FETCH_SIZE
and WRITE_SIZE are in KiB).
"""
import csv
import re
import sys
from collections import defaultdict


def short_name(name):
    """Kernel name without namespace and arguments; template arguments are
    kept (without spaces) so that instantiations stay apart."""
    name = re.sub(r"\(.*", "", name)
    name = re.sub(r"^void ", "", name.strip())
    m = re.match(r"(.*?)(<.*>)?$", name)
    base, targs = m.group(1), (m.group(2) or "")
    return base.split("::")[-1].strip() + targs.replace(" ", "")


def stats(path):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        calls = int(r.get("Calls", 0) or 0)
        total = float(r.get("TotalDurationNs", 0) or 0)
        avg = float(r.get("AverageNs", 0) or (total / calls if calls else 0))
        out.append((total, short_name(r.get("Name", "")), calls, avg, float(r.get("Percentage", 0) or 0)))
    out.sort(reverse=True)
    print(f"{'kernel':34s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s} {'pct':>6s}")
    for total, name, calls, avg, pct in out:
        print(f"{name:34s} {calls:7d} {total / 1e6:10.3f} {avg / 1e3:10.2f} {pct:6.2f}")


def counters(path, counter, pattern=None):
    acc = defaultdict(lambda: [0, 0.0])
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        name = short_name(r.get("Kernel_Name", ""))
        if pattern and not re.search(pattern, name):
            continue
        a = acc[name]
        a[0] += 1
        a[1] += float(r.get("Counter_Value", 0) or 0)
    print(f"{'kernel':34s} {'dispatches':>10s} {'avg_' + counter:>18s}")
    for name, (n, tot) in sorted(acc.items(), key=lambda kv: -kv[1][1]):
        print(f"{name:34s} {n:10d} {tot / n:18.1f}")


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "stats":
        stats(sys.argv[2])
    elif len(sys.argv) >= 4 and sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], sys.argv[4] if len(sys.argv) > 4 else None)
    else:
        print(__doc__)
        sys.exit(2)
