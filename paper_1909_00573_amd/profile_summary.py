"""Summaries of rocprofv3 CSV output for the library's kernels.

    python -m paper_1909_00573_amd.profile_summary stats <kernel_stats.csv>
    python -m paper_1909_00573_amd.profile_summary counters <counter_collection.csv> <counter> [name regex]
    python -m paper_1909_00573_amd.profile_summary table <counter_collection.csv>... [name regex]

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


def counter_table(paths, pattern=None):
    """Per kernel, the average per dispatch of every counter found in the
    given counter-collection CSVs (one pass per file), and the ratios that
    read them: wave time waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES), VALU busy
    per wave (SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES), vector L1 hit rate
    (1 - TCP_TCC_READ_REQ / TCP_TOTAL_CACHE_ACCESSES), L2 hit rate
    (TCC_HIT / (TCC_HIT + TCC_MISS)), matrix-core busy per SIMD
    (SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 x 4 x 256): the GPU-busy
    count arrives summed over the 8 XCDs, there are 4 SIMDs in each of the
    256 CUs), and the bf16 matrix FLOPs (SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512)."""
    acc = defaultdict(lambda: defaultdict(lambda: [0, 0.0]))
    for path in paths:
        for r in csv.DictReader(open(path)):
            name = short_name(r.get("Kernel_Name", ""))
            if pattern and not re.search(pattern, name):
                continue
            a = acc[name][r.get("Counter_Name")]
            a[0] += 1
            a[1] += float(r.get("Counter_Value", 0) or 0)
    for name in sorted(acc):
        c = {k: v[1] / v[0] for k, v in acc[name].items() if v[0]}
        n = max(v[0] for v in acc[name].values())
        print(f"{name}  ({n} dispatches per counter)")
        for k in sorted(c):
            print(f"    {k:34s} {c[k]:18.1f}")
        ratios = []
        if "SQ_WAVE_CYCLES" in c and c["SQ_WAVE_CYCLES"] > 0:
            if "SQ_WAIT_ANY" in c:
                ratios.append(("wave cycles waiting", c["SQ_WAIT_ANY"] / c["SQ_WAVE_CYCLES"]))
            if "SQ_ACTIVE_INST_VALU" in c:
                ratios.append(("wave cycles issuing VALU", c["SQ_ACTIVE_INST_VALU"] / c["SQ_WAVE_CYCLES"]))
        if c.get("TCP_TOTAL_CACHE_ACCESSES_sum", 0) > 0 and "TCP_TCC_READ_REQ_sum" in c:
            ratios.append(("vector L1 hit rate", 1 - c["TCP_TCC_READ_REQ_sum"] / c["TCP_TOTAL_CACHE_ACCESSES_sum"]))
        if c.get("TCC_HIT_sum", 0) + c.get("TCC_MISS_sum", 0) > 0:
            ratios.append(("L2 hit rate", c["TCC_HIT_sum"] / (c["TCC_HIT_sum"] + c["TCC_MISS_sum"])))
        if c.get("GRBM_GUI_ACTIVE", 0) > 0 and "SQ_VALU_MFMA_BUSY_CYCLES" in c:
            ratios.append(("matrix-core busy per SIMD",
                           c["SQ_VALU_MFMA_BUSY_CYCLES"] / (c["GRBM_GUI_ACTIVE"] / 8 * 4 * 256)))
        if "SQ_INSTS_VALU_MFMA_MOPS_BF16" in c:
            ratios.append(("bf16 matrix GFLOP per dispatch", c["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * 512 / 1e9))
        for label, v in ratios:
            print(f"    = {label:32s} {v:18.4f}")


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "stats":
        stats(sys.argv[2])
    elif len(sys.argv) >= 4 and sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], sys.argv[4] if len(sys.argv) > 4 else None)
    elif len(sys.argv) >= 3 and sys.argv[1] == "table":
        files = [a for a in sys.argv[2:] if a.endswith(".csv")]
        pat = next((a for a in sys.argv[2:] if not a.endswith(".csv")), None)
        counter_table(files, pat)
    else:
        print(__doc__)
        sys.exit(2)
