"""Summaries of rocprofv3 output as markdown tables.

    python profile_summary.py stats DIR          # --kernel-trace --stats --output-format csv
    python profile_summary.py counters DIR COPY  # --pmc <one counter> --output-format csv,
                                                 # COPY = the same counter over `bench.py --copy-probe`
    python profile_summary.py mfma DIR           # --pmc MfmaUtil MfmaFlopsBF16 MfmaFlopsF32 --kernel-trace

`stats` lists every kernel's dispatch count and average / min / max / total
duration.  `counters` lists the per-dispatch average of the counter (KiB) for
every kernel and the calibrated bytes: the copy probe moves exactly 1 GiB per
dispatch in each direction, so bytes = counter x (1 GiB / counter of the copy
kernel).  `mfma` lists, per kernel, the per-dispatch average of every counter
of the run, the matrix-core flops per dispatch and, when the run also traced
kernels, the achieved matrix-core rate against the dense peak of its type."""
import collections
import csv
import glob
import os
import sys


def _one(pattern):
    hits = glob.glob(pattern, recursive=True)
    if not hits:
        raise SystemExit(f"nothing matches {pattern}")
    return hits[0]


def stats(d):
    path = _one(os.path.join(d, "**", "*kernel_stats.csv"))
    rows = list(csv.DictReader(open(path)))
    print("| kernel | dispatches | avg us | min us | max us | total ms |")
    print("|---|---|---|---|---|---|")
    for r in rows:
        print(f"| `{r['Name']}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
              f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
              f"{float(r['TotalDurationNs']) / 1e6:.3f} |")


def _counter(d):
    path = _one(os.path.join(d, "**", "*counter_collection.csv"))
    per = collections.defaultdict(list)
    name = None
    for r in csv.DictReader(open(path)):
        per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        name = r["Counter_Name"]
    return name, {k: sum(v) / len(v) for k, v in per.items()}, {k: len(v) for k, v in per.items()}


def counters(d, copy_dir):
    name, avg, cnt = _counter(d)
    _, cavg, _ = _counter(copy_dir)
    probe = [v for k, v in cavg.items() if "neg_kernel" in k]
    if not probe:
        raise SystemExit("the copy probe's kernel is missing")
    scale = 1048576.0 / probe[0]
    print(f"counter {name}; copy probe reads {probe[0]:.1f} KiB per GiB moved -> scale {scale:.5f}")
    print()
    print(f"| kernel | dispatches | {name} KiB/dispatch | calibrated MB/dispatch |")
    print("|---|---|---|---|")
    for k, v in sorted(avg.items(), key=lambda kv: -kv[1]):
        print(f"| `{k}` | {cnt[k]} | {v:.1f} | {v * scale * 1024 / 1e6:.2f} |")


# dense matrix-core peaks of one MI355X, TFLOP/s
MFMA_PEAK = {"MfmaFlopsBF16": 2500.0, "MfmaFlopsF32": 157.3}


def mfma(d):
    path = _one(os.path.join(d, "**", "*counter_collection.csv"))
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(path)):
        per[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    dur = {}
    hits = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if hits:
        for r in csv.DictReader(open(hits[0])):
            dur[r["Name"]] = float(r["AverageNs"])
    names = sorted({c for v in per.values() for c in v})
    print("| kernel | dispatches | " + " | ".join(f"{n} avg" for n in names) + " | matrix-core rate |")
    print("|---" * (len(names) + 3) + "|")
    for k, v in sorted(per.items(), key=lambda kv: -sum(sum(x) for x in kv[1].values())):
        n = max(len(x) for x in v.values())
        avg = {c: sum(x) / len(x) for c, x in v.items()}
        rate = []
        for c, peak in MFMA_PEAK.items():
            if avg.get(c, 0) > 0 and k in dur:
                t = avg[c] / dur[k] / 1e3  # FLOP/ns = GFLOP/s; /1e3 -> TFLOP/s
                rate.append(f"{c[9:]} {t:.3f} TFLOP/s = {100 * t / peak:.3f}% of {peak:g}")
        print(f"| `{k}` | {n} | " + " | ".join(f"{avg.get(c, 0):.4g}" for c in names) +
              f" | {'; '.join(rate) or '-'} |")


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "stats":
        stats(sys.argv[2])
    elif len(sys.argv) >= 3 and sys.argv[1] == "mfma":
        mfma(sys.argv[2])
    elif len(sys.argv) >= 4 and sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3])
    else:
        raise SystemExit(__doc__)
