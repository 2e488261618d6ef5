"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2403_04946_amd.profile_summary stats <kernel_stats.csv>
        Markdown table of kernel time per kernel (all template variants of a
        kernel family are also summed into one line per family).
    python -m paper_2403_04946_amd.profile_summary pmc <counter_collection.csv> <counter> [kernel-substring]
        Per-kernel-family totals and per-dispatch averages of one counter
        (summed over its hardware instances; FETCH_SIZE and WRITE_SIZE in KiB
        as rocprofv3 reports them, other counters as counts).
"""
import collections
import csv
import re
import sys


def family(name):
    # "void ttf::zgemm_kernel<0, 0, 64, 64>(ttf::GemmParams)" -> "ttf::zgemm_kernel"
    name = re.sub(r"^void ", "", name)
    name = name.split("(")[0]
    return re.sub(r"<.*>$", "", name)


def stats(path):
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    fam = collections.defaultdict(lambda: [0, 0.0])
    print("| kernel | calls | total ms | avg us | % |")
    print("|---|---:|---:|---:|---:|")
    for r in rows:
        ns = float(r["TotalDurationNs"])
        fam[family(r["Name"])][0] += int(r["Calls"])
        fam[family(r["Name"])][1] += ns
        if ns / tot >= 0.005:
            print(f"| `{r['Name'][:70]}` | {r['Calls']} | {ns / 1e6:.1f} | {float(r['AverageNs']) / 1e3:.1f} | "
                  f"{100 * ns / tot:.1f} |")
    print()
    print("| kernel family | calls | total ms | avg us |")
    print("|---|---:|---:|---:|")
    for k, (n, ns) in sorted(fam.items(), key=lambda kv: -kv[1][1]):
        if ns / tot >= 0.002:
            print(f"| `{k}` | {n} | {ns / 1e6:.1f} | {ns / n / 1e3:.1f} |")
    print(f"\ntotal kernel time {tot / 1e6:.1f} ms")


def pmc(path, counter, sub=None):
    per = collections.defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        did = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per[did] += float(r["Counter_Value"])
        names[did] = r.get("Kernel_Name", "")
    fam = collections.defaultdict(lambda: [0, 0.0])
    for did, v in per.items():
        f = family(names[did])
        if sub and sub not in f:
            continue
        fam[f][0] += 1
        fam[f][1] += v
    unit = " KiB" if counter in ("FETCH_SIZE", "WRITE_SIZE") else ""
    print(f"| kernel family | dispatches | {counter} total{unit} | per dispatch{unit} |")
    print("|---|---:|---:|---:|")
    for k, (n, v) in sorted(fam.items(), key=lambda kv: -kv[1][1]):
        print(f"| `{k}` | {n} | {v:.0f} | {v / n:.1f} |")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2])
    else:
        pmc(sys.argv[2], sys.argv[3], sys.argv[4] if len(sys.argv) > 4 else None)
