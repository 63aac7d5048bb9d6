"""Summaries of rocprofv3 CSV output (kernel stats; PMC counters scaled by a copy).

Usage:
  python -m paper_1603_02524_amd.rocprof_summary stats <run_kernel_stats.csv> [top]
  python -m paper_1603_02524_amd.rocprof_summary pmc <solve_counter_collection.csv> <copy_counter_collection.csv>
                                  <counter> <bytes moved per copy>
  python -m paper_1603_02524_amd.rocprof_summary counters <counter_collection.csv> [<csv> ...] -- <kernel> [<kernel> ...]
      (per kernel whose short name starts with one of the given prefixes: each counter's mean
       per dispatch and, where SQ_WAVES was collected, per wave)
"""
import collections
import csv
import sys


def short(name):
    """Kernel name without its argument list ("(anonymous namespace)::" kept)."""
    name = name.replace("void ", "", 1)
    anon = "(anonymous namespace)::"
    pre = anon if name.startswith(anon) else ""
    rest = name[len(pre):]
    depth, cut = 0, len(rest)
    for i, ch in enumerate(rest):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    return (pre + rest[:cut]) or "(unnamed)"


def stats(path, top=24):
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    print("| kernel | calls | avg us | total ms | % |\n|---|---|---|---|---|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        name = short(r["Name"])
        print(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
              f"{float(r['TotalDurationNs']) / 1e6:.3f} | {100 * float(r['TotalDurationNs']) / tot:.1f} |")
    print(f"\nTotal GPU kernel time {tot / 1e6:.3f} ms.")


def pmc(solve, copy, counter, copy_bytes):
    def load(p):
        agg = collections.defaultdict(list)
        for r in csv.DictReader(open(p)):
            if r["Counter_Name"] == counter:
                agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return agg
    c = load(copy)["__amd_rocclr_copyBuffer"]
    kib = sum(c) / len(c)
    scale = float(copy_bytes) / (kib * 1024.0)
    print(f"{counter}: plain copy of {int(copy_bytes)} B reads as {kib:.0f} KiB per dispatch "
          f"-> scale {scale:.4f} B per counted byte\n")
    print(f"| kernel | dispatches | {counter} KiB avg | HBM MB per dispatch (scaled) |\n|---|---|---|---|")
    a = load(solve)
    for k, v in sorted(a.items(), key=lambda kv: -sum(kv[1]))[:16]:
        name = short(k)
        avg = sum(v) / len(v)
        print(f"| `{name}` | {len(v)} | {avg:.0f} | {avg * 1024 * scale / 1e6:.1f} |")


def counters(paths, kernels):
    per = collections.defaultdict(lambda: collections.defaultdict(lambda: collections.defaultdict(float)))
    for p in paths:
        for r in csv.DictReader(open(p)):
            name = short(r["Kernel_Name"])
            if any(name.startswith(k) for k in kernels):
                per[name][r["Counter_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
    for name in sorted(per):
        cs = per[name]
        mean = {c: sum(d.values()) / len(d) for c, d in cs.items()}
        waves = mean.get("SQ_WAVES")
        print(f"\n`{name}`\n\n| counter | dispatches | mean per dispatch | per wave |\n|---|---|---|---|")
        for c in sorted(mean):
            pw = f"{mean[c] / waves:.1f}" if waves else "-"
            print(f"| {c} | {len(cs[c])} | {mean[c]:.0f} | {pw} |")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 24)
    elif sys.argv[1] == "counters":
        cut = sys.argv.index("--")
        counters(sys.argv[2:cut], sys.argv[cut + 1:])
    else:
        pmc(sys.argv[2], sys.argv[3], sys.argv[4], float(sys.argv[5]))
