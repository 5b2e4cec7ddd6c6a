"""Summaries of rocprofv3 output for profiles/ (runs on the host, no GPU).

    python -m paper_2406_11185_amd.profile_summary stats KERNEL_STATS_CSV BENCH_JSON OUT.md --command CMD
    python -m paper_2406_11185_amd.profile_summary valu COUNTER_CSV BENCH_JSON OUT.md --command CMD

`stats`: per-kernel calls and durations from a `--kernel-trace --stats` run of
bench.py, with each J/K class kernel's algorithmic rate (flops of the generated
code per quartet, from classes.json, times the quartets the benchmark line of
the same run reports for that class, over the kernel's mean duration).
`valu`: VALU instruction counters per J/K class kernel (`--pmc` runs) turned
into counter flops -- 64 lanes x (2 per FMA, 1 per add, multiply or
transcendental) per wavefront instruction, an upper bound that counts inactive
lanes -- next to the algorithmic flops, both over the kernel durations of the
stats run, and the memory-side atomic requests of each kernel.
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PEAK = 78.6   # TFLOP/s: FP64 vector, and FP32 without packed instructions
FINGERPRINT_SOURCES = ["paper_2406_11185_amd/csrc/gen_hgp.py", "paper_2406_11185_amd/csrc/jk_device.hpp",
                       "paper_2406_11185_amd/csrc/jk_host.hip", "paper_2406_11185_amd/csrc/jk_classes.hpp"]


def source_fingerprint() -> str:
    """Hash of the sources that decide the J/K kernels' code and launches."""
    import hashlib
    h = hashlib.sha256()
    for rel in FINGERPRINT_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def class_infos():
    with open(os.path.join(HERE, "classes.json")) as fh:
        return {i["name"]: i for i in json.load(fh)}


def flops_per_quartet(info, npp=81, n_dm=1):
    return npp * (info["vrr_flops_alg"] + 71 + 4 * info["L"]) + info["hrr_flops"] + \
        n_dm * info["digest_flops"]


def kernel_key(name):
    """(class, 'fp64'|'fp32', kernel kind) for a J/K class kernel, else None."""
    m = re.search(r"eri_jk(_lds|_split|_rows)?_kernel<jk::Cls_(\w{4})\w*, (double|float)", name)
    if not m:
        return None
    return m.group(2), "fp64" if m.group(3) == "double" else "fp32", (m.group(1) or "_single")[1:]


def load_bench(path):
    """The JSON line bench.py printed (the last line that parses)."""
    line = None
    with open(path) as fh:
        for ln in fh:
            ln = ln.strip()
            if ln.startswith("{") and ln.endswith("}"):
                line = ln
    return json.loads(line)


def read_stats(path):
    out = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            name = r.get("Name") or r.get("Kernel_Name") or ""
            out[name] = (int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6,
                         float(r["AverageNs"]) / 1e6)
    return out


def stats(args):
    st = read_stats(args.csv)
    bench = load_bench(args.bench)
    infos = class_infos()
    n_dm = bench["config"]["n_dm"]
    builds = bench["warmup"] + bench["steps"]   # builds in the profiled run (no extra legs)
    total = sum(v[1] for v in st.values())
    lines = [f"# rocprofv3 kernel statistics: {args.title}", "",
             "Command (from the repository root, on an MI355X):", "", "```", args.command, "```",
             "", f"Total kernel time over the profiled run: {total:.2f} ms ({len(st)} kernels).  "
             "Class kernels run one at a time (serial launches), so each duration is the "
             "kernel's own.  Algorithmic TFLOP/s = generated-code flops per quartet (each "
             "quartet's integrals once, its digestion once per density) x the quartets of the "
             "class in one build (benchmark line of the same run) x the builds of the run / the "
             "kernel's total time "
             "(a class launched once per density, recomputing its integrals, shows that "
             f"work as lost rate); fraction of {PEAK} TFLOP/s.", "",
             "| kernel | calls | total ms | avg ms | % | quartets per build | TFLOP/s | frac |",
             "|---|---|---|---|---|---|---|---|"]
    for name, (calls, tot, avg) in sorted(st.items(), key=lambda kv: -kv[1][1]):
        k = kernel_key(name)
        q = tf = fr = ""
        if k:
            c = bench["classes"].get(f"{k[0]}_{k[1]}")
            if c:
                qn = c["quartets"]
                rate = flops_per_quartet(infos[k[0]], n_dm=n_dm) * qn * builds / (tot / 1e3) / 1e12
                q, tf, fr = str(qn), f"{rate:.1f}", f"{rate / PEAK:.3f}"
        short = re.sub(r"\(.*\)$", "", name).replace("jk::", "").replace("void ", "")
        lines.append(f"| `{short[:90]}` | {calls} | {tot:.3f} | {avg:.4f} | "
                     f"{100 * tot / total:.2f} | {q} | {tf} | {fr} |")
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines[:40]))


VALU = {"SQ_INSTS_VALU_FMA_F64": 2, "SQ_INSTS_VALU_ADD_F64": 1, "SQ_INSTS_VALU_MUL_F64": 1,
        "SQ_INSTS_VALU_TRANS_F64": 1, "SQ_INSTS_VALU_FMA_F32": 2, "SQ_INSTS_VALU_ADD_F32": 1,
        "SQ_INSTS_VALU_MUL_F32": 1, "SQ_INSTS_VALU_TRANS_F32": 1}
ATOMIC = ("TCC_EA0_ATOMIC_sum", "TCC_ATOMIC_sum")


def valu(args):
    per = defaultdict(lambda: defaultdict(float))
    calls = defaultdict(set)
    for path in args.csv.split(","):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                k = kernel_key(r["Kernel_Name"])
                if not k or (r["Counter_Name"] not in VALU and r["Counter_Name"] not in ATOMIC):
                    continue
                per[k][r["Counter_Name"]] += float(r["Counter_Value"])
                calls[(k, r["Counter_Name"])].add(r.get("Dispatch_Id", r.get("Correlation_Id", "")))
    st = read_stats(args.stats) if args.stats else {}
    avg = {}
    for name, (_, _, a) in st.items():
        k = kernel_key(name)
        if k:
            avg[k] = a
    bench = load_bench(args.bench)
    infos = class_infos()
    n_dm = bench["config"]["n_dm"]
    lines = [f"# VALU and atomic counters per class kernel: {args.title}", "", "Commands:", "", "```",
             *args.command.split(";;"), "```", "",
             "Counter flops = 64 x (2 FMA + ADD + MUL + TRANS) per wavefront instruction, FP64 and "
             "FP32 counted separately (an upper bound: inactive lanes are counted).  Algorithmic "
             "flops from the generated code.  Rates over the kernel's mean duration in the "
             f"kernel-statistics run; fractions of {PEAK} TFLOP/s.  Atomics: TCC_EA0_ATOMIC, the "
             "atomic requests the L2 forwards to the memory side (device-scope atomics on this "
             "chip are all executed there; TCC_ATOMIC reads the same), per screened quartet and "
             "per second.", "", f"source fingerprint: `{source_fingerprint()}`", "",
             "| kernel | counter GFLOP fp64 | counter GFLOP fp32 | algorithmic GFLOP | "
             "counter / algorithmic | counter TFLOP/s | algorithmic TFLOP/s | frac (counter) | "
             "atomics per quartet | atomic G/s |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    rows = []
    for k, cnt in per.items():
        def pc(c):   # per dispatch
            return cnt.get(c, 0.0) / max(1, len(calls.get((k, c), ())))
        f64 = 64 * sum(VALU[c] * pc(c) for c in VALU if c.endswith("F64")) / 1e9
        f32 = 64 * sum(VALU[c] * pc(c) for c in VALU if c.endswith("F32")) / 1e9
        c = bench["classes"].get(f"{k[0]}_{k[1]}")
        nq = c["quartets"] if c else 0
        alg = flops_per_quartet(infos[k[0]], n_dm=n_dm) * nq / 1e9
        a = avg.get(k)
        at = pc("TCC_EA0_ATOMIC_sum")
        nan = float("nan")
        ct = (f64 + f32) / a if a else nan   # GFLOP per ms = TFLOP/s
        rows.append((-(f64 + f32), f"| eri_jk {k[0]} {k[1]} ({k[2]}) | {f64:.2f} | {f32:.2f} | "
                                   f"{alg:.2f} | {(f64 + f32) / alg if alg else nan:.2f} | "
                                   f"{ct:.1f} | {alg / a if a else nan:.1f} | "
                                   f"{ct / PEAK:.3f} | {at / nq if nq else nan:.2f} | "
                                   f"{at / (a / 1e3) / 1e9 if a else nan:.1f} |"))
    lines += [r for _, r in sorted(rows)]
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("bench")
    s.add_argument("out")
    s.add_argument("--command", default="")
    s.add_argument("--title", default="")
    v = sub.add_parser("valu")
    v.add_argument("csv", help="counter_collection.csv files, comma separated")
    v.add_argument("bench")
    v.add_argument("out")
    v.add_argument("--stats", default="")
    v.add_argument("--command", default="")
    v.add_argument("--title", default="")
    a = ap.parse_args()
    stats(a) if a.what == "stats" else valu(a)


if __name__ == "__main__":
    main()
