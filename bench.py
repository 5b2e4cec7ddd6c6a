"""Benchmark of the direct-SCF J/K build on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload w30] [--precision fp64]
                    [--no-cpu] [--no-extra]

A step is one complete jk_build call: shell-pair data, Cauchy-Schwarz bounds,
Q sort, screening and work lists, every integral+digestion kernel and the
symmetrisation of J and K, on a seeded synthetic molecule whose density is
already resident in device memory.  The default workload is the 30-atom,
270-function molecule screened at 1e-10 in FP64.

Prints one JSON line.  `value` is screened quartets per second (unique shell
quartets that pass the Schwarz screen, per build).  `roofline` describes the
kernel with the most algorithmic work, which the library runs alone before
spreading the other classes over three streams: algorithmic work per launch (flops
of the generated recurrence, horizontal-recurrence and digestion code per
quartet, plus a fixed count per primitive quartet for the Boys function and
prefactors) divided by its mean launch time from HIP events recorded on the
launch stream.  `cpu_baseline` is the CPU oracle timed on a bounded sample of
bra pairs of the same molecule.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6     # MI355X vector FP64 (256 CU x 2.4 GHz x 128 flop/clk)
FP32_PEAK_TFLOPS = 157.3    # with packed FP32 (not used by these kernels: 78.6 unpacked)


def prim_setup_flops(L: int) -> int:
    """Flops of one primitive quartet outside the recurrences (see jk_device.hpp
    prim_setup/boys_f64): reciprocal, Gaussian-product distances, Boys Taylor
    step and e^-T series, downward recursion (3 per order), prefactor scaling
    and recurrence coefficients."""
    return 71 + 4 * L


def class_info():
    """Per-class operation counts written by the code generator at build time."""
    path = os.path.join(ROOT, "paper_2406_11185_amd", "classes.json")
    with open(path) as fh:
        return json.load(fh)


def flops_per_quartet(info, npp_b=9, npp_k=9, n_dm=1):
    return (npp_b * npp_k * (info["vrr_flops_alg"] + prim_setup_flops(info["L"]))
            + info["hrr_flops"] + n_dm * info["digest_flops"])


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_w30_fp64.md")
FINGERPRINT_SOURCES = ["paper_2406_11185_amd/csrc/gen_hgp.py", "paper_2406_11185_amd/csrc/jk_device.hpp",
                       "paper_2406_11185_amd/csrc/jk_host.hip", "paper_2406_11185_amd/csrc/jk_classes.hpp"]


def source_fingerprint() -> str:
    """Hash of the sources that decide the J/K kernels' code: counter data taken
    with another fingerprint describe other kernels."""
    import hashlib
    h = hashlib.sha256()
    for rel in FINGERPRINT_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_key(name: str):
    """'eri_jk <class> fp64|fp32' for a J/K class kernel name, else None."""
    import re
    m = re.search(r"jk::eri_jk(?:_lds|_split)?_kernel<jk::Cls_(\w+), (double|float)", name)
    if not m:
        return None
    return f"eri_jk {m.group(1)} {'fp64' if m.group(2) == 'double' else 'fp32'}"


def pmc_summary(fetch_csv: str, write_csv: str, out: str, calib_mib: int, command: str) -> None:
    """Per-dispatch HBM bytes of every J/K class kernel from two rocprofv3 --pmc
    runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), scaled by what the same
    counters read for the copy of calib_mib MiB made before the steps."""
    import csv
    from collections import defaultdict

    def load(path, counter):
        per = defaultdict(list)
        copy = []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"])
                if "copyBuffer" in r["Kernel_Name"]:
                    copy.append(v)
                k = kernel_key(r["Kernel_Name"])
                if k:
                    per[k].append(v)
        return per, max(copy) if copy else None

    fetch, fcopy = load(fetch_csv, "FETCH_SIZE")
    write, wcopy = load(write_csv, "WRITE_SIZE")
    known = calib_mib * 1024.0
    fs, ws = known / fcopy, known / wcopy
    lines = ["# HBM traffic per dispatch: J/K build, 30 atoms / 270 functions, tol 1e-10, FP64", "",
             "Two rocprofv3 counter runs of the benchmark (kernels are serialised while counters "
             "are collected), from the repository root on the GPU box:", "", "```",
             command.replace("PMC", "FETCH_SIZE"), command.replace("PMC", "WRITE_SIZE"), "```", "",
             f"Calibration: the {calib_mib} MiB device-to-device copy made before the steps reads "
             f"FETCH_SIZE = {fcopy:.1f} KiB and WRITE_SIZE = {wcopy:.1f} KiB for {known:.0f} KiB "
             f"moved each way, so read bytes = FETCH_SIZE x {fs:.3f} and written bytes = "
             f"WRITE_SIZE x {ws:.3f}.", "",
             f"source fingerprint: `{source_fingerprint()}`", "",
             "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB | written MB | traffic MB |",
             "|---|---|---|---|---|---|---|"]
    rows = []
    for k in sorted(set(fetch) & set(write)):
        f = sum(fetch[k]) / len(fetch[k])
        w = sum(write[k]) / len(write[k])
        rd, wr = f * fs * 1024 / 1e6, w * ws * 1024 / 1e6
        rows.append((rd + wr, f"| {k} | {len(fetch[k])} | {f:.1f} | {w:.1f} | {rd:.3f} | {wr:.3f} | "
                              f"{rd + wr:.3f} |"))
    lines += [r for _, r in sorted(rows, reverse=True)]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def traffic_of(kernel: str):
    """HBM bytes per dispatch of `kernel` from the committed counter summary, or
    None if there is none or the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            text = fh.read()
    except OSError:
        return None
    if f"source fingerprint: `{source_fingerprint()}`" not in text:
        return None
    for ln in text.splitlines():
        cells = [c.strip() for c in ln.strip().strip("|").split("|")]
        if len(cells) == 7 and cells[0] == kernel:
            return float(cells[6]) * 1e6
    return None


def cpu_baseline(mol, tol, seconds_target=15.0):
    """Oracle timed on a growing sample of unique bra pairs (all their kets)."""
    import numpy as np
    import oracle
    npair = mol.n_shells * (mol.n_shells + 1) // 2
    rng = np.random.default_rng(12345)
    order = rng.permutation(npair)
    cores = len(os.sched_getaffinity(0))
    nthreads = int(os.environ.get("OMP_NUM_THREADS", cores))
    nthreads = max(1, min(nthreads, cores))
    take, spent, kept_total, used = 8, 0.0, 0, 0
    while spent < seconds_target and used < npair:
        idx = order[used:used + take]
        t = time.perf_counter()
        _, _, kept = oracle.jk_bra_sample(mol, tol, idx, nthreads=nthreads)
        spent += time.perf_counter() - t
        kept_total += kept
        used += len(idx)
        take *= 2
    return {"value": kept_total / spent, "unit": "quartets/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"{used} of {npair} unique bra shell pairs (seeded), all their ket pairs: "
                      f"{kept_total} screened quartets in {spent:.1f} s"}


def run_steps(jkb, ctx, basis, D, J, K, tol, opts, steps, torch):
    per_step = []
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        jkb.jk_build(ctx, basis, D, J, K, tol, opts)
        st = ctx.stats()          # waits for this step's events
        per_step.append(time.perf_counter() - ts)
        stats.append(st)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, per_step, stats


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="w30")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="before the steps, copy a buffer of this many MiB once (a kernel of "
                         "known traffic for scaling hardware byte counters)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the per-dispatch HBM traffic summary from two rocprofv3 "
                         "counter_collection.csv files and exit (no GPU use)")
    ap.add_argument("--pmc-command", default="",
                    help="with --pmc-summary: the profiled command, PMC standing for the counter")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], TRAFFIC_FILE,
                    args.copy_calib_mib or 256, args.pmc_command)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2406_11185_amd import jk as jkb
    from paper_2406_11185_amd import molgen

    w = molgen.WORKLOADS[args.workload]
    precision = args.precision or w["precision"]
    tol = w["tol"]
    mol = molgen.workload(args.workload)
    basis = jkb.Basis(mol)
    dev = torch.device("cuda:0")
    D = torch.as_tensor(mol.D, device=dev).contiguous()
    J = torch.empty_like(D)
    K = torch.empty_like(D)
    ctx = jkb.Context(0)
    opts = jkb.make_opts(precision, n_dm=D.shape[0], timing=True)

    if args.copy_calib_mib:
        src = torch.ones(args.copy_calib_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        jkb.jk_build(ctx, basis, D, J, K, tol, opts)
    torch.cuda.synchronize()
    total, per_step, stats = run_steps(jkb, ctx, basis, D, J, K, tol, opts, args.steps, torch)
    ms_per_step = 1e3 * total / args.steps
    st = stats[-1]
    quartets = sum(st.quartets_fp64) + sum(st.quartets_fp32)

    # dominant kernel: the class launch with the most algorithmic work per step
    # (the library runs its largest launch alone, so its event interval is its
    # own run time; launches that share the GPU have stretched intervals)
    infos = class_info()
    agg = {}
    for s in stats:
        for q in range(jkb.JK_NCLASS):
            for pr, ms_arr, n_arr, qa in ((0, s.ms_kernel_fp64, s.launches_fp64, s.quartets_fp64),
                                          (1, s.ms_kernel_fp32, s.launches_fp32, s.quartets_fp32)):
                if n_arr[q]:
                    a = agg.setdefault((q, pr), [0.0, 0, 0])
                    a[0] += ms_arr[q]
                    a[1] += n_arr[q]
                    a[2] += qa[q]
    (qd, prd), (ms_sum, nlaunch, nq) = max(
        agg.items(), key=lambda kv: flops_per_quartet(infos[kv[0][0]], n_dm=D.shape[0]) * kv[1][2])
    info = infos[qd]
    flops_launch = flops_per_quartet(info, n_dm=D.shape[0]) * nq / nlaunch
    mean_s = ms_sum / nlaunch / 1e3
    achieved = flops_launch / mean_s / 1e12
    peak = FP64_PEAK_TFLOPS if prd == 0 else FP32_PEAK_TFLOPS
    kname = f"eri_jk {info['name']} {'fp32' if prd else 'fp64'}"
    total_kernel_ms = sum(a[0] for a in agg.values()) / len(stats)
    total_flops = 0.0
    for (q, pr), a in agg.items():
        total_flops += flops_per_quartet(infos[q], n_dm=D.shape[0]) * a[2] / len(stats)
    result = {
        "metric": "screened ERI quartets/s of the J+K build",
        "value": quartets / (total / args.steps),
        "unit": "quartets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {w['desc']}", "atoms": mol.n_atoms,
                   "basis_functions": mol.n_bf, "tol": tol, "precision": precision,
                   "n_dm": int(D.shape[0]), "screened_quartets": int(quartets),
                   "skipped_quartets": int(st.quartets_skipped)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": traffic_of(kname) if args.workload == "w30" and precision == "fp64"
                     else None,
                     "kernel": kname,
                     "flops_per_launch": flops_launch, "mean_launch_ms": mean_s * 1e3,
                     "launches": nlaunch},
        "build_kernel_ms": total_kernel_ms,
        "classes": {f"{infos[q]['name']}_{'fp32' if pr else 'fp64'}":
                    {"ms": round(a[0] / len(stats), 3), "quartets": int(a[2] / len(stats)),
                     "tflops": round(flops_per_quartet(infos[q], n_dm=D.shape[0]) * a[2]
                                     / (a[0] / 1e3) / 1e12, 3) if a[0] > 0 else None}
                    for (q, pr), a in sorted(agg.items())},
        # algorithmic flops of all class launches of a step over the step time
        "build_tflops": total_flops / (ms_per_step / 1e3) / 1e12,
        "setup_ms": st.ms_setup,
    }

    if not args.no_extra and args.workload == "w30":
        ex = {}
        mol2 = molgen.workload("w120")
        b2 = jkb.Basis(mol2)
        D2 = torch.as_tensor(mol2.D, device=dev).contiguous()
        J2, K2 = torch.empty_like(D2), torch.empty_like(D2)
        res = {}
        for prec in ("fp64", "mixed"):
            o2 = jkb.make_opts(prec, timing=True)
            jkb.jk_build(ctx, b2, D2, J2, K2, 1e-10, o2)
            tt, _, sts = run_steps(jkb, ctx, b2, D2, J2, K2, 1e-10, o2, 2, torch)
            res[prec] = (J2.double().cpu().numpy(), K2.double().cpu().numpy())
            ex[f"w120_{prec}_ms"] = 1e3 * tt / 2
            ex[f"w120_{prec}_quartets_fp32"] = int(sum(sts[-1].quartets_fp32))
        EJ = {p: 0.5 * float(np.sum(mol2.D[0] * res[p][0][0])) for p in res}
        EK = {p: 0.25 * float(np.sum(mol2.D[0] * res[p][1][0])) for p in res}
        ex["w120_mixed_speedup"] = ex["w120_fp64_ms"] / ex["w120_mixed_ms"]
        # nuclear gradient of the 30-atom molecule (same geometry and density)
        G = torch.empty((D.shape[0], mol.n_atoms, 3), dtype=torch.float64, device=dev)
        og = jkb.make_opts("fp64", n_dm=D.shape[0])
        jkb.jk_grad(ctx, basis, D, G, tol, og)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(2):
            jkb.jk_grad(ctx, basis, D, G, tol, og)
        torch.cuda.synchronize()
        ex["w30_grad_ms"] = 1e3 * (time.perf_counter() - tg) / 2
        ex["w120_dEJ"] = EJ["mixed"] - EJ["fp64"]
        ex["w120_dEK"] = EK["mixed"] - EK["fp64"]
        result["extra"] = ex

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(mol, tol)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
