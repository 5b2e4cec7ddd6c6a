"""Benchmark of the direct-SCF J/K build on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload w120] [--precision mixed]
                    [--no-cpu] [--no-extra]

A step is one complete jk_build call: shell-pair data, Cauchy-Schwarz bounds,
Q sort, screening and work lists, every integral+digestion kernel, the
symmetrisation of J and K and the energies E_J, E_K, on a seeded synthetic
molecule whose density is already resident in device memory.  The default
workload is the 120-atom, 1080-function molecule screened at 1e-10 with the
mixed-precision dispatch (FP32 integrals for Schwarz bounds below 1e-4); the
same build in plain FP64 is timed beside it.

Prints one JSON line.  `value` is screened quartets per second of the headline
build (unique shell quartets that pass the Schwarz screen, per build).  The
timed builds launch every class kernel on one stream in turn, so the HIP
events the library records around each launch bracket that kernel's own run
time; `roofline` describes the kernel with the largest share of the step time:
its algorithmic work per launch (flops of the generated recurrence,
horizontal-recurrence and digestion code per quartet, plus a fixed count per
primitive quartet for the Boys function and prefactors) divided by its mean
launch time.  `cpu_baseline` is the CPU oracle timed on a bounded, seeded
sample of bra pairs of the same molecule.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X vector peaks: 256 CU x 2.4 GHz x 64 lanes x 2 flop per FMA.  FP64 and
# unpacked FP32 run one FMA per lane per clock; the FP32 vendor peak (157.3)
# counts packed two-wide FP32 instructions, which these kernels do not use.
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 78.6
FP32_PACKED_PEAK_TFLOPS = 157.3


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


def traffic_file(workload, precision):
    return os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}_{precision}.md")


def atomics_file(workload, precision):
    return os.path.join(ROOT, "profiles", f"valu_atomics_{workload}_{precision}.md")


def source_fingerprint() -> str:
    """Hash of the sources that decide the J/K kernels' code (counter data taken
    with another fingerprint describe other kernels)."""
    from paper_2406_11185_amd.profile_summary import source_fingerprint as fp
    return fp()


def kernel_key(name: str):
    """'eri_jk <class> fp64|fp32' for a J/K class kernel name, else None."""
    import re
    m = re.search(r"jk::eri_jk(?:_lds|_split|_rows)?_kernel<jk::Cls_([a-z]{4})\w*, (double|float)", name)
    if not m:
        return None
    return f"eri_jk {m.group(1)} {'fp64' if m.group(2) == 'double' else 'fp32'}"


def pmc_summary(fetch_csv: str, write_csv: str, out: str, calib_mib: int, command: str,
                title: str) -> None:
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
    lines = [f"# HBM traffic per dispatch: J/K build, {title}", "",
             "Two rocprofv3 counter runs of the benchmark (kernels are serialised while counters "
             "are collected), from the repository root, on an MI355X:", "", "```",
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


def traffic_of(kernel: str, workload: str, precision: str):
    """HBM bytes per dispatch of `kernel` from the committed counter summary, or
    None if there is none or the kernel sources changed since it was taken."""
    try:
        with open(traffic_file(workload, precision)) as fh:
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


def counters_of(kernel: str, workload: str, precision: str):
    """(memory-side atomics per screened quartet, counter VALU fraction of peak) of
    `kernel` from the committed counter summary, or None if there is none or the
    kernel sources changed since it was taken."""
    try:
        with open(atomics_file(workload, precision)) as fh:
            text = fh.read()
    except OSError:
        return None
    if f"source fingerprint: `{source_fingerprint()}`" not in text:
        return None
    for ln in text.splitlines():
        cells = [c.strip() for c in ln.strip().strip("|").split("|")]
        if len(cells) == 10 and cells[0].split(" (")[0] == kernel:
            return float(cells[8]), float(cells[7])
    return None


def cpu_baseline(mol, tol, gpu_quartets, seconds_target=15.0):
    """Oracle timed on a growing seeded sample of unique bra pairs (all their
    kets), its rate extrapolated to the whole build by screened-quartet count."""
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
    rate = kept_total / spent
    return {"value": rate, "unit": "quartets/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{used} of {npair} unique bra shell pairs (seeded), all their ket pairs: "
                      f"{kept_total} screened quartets in {spent:.1f} s; extrapolated to the "
                      f"{gpu_quartets} screened quartets of one build: {gpu_quartets / rate:.0f} s "
                      f"per build (extrapolated)"}


def run_steps(jkb, ctx, basis, D, J, K, tol, opts, steps, torch):
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        jkb.jk_build(ctx, basis, D, J, K, tol, opts)
        stats.append(ctx.stats())     # waits for this step's events
    torch.cuda.synchronize()
    return time.perf_counter() - t0, stats


def class_table(stats, infos, n_dm):
    """Per (class, precision): summed event ms, launches and quartets over the steps."""
    agg = {}
    for s in stats:
        for q in range(21):
            for pr, ms_arr, n_arr, qa in ((0, s.ms_kernel_fp64, s.launches_fp64, s.quartets_fp64),
                                          (1, s.ms_kernel_fp32, s.launches_fp32, s.quartets_fp32)):
                if n_arr[q]:
                    a = agg.setdefault((q, pr), [0.0, 0, 0])
                    a[0] += ms_arr[q]
                    a[1] += n_arr[q]
                    a[2] += qa[q]
    return agg


def progress(msg):
    print(f"[bench] {msg} ({time.strftime('%H:%M:%S')})", file=sys.stderr, flush=True)


def extra_measurements(args, jkb, molgen, ctx, mol, basis, D, J, K, E_head, tol, precision,
                       ms_per_step, torch):
    """The same build in the other precision (time, speedup, energy differences),
    the paper's own FP32 threshold (tolerance x 1e5), the long-range build of a
    range-separated hybrid (omega = 0.3), the SCF steps beside the build
    (diagonalisation, DIIS), the XC integration's grid part, and the nuclear
    gradient:
    of the 30-atom molecule, or of the workload itself (autograd through
    JKEnergy) when it carries several densities."""
    import numpy as np
    dev = D.device
    n_dm = int(D.shape[0])
    ex = {}
    other = "fp64" if precision == "mixed" else "mixed"
    E2 = torch.empty((n_dm, 3), dtype=torch.float64, device=dev)
    J_head, K_head = J.clone(), K.clone()
    o2 = jkb.make_opts(other, n_dm=n_dm, timing=True, serial=True, energy=E2)
    nrep = 2 if n_dm == 1 else 1
    if n_dm == 1:
        jkb.jk_build(ctx, basis, D, J, K, tol, o2)
    t2, _ = run_steps(jkb, ctx, basis, D, J, K, tol, o2, nrep, torch)
    progress(f"{other} builds done")
    E_other = E2.cpu().numpy()
    ex[f"{other}_ms"] = 1e3 * t2 / nrep
    ex[f"{precision}_ms"] = ms_per_step
    fp64_ms = ex["fp64_ms"]
    ex["mixed_speedup_over_fp64"] = fp64_ms / ex["mixed_ms"]
    E64 = E_other if other == "fp64" else E_head
    Emx = E_head if other == "fp64" else E_other
    ex["mixed_dEJ"] = float(np.abs(Emx[:, 0] - E64[:, 0]).max())
    ex["mixed_dEK"] = float(np.abs(Emx[:, 1] - E64[:, 1]).max())
    ex["mixed_max_abs_dJ"] = float((J - J_head).abs().max())
    ex["mixed_max_abs_dK"] = float((K - K_head).abs().max())
    del J_head, K_head
    if n_dm == 1:
        # the paper's own single-precision threshold, tolerance x 1e5
        o3 = jkb.make_opts("mixed", fp32_below=tol * 1e5, n_dm=n_dm, timing=True, serial=True,
                           energy=E2)
        t3, s3 = run_steps(jkb, ctx, basis, D, J, K, tol, o3, 1, torch)
        E3 = E2.cpu().numpy()
        ex["mixed_paper_threshold"] = {
            "fp32_below": tol * 1e5, "ms": 1e3 * t3, "speedup_over_fp64": fp64_ms / (1e3 * t3),
            "quartets_fp32": int(sum(s3[-1].quartets_fp32)),
            "dEJ": float(E3[0, 0] - E64[0, 0]), "dEK": float(E3[0, 1] - E64[0, 1])}
    if n_dm == 1:
        # the long-range exchange integrals of a range-separated hybrid:
        # erf(omega r12)/r12 at omega = 0.3 bohr^-1 (the omegaB97X value), same
        # screening and precision as the headline build
        o4 = jkb.make_opts(precision, n_dm=n_dm, timing=True, serial=True, energy=E2, omega=0.3)
        jkb.jk_build(ctx, basis, D, J, K, tol, o4)
        t4, _ = run_steps(jkb, ctx, basis, D, J, K, tol, o4, 1, torch)
        E4 = E2.cpu().numpy()
        ex["long_range_omega_0.3"] = {
            "precision": precision, "ms": 1e3 * t4, "time_over_1_r12_build": 1e3 * t4 / ms_per_step,
            "E_J": float(E4[0, 0]), "E_K": float(E4[0, 1])}
        progress("long-range (omega 0.3) build done")
    if n_dm == 1:
        # the SCF steps beside the build at the workload's size: Roothaan
        # diagonalisation with the density (n_occ = n/4) and one DIIS step over a
        # full history of 8 pairs; F = J - K/2 of the last build above, S a seeded
        # overlap-like positive-definite matrix
        import math
        n = int(D.shape[1])
        rng = np.random.default_rng(7)
        X = rng.normal(size=(n, n)) * 0.3 / math.sqrt(n)
        S = torch.as_tensor(1.3 * np.eye(n) + 0.5 * (X + X.T), device=dev)
        F = (J[0] - 0.5 * K[0]).contiguous()
        h = jkb.ScfSteps(n, depth=8)
        h.diag(F, S, n // 4)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            _, _, Dn = h.diag(F, S, n // 4)
        torch.cuda.synchronize()
        diag_ms = 1e3 * (time.perf_counter() - t) / 3
        for _ in range(8):
            h.diis(F, Dn, S)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            h.diis(F, Dn, S)
        torch.cuda.synchronize()
        ex["scf_steps"] = {"n": n, "diag_with_density_ms": diag_ms,
                           "diis_depth8_ms": 1e3 * (time.perf_counter() - t) / 3}
        h.close()
        progress("SCF steps (diagonalisation, DIIS) done")
    if n_dm == 1:
        # the XC integration's grid part at the workload's size: a synthetic grid of
        # 50 radial x 110 angular points per atom, rho of the workload's density and
        # V for the grid weight times a smooth synthetic potential; algorithmic work
        # = the 32 x 32 x 32 block products the calls ran (2 * 32^3 flops each)
        pts, wgt = molgen.atom_grid(mol, 50, 110)
        Gd = torch.as_tensor(pts, device=dev)
        wvd = torch.as_tensor(wgt * np.exp(-0.02 * np.sum(pts ** 2, axis=1)), device=dev)
        D0 = D[0].contiguous()
        jkb.xc_rho(mol, Gd, D0)
        jkb.xc_vmat(mol, Gd, wvd)
        xc = {"points": int(len(pts))}
        for name, call in (("rho", lambda t: jkb.xc_rho(mol, Gd, D0, tiles=t)),
                           ("vmat", lambda t: jkb.xc_vmat(mol, Gd, wvd, tiles=t))):
            tiles = torch.zeros(1, dtype=torch.int64, device=dev)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(2):
                call(tiles)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 2
            tf = int(tiles.cpu()[0]) / 2 * 2 * 32 ** 3 / (ms / 1e3) / 1e12
            xc[name] = {"ms": ms, "block_products": int(tiles.cpu()[0]) // 2,
                        "tflops_algorithmic": tf, "frac_of_fp64_vector_peak": tf / 78.6}
        # gradient-corrected terms: rho with grad rho, and V with the grad-rho
        # derivative terms (synthetic derivative weights)
        wgd = torch.stack([wvd * (0.5 + 0.1 * c) for c in range(3)]).contiguous()
        jkb.xc_rho_gga(mol, Gd, D0)
        jkb.xc_vmat_gga(mol, Gd, wvd, wgd)
        for name, call in (("rho_gga", lambda: jkb.xc_rho_gga(mol, Gd, D0)),
                           ("vmat_gga", lambda: jkb.xc_vmat_gga(mol, Gd, wvd, wgd))):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(2):
                call()
            e1.record()
            torch.cuda.synchronize()
            xc[name] = {"ms": e0.elapsed_time(e1) / 2}
        ex["xc_grid"] = xc
        progress("XC grid part (rho, V, and their gradient-corrected forms) done")
    if n_dm == 1 and args.with_grad:
        # nuclear gradient of the 30-atom molecule, FP64 and mixed
        mg = molgen.workload("w30grad")
        bg = jkb.Basis(mg)
        tg_tol = molgen.WORKLOADS["w30grad"]["tol"]
        Dg = torch.as_tensor(mg.D, device=dev).contiguous()
        G = torch.empty((Dg.shape[0], mg.n_atoms, 3), dtype=torch.float64, device=dev)
        for prec in ("fp64", "mixed"):
            og = jkb.make_opts(prec, n_dm=int(Dg.shape[0]))
            jkb.jk_grad(ctx, bg, Dg, G, tg_tol, og)
            torch.cuda.synchronize()
            tg = time.perf_counter()
            for _ in range(2):
                jkb.jk_grad(ctx, bg, Dg, G, tg_tol, og)
            torch.cuda.synchronize()
            ex[f"w30_grad_{prec}_ms"] = 1e3 * (time.perf_counter() - tg) / 2
    elif args.with_grad:
        # the workload's own gradient, mixed through autograd (forward build and
        # backward derivative kernels), and the FP64 gradient for the error
        xyz = torch.tensor(mol.xyz, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        Eg = jkb.JKEnergy.apply(xyz, D, mol, tol, "mixed")
        torch.cuda.synchronize()
        ex["autograd_forward_mixed_s"] = time.perf_counter() - t
        progress("autograd forward done")
        t = time.perf_counter()
        Eg.sum().backward()
        torch.cuda.synchronize()
        ex["grad_mixed_s"] = time.perf_counter() - t
        progress("autograd backward (mixed gradient) done")
        Gm = xyz.grad.numpy().copy()
        G = torch.empty((n_dm, mol.n_atoms, 3), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        jkb.jk_grad(ctx, basis, D, G, tol, jkb.make_opts("fp64", n_dm=n_dm))
        torch.cuda.synchronize()
        ex["grad_fp64_s"] = time.perf_counter() - t
        progress("FP64 gradient done")
        G64 = G.cpu().numpy().sum(axis=0)
        ex["grad_mixed_max_abs_err_vs_fp64"] = float(np.abs(Gm - G64).max())
    return ex


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="w120")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--with-grad", action="store_true",
                    help="also time the nuclear gradient (jk_grad), which is kept off the GPU "
                         "by default while a fault in it is open")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="before the steps, copy a buffer of this many MiB once (a kernel of "
                         "known traffic for scaling hardware byte counters)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the per-dispatch HBM traffic summary from two rocprofv3 "
                         "counter_collection.csv files and exit (no GPU use)")
    ap.add_argument("--pmc-command", default="",
                    help="with --pmc-summary: the profiled command, PMC standing for the counter")
    args = ap.parse_args()
    from paper_2406_11185_amd import molgen
    w = molgen.WORKLOADS[args.workload]
    precision = args.precision or w["precision"]
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], traffic_file(args.workload, precision),
                    args.copy_calib_mib or 256, args.pmc_command, f"{w['desc']}, {precision}")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2406_11185_amd import jk as jkb

    tol = w["tol"]
    mol = molgen.workload(args.workload)
    basis = jkb.Basis(mol)
    dev = torch.device("cuda:0")
    D = torch.as_tensor(mol.D, device=dev).contiguous()
    n_dm = int(D.shape[0])
    J = torch.empty_like(D)
    K = torch.empty_like(D)
    E = torch.empty((n_dm, 3), dtype=torch.float64, device=dev)
    ctx = jkb.Context(0)
    opts = jkb.make_opts(precision, n_dm=n_dm, timing=True, serial=True, energy=E)

    if args.copy_calib_mib:
        src = torch.ones(args.copy_calib_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        jkb.jk_build(ctx, basis, D, J, K, tol, opts)
    torch.cuda.synchronize()
    if args.warmup:
        progress(f"{args.warmup} warmup {precision} builds done")
    total, stats = run_steps(jkb, ctx, basis, D, J, K, tol, opts, args.steps, torch)
    progress(f"{args.steps} timed {precision} builds done")
    ms_per_step = 1e3 * total / args.steps
    st = stats[-1]
    quartets = sum(st.quartets_fp64) + sum(st.quartets_fp32)
    E_head = E.cpu().numpy().copy()

    # dominant kernel: the class launch with the largest share of the step time
    # (serial launches: each event interval is that kernel's own run time)
    infos = class_info()
    agg = class_table(stats, infos, n_dm)
    (qd, prd), (ms_sum, nlaunch, nq) = max(agg.items(), key=lambda kv: kv[1][0])
    info = infos[qd]
    flops_launch = flops_per_quartet(info, n_dm=n_dm) * nq / nlaunch
    mean_s = ms_sum / nlaunch / 1e3
    achieved = flops_launch / mean_s / 1e12
    peak = FP64_PEAK_TFLOPS if prd == 0 else FP32_PEAK_TFLOPS
    kname = f"eri_jk {info['name']} {'fp32' if prd else 'fp64'}"
    total_kernel_ms = sum(a[0] for a in agg.values()) / len(stats)
    total_flops = 0.0
    for (q, pr), a in agg.items():
        total_flops += flops_per_quartet(infos[q], n_dm=n_dm) * a[2] / len(stats)
    roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic_of(kname, args.workload, precision),
            "kernel": kname, "flops_per_launch": flops_launch, "mean_launch_ms": mean_s * 1e3,
            "launches": nlaunch}
    cn = counters_of(kname, args.workload, precision)
    if cn:
        # FETCH_SIZE / WRITE_SIZE of these kernels are mostly memory-side FP64 atomics
        roof["memory_side_atomics_per_launch"] = cn[0] * nq / nlaunch
        roof["counter_valu_frac"] = cn[1]
    if prd == 1:
        roof["peak_packed_fp32"] = FP32_PACKED_PEAK_TFLOPS
        roof["frac_of_packed_fp32"] = achieved / FP32_PACKED_PEAK_TFLOPS
    result = {
        "metric": "J+K build: screened ERI quartets/s (FP64 vs mixed build seconds and gradient "
                  "seconds in extra)",
        "value": quartets / (total / args.steps),
        "unit": "quartets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {w['desc']}", "atoms": mol.n_atoms,
                   "basis_functions": mol.n_bf, "tol": tol, "precision": precision,
                   "fp32_below": 1e-4 if precision == "mixed" else None,
                   "n_dm": n_dm, "screened_quartets": int(quartets),
                   "quartets_fp32": int(sum(st.quartets_fp32)),
                   "skipped_quartets": int(st.quartets_skipped), "launches": "serial"},
        "roofline": roof,
        "build_kernel_ms": total_kernel_ms,
        "classes": {f"{infos[q]['name']}_{'fp32' if pr else 'fp64'}":
                    {"ms": round(a[0] / len(stats), 3), "quartets": int(a[2] / len(stats)),
                     "tflops": round(flops_per_quartet(infos[q], n_dm=n_dm) * a[2]
                                     / (a[0] / 1e3) / 1e12, 3) if a[0] > 0 else None}
                    for (q, pr), a in sorted(agg.items())},
        # algorithmic flops of all class launches of a step over the step time
        "build_tflops": total_flops / (ms_per_step / 1e3) / 1e12,
        "setup_ms": st.ms_setup,
        "energies": {"E_J": float(E_head[0, 0]), "E_K": float(E_head[0, 1])},
    }

    if not args.no_extra:
        result["extra"] = extra_measurements(args, jkb, molgen, ctx, mol, basis, D, J, K, E_head,
                                             tol, precision, ms_per_step, torch)

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(mol, tol, quartets)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
