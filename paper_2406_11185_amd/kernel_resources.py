"""Per-kernel register, LDS and scratch use of the built libjk.so (gfx950).

    python -m paper_2406_11185_amd.kernel_resources [--md OUT.md]

Reads the AMDGPU code-object metadata of this repository's own build: the
object files under _build/obj carry a .hip_fatbin section whose gfx950 code
object lists, per kernel, the unified register count (architectural plus
accumulation VGPRs), the AGPR part of it, the spill counts, the private
(scratch) bytes per lane and the static LDS bytes.  Waves per SIMD follow from
the 512 registers of a lane on CDNA4, allocated in granules of 8.
"""
from __future__ import annotations

import argparse
import os
import re
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OBJ = os.path.join(ROOT, "_build", "obj")
LLVM = "/opt/rocm/llvm/bin"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"


def demangle(names):
    r = subprocess.run(["c++filt"], input="\n".join(names),
                       capture_output=True, text=True, check=True)
    return r.stdout.splitlines()


def kernels_of(obj: str):
    with tempfile.TemporaryDirectory() as td:
        fat = os.path.join(td, "fat")
        co = os.path.join(td, "co")
        r = subprocess.run([os.path.join(LLVM, "llvm-objcopy"), f"--dump-section=.hip_fatbin={fat}",
                            obj, os.path.join(td, "scratch.o")], capture_output=True)
        if r.returncode != 0:   # a host-only object: no device code
            return []
        subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o",
                        f"--input={fat}", f"--targets={TARGET}", f"--output={co}"], check=True,
                       capture_output=True)
        notes = subprocess.run([os.path.join(LLVM, "llvm-readelf"), "--notes", co],
                               capture_output=True, text=True, check=True).stdout
    out = []
    # kernel entries of the amdhsa.kernels list sit at two spaces of indentation
    for blk in re.split(r"\n  - \.", notes)[1:]:
        def f(key):
            m = re.search(rf"(?m)^\s*{key}:\s+(\S+)", "." + blk)
            return m.group(1) if m else None
        name = f(r"\.name")
        if not name or f(r"\.vgpr_count") is None:
            continue
        m = re.search(r"\.args:\s*\n\s*- \.offset:\s+0\s*\n\s*\.size:\s+(\d+)", "." + blk)
        out.append(dict(name=name, vgpr=int(f(r"\.vgpr_count")), agpr=int(f(r"\.agpr_count") or 0),
                        arg0=int(m.group(1)) if m else -1,
                        vspill=int(f(r"\.vgpr_spill_count") or 0),
                        scratch=int(f(r"\.private_segment_fixed_size") or 0),
                        lds=int(f(r"\.group_segment_fixed_size") or 0)))
    return out


def waves_per_simd(vgpr):
    # .vgpr_count is the unified count (architectural + accumulation registers) out of
    # the 512 a lane has on CDNA4, allocated in granules of 8
    return min(8, 512 // max(8, ((vgpr + 7) // 8) * 8))


def host_arg_sizes():
    """sizeof(EriLaunch), sizeof(GradLaunch) as the host compiler lays them out."""
    src = ('#include "jk_grad_device.hpp"\n#include <cstdio>\n'
           'int main() { std::printf("%zu %zu\\n", sizeof(jk::EriLaunch), sizeof(jk::GradLaunch)); }\n')
    with tempfile.TemporaryDirectory() as td:
        p = os.path.join(td, "sz.hip")
        with open(p, "w") as fh:
            fh.write(src)
        exe = os.path.join(td, "sz")
        csrc = os.path.join(ROOT, "paper_2406_11185_amd", "csrc")
        subprocess.run(["/opt/rocm/bin/hipcc", "-std=c++17", "--offload-host-only", "-O0", "-I",
                        os.path.join(ROOT, "include"), "-I", csrc, "-I",
                        os.path.join(ROOT, "_build", "gen"), p, "-o", exe], check=True,
                       capture_output=True)
        e, g = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    return int(e), int(g)


def table():
    rows = []
    for f in sorted(os.listdir(OBJ)):
        if f.endswith(".o"):
            rows += kernels_of(os.path.join(OBJ, f))
    names = demangle([r["name"] for r in rows])
    for r, n in zip(rows, names):
        r["name"] = n.replace("jk::", "").replace("(jk::EriLaunch)", "").replace(
            "(jk::GradLaunch)", "").replace("void ", "")
        r["waves"] = waves_per_simd(r["vgpr"])
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--md", default="")
    a = ap.parse_args()
    rows = table()
    lines = ["| kernel | VGPR (unified) | of which AGPR | VGPR spills | scratch B/lane | static LDS B "
             "| waves/SIMD |",
             "|---|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: r["name"]):
        if r["name"].startswith(("rocprim::", "hipcub::")):
            continue   # the sort and scan kernels of the ROCm libraries
        lines.append(f"| `{r['name']}` | {r['vgpr']} | {r['agpr']} | {r['vspill']} | {r['scratch']} "
                     f"| {r['lds']} | {r['waves']} |")
    text = "\n".join(lines) + "\n"
    if a.md:
        text = ("# Registers, spills, scratch and LDS of every kernel of libjk.so (gfx950)\n\n"
                "From the code-object metadata of this repository's build, written by\n\n"
                "```\npython -m paper_2406_11185_amd.build && "
                f"python -m paper_2406_11185_amd.kernel_resources --md {os.path.relpath(a.md, ROOT)}\n```\n\n"
                "waves/SIMD: the limit the unified register count alone sets (512 per lane).\n\n"
                + text)
        with open(a.md, "w") as fh:
            fh.write(text)
    print(text)


if __name__ == "__main__":
    main()
