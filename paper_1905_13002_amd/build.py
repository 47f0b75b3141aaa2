"""Build libpks.so (HIP for gfx950) in-tree.

    python -m paper_1905_13002_amd.build

Every translation unit is compiled with hipcc for gfx950 only, with packed
FP32 instructions disabled (``-Xclang -target-feature -Xclang
-packed-fp32-ops``), then linked into ``paper_1905_13002_amd/libpks.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpks.so")
BUILD = os.path.join(os.path.dirname(HERE), "_build")

SOURCES = (["scan_large_f64.hip", "scan_large_f32.hip", "scan_large_f64_seg.hip", "scan_large_f32_seg.hip",
            "api.cpp", "plan.cpp", "precompute.hip", "scan_small.hip", "scan_large.hip", "loglik.hip",
            "hmm.hip", "noalloc.hip", "scan_w16.hip"]
           + ["scan_small_n%d_%s.hip" % (n, t) for n in (4, 3, 2, 1) for t in ("f64", "f32")])

# The small-state scan units hold the top-level kernels, whose 4 x 4 products
# run on v_mfma_f64_4x4x4f64.  They are built with MFMA results kept in
# ordinary VGPRs: when a workgroup size left the compiler room for the
# accumulation registers (AGPR form), the same top-level kernel returned wrong
# carries for every item after the first, while the VGPR form (forced here,
# or chosen by the compiler under a tighter register budget) is exact.
PER_FILE = {"scan_small_n%d_%s.hip" % (n, t): ["-mllvm", "-amdgpu-mfma-vgpr-form"]
            for n in (4, 3, 2, 1) for t in ("f64", "f32")}
PER_FILE["scan_w16.hip"] = ["-mllvm", "-amdgpu-mfma-vgpr-form"]

ARCH = os.environ.get("PKS_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unknown-pragmas",
          "-Wno-unused-result", "-Wno-unused-value", "-I" + os.path.join(os.path.dirname(HERE), "include")]


def _compile(src: str, extra) -> str:
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC] + COMMON + PER_FILE.get(src, []) + list(extra) + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stdout))
    msgs = [l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if msgs:
        sys.stderr.write("\n".join(msgs[-40:]) + "\n")
    return obj


def build(extra=(), jobs=None, verbose=True) -> str:
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra), srcs))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stdout))
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT, file=sys.stderr)
    return OUT


def resource_usage(out_md: str) -> None:
    """Compile every unit with the compiler's kernel-resource remarks and
    write a table (registers, scratch, LDS, waves per SIMD per kernel) to
    `out_md`."""
    import re
    rows = {}
    for src in SOURCES:
        if not src.endswith(".hip"):
            continue
        cmd = ([HIPCC] + COMMON + PER_FILE.get(src, []) + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o",
               os.devnull, "-Rpass-analysis=kernel-resource-usage"])
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        cur = None
        for line in r.stdout.splitlines():
            m = re.search(r"remark:\s+Function Name: (\S+)", line)
            if m:
                cur = m.group(1)
                rows.setdefault(cur, {})
                continue
            m = re.search(r"remark:\s+(VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]|"
                          r"LDS Size \[bytes/block\]): (\d+)", line)
            if m and cur:
                rows[cur][m.group(1).split(" ")[0]] = int(m.group(2))
    demangle = shutil.which("llvm-cxxfilt") or shutil.which("c++filt") or "c++filt"
    names = list(rows)
    try:
        dem = subprocess.run([demangle], input="\n".join(names), stdout=subprocess.PIPE, text=True).stdout.split("\n")
    except OSError:
        dem = names
    lines = ["# Kernel resources (compiler: hipcc -Rpass-analysis=kernel-resource-usage, gfx950)", "",
             "Command: `python -m paper_1905_13002_amd.build --resource-usage profiles/kernel_resources.md`.", "",
             "| kernel | VGPRs | AGPRs | scratch B/lane | LDS B/block | waves/SIMD |", "|---|---:|---:|---:|---:|---:|"]
    for raw, d in sorted(zip(names, dem), key=lambda x: x[1]):
        v = rows[raw]
        if not v:
            continue
        short = re.sub(r"pks::(\(anonymous namespace\)::|lg::)?", "", d.strip() or raw)
        short = re.sub(r"\(.*\)$", "", short).replace("void ", "")
        # small-state scans: the nx = 4 instantiations only (nx = 1..3 are alike)
        if re.match(r"k_(filter|smoother)_\w+<[123],", short):
            continue
        lines.append("| `%s` | %s | %s | %s | %s | %s |" % (short, v.get("VGPRs", ""), v.get("AGPRs", ""),
                                                           v.get("ScratchSize", ""), v.get("LDS", ""),
                                                           v.get("Occupancy", "")))
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote", out_md, file=sys.stderr)


if __name__ == "__main__":
    if len(sys.argv) == 3 and sys.argv[1] == "--resource-usage":
        resource_usage(sys.argv[2])
    else:
        build(extra=sys.argv[1:])
