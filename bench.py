#!/usr/bin/env python3
"""Benchmark: parallel Kalman filter + RTS smoother on one MI355X.

Default workload: the 2-D constant-velocity tracking model (Section V of the
paper), one sequence of T = 2**20 steps, nx = 4, ny = 2.  One "step" of the
benchmark is one full pass of the hot path: model precompute, the forward
filtering scan (Lemmas 1-2) and the reverse smoothing scan (Lemmas 3-4) over
all T time steps, through the C ABI (pks_filter_smooth) on device-resident
inputs.  The headline value is FP64 smoothed time steps per second; the mixed
FP32 mode is measured the same way and reported beside it, with the maximum
per-step relative error of every result against the sequential FP64 oracle.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 2|4]
    python bench.py --op loglik [--workload 2|4]

With --op loglik a step is instead one evaluation of the marginal likelihood
(Section III-C) from filtered moments already in HBM: every factor
log p(y_k | y_1:k-1), every partial sum log p(y_1:k) and the totals
(pks_loglik with cumulative output).

Prints exactly one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector (= 256 CU x 2.4 GHz x 128 flop/clk)
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector, published

# Algorithmic work per time step and kernel.  Flops of the operators,
# counted as the paper's experiment counts them (matrix product 2mnk, LU
# 2n^3/3, Cholesky n^3/3, triangular solve pair 2n^2 per right-hand side):
#   filtering combine (Lemma 2)               16.7 n^3 + 10 n^2
#   filtering combine, prefix with A = 0       8.7 n^3 +  6 n^2
#   filtering element (Lemma 1, b_k, eta_k)    4 n ny
#   smoothing element (Lemma 3)                8.3 n^3 +  6 n^2
#   smoothing combine (Lemma 4)                6 n^3   +  2 n^2
#   smoothing combine, suffix with E = 0       4 n^3   +  2 n^2
# (at n = 4: 1227, 651, 32, 629, 416, 288).  Bytes: the method's own traffic
# (y in, filtered moments out; filtered moments in, smoothed moments out).
def op_flops(n, ny):
    return dict(f_full=16.67 * n ** 3 + 10 * n * n, f_carry=8.67 * n ** 3 + 6 * n * n, f_elem=4 * n * ny,
                s_elem=8.33 * n ** 3 + 6 * n * n, s_full=6 * n ** 3 + 2 * n * n, s_carry=4 * n ** 3 + 2 * n * n)


def kernel_model(nx, ny, rs, tv=False):
    mom = (nx + nx * nx) * rs
    f = op_flops(nx, ny)
    # time-varying model: the precompute builds every step's constants from its
    # own model rows (F, Q, u, H, d, R in; the Lemma 1 factors S = L L^T, K,
    # A, C, J, W and the first-step element are counted as products/solves)
    rows = (2 * nx * nx + nx + ny * nx + ny + ny * ny) * 8
    pre_flops = (2 * ny * nx * nx + 2 * ny * ny * nx + ny ** 3 / 3 + 4 * ny * ny * nx
                 + 3 * 2 * nx * nx * ny + 2 * nx * nx * nx)
    per_step = {
        "reduce_f": dict(bytes=ny * rs, flops=f["f_full"] + f["f_elem"]),
        "down_f": dict(bytes=ny * rs + mom, flops=f["f_carry"] + f["f_elem"]),
        "reduce_s": dict(bytes=mom, flops=f["s_elem"] + f["s_full"]),
        "down_s": dict(bytes=2 * mom, flops=f["s_elem"] + f["s_carry"]),
        # filter down-sweep fused with the smoother reduce: the filtered moments
        # are written once and folded into smoothing elements from registers
        "down_f_reduce_s": dict(bytes=ny * rs + mom, flops=f["f_carry"] + f["f_elem"] + f["s_elem"] + f["s_full"]),
    }
    out = {
        "k_filter_down_smooth_reduce": per_step["down_f_reduce_s"],
        "k_filter_reduce": per_step["reduce_f"], "k_large_filter_reduce": per_step["reduce_f"],
        "k_filter_down": per_step["down_f"], "k_large_filter_down": per_step["down_f"],
        "k_smoother_reduce": per_step["reduce_s"], "k_large_smoother_reduce": per_step["reduce_s"],
        "k_smoother_down": per_step["down_s"], "k_large_smoother_down": per_step["down_s"],
        "k_w16_filter_reduce": per_step["reduce_f"], "k_w16_filter_down": per_step["down_f"],
        "k_w16_smoother_reduce": per_step["reduce_s"], "k_w16_smoother_down": per_step["down_s"],
    }
    if tv:
        out["k_precompute"] = dict(bytes=rows, flops=pre_flops)
    return out


def ll_kernel_model(nx, ny, rs):
    """Per-step algorithmic work of the likelihood kernels: the factor kernel
    reads y_k and the moments of step k-1 and writes one double; its flops are
    G P G^T (lower half), the residual, a Cholesky factorisation and one
    triangular solve.  The block scan reads and writes one double per step."""
    flops = 2 * ny * nx * nx + ny * (ny + 1) * nx + 2 * ny * nx + ny ** 3 / 3 + ny * ny + 6 * ny
    k = dict(bytes=(ny + nx + nx * nx) * rs + 8, flops=flops)
    return {"k_ll_steps": k, "k_ll_block_scan": dict(bytes=16, flops=1), "k_ll_fixup": dict(bytes=16, flops=1)}


KERNEL_SOURCES = ["paper_1905_13002_amd/csrc/small_ops.hpp", "paper_1905_13002_amd/csrc/scan_small_impl.hpp",
                  "paper_1905_13002_amd/csrc/top_epl.hpp", "paper_1905_13002_amd/csrc/precompute.hip"]


def sources_sha():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name, precision, kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload_name)
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("sources_sha") != sources_sha():
        return None
    ent = rec.get("kernels", {}).get("%s/%s" % (precision, kernel))
    if not ent:
        return None
    return ent.get("hbm_bytes_per_launch")


def measured_pass_traffic(workload_name, precision):
    """HBM bytes of one whole pass (every kernel's counter bytes per launch,
    summed) from the committed counter summary, if it was taken on the current
    kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload_name)
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("sources_sha") != sources_sha():
        return None
    ks = [v for k, v in rec.get("kernels", {}).items() if k.startswith(precision + "/")]
    if not ks:
        return None
    return int(sum(v.get("hbm_bytes_per_launch", 0) for v in ks))


# rocprofv3 runs that the committed kernel profile of the default workload
# comes from (run from the repository root, then summarised with
# `python bench.py --summarize-profiles gpurun_out`)
PROFILE_COMMANDS = [
    "rocprofv3 --kernel-trace --stats -d gpurun_out/prof_trace -o trace -- "
    "python bench.py --steps 5 --warmup 2 --no-cpu-baseline",
    "rocprofv3 --pmc FETCH_SIZE -d gpurun_out/prof_fetch -o fetch -- "
    "python bench.py --steps 2 --warmup 1 --no-cpu-baseline --copy-calibration",
    "rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof_write -o write -- "
    "python bench.py --steps 2 --warmup 1 --no-cpu-baseline --copy-calibration",
]


def summarize_profiles(base, workload_name):
    """Write profiles/<workload>_kernels.md and profiles/traffic_<workload>.json
    from the three rocprofv3 databases under `base` (kernel trace statistics,
    FETCH_SIZE and WRITE_SIZE per dispatch).  The HBM byte counters are scaled
    by what they read for the calibration kernel of --copy-calibration (an
    elementwise multiply that reads 1 GiB and writes 1 GiB)."""
    import collections
    import re
    import sqlite3

    def short(n):
        n = n.replace("pks::(anonymous namespace)::", "").replace("pks::", "")
        m = re.match(r"void (\w+<[^>]*>)", n)
        return m.group(1) if m else n

    def find_db(d):
        for f in sorted(os.listdir(d)):
            if f.endswith("_results.db"):
                return os.path.join(d, f)
        raise FileNotFoundError("no *_results.db under %s" % d)

    cur = sqlite3.connect(find_db(os.path.join(base, "prof_trace"))).cursor()
    # top_kernels: name, total_calls, total_duration, average (microseconds), percentage
    trace = [(short(r[0]), int(r[1]), float(r[3])) for r in
             cur.execute("select name, total_calls, total_duration, average from top_kernels")]

    def counters(sub, name):
        c = sqlite3.connect(find_db(os.path.join(base, sub))).cursor()
        d = collections.defaultdict(list)
        for kn, v in c.execute("select kernel_name, value from counters_collection where counter_name=?", (name,)):
            d[short(kn)].append(float(v))
        return d

    fetch = counters("prof_fetch", "FETCH_SIZE")
    write = counters("prof_write", "WRITE_SIZE")
    calib = [k for k in fetch if "elementwise" in k and "Mul" in k]
    if not calib:
        raise RuntimeError("calibration kernel not found: run the counter passes with --copy-calibration")
    cal_f = statistics.median(fetch[calib[0]])
    cal_w = statistics.median(write[calib[0]])
    gib_kib = float(1 << 20)
    fs, ws_ = gib_kib / cal_f, gib_kib / cal_w
    med = lambda v: statistics.median(v) if v else float("nan")
    rows, kernels = [], {}
    for name, calls, avg in trace:
        if not name.startswith("k_"):
            continue
        f_k, w_k = med(fetch.get(name, [])), med(write.get(name, []))
        hbm = (f_k * fs + w_k * ws_) * 1024.0
        rows.append((name, calls, avg, f_k / 1024.0, w_k / 1024.0, hbm / (1 << 20)))
        prec = "fp64" if "double" in name else "mixed"
        key = "%s/%s" % (prec, name.split("<")[0])
        if key not in kernels:
            kernels[key] = dict(kernel=name, avg_us=round(avg, 3), fetch_kib_raw=f_k, write_kib_raw=w_k,
                                hbm_bytes_per_launch=int(round(hbm)))
    rec = dict(workload=workload_name, sources_sha=sources_sha(), fetch_scale=round(fs, 4),
               write_scale=round(ws_, 4),
               note="HBM bytes per launch = FETCH_SIZE*fetch_scale + WRITE_SIZE*write_scale (KiB), "
                    "median over dispatches", kernels=kernels)
    with open(os.path.join(ROOT, "profiles", "traffic_%s.json" % workload_name), "w") as fh:
        json.dump(rec, fh, indent=1)
    lines = ["# Kernel profile: %s, filter + smoother" % workload_name, "",
             "`rocprofv3` on one MI355X, library built from this tree.  Commands (repository root):", "", "```"]
    lines += PROFILE_COMMANDS + ["python bench.py --summarize-profiles gpurun_out", "```", "",
                                 "Each bench run times the FP64 path and then the mixed path; `avg_us` is "
                                 "rocprofv3's mean kernel duration over all dispatches (warm-up included).", "",
                                 "Counter calibration (`--copy-calibration`, elementwise multiply of 2^28 float32: "
                                 "1 GiB read, 1 GiB written): FETCH_SIZE %.0f KiB, WRITE_SIZE %.0f KiB per dispatch, "
                                 "so HBM bytes = FETCH_SIZE x %.3f + WRITE_SIZE x %.3f." % (cal_f, cal_w, fs, ws_), "",
                                 "| kernel | calls | avg_us | FETCH_SIZE MiB (raw) | WRITE_SIZE MiB (raw) | "
                                 "HBM MiB (scaled) |", "|---|---:|---:|---:|---:|---:|"]
    for name, calls, avg, f_m, w_m, h_m in rows:
        lines.append("| `%s` | %d | %.1f | %.1f | %.1f | %.1f |" % (name, calls, avg, f_m, w_m, h_m))
    with open(os.path.join(ROOT, "profiles", "%s_kernels.md" % workload_name), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote profiles/%s_kernels.md and profiles/traffic_%s.json" % (workload_name, workload_name))


COUNTER_PASSES = [
    "SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_WAIT_INST_ANY SQ_INSTS_LDS "
    "SQ_INSTS_VALU_FMA_F64 GRBM_GUI_ACTIVE",
    "SQ_LDS_BANK_CONFLICT SQ_INSTS_SALU SQ_INSTS_VMEM SQ_INSTS_VALU_TRANS_F64 SQ_INSTS_VALU_MUL_F64 "
    "SQ_INSTS_VALU_ADD_F64 SQ_WAIT_ANY SQ_THREAD_CYCLES_VALU",
    "SQ_INSTS_MFMA SQ_VALU_MFMA_BUSY_CYCLES SQ_WAVE_CYCLES SQ_WAVES",
]


def counter_commands(wid, base="gpurun_out"):
    """The rocprofv3 passes behind profiles/<workload>_counters.md (one timed
    step each; the large-state workloads without the oracle check)."""
    extra = " --steps 2 --warmup 1" if wid == 2 else " --workload %d --steps 1 --warmup 0 --no-check" % wid
    return ["rocprofv3 --pmc %s -d %s/pmc_%s -o pmc -- python bench.py%s --no-cpu-baseline"
            % (cnt, base, "abc"[i], extra) for i, cnt in enumerate(COUNTER_PASSES)]


def summarize_counters(base, wid):
    """Write profiles/<workload>_counters.md from the rocprofv3 --pmc
    databases under base/pmc_a, pmc_b and pmc_c (median over dispatches):
    instruction mix, how busy the vector unit and the matrix cores are, LDS
    bank conflicts, per kernel."""
    from paper_1905_13002_amd import workloads as wl
    workload_name = wl.WORKLOAD_NAMES[wid]
    import collections
    import re
    import sqlite3

    def short(n):
        n = n.replace("pks::(anonymous namespace)::", "").replace("pks::", "").replace("lg::", "").replace("w16::", "")
        m = re.match(r"void (\w+<[^>]*>)", n)
        return m.group(1) if m else n

    vals = collections.defaultdict(dict)
    for sub in ("pmc_a", "pmc_b", "pmc_c"):
        d = os.path.join(base, sub)
        if not os.path.isdir(d):
            continue
        dbs = [f for f in sorted(os.listdir(d)) if f.endswith("_results.db")]
        cur = sqlite3.connect(os.path.join(d, dbs[0])).cursor()
        acc = collections.defaultdict(list)
        for kn, cn, v in cur.execute("select kernel_name, counter_name, value from counters_collection"):
            acc[(short(kn), cn)].append(float(v))
        for (kn, cn), v in acc.items():
            vals[kn][cn + ("_C" if sub == "pmc_c" and cn in ("SQ_WAVE_CYCLES", "SQ_WAVES") else "")] = \
                statistics.median(v)
    lines = ["# Counter profile: %s" % workload_name, "",
             "`rocprofv3 --pmc` on one MI355X, library built from this tree; two passes (repository root):", "",
             "```"]
    lines += counter_commands(wid, base)
    lines += ["python bench.py --summarize-counters %s%s" % (base, "" if wid == 2 else " --workload %d" % wid),
              "```", "",
              "Per kernel (median over dispatches): `VALU/wave` = SQ_INSTS_VALU / SQ_WAVES; `VALU busy` = "
              "SQ_ACTIVE_INST_VALU x 4 / (SQ_WAVE_CYCLES x 4): the share of a wave's lifetime spent issuing "
              "vector instructions (both counters in quad-cycles); `FMA64 share` = SQ_INSTS_VALU_FMA_F64 / "
              "SQ_INSTS_VALU; `wait` = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES; `MFMA/wave` = SQ_INSTS_MFMA / "
              "SQ_WAVES; `MFMA busy` = SQ_VALU_MFMA_BUSY_CYCLES / SQ_WAVE_CYCLES (third pass: matrix-core busy "
              "cycles per wave cycle); `bank conflicts/LDS` = "
              "SQ_LDS_BANK_CONFLICT / SQ_INSTS_LDS (conflict cycles per LDS instruction).  Register counts "
              "and waves per SIMD are the compiler's (`hipcc -Rpass-analysis=kernel-resource-usage`).", "",
              "| kernel | waves | VALU/wave | VALU busy | FMA64 share | LDS/wave | VMEM/wave | wait | "
              "bank conflicts/LDS | MFMA/wave | MFMA busy |",
              "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for kn in sorted(vals):
        if not kn.startswith("k_"):
            continue
        v = vals[kn]
        w = max(1.0, v.get("SQ_WAVES", 1.0))
        wc = max(1.0, v.get("SQ_WAVE_CYCLES", 1.0))
        lines.append("| `%s` | %d | %.0f | %.2f | %.2f | %.0f | %.0f | %.2f | %.2f | %.0f | %.2f |" % (
            kn, w, v.get("SQ_INSTS_VALU", 0) / w, v.get("SQ_ACTIVE_INST_VALU", 0) / wc,
            v.get("SQ_INSTS_VALU_FMA_F64", 0) / max(1.0, v.get("SQ_INSTS_VALU", 1.0)),
            v.get("SQ_INSTS_LDS", 0) / w, v.get("SQ_INSTS_VMEM", 0) / w, v.get("SQ_WAIT_INST_ANY", 0) / wc,
            v.get("SQ_LDS_BANK_CONFLICT", 0) / max(1.0, v.get("SQ_INSTS_LDS", 1.0)),
            v.get("SQ_INSTS_MFMA", 0) / w,
            v.get("SQ_VALU_MFMA_BUSY_CYCLES", 0) / max(1.0, v.get("SQ_WAVE_CYCLES_C", v.get("SQ_WAVE_CYCLES", 1.0)))))
    with open(os.path.join(ROOT, "profiles", "%s_counters.md" % workload_name), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote profiles/%s_counters.md" % workload_name)


def progress(msg):
    """One line per finished phase on stderr (the JSON result alone goes to stdout)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def summarize_trace(base, wid, op="filter_smooth"):
    """Write profiles/<workload>_kernels.md (loglik_<workload>_kernels.md for
    --op loglik) from a rocprofv3 kernel trace of `bench.py --workload wid`
    under `base` (calls and mean duration per kernel)."""
    import sqlite3
    import re
    from paper_1905_13002_amd import workloads as wl
    name = wl.WORKLOAD_NAMES[wid]
    ll = op == "loglik"
    hmm = op == "hmm"
    if hmm:
        name, wid = wl.WORKLOAD_NAMES[7], 7
    opt = " --op loglik" if ll else (" --op hmm" if hmm else "")
    db = [f for f in sorted(os.listdir(base)) if f.endswith("_results.db")]
    if not db:
        raise FileNotFoundError("no *_results.db under %s" % base)
    cur = sqlite3.connect(os.path.join(base, db[0])).cursor()
    rows = []
    for n, calls, tot, avg in cur.execute("select name, total_calls, total_duration, average from top_kernels"):
        n = n.replace("pks::(anonymous namespace)::", "").replace("pks::lg::", "").replace("pks::w16::", "").replace("pks::", "")
        m = re.match(r"void (\w+<[^>]*>)", n)
        n = m.group(1) if m else n
        if n.startswith("k_"):
            rows.append((n, int(calls), float(avg), float(tot)))
    cmd = ("rocprofv3 --kernel-trace --stats -d %s -o trace -- python bench.py --workload %d%s --steps 2 "
           "--warmup 1 --no-cpu-baseline --no-check" % (base.rstrip("/"), wid, opt))
    what = ("marginal likelihood (filter, then factors + partial sums + totals)" if ll else
            ("discrete-state filter + smoother (FP64)" if hmm else "filter + smoother"))
    lines = ["# Kernel profile: %s, %s" % (name, what), "",
             "`rocprofv3` kernel trace on one MI355X, library built from this tree.  Commands (repository root):", "",
             "```", cmd, "python bench.py --summarize-trace %s --workload %d%s" % (base.rstrip("/"), wid, opt),
             "```", "",
             ("The bench runs the FP64 pass (warm-up, timed passes and passes with HIP events); " if hmm else
              "The bench runs the FP64 path and then the mixed path (warm-up, timed passes and one pass with HIP "
              "events each); ") + "`avg_us` is the mean kernel duration over all dispatches, `total_ms` the sum.", "",
             "| kernel | calls | avg_us | total_ms |", "|---|---:|---:|---:|"]
    for n, calls, avg, tot in rows:
        lines.append("| `%s` | %d | %.1f | %.2f |" % (n, calls, avg, tot / 1e3))
    out = ("loglik_" if ll else "") + name
    with open(os.path.join(ROOT, "profiles", "%s_kernels.md" % out), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote profiles/%s_kernels.md" % out)


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", type=int, default=2, choices=[1, 2, 3, 4, 5, 6, 7])
    ap.add_argument("--op", default="filter_smooth", choices=["filter_smooth", "loglik", "hmm"],
                    help="what a timed step runs (default: the filter + smoother pass)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the comparison with the oracle (profiling runs; the line then has no max_rel_err)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle time for the CPU baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters under rocprofv3)")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="summarise the rocprofv3 databases under DIR into profiles/ and exit")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="summarise the two rocprofv3 --pmc counter passes under DIR into profiles/ and exit")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="summarise a rocprofv3 kernel trace of --workload under DIR into profiles/ and exit")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles, "cv_T1048576")
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.workload)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.workload, args.op)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on exactly one GPU (the scan of one GPU's share); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import oracle
    from paper_1905_13002_amd import pks, workloads as wl

    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # an elementwise kernel that reads 1 GiB and writes 1 GiB once
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.op == "hmm" or args.workload == 7:   # workload 7 is the discrete-state model
        bench_hmm(args, np, torch, oracle, pks, wl)
        return
    w = wl.workload(args.workload)
    progress("workload %s generated (%d steps, %d sequences)" % (w.name, w.total, w.B))
    if args.op == "loglik":
        bench_loglik(args, w, np, torch, oracle, pks, wl, dev)
        return
    T = w.total
    nx, ny = w.model.nx, w.model.ny
    batched = w.B > 1
    tv = w.time_varying
    dm = pks.to_device(w.model, device=dev, per_sequence=w.per_sequence, time_varying=tv)
    off = torch.as_tensor(w.offsets).to(dev) if batched else None

    results = {}
    for prec in ("fp64", "mixed"):
        rdt = torch.float64 if prec == "fp64" else torch.float32
        y = torch.as_tensor(w.y).to(dev, rdt)
        m = torch.empty((T, nx), dtype=rdt, device=dev)
        P = torch.empty((T, nx, nx), dtype=rdt, device=dev)
        ms = torch.empty_like(m)
        Ps = torch.empty_like(P)
        ws = pks.workspace(nx, ny, T, w.B, prec, dev, time_varying=tv)
        # the pass two ways: replays of the captured pass (pks_plan_create /
        # pks_plan_launch: precompute, filter and smoother in one HIP graph)
        # and the eager calls (into buffers of their own).  The timed step is
        # the plan for packed sequences and the eager call for one sequence
        # (where the replay measured a few per cent slower); the other is
        # reported beside it.
        plan = pks.Plan(dm, y, off, prec)
        plan_sec = time_steps(plan.launch, args.steps, args.warmup, torch)
        if batched:
            eager = lambda: (pks.smooth_batched(dm, off, *pks.filter_batched(dm, off, y, prec, ws=ws, out=(m, P)),
                                                prec, ws=ws, out=(ms, Ps)))
        else:
            eager = lambda: pks.filter_smooth(dm, y, prec, ws=ws, out=(m, P, ms, Ps))
        eager_sec = time_steps(eager, args.steps, args.warmup, torch)
        sec = plan_sec if batched else eager_sec
        # per-kernel durations: HIP events around every launch of the eager
        # path (graph replays hide individual launches), same workload
        pks.profile_start()
        for _ in range(args.steps):
            eager()
        prof = pks.profile_stop()
        torch.cuda.synchronize()
        # the checked outputs: the timed path's
        src = (plan.m, plan.P, plan.ms, plan.Ps) if batched else (m, P, ms, Ps)
        out = {k: v.double().cpu().numpy() for k, v in zip(("m", "P", "ms", "Ps"), src)}
        plan.close()
        results[prec] = dict(sec=sec, plan_sec=plan_sec, eager_sec=eager_sec, prof=prof, out=out)
        progress("%s timed: %.4f ms per pass (plan replay %.4f ms, eager calls %.4f ms)"
                 % (prec, sec * 1e3, plan_sec * 1e3, eager_sec * 1e3))

    # accuracy against the oracle (FP64; the mixed reference uses the float32-rounded y).
    # Batched workloads: a sample of sequences (first, last and evenly spaced).
    sample = list(range(w.B))
    if batched:
        budget = 3e10                                  # oracle flops allowed for the check
        per_seq = max(1.0, T / w.B * 20.0 * nx ** 3)
        k = int(max(2, min(w.B, budget // per_seq)))
        sample = sorted(set([0, w.B - 1] + list(range(0, w.B, max(1, w.B // k)))[:k]))

    def ref_for(prec, b=None):
        yy = w.y if prec == "fp64" else w.y.astype(np.float32).astype(np.float64)
        if b is None:
            run = oracle.kf_rts_tv if tv else oracle.kf_rts
            return run(w.model.F, w.model.Q, w.model.H, w.model.R, w.model.m0, w.model.P0, yy)
        mo = w.model_of(b)
        return oracle.kf_rts(mo.F, mo.Q, mo.H, mo.R, mo.m0, mo.P0, yy[w.seq(b)])

    errs = {}
    for prec in ("fp64", "mixed"):
        out = results[prec]["out"]
        if args.no_check:
            errs[prec] = {k: float("nan") for k in ("m", "P", "ms", "Ps")}
            continue
        if not batched:
            ref = ref_for(prec)
            errs[prec] = {k: wl.max_rel_err(out[k], ref[k]) for k in ("m", "P", "ms", "Ps")}
            progress("%s checked against the oracle" % prec)
        else:
            e = {k: 0.0 for k in ("m", "P", "ms", "Ps")}
            for i, b in enumerate(sample):
                ref = ref_for(prec, b)
                for key in e:
                    e[key] = max(e[key], wl.max_rel_err(out[key][w.seq(b)], ref[key]))
                if (i + 1) % 512 == 0:
                    progress("%s: %d of %d sampled sequences checked" % (prec, i + 1, len(sample)))
            errs[prec] = e
            progress("%s checked against the oracle on %d sequences" % (prec, len(sample)))

    # one sequence of one model with 5 <= nx <= 16 runs the register-resident
    # path, whose arithmetic is FP64 in both precisions
    f64_mixed = (not batched) and (not tv) and 5 <= nx <= 16 and ny <= 16

    # roofline of the dominant kernel (FP64 headline)
    def roofline(prec):
        rs = 8 if prec == "fp64" else 4
        model = kernel_model(nx, ny, rs, tv)
        prof = results[prec]["prof"]
        per_launch = {k: tot / max(1, n) for k, (tot, n) in prof.items()}
        dom = max(per_launch, key=per_launch.get)
        dur_s = per_launch[dom] * 1e-3
        km = model.get(dom)
        if km is None:
            return dom, per_launch, None
        t_mem = km["bytes"] * T / (HBM_PEAK_GBS * 1e9)
        peak_f = FP64_PEAK_TFLOPS if (prec == "fp64" or f64_mixed) else FP32_PEAK_TFLOPS
        t_alu = km["flops"] * T / (peak_f * 1e12)
        tr = measured_traffic(w.name, prec, dom)
        if t_mem >= t_alu:
            ach = km["bytes"] * T / dur_s / 1e9
            rl = dict(bound="hbm", achieved=round(ach, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(ach / HBM_PEAK_GBS, 4), traffic=tr)
        else:
            ach = km["flops"] * T / dur_s / 1e12
            rl = dict(bound="alu", achieved=round(ach, 3), peak=peak_f, unit="TFLOP/s",
                      frac=round(ach / peak_f, 4), traffic=tr)
        rl.update(kernel=dom, kernel_ms=round(per_launch[dom], 4),
                  algorithmic_bytes_per_launch=km["bytes"] * T, algorithmic_flops_per_launch=km["flops"] * T)
        return dom, per_launch, rl

    def pass_roofline(prec, sec, dom_rl):
        """The whole pass against its binding roofline: the method's own
        traffic, ny + 3 (nx + nx^2) words per step (y in; filtered moments out;
        filtered moments in; smoothed moments out; plus the per-step model rows
        of a time-varying model), over the measured time per pass.  The
        dominant kernel's own roofline is reported beside it."""
        rs = 8 if prec == "fp64" else 4
        f = op_flops(nx, ny)
        bytes_step = (ny + 3 * (nx + nx * nx)) * rs
        if tv:
            bytes_step += (2 * nx * nx + nx + ny * nx + ny + ny * ny) * 8
        flops_step = (f["f_full"] + f["f_carry"] + 2 * f["f_elem"] + 2 * f["s_elem"] + f["s_full"]
                      + f["s_carry"])
        peak_f = FP64_PEAK_TFLOPS if (prec == "fp64" or f64_mixed) else FP32_PEAK_TFLOPS
        t_mem = bytes_step * T / (HBM_PEAK_GBS * 1e9)
        t_alu = flops_step * T / (peak_f * 1e12)
        tr = measured_pass_traffic(w.name, prec)
        if t_mem >= t_alu:
            ach = bytes_step * T / sec / 1e9
            rl = dict(bound="hbm", achieved=round(ach, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(ach / HBM_PEAK_GBS, 4), traffic=tr)
        else:
            ach = flops_step * T / sec / 1e12
            rl = dict(bound="alu", achieved=round(ach, 3), peak=peak_f, unit="TFLOP/s",
                      frac=round(ach / peak_f, 4), traffic=tr)
        rl.update(scope="whole pass (all kernels of one filter + smoother pass)",
                  algorithmic_bytes_per_step=bytes_step, algorithmic_flops_per_step=round(flops_step, 1),
                  dominant_kernel=dom_rl)
        return rl

    dom64, kern64, rl64k = roofline("fp64")
    domm, kernm, rlmk = roofline("mixed")
    rl64 = pass_roofline("fp64", results["fp64"]["sec"], rl64k)
    rlm = pass_roofline("mixed", results["mixed"]["sec"], rlmk)

    # CPU baseline: the oracle as it stands, one host thread, on the same workload
    cpu = None
    if not args.no_cpu_baseline:
        if batched:
            # a bounded sample of sequences, run one after another on one thread
            steps_s, nseq, dt = 0, 0, 0.0
            t_start = time.perf_counter()
            for b in range(0, w.B, max(1, w.B // 64)):
                mo = w.model_of(b)
                s_ = w.seq(b)
                t0 = time.perf_counter()
                oracle.kf_rts(mo.F, mo.Q, mo.H, mo.R, mo.m0, mo.P0, w.y[s_])
                dt += time.perf_counter() - t0
                steps_s += s_.stop - s_.start
                nseq += 1
                if time.perf_counter() - t_start > args.cpu_seconds:
                    break
            cpu = dict(value=steps_s / dt, unit="smoothed time steps/s", cores=1, kind="oracle",
                       sample="%d of %d sequences (%d steps), sequential C FP64 KF+RTS, 1 thread"
                       % (nseq, w.B, steps_s))
        else:
            times = []
            t_start = time.perf_counter()
            run = oracle.kf_rts_tv if tv else oracle.kf_rts
            while True:
                t0 = time.perf_counter()
                run(w.model.F, w.model.Q, w.model.H, w.model.R, w.model.m0, w.model.P0, w.y)
                times.append(time.perf_counter() - t0)
                if time.perf_counter() - t_start > args.cpu_seconds or len(times) >= 50:
                    break
            med = statistics.median(times)
            cpu = dict(value=T / med, unit="smoothed time steps/s", cores=1, kind="oracle",
                       sample="full workload (T=%d), %d runs, median; sequential C FP64 KF+RTS, 1 thread"
                       % (T, len(times)))

    if cpu is not None:
        progress("oracle baseline on the host: %.3e steps/s" % cpu["value"])
    sec64 = results["fp64"]["sec"]
    secm = results["mixed"]["sec"]
    line = {
        "metric": "smoothed time steps/sec (filter+smoother) vs FP64 scan; max rel err vs oracle",
        "value": T / sec64,
        "unit": "smoothed time steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded simulation of the model)",
        "config": {"workload": w.name, "T": T, "B": w.B, "nx": nx, "ny": ny, "time_varying": tv,
                   "path": ("plan (hipGraph: pks_plan_create%s / pks_plan_launch)" % ("_tv" if tv else "")) if batched
                   else ("pks_filter_smooth_tv" if tv else "pks_filter_smooth")},
        "plan_ms_per_step": results["fp64"]["plan_sec"] * 1e3,
        "eager_ms_per_step": results["fp64"]["eager_sec"] * 1e3,
        "max_rel_err": {k: float("%.3e" % v) for k, v in errs["fp64"].items()},
        "err_sample": "all steps" if not batched else "%d of %d sequences" % (len(sample), w.B),
        "roofline": rl64,
        "kernels_ms": {k: round(v, 4) for k, v in kern64.items()},
        "mixed": {
            "value": T / secm, "ms_per_step": secm * 1e3,
            "plan_ms_per_step": results["mixed"]["plan_sec"] * 1e3,
            "eager_ms_per_step": results["mixed"]["eager_sec"] * 1e3,
            "dtype": "f32 storage, f64 arithmetic" if f64_mixed else "f32 storage/products, f64 solves",
            "speedup_vs_fp64": sec64 / secm,
            "max_rel_err": {k: float("%.3e" % v) for k, v in errs["mixed"].items()},
            "roofline": rlm,
            "kernels_ms": {k: round(v, 4) for k, v in kernm.items()},
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_hmm(args, np, torch, oracle, pks, wl):
    """Discrete-state HMM (workload 7: K = 64 states, T = 2^16): one step is
    the filter (filtered marginals and log p(y_1:k)) plus the smoother.
    Roofline: FP64 matrix products, 2 K^3 flops per step for each pass's
    block elements (the GEMM of one step of the running product), against
    the FP64 peak (matrix = vector on MI355X)."""
    w = wl.hmm_workload()
    T, K = w.T, w.K
    progress("workload %s generated" % w.name)
    dm = pks.hmm_to_device(w.Pi, w.p0)
    L = torch.as_tensor(w.L).cuda()
    ws = pks.hmm_workspace(K, T)
    alpha = torch.empty((T, K), dtype=torch.float64, device="cuda")
    logp = torch.empty(T, dtype=torch.float64, device="cuda")
    gamma = torch.empty_like(alpha)
    step = lambda: pks.hmm_filter_smooth(dm, L, ws=ws, out=(alpha, logp, gamma))
    sec = time_steps(step, args.steps, args.warmup, torch)
    pks.profile_start()
    for _ in range(args.steps):
        step()
    prof = pks.profile_stop()
    torch.cuda.synchronize()
    kern = {k: tot / max(1, n) for k, (tot, n) in prof.items()}
    if args.no_check:
        errs = {"alpha_abs": float("nan"), "gamma_abs": float("nan"), "logp_rel": float("nan")}
    else:
        ref = oracle.hmm_fb(w.Pi, w.p0, w.L)
        a, g, lp = alpha.cpu().numpy(), gamma.cpu().numpy(), logp.cpu().numpy()
        errs = {"alpha_abs": float(np.max(np.abs(a - ref["alpha"]))),
                "gamma_abs": float(np.max(np.abs(g - ref["gamma"]))),
                "logp_rel": float(np.max(np.abs(lp - np.cumsum(ref["ll"])) /
                                         np.maximum(1.0, np.cumsum(np.abs(ref["ll"])))))}
    flops_step = 2 * 2.0 * K ** 3
    ach = flops_step * T / sec / 1e12
    dom = max(kern, key=kern.get)
    rl = dict(bound="mfma", achieved=round(ach, 3), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
              frac=round(ach / FP64_PEAK_TFLOPS, 4), traffic=None, scope="whole pass",
              algorithmic_flops_per_step=flops_step, dominant_kernel=dom, dominant_kernel_ms=round(kern[dom], 4))
    cpu = None
    if not args.no_cpu_baseline:
        times = []
        t_start = time.perf_counter()
        while True:
            t0 = time.perf_counter()
            oracle.hmm_fb(w.Pi, w.p0, w.L)
            times.append(time.perf_counter() - t0)
            if time.perf_counter() - t_start > args.cpu_seconds or len(times) >= 20:
                break
        cpu = dict(value=T / statistics.median(times), unit="smoothed time steps/s", cores=1, kind="oracle",
                   sample="full workload (T=%d, K=%d), %d runs, median; sequential C forward-backward, 1 thread"
                   % (T, K, len(times)))
    line = {"metric": "HMM smoothed time steps/sec (filter+smoother), K=%d states" % K, "value": T / sec,
            "unit": "smoothed time steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic (seeded sticky chain, Gaussian emissions)",
            "config": {"workload": w.name, "T": T, "K": K, "path": "pks_hmm_filter_smooth"},
            "max_err": errs, "roofline": rl, "kernels_ms": {k: round(v, 4) for k, v in kern.items()},
            "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)


def bench_loglik(args, w, np, torch, oracle, pks, wl, dev):
    T, B = w.total, w.B
    nx, ny = w.model.nx, w.model.ny
    batched = B > 1
    tv = w.time_varying
    dm = pks.to_device(w.model, device=dev, per_sequence=w.per_sequence, time_varying=tv)
    off = torch.as_tensor(w.offsets).to(dev) if batched else None
    orun = oracle.kf_rts_tv if tv else oracle.kf_rts
    results = {}
    for prec in ("fp64", "mixed"):
        rdt = torch.float64 if prec == "fp64" else torch.float32
        y = torch.as_tensor(w.y).to(dev, rdt)
        ws = pks.workspace(nx, ny, T, B, prec, dev, time_varying=tv)
        if batched:
            m, P = pks.filter_batched(dm, off, y, prec, ws=ws)
            step = lambda: pks.loglik_batched(dm, off, y, m, P, prec, cumulative=True, ws=ws)
        else:
            m, P = pks.filter(dm, y, prec, ws=ws)
            step = lambda: pks.loglik(dm, y, m, P, prec, cumulative=True, ws=ws)
        sec = time_steps(step, args.steps, args.warmup, torch)
        pks.profile_start()
        for _ in range(args.steps):
            out = step()
        prof = pks.profile_stop()
        torch.cuda.synchronize()
        results[prec] = dict(sec=sec, prof=prof, cum=out[0].cpu().numpy(), tot=out[1].cpu().numpy())
        progress("%s timed: %.4f ms per evaluation" % (prec, sec * 1e3))

    # accuracy: the oracle's factors summed per sequence (sampled sequences when batched)
    sample = list(range(B)) if not batched else sorted(set([0, B - 1] + list(range(0, B, max(1, B // 64)))))
    if args.no_check:
        sample = []
    errs = {}
    for prec in ("fp64", "mixed"):
        yy = w.y if prec == "fp64" else w.y.astype(np.float32).astype(np.float64)
        e_tot, e_cum = 0.0, 0.0
        for b in sample:
            mo = w.model_of(b) if batched else w.model
            s_ = w.seq(b) if batched else slice(0, T)
            ref = orun(mo.F, mo.Q, mo.H, mo.R, mo.m0, mo.P0, yy[s_], smooth=False, loglik=True)["ll"]
            rc = np.cumsum(ref)
            g = results[prec]["cum"][s_]
            e_cum = max(e_cum, float(np.max(np.abs(g - rc) / np.maximum(1.0, np.abs(rc)))))
            e_tot = max(e_tot, abs(results[prec]["tot"][b] - rc[-1]) / max(1.0, abs(rc[-1])))
        errs[prec] = dict(total=float("%.3e" % e_tot), partial_sums=float("%.3e" % e_cum))
        progress("%s checked against the oracle on %d sequences" % (prec, len(sample)))

    def roofline(prec):
        rs = 8 if prec == "fp64" else 4
        km = ll_kernel_model(nx, ny, rs)["k_ll_steps"]
        prof = results[prec]["prof"]
        per_launch = {k: tot / max(1, n) for k, (tot, n) in prof.items()}
        dur_s = per_launch["k_ll_steps"] * 1e-3
        ach = km["bytes"] * T / dur_s / 1e9
        rl = dict(bound="hbm", achieved=round(ach, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                  frac=round(ach / HBM_PEAK_GBS, 4), traffic=None, kernel="k_ll_steps",
                  kernel_ms=round(per_launch["k_ll_steps"], 4), algorithmic_bytes_per_launch=km["bytes"] * T,
                  algorithmic_flops_per_launch=km["flops"] * T)
        return per_launch, rl

    kern64, rl64 = roofline("fp64")
    kernm, rlm = roofline("mixed")
    cpu = None
    if not args.no_cpu_baseline:
        nsteps, dt, nseq = 0, 0.0, 0
        t_start = time.perf_counter()
        while time.perf_counter() - t_start < args.cpu_seconds:
            for b in (sample if batched else [0]):
                mo = w.model_of(b) if batched else w.model
                s_ = w.seq(b) if batched else slice(0, T)
                offs = np.array([0, s_.stop - s_.start])
                t0 = time.perf_counter()
                ll = orun(mo.F, mo.Q, mo.H, mo.R, mo.m0, mo.P0, w.y[s_], smooth=False, loglik=True)["ll"]
                oracle.loglik_prefix(ll, offs)
                dt += time.perf_counter() - t0
                nsteps += s_.stop - s_.start
                nseq += 1
                if time.perf_counter() - t_start > args.cpu_seconds:
                    break
        cpu = dict(value=nsteps / dt, unit="time steps/s", cores=1, kind="oracle",
                   sample="%d sequence runs (%d steps): sequential C FP64 Kalman filter with the per-step "
                          "factors, then their running sums; 1 thread; includes the filter, which the GPU "
                          "figure does not" % (nseq, nsteps))
        progress("oracle baseline on the host: %.3e steps/s" % cpu["value"])
    sec64, secm = results["fp64"]["sec"], results["mixed"]["sec"]
    line = {
        "metric": "log-likelihood time steps/sec (every factor, partial sum and total from filtered moments)",
        "value": T / sec64,
        "unit": "time steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded simulation of the model)",
        "config": {"workload": w.name, "T": T, "B": B, "nx": nx, "ny": ny, "time_varying": tv,
                   "path": "pks_loglik_batched" if batched else ("pks_loglik_tv" if tv else "pks_loglik"),
                   "cumulative": True},
        "max_rel_err": errs["fp64"],
        "err_sample": "all steps" if not batched else "%d of %d sequences" % (len(sample), B),
        "roofline": rl64,
        "kernels_ms": {k: round(v, 4) for k, v in kern64.items()},
        "mixed": {"value": T / secm, "ms_per_step": secm * 1e3, "dtype": "f32 inputs, f64 arithmetic",
                  "max_rel_err": errs["mixed"], "roofline": rlm,
                  "kernels_ms": {k: round(v, 4) for k, v in kernm.items()}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
