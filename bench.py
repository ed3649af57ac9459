"""Benchmark of the batched Lorentz-vector hot path on one MI355X.

One step is one pass of every kernel of the path over one batch of synthetic,
collider-shaped input already resident in HBM:

  mass_fwd / mass_fwd32     pair mass, PtEtaPhiM, 2^24 pairs     (72 / 36 B/pair)
  mass_bwd / mass_bwd32     reverse mode of the same pairs        (136 / 68 B/pair)
  boost_fwd / boost_fwd32   boost, per-item beta, 2^24 vectors    (88 / 44 B/vector)
  boost_bwd / boost_bwd32   reverse mode of the boost             (144 / 72 B/vector)
                            (FP64, then the same inputs rounded to FP32)
  mass_comp32  FP32 compensated pair mass, 2^26 light pairs with
               10 % nearly collinear (the precision-stress workload) (36 B/pair)
  event_reduce FP64 jagged reduction, 2^20 Poisson(8) events:
               totals, event mass and all pair masses           (~568 B/event)
  event_reduce32c  the same events in FP32, compensated mode     (~292 B/event)
  event_reduce_bwd FP64 reverse mode of the jagged reduction     (~824 B/event)

value = kernel-items processed per second, in Gevents/s: every kernel of the
step counts the items it processes (a pair, a vector or a collider event), so
a pair through the FP64 forward and backward counts twice.  Every kernel is
also reported separately with its algorithmic bytes, achieved GB/s and
fraction of the 8 TB/s HBM peak.  Per-kernel times come from HIP events
recorded on the stream the kernels run on, inside the timed steps.

cpu_baseline: the CPU oracle (test infrastructure) timed on the host cores on
one step's workload, repeated until about 10 s have passed, in the same unit.
Its accurate (cancellation-free, binary64) masses of the 2^26 stress pairs
are kept as the reference of the precision comparison below.

fp32_comp_vs_fp64_plain: the FP32 compensated, plain FP64 and plain FP32
masses of the 2^26 stress pairs, each launch timed and each result compared,
pair by pair, with that oracle reference (max and 99.9th percentile, in GeV
and relative, collinear and generic pairs apart, and the FP64 redo count).

convert: the stand-alone coordinate conversions (Sec. 3.1), FP64 and FP32,
forward (2 x 4 columns per vector) and reverse mode (3 x 4 columns), each
timed on its own over 2^24 vectors after the step; they are not part of the
step and not of `value`.

transform: general Lorentz transformations (4x4) and rotations (3x3 matrix,
axis and angle), one for all vectors or one per vector, and the per-item
reverse mode with the matrix gradient, timed the same way.

analysis: a 1000-bin histogram of 2^26 FP64 pair masses (512 MiB, twice the
last-level cache) and the per-event pair closest to 91.1876 GeV over the
jagged events' pair masses, and the reverse mode of the cancellation-free mass
on 2^24 FP32 stress pairs (68 B/pair), timed the same way.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-compare] [--no-convert]
                       [--no-transform] [--no-analysis] [--calib-copy] [--kernels a,b,...]
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gevents/s & HBM GB/s (% of peak): mass/boost fwd+bwd, FP32-comp vs FP64 plain"
HBM_PEAK_GBS = 8000.0
N_ITEMS = 1 << 24
N_STRESS = 1 << 26
N_EVENTS = 1 << 20
TILING_FIELDS = ("block", "events_per_tile", "lds_particles", "pairs_per_round")
KERNELS = ["mass_fwd", "mass_bwd", "boost_fwd", "boost_bwd", "mass_fwd32", "mass_bwd32", "boost_fwd32",
           "boost_bwd32", "mass_comp32", "event_reduce", "event_reduce32c", "event_reduce_bwd"]
KERNEL_SYMBOL = {
    "mass_fwd": "k_stream<MassPlain<double, 1>, 2>", "mass_bwd": "k_stream<MassBwd<double, 1>, 2>",
    "boost_fwd": "k_stream<BoostFwd<double, 1>, 2>", "boost_bwd": "k_stream<BoostBwd<double, 1, true>, 2>",
    "mass_fwd32": "k_stream<MassPlain<float, 1>, 4>", "mass_bwd32": "k_stream<MassBwd<float, 1>, 4>",
    "boost_fwd32": "k_stream<BoostFwd<float, 1>, 4>", "boost_bwd32": "k_stream<BoostBwd<float, 1, true>, 4>",
    "mass_comp32": "k_stream<MassComp<float>, 4>",
    "event_reduce": "k_event_reduce<double, 1, 0, false>", "event_reduce32c": "k_event_reduce<float, 1, 1, false>",
    "event_reduce_bwd": "k_event_reduce_bwd<double, 1>",
}
# Coordinate conversions, measured after the step: (dtype, from, to, reverse mode) and kernel symbol.
CONVERT_CASES = {
    "convert_ptm_to_cart": ("f64", "PtEtaPhiM", "PxPyPzE", False, "Convert<double, 1, 0>"),
    "convert_cart_to_ptm": ("f64", "PxPyPzE", "PtEtaPhiM", False, "Convert<double, 0, 1>"),
    "convert_ptm_to_cart_bwd": ("f64", "PtEtaPhiM", "PxPyPzE", True, "ConvertBwd<double, 1, 0>"),
    "convert_cart_to_ptm_bwd": ("f64", "PxPyPzE", "PtEtaPhiM", True, "ConvertBwd<double, 0, 1>"),
    "convert_ptm_to_cart_f32": ("f32", "PtEtaPhiM", "PxPyPzE", False, "Convert<float, 1, 0>"),
    "convert_cart_to_ptm_f32": ("f32", "PxPyPzE", "PtEtaPhiM", False, "Convert<float, 0, 1>"),
    "convert_cart_to_ptm_bwd_f32": ("f32", "PxPyPzE", "PtEtaPhiM", True, "ConvertBwd<float, 0, 1>"),
}
# General transformations, measured after the step: kernel symbol and algorithmic bytes per vector.
TRANSFORM_CASES = {
    "lorentz_broadcast": ("TransformFwd<double, 0, 0>", 64),
    "lorentz_per_item": ("TransformFwd<double, 0, 1>", 192),
    "lorentz_per_item_bwd": ("TransformBwd<double, 0, 1, true>", 352),
    "rotate_broadcast": ("TransformFwd<double, 1, 0>", 64),
    "axis_angle_per_item": ("TransformFwd<double, 2, 1>", 96),
    "lorentz_broadcast_f32": ("TransformFwd<float, 0, 0>", 32),
}
# The analysis step, measured after the step: kernel symbols.
ANALYSIS_SYMBOL = {"mass_histogram": "k_hist_lds<double, 2>", "event_best_pair": "k_best_pair<double>",
                   "mass_comp32_bwd": "k_stream<MassCompBwd<float>, 4>",
                   "mass_histogram_fused": "k_mass_hist<MassPlain<double, 1>, 2, true>",
                   "event_best_pair_fused": "k_event_reduce<double, 1, 0, true>"}
ALL_SYMBOLS = {**KERNEL_SYMBOL, **{k: v[4] for k, v in CONVERT_CASES.items()},
               **{k: v[0] for k, v in TRANSFORM_CASES.items()}, **ANALYSIS_SYMBOL}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the FP32-compensated vs plain FP64 comparison (profiling runs: only the step's "
                         "launches)")
    ap.add_argument("--no-convert", action="store_true", help="skip the coordinate-conversion measurements")
    ap.add_argument("--no-transform", action="store_true", help="skip the general-transformation measurements")
    ap.add_argument("--no-analysis", action="store_true", help="skip the histogram and best-pair measurements")
    ap.add_argument("--kernels", default=None,
                    help="comma-separated subset of the step's kernels to run (profiling runs); default all")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the steps, run one 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter_collection.csv files (FETCH_SIZE, WRITE_SIZE) of a "
                         "--calib-copy run into profiles/hbm_traffic.txt and exit")
    ap.add_argument("--summarize-sq", nargs="+", metavar="COUNTER_CSV",
                    help="write profiles/jagged_sq_counters.md from rocprofv3 SQ counter passes")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_CSV", "BENCH_JSON"),
                    help="turn a rocprofv3 --kernel-trace kernel_trace.csv and the JSON line the same run printed "
                         "into profiles/step_kernel_trace.md and exit")
    return ap.parse_args()


TRACE_CMD = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats --output-format csv "
             "-d $R/gpurun_out/prof_trace -o bench -- python3 $R/bench.py --steps 20 --warmup 3 --no-cpu --no-compare "
             "> $R/gpurun_out/trace_bench.json")


def summarize_trace(trace_csv, bench_json):
    """Per-kernel launch durations from a rocprofv3 kernel trace beside the
    benchmark's own HIP-event averages of the same run.  For the step's
    kernels only their last warmup + steps dispatches of the step's launch
    shape count (the jagged autotuner's trial launches come before them)."""
    import collections
    import csv
    import re

    bench = None
    for line in open(bench_json):
        if line.startswith("{"):
            bench = json.loads(line)
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        per[r["Kernel_Name"]].append((int(r["Dispatch_Id"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
                                      * 1e-3, r["Workgroup_Size_X"], r["Grid_Size_X"], r["LDS_Block_Size"]))
    n_step = bench["warmup"] + bench["steps"]
    rows = []
    for name, ds in per.items():
        ds.sort()
        short = re.sub(r"glv::\(anonymous namespace\)::", "", name)
        key = next((k for k, sym in ALL_SYMBOLS.items() if sym in short), None)
        if key:
            # the step's own launch shape (the most frequent grid: the settle
            # and timed steps), so that launches of the same kernel on other
            # sizes -- autotuner trials, the analysis inputs -- do not count
            grid = collections.Counter(d[3] for d in ds).most_common(1)[0][0]
            ds = [d for d in ds if d[3] == grid]
        extra = len(ds) - n_step if key else 0
        if key:
            ds = ds[-n_step:]
        us = np.array([d[1] for d in ds])
        rows.append((us.sum(), short, key, len(ds), float(us.mean()), float(us.min()), extra, ds[-1][2:]))
    total = sum(r[0] for r in rows)
    out = ["# Kernel trace: one benchmark step (2^24 items per element-wise kernel, 2^20 jagged events)", "",
           "Command (from the repository root `R` on one MI355X):", "", "```", TRACE_CMD, "```", "",
           f"Source: `bench_kernel_trace.csv`; per step kernel its last {bench['warmup']} warm-up + "
           f"{bench['steps']} timed dispatches of the step's launch shape; jagged tilings (block, events per tile, LDS particles) "
           f"{tuple((bench['config'].get('event_tiling') or {}).values())} FP64, "
           f"{tuple((bench['config'].get('event_tiling_fp32_comp') or {}).values())} FP32 compensated, "
           f"{tuple((bench['config'].get('event_tiling_bwd') or {}).values())} backward (autotuned on "
           "these events, the trial launches excluded); the coordinate conversions, general "
           "transformations and the analysis step run after the step, each warm-up + steps times.  Algorithmic bytes per launch as in `bench.py`.", "",
           "| kernel | calls | avg µs | min µs | share % | block, grid, LDS B | alg. bytes / launch | alg. GB/s (avg) "
           "| % of 8 TB/s |", "|---|---|---|---|---|---|---|---|---|"]
    for tot, name, key, calls, avg, mn, extra, geo in sorted(rows, key=lambda r: -r[0]):
        label = f"`{name[:100]}`" + (f" ({key})" if key else "")
        g = f"{geo[0]}, {geo[1]}, {geo[2]}"
        measured = {**bench["kernels"], **(bench.get("convert") or {}), **(bench.get("transform") or {}),
                    **(bench.get("analysis") or {})}
        if key and key in measured:
            ab = measured[key]["alg_bytes"]
            gbs = ab / (avg * 1e-6) / 1e9
            out.append(f"| {label} | {calls} | {avg:.1f} | {mn:.1f} | {100 * tot / total:.2f} | {g} | {ab} | "
                       f"{gbs:.0f} | {100 * gbs / HBM_PEAK_GBS:.1f} |")
        else:
            out.append(f"| {label} | {calls} | {avg:.1f} | {mn:.1f} | {100 * tot / total:.2f} | {g} | — | — | — |")
    out += ["", "The benchmark's own HIP-event averages in the same run (under the tracer):", ""]
    for k, v in {**bench["kernels"], **(bench.get("convert") or {}), **(bench.get("transform") or {}),
                 **(bench.get("analysis") or {})}.items():
        out.append(f"* {k}: {v['avg_us']} µs, {v['alg_GBps']} GB/s ({100 * v['frac_hbm_peak']:.1f} % of peak)")
    path = os.path.join(ROOT, "profiles", "step_kernel_trace.md")
    with open(path, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))


COPY_BYTES = 1 << 30


def summarize_pmc(fetch_csv, write_csv):
    """Per-kernel HBM bytes per launch from FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch), each scaled so that the 1 GiB calibration copy reads and
    writes exactly 1 GiB."""
    import collections
    import csv
    import re

    def load(path, counter):
        vals = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                vals[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)
        return vals

    fetch, write = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    copy = [k for k in fetch if "copyBuffer" in k]
    f_copy = max(max(fetch[k]) for k in copy)
    w_copy = max(max(write[k]) for k in copy)
    f_scale, w_scale = COPY_BYTES / f_copy, COPY_BYTES / w_copy
    lines = [f"# HBM traffic per launch: rocprofv3 FETCH_SIZE x {f_scale:.4f} + WRITE_SIZE x {w_scale:.4f}",
             "# (scales from a 1 GiB device copy in the same runs).  Commands, from the repository root R:",
             "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d $R/gpurun_out/pmc_fetch -o fetch -- "
             "python3 $R/bench.py --steps 2 --warmup 1 --no-cpu --no-compare --calib-copy",
             "#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d $R/gpurun_out/pmc_write -o write -- "
             "python3 $R/bench.py --steps 2 --warmup 1 --no-cpu --no-compare --calib-copy",
             "#   python3 bench.py --summarize-pmc gpurun_out/pmc_fetch/fetch_counter_collection.csv "
             "gpurun_out/pmc_write/write_counter_collection.csv",
             "# sources = digest of the kernel's source file and the shared headers at measurement time"]
    for key, sym in ALL_SYMBOLS.items():
        names = [k for k in fetch if sym in re.sub(r"glv::\(anonymous namespace\)::", "", k)]
        if not names:
            continue
        n = names[0]
        fb = float(np.median(fetch[n])) * f_scale
        wb = float(np.median(write.get(n, [0.0]))) * w_scale
        lines.append(f"traffic kernel={key} sources={source_digest(key)} fetch_bytes={fb:.0f} write_bytes={wb:.0f} "
                     f"bytes_per_launch={fb + wb:.0f}")
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


SQ_PASSES = [
    "SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_BUSY_CYCLES SQ_WAVE_CYCLES",
    "SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_ANY SQ_WAIT_INST_LDS SQ_WAIT_ANY SQ_LDS_BANK_CONFLICT "
    "SQ_INSTS_VALU_TRANS_F32 SQ_INSTS_VALU_TRANS_F64",
    "SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_INT32 SQ_INSTS_VALU_INT64 "
    "SQ_INSTS_VALU_FMA_F32 SQ_INSTS_VALU_MUL_F32 SQ_INSTS_VALU_ADD_F32",
]
SQ_KERNELS = ("event_reduce", "event_reduce32c", "event_reduce_bwd", "event_best_pair_fused", "mass_comp32",
              "mass_comp32_bwd")
SQ_LAST = 5  # dispatches per kernel and pass: the timed steps, after the autotuners' trials
SIMDS, CLOCK_GHZ = 1024, 2.4  # MI355X: 256 CUs x 4 SIMDs


def summarize_sq(csvs):
    """Per-kernel averages of SQ counters over the dispatches of each pass and
    the VALU issue time they imply (a wave64 VALU instruction occupies a SIMD
    for 4 cycles), next to the dispatch's own duration in the same run."""
    import collections
    import csv
    import re

    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    dur = collections.defaultdict(list)
    meta = {}
    for path in csvs:
        # per kernel, the last SQ_LAST dispatches of this pass (the timed
        # steps, not the autotuners' trial tilings)
        rows = collections.defaultdict(lambda: collections.defaultdict(list))
        for r in csv.DictReader(open(path)):
            name = re.sub(r"glv::\(anonymous namespace\)::", "", r["Kernel_Name"])
            key = next((k for k in SQ_KERNELS if ALL_SYMBOLS[k] in name), None)
            if key is not None:
                rows[key][int(r["Dispatch_Id"])].append(r)
        for key, by_id in rows.items():
            for d in sorted(by_id)[-SQ_LAST:]:
                for r in by_id[d]:
                    vals[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
                    meta[key] = (r["Workgroup_Size"], r["Grid_Size"], r["VGPR_Count"], r["SGPR_Count"])
                r = by_id[d][0]
                dur[key].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    cmd = " ".join(f'"{p}"' for p in SQ_PASSES)
    lines = ["# SQ counters of the jagged kernels and the compensated FP32 mass (2^20 Poisson(8) events, 2^26 pairs)",
             "",
             "Commands (from the repository root `R` on one MI355X; one rocprofv3 pass per counter group):",
             "",
             "```",
             f"i=0; for P in {cmd}; do",
             "  i=$((i+1)); cd /tmp && export TMPDIR=/tmp && timeout -s KILL 240 rocprofv3 --pmc $P --output-format csv "
             "-d $R/gpurun_out/sq_$i -o sq -- python3 $R/bench.py --kernels event_reduce,event_reduce32c,"
             "event_reduce_bwd,mass_comp32 --steps 2 --warmup 1 --no-cpu --no-compare --no-convert --no-transform",
             "done",
             "python3 bench.py --summarize-sq gpurun_out/sq_*/sq_counter_collection.csv",
             "```",
             "",
             f"Counters are per dispatch, averaged over the last {SQ_LAST} dispatches of each kernel in each pass (the "
             "timed steps, after the autotuners' trial launches); `VALU issue` = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x 2.4 GHz), the time the VALU "
             "instructions alone occupy the SIMDs; `dispatch` = the dispatch's duration under counter collection.",
             ""]
    derived = ["| kernel | block, grid (work-items), VGPR, SGPR | dispatch us | VALU insts | VALU issue us | "
               "VALU/dispatch | LDS insts | LDS bank-conflict cycles | SALU insts |",
               "|---|---|---|---|---|---|---|---|---|"]
    for k in SQ_KERNELS:
        if k not in vals:
            continue
        c = {n: float(np.mean(v)) for n, v in vals[k].items()}
        d = float(np.median(dur[k]))
        vi = c.get("SQ_INSTS_VALU", 0.0)
        issue = vi * 4 / (SIMDS * CLOCK_GHZ * 1e3)
        derived.append(f"| {k} (`{ALL_SYMBOLS[k]}`) | {', '.join(meta[k])} | {d:.0f} | {vi:.3g} | {issue:.0f} | "
                       f"{issue / d:.2f} | {c.get('SQ_INSTS_LDS', 0):.3g} | {c.get('SQ_LDS_BANK_CONFLICT', 0):.3g} | "
                       f"{c.get('SQ_INSTS_SALU', 0):.3g} |")
    lines += derived + ["", "All counters (per dispatch):", ""]
    names = sorted({n for k in vals for n in vals[k]})
    lines.append("| counter | " + " | ".join(k for k in SQ_KERNELS if k in vals) + " |")
    lines.append("|---|" + "---|" * sum(1 for k in SQ_KERNELS if k in vals))
    for n in names:
        row = [f"{float(np.mean(vals[k][n])):.4g}" if vals[k].get(n) else "-" for k in SQ_KERNELS if k in vals]
        lines.append(f"| {n} | " + " | ".join(row) + " |")
    path = os.path.join(ROOT, "profiles", "jagged_sq_counters.md")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


# Sources that define each kernel and its launch configuration.
KERNEL_SOURCES = {k: ["kernels_jagged.hip", "glv_abi.hip"] for k in ("event_reduce", "event_reduce32c",
                                                                       "event_reduce_bwd")}
KERNEL_SOURCES.update({k: ["kernels_analysis.hip"] for k in ("mass_histogram", "event_best_pair")})
KERNEL_SOURCES["event_best_pair_fused"] = ["kernels_jagged.hip", "glv_abi.hip"]
SHARED_SOURCES = ["glv_device.h", "glv_math.h", "glv_launch.h"]


def source_digest(kernel):
    """Digest of the sources that define `kernel` and its launch (its kernel
    file and the shared headers), to tell whether stored counter readings still
    describe it."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2312_02756_amd", "csrc")
    for f in sorted(SHARED_SOURCES + KERNEL_SOURCES.get(kernel, ["kernels_elementwise.hip"])):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from profiles/hbm_traffic.txt (rocprofv3
    FETCH_SIZE / WRITE_SIZE, scaled by a copy-kernel calibration), or None if
    absent or recorded for other kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    digest = source_digest(kernel)
    for line in open(path):
        if not line.startswith("traffic "):
            continue
        kv = dict(tok.split("=", 1) for tok in line.split()[1:])
        if kv.get("kernel") == kernel and kv.get("sources") == digest:
            return float(kv["bytes_per_launch"])
    return None


def main():
    args = parse()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_sq:
        summarize_sq(args.summarize_sq)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path has no cross-GPU step: "
              "each GPU would reduce its own share of items and events independently)", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2312_02756_amd import glv

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def gpu(cols, dt):
        return tuple(torch.from_numpy(np.ascontiguousarray(c)).to(dev).to(dt).contiguous() for c in cols)

    # ---------------------------------------------------------- inputs (host)
    t0 = time.time()
    a, b = synth.pairs_generic(synth.rng(synth.LARGE), N_ITEMS)
    x, beta = synth.boost_items(synth.rng(synth.LARGE), N_ITEMS)
    gr = synth.rng(synth.GRADS)
    gm = synth.upstream(gr, N_ITEMS, 1)[0]
    gy = synth.upstream(gr, N_ITEMS, 4)
    sa, sb, collinear = synth.pairs_stress(synth.rng(synth.STRESS), N_STRESS)
    sa, sb = synth.as_dtype(sa, np.float32), synth.as_dtype(sb, np.float32)
    off, parts = synth.jagged_events(synth.rng(synth.JAGGED), N_EVENTS)
    parts32 = synth.as_dtype(parts, np.float32)
    n_pairs_h = int(np.sum((np.diff(off) * (np.diff(off) - 1)) // 2))
    gj = synth.rng(synth.JAGGED_GRADS)
    g_tot = synth.upstream(gj, N_EVENTS, 4)
    g_em = synth.upstream(gj, N_EVENTS, 1)[0]
    g_pair = synth.upstream(gj, n_pairs_h, 1)[0]
    gen_s = time.time() - t0

    # -------------------------------------------------------- inputs (device)
    A, B = gpu(a, torch.float64), gpu(b, torch.float64)
    GM = gpu([gm], torch.float64)[0]
    X, BETA = gpu(x, torch.float64), gpu(beta, torch.float64)
    GY = gpu(gy, torch.float64)
    # the FP32 rows take the same inputs rounded to FP32
    to32 = lambda cols: tuple(t.to(torch.float32) for t in cols)  # noqa: E731
    A32, B32, GM32, X32, BETA32, GY32 = to32(A), to32(B), GM.to(torch.float32), to32(X), to32(BETA), to32(GY)
    SA, SB = gpu(sa, torch.float32), gpu(sb, torch.float32)
    P = gpu(parts, torch.float64)
    P32 = gpu(parts32, torch.float32)
    OFF = torch.from_numpy(off).to(dev)
    PO = glv.glv_pair_offsets(OFF)
    n_pairs = int(PO[-1].item())
    assert n_pairs == n_pairs_h
    n_part = int(off[-1])
    GTOT = gpu(g_tot, torch.float64)
    GEM = gpu([g_em], torch.float64)[0]
    GPAIR = gpu([g_pair], torch.float64)[0]
    run = KERNELS if not args.kernels else [k for k in KERNELS if k in args.kernels.split(",")]
    # the jagged reductions run with the tilings the autotuners pick on these events
    tiling = glv.glv_autotune_event_reduce(P, OFF, PO) if "event_reduce" in run else None
    tiling32c = (glv.glv_autotune_event_reduce(P32, OFF, PO, mode="compensated") if "event_reduce32c" in run
                 else None)
    tiling_bwd = (glv.glv_autotune_event_reduce_bwd(P, OFF, PO, grad_total=GTOT, grad_event_m=GEM,
                                                    grad_pair_m=GPAIR) if "event_reduce_bwd" in run else None)
    # outputs preallocated once, reused every step
    new = lambda n, dt, k: tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(k))  # noqa: E731
    (M,) = new(N_ITEMS, torch.float64, 1)
    (M32,) = new(N_ITEMS, torch.float32, 1)
    (MC,) = new(N_STRESS, torch.float32, 1)
    FB = torch.zeros(1, dtype=torch.int64, device=dev)
    Y, GA, GB, GX = new(N_ITEMS, torch.float64, 4), new(N_ITEMS, torch.float64, 4), new(N_ITEMS, torch.float64, 4), \
        new(N_ITEMS, torch.float64, 4)
    GBETA = new(N_ITEMS, torch.float64, 3)
    Y32, GA32, GB32, GX32 = new(N_ITEMS, torch.float32, 4), new(N_ITEMS, torch.float32, 4), \
        new(N_ITEMS, torch.float32, 4), new(N_ITEMS, torch.float32, 4)
    GBETA32 = new(N_ITEMS, torch.float32, 3)
    TOT, (EM,), (PM,) = new(N_EVENTS, torch.float64, 4), new(N_EVENTS, torch.float64, 1), new(n_pairs, torch.float64, 1)
    TOT32, (EM32,), (PM32,) = new(N_EVENTS, torch.float32, 4), new(N_EVENTS, torch.float32, 1), \
        new(n_pairs, torch.float32, 1)
    FBJ = torch.zeros(1, dtype=torch.int64, device=dev)
    GP = new(n_part, torch.float64, 4)
    torch.cuda.synchronize()

    from paper_2312_02756_amd import _lib
    lib = _lib.load()
    P4, P3 = _lib.P4, _lib.P3
    stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream
    ptr4 = lambda cols: P4(*[t.data_ptr() for t in cols])  # noqa: E731
    ptr3 = lambda cols: P3(*[t.data_ptr() for t in cols])  # noqa: E731

    # C-ABI calls with pointers marshalled once
    cA, cB, cX, cBETA, cGY = ptr4(A), ptr4(B), ptr4(X), ptr3(BETA), ptr4(GY)
    cGA, cGB, cY, cGX, cGBETA = ptr4(GA), ptr4(GB), ptr4(Y), ptr4(GX), ptr3(GBETA)
    cA32, cB32, cX32, cBETA32, cGY32 = ptr4(A32), ptr4(B32), ptr4(X32), ptr3(BETA32), ptr4(GY32)
    cGA32, cGB32, cY32, cGX32, cGBETA32 = ptr4(GA32), ptr4(GB32), ptr4(Y32), ptr4(GX32), ptr3(GBETA32)
    cSA, cSB, cP, cTOT = ptr4(SA), ptr4(SB), ptr4(P), ptr4(TOT)
    cP32, cTOT32, cGTOT, cGP = ptr4(P32), ptr4(TOT32), ptr4(GTOT), ptr4(GP)
    F32, F64, PTM, CART = _lib.GLV_F32, _lib.GLV_F64, _lib.GLV_PTETAPHIM, _lib.GLV_PXPYPZE
    PLAIN, COMP = _lib.GLV_PLAIN, _lib.GLV_COMPENSATED

    calls = {
        "mass_fwd": lambda: lib.glv_invariant_mass(F64, PTM, PLAIN, N_ITEMS, cA, cB, M.data_ptr(), None, sp),
        "mass_bwd": lambda: lib.glv_invariant_mass_bwd(F64, PTM, N_ITEMS, cA, cB, GM.data_ptr(), cGA, cGB, sp),
        "boost_fwd": lambda: lib.glv_boost(F64, N_ITEMS, cX, cBETA, 1, cY, sp),
        "boost_bwd": lambda: lib.glv_boost_bwd(F64, N_ITEMS, cX, cBETA, 1, cGY, cGX, cGBETA, sp),
        "mass_fwd32": lambda: lib.glv_invariant_mass(F32, PTM, PLAIN, N_ITEMS, cA32, cB32, M32.data_ptr(), None, sp),
        "mass_bwd32": lambda: lib.glv_invariant_mass_bwd(F32, PTM, N_ITEMS, cA32, cB32, GM32.data_ptr(), cGA32,
                                                         cGB32, sp),
        "boost_fwd32": lambda: lib.glv_boost(F32, N_ITEMS, cX32, cBETA32, 1, cY32, sp),
        "boost_bwd32": lambda: lib.glv_boost_bwd(F32, N_ITEMS, cX32, cBETA32, 1, cGY32, cGX32, cGBETA32, sp),
        "mass_comp32": lambda: lib.glv_invariant_mass(F32, PTM, COMP, N_STRESS, cSA, cSB, MC.data_ptr(),
                                                      FB.data_ptr(), sp),
        "event_reduce": lambda: lib.glv_event_reduce(F64, PTM, PLAIN, N_EVENTS, OFF.data_ptr(), PO.data_ptr(), cP,
                                                     cTOT, EM.data_ptr(), PM.data_ptr(), None, None, sp),
        "event_reduce32c": lambda: lib.glv_event_reduce(F32, PTM, COMP, N_EVENTS, OFF.data_ptr(), PO.data_ptr(),
                                                        cP32, cTOT32, EM32.data_ptr(), PM32.data_ptr(),
                                                        FBJ.data_ptr(), None, sp),
        "event_reduce_bwd": lambda: lib.glv_event_reduce_bwd(F64, PTM, N_EVENTS, OFF.data_ptr(), PO.data_ptr(), cP,
                                                             cGTOT, GEM.data_ptr(), GPAIR.data_ptr(), cGP, None,
                                                             sp),
    }
    # algorithmic bytes per launch: what each kernel must read and write once
    alg_bytes = {
        "mass_fwd": 72 * N_ITEMS, "mass_bwd": 136 * N_ITEMS, "boost_fwd": 88 * N_ITEMS,
        "boost_bwd": 144 * N_ITEMS, "mass_fwd32": 36 * N_ITEMS, "mass_bwd32": 68 * N_ITEMS,
        "boost_fwd32": 44 * N_ITEMS, "boost_bwd32": 72 * N_ITEMS, "mass_comp32": 36 * N_STRESS,
        "event_reduce": 32 * n_part + 16 * (N_EVENTS + 1) + 40 * N_EVENTS + 8 * n_pairs,
        "event_reduce32c": 16 * n_part + 16 * (N_EVENTS + 1) + 20 * N_EVENTS + 4 * n_pairs,
        "event_reduce_bwd": 64 * n_part + 16 * (N_EVENTS + 1) + 40 * N_EVENTS + 8 * n_pairs,
    }
    units = {k: (N_EVENTS if k.startswith("event_reduce") else N_STRESS if k == "mass_comp32" else N_ITEMS)
             for k in KERNELS}
    items_per_step = sum(units[k] for k in run)

    def step(evs=None):
        for k in run:
            if evs is not None:
                evs[k][0].record(stream)
            rc = calls[k]()
            if rc != 0:
                raise RuntimeError(f"{k}: status {rc}")
            if evs is not None:
                evs[k][1].record(stream)

    # settle: about a second of untimed steps first, so that clocks and memory
    # reach their steady state (cold launches measured 15-25 % slower), then
    # the W warm-up steps
    t_settle = time.perf_counter()
    while time.perf_counter() - t_settle < 1.0:
        step()
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    K = args.steps
    evs = [{k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for k in run}
           for _ in range(K)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(K):
        step(evs[s])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start

    per_kernel = {}
    for k in run:
        ts = np.array([e[k][0].elapsed_time(e[k][1]) for e in evs]) * 1e-3  # seconds
        avg = float(ts.mean())
        gbs = alg_bytes[k] / avg / 1e9
        per_kernel[k] = {
            "avg_us": round(avg * 1e6, 2), "median_us": round(float(np.median(ts)) * 1e6, 2),
            "min_us": round(float(ts.min()) * 1e6, 2),
            "alg_bytes": int(alg_bytes[k]), "alg_GBps": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
            "units": units[k], "Gunits_per_s": round(units[k] / avg / 1e9, 3),
            "traffic": stored_traffic(k),
        }
    if "event_reduce" in per_kernel:
        per_kernel["event_reduce"]["pairs"] = n_pairs
        per_kernel["event_reduce"]["particles"] = n_part
    if "mass_comp32" in per_kernel:
        per_kernel["mass_comp32"]["fp64_redo_per_launch"] = int(FB.item()) // max(1, args.warmup + K)
    if "event_reduce32c" in per_kernel:
        per_kernel["event_reduce32c"]["fp64_redo_per_launch"] = int(FBJ.item()) // max(1, args.warmup + K)

    ms_per_step = elapsed / K * 1e3
    value = items_per_step / (elapsed / K) / 1e9
    dom = max(run, key=lambda k: per_kernel[k]["avg_us"])
    ach = per_kernel[dom]["alg_GBps"]
    roofline = {"bound": "hbm", "kernel": KERNEL_SYMBOL[dom], "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": stored_traffic(dom)}
    step_bytes = sum(alg_bytes[k] for k in run)

    # the oracle on the host cores (its accurate masses of the stress pairs are
    # the reference of the precision comparison)
    cpu, ref_host = None, None
    if not args.no_cpu:
        cpu, ref_host = cpu_baseline(a, b, gm, x, beta, gy, sa, sb, off, parts, parts32, g_tot, g_em, g_pair)

    SA64 = SB64 = None
    if not (args.no_compare and args.no_analysis):
        SA64, SB64 = tuple(t.to(torch.float64) for t in SA), tuple(t.to(torch.float64) for t in SB)
    comparison = None if args.no_compare else compare_precisions(
        lib, SA, SB, SA64, SB64, MC, FB, torch.from_numpy(collinear).to(dev), ref_host, sp, args.warmup, K)

    convert = None if args.no_convert else measure_convert(lib, A, X, GY, A32, stream, args.warmup, K)
    transform = None if args.no_transform else measure_transform(lib, A, B, GA, GB, X, GY, BETA, GM, stream,
                                                                 args.warmup, K)
    analysis = None
    if not args.no_analysis:
        counts = torch.zeros(1002, dtype=torch.int64, device=dev)
        rank = torch.empty(N_EVENTS, dtype=torch.int64, device=dev)
        best = torch.empty(N_EVENTS, dtype=torch.float64, device=dev)
        # 2^26 FP64 masses (512 MiB, twice the last-level cache): the plain
        # FP64 masses of the widened stress pairs
        MH = torch.empty(N_STRESS, dtype=torch.float64, device=dev)
        rc = lib.glv_invariant_mass(F64, PTM, PLAIN, N_STRESS, ptr4(SA64), ptr4(SB64), MH.data_ptr(), None, sp)
        if rc != 0:
            raise RuntimeError(f"histogram input: status {rc}")
        if "event_reduce" not in run:
            rc = calls["event_reduce"]()
            if rc != 0:
                raise RuntimeError(f"best-pair input: status {rc}")
        analysis = {
            "mass_histogram": time_launches(
                "mass_histogram", lambda: lib.glv_mass_histogram(F64, N_STRESS, MH.data_ptr(), 0.0, 200.0, 1000,
                                                                 counts.data_ptr(), sp),
                stream, args.warmup, K, N_STRESS, 8 * N_STRESS),
            "event_best_pair": time_launches(
                "event_best_pair", lambda: lib.glv_event_best_pair(F64, N_EVENTS, PO.data_ptr(), PM.data_ptr(),
                                                                   91.1876, rank.data_ptr(), best.data_ptr(), sp),
                stream, args.warmup, K, N_EVENTS, 8 * n_pairs + 8 * (N_EVENTS + 1) + 16 * N_EVENTS),
        }
        GMS = GM32  # 2^24 FP32 upstreams for the first 2^24 stress pairs
        GAS, GBS = new(N_ITEMS, torch.float32, 4), new(N_ITEMS, torch.float32, 4)
        cSA24, cSB24 = ptr4(tuple(t[:N_ITEMS] for t in SA)), ptr4(tuple(t[:N_ITEMS] for t in SB))
        cGAS, cGBS = ptr4(GAS), ptr4(GBS)
        analysis["mass_comp32_bwd"] = time_launches(
            "mass_comp32_bwd", lambda: lib.glv_invariant_mass_comp_bwd(F32, N_ITEMS, cSA24, cSB24, GMS.data_ptr(),
                                                                       cGAS, cGBS, sp),
            stream, args.warmup, K, N_ITEMS, 68 * N_ITEMS)
        analysis["mass_histogram"]["bins"] = 1000
        analysis["event_best_pair"]["pairs"] = n_pairs
        # the same analysis fused into the kernels: the step's 2^24 FP64 pairs
        # binned as their masses are computed (legs read, nothing stored: 64
        # B/pair against 72 + 8 B/pair for the mass kernel then the
        # histogram), and each jagged event's best pair chosen inside the
        # reduction (no pair masses written and read back: 32 B/particle,
        # 16 B/event of offsets and 16 B/event of outputs)
        analysis["mass_histogram_fused"] = time_launches(
            "mass_histogram_fused", lambda: lib.glv_invariant_mass_histogram(
                F64, PTM, PLAIN, N_ITEMS, cA, cB, 0.0, 200.0, 1000, counts.data_ptr(), None, sp),
            stream, args.warmup, K, N_ITEMS, 64 * N_ITEMS)
        analysis["mass_histogram_fused"]["unfused_alg_bytes"] = 80 * N_ITEMS
        analysis["event_best_pair_fused"] = time_launches(
            "event_best_pair_fused", lambda: lib.glv_event_reduce_best_pair(
                F64, PTM, PLAIN, N_EVENTS, OFF.data_ptr(), PO.data_ptr(), cP, 91.1876, rank.data_ptr(),
                best.data_ptr(), None, None, sp),
            stream, args.warmup, K, N_EVENTS, 32 * n_part + 16 * (N_EVENTS + 1) + 16 * N_EVENTS)
        analysis["event_best_pair_fused"]["unfused_alg_bytes"] = (
            alg_bytes["event_reduce"] - 40 * N_EVENTS + 8 * n_pairs + 8 * (N_EVENTS + 1) + 16 * N_EVENTS)

    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gevents/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {
            "workload": "per step: 2^24 PtEtaPhiM pairs (mass fwd+bwd) and 2^24 PxPyPzE vectors with per-item "
                        "beta (boost fwd+bwd), each in FP64 and in FP32; 2^26 FP32 light pairs, 10% nearly "
                        "collinear (compensated mass); 2^20 jagged events, Poisson(8) particles (totals, event "
                        "mass, all pair masses; FP64 fwd+bwd and FP32 compensated fwd)",
            "kernels": run, "items_per_step": items_per_step,
            "item": "one pair, vector or collider event through one kernel of the step",
            "step_alg_bytes": step_bytes,
            "step_alg_GBps": round(step_bytes / (elapsed / K) / 1e9, 1),
            "pairs_in_events": n_pairs, "particles": n_part,
            "event_tiling": None if tiling is None else dict(zip(TILING_FIELDS, tiling)),
            "event_tiling_fp32_comp": None if tiling32c is None else dict(zip(TILING_FIELDS, tiling32c)),
            "event_tiling_bwd": None if tiling_bwd is None else dict(zip(TILING_FIELDS, tiling_bwd)),
            "parallelism": "single GPU", "input_gen_s": round(gen_s, 1),
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": per_kernel,
        "fp32_comp_vs_fp64_plain": comparison,
        "convert": convert,
        "transform": transform,
        "analysis": analysis,
    }
    print(json.dumps(out), flush=True)


def time_launches(key, call, stream, warmup, steps, n, alg_bytes):
    """HIP events on the kernels' stream around each of `steps` launches of
    `call` (after `warmup` untimed ones): times, achieved GB/s from the
    algorithmic bytes, and the stored traffic."""
    import torch

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for _ in range(warmup):
        call()
    for e0, e1 in evs:
        e0.record(stream)
        rc = call()
        e1.record(stream)
        if rc != 0:
            raise RuntimeError(f"{key}: status {rc}")
    torch.cuda.synchronize()
    ts = np.array([e0.elapsed_time(e1) for e0, e1 in evs]) * 1e-3
    avg = float(ts.mean())
    gbs = alg_bytes / avg / 1e9
    return {"avg_us": round(avg * 1e6, 2), "median_us": round(float(np.median(ts)) * 1e6, 2),
            "min_us": round(float(ts.min()) * 1e6, 2), "alg_bytes": int(alg_bytes), "alg_GBps": round(gbs, 1),
            "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4), "Gvectors_per_s": round(n / avg / 1e9, 3),
            "traffic": stored_traffic(key)}


def measure_transform(lib, A, B, GA, GB, X, GY, BETA, GM, stream, warmup, steps):
    """Each general transformation on its own over the boost workload's 2^24
    vectors.  Per-vector matrices take 16 resident columns as entries (the
    mass legs and the mass gradients of the step: the arithmetic does not
    depend on the values), none of them the vectors or upstreams themselves,
    so that every column is a separate HBM stream; axis and angle are the
    boost velocities and the mass upstream; broadcast matrices are a
    rotation-boost product."""
    import torch

    from paper_2312_02756_amd import _lib

    sp = stream.cuda_stream
    dev = X[0].device
    n = X[0].numel()
    P4, P9, P16 = _lib.P4, _lib.P9, _lib.P16
    ptr = lambda arr, cols: arr(*[t.data_ptr() for t in cols])  # noqa: E731
    per_item = list(A) + list(B) + list(GA) + list(GB)
    aa = list(BETA) + [GM]
    th, b = 0.3, 0.6  # rotation about z by 0.3 rad, then a boost along x with beta 0.6
    g = 1.0 / np.sqrt(1.0 - b * b)
    rz = np.array([[np.cos(th), -np.sin(th), 0, 0], [np.sin(th), np.cos(th), 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]])
    bx = np.array([[g, 0, 0, g * b], [0, 1, 0, 0], [0, 0, 1, 0], [g * b, 0, 0, g]])
    lb = bx @ rz
    one64 = [torch.tensor([v], dtype=torch.float64, device=dev) for v in lb.ravel()]
    one32 = [t.to(torch.float32) for t in one64]
    rot = [torch.tensor([v], dtype=torch.float64, device=dev) for v in rz[:3, :3].ravel()]
    Y64 = tuple(torch.empty(n, dtype=torch.float64, device=dev) for _ in range(4))
    GL = tuple(torch.empty(n, dtype=torch.float64, device=dev) for _ in range(16))
    X32 = tuple(t.to(torch.float32) for t in X)
    Y32 = tuple(torch.empty(n, dtype=torch.float32, device=dev) for _ in range(4))
    F64, F32 = _lib.GLV_F64, _lib.GLV_F32
    cX, cY, cX32, cY32 = ptr(P4, X), ptr(P4, Y64), ptr(P4, X32), ptr(P4, Y32)
    cL1, cLn, cR1, cAA = ptr(P16, one64), ptr(P16, per_item), ptr(P9, rot), ptr(P4, aa)
    cL32, cGY, cGL = ptr(P16, one32), ptr(P4, GY), ptr(P16, GL)
    calls = {
        "lorentz_broadcast": lambda: lib.glv_lorentz_transform(F64, n, cX, cL1, 0, cY, sp),
        "lorentz_per_item": lambda: lib.glv_lorentz_transform(F64, n, cX, cLn, 1, cY, sp),
        "lorentz_per_item_bwd": lambda: lib.glv_lorentz_transform_bwd(F64, n, cX, cLn, 1, cGY, cY, cGL, sp),
        "rotate_broadcast": lambda: lib.glv_rotate(F64, n, cX, cR1, 0, cY, sp),
        "axis_angle_per_item": lambda: lib.glv_rotate_axis_angle(F64, n, cX, cAA, 1, cY, sp),
        "lorentz_broadcast_f32": lambda: lib.glv_lorentz_transform(F32, n, cX32, cL32, 0, cY32, sp),
    }
    return {key: time_launches(key, calls[key], stream, warmup, steps, n, TRANSFORM_CASES[key][1] * n)
            for key in TRANSFORM_CASES}


def measure_convert(lib, A, X, GY, SA, stream, warmup, steps):
    """Each coordinate conversion on its own, 2^24 vectors: PtEtaPhiM inputs
    are the mass workload's first legs (FP64, or rounded to FP32), PxPyPzE
    inputs the boost workload's vectors (FP64) or the FP32 legs converted once
    beforehand; the
    reverse modes take the boost workload's upstream gradients.  HIP events on
    the kernels' stream around each launch; algorithmic bytes = 4 columns in
    and 4 out (forward), 8 in and 4 out (reverse mode)."""
    import torch

    from paper_2312_02756_amd import _lib

    P4 = _lib.P4
    sp = stream.cuda_stream
    dev = A[0].device
    code = {"PxPyPzE": _lib.GLV_PXPYPZE, "PtEtaPhiM": _lib.GLV_PTETAPHIM}
    ptr4 = lambda cols: P4(*[t.data_ptr() for t in cols])  # noqa: E731
    n = A[0].numel()
    new = lambda dt: tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(4))  # noqa: E731
    O64, O32, C32, G32 = new(torch.float64), new(torch.float32), new(torch.float32), new(torch.float32)
    for k in range(4):
        G32[k].copy_(GY[k])
    rc = lib.glv_convert(_lib.GLV_F32, code["PtEtaPhiM"], code["PxPyPzE"], n, ptr4(SA), ptr4(C32), sp)
    if rc != 0:
        raise RuntimeError(f"glv_convert: status {rc}")
    inputs = {("f64", "PtEtaPhiM"): A, ("f64", "PxPyPzE"): X, ("f32", "PtEtaPhiM"): SA, ("f32", "PxPyPzE"): C32}
    out = {}
    for key, (dt, src, dst, bwd, _) in CONVERT_CASES.items():
        dcode = _lib.GLV_F64 if dt == "f64" else _lib.GLV_F32
        cin, cout = ptr4(inputs[(dt, src)]), ptr4(O64 if dt == "f64" else O32)
        cg = ptr4(GY if dt == "f64" else G32)
        if bwd:
            call = lambda: lib.glv_convert_bwd(dcode, code[src], code[dst], n, cin, cg, cout, sp)  # noqa: E731
        else:
            call = lambda: lib.glv_convert(dcode, code[src], code[dst], n, cin, cout, sp)  # noqa: E731
        es = 8 if dt == "f64" else 4
        out[key] = time_launches(key, call, stream, warmup, steps, n, (12 if bwd else 8) * es * n)
    return out


def compare_precisions(lib, SA, SB, SA64, SB64, MC, FB, collinear, ref_host, sp, warmup, steps):
    """The FP32 compensated mass against plain FP64 and plain FP32 on the same
    2^26 stress pairs (light legs, 10 % nearly collinear): time per launch and
    the error, relative and in GeV, each against the oracle's accurate
    (cancellation-free, binary64) mass of the same FP32 inputs, computed by the
    CPU-baseline leg (``ref_host``; without it the errors are not reported):
    the largest and the 99.9th percentile, over all pairs and over the
    collinear and the generic pairs apart, and the compensated launch's FP64
    redo count.  Outside the timed step."""
    import torch

    from paper_2312_02756_amd import _lib

    n = SA[0].numel()
    P4 = _lib.P4
    ptr4 = lambda cols: P4(*[t.data_ptr() for t in cols])  # noqa: E731
    dev = SA[0].device
    m64 = torch.empty(n, dtype=torch.float64, device=dev)
    m32 = torch.empty(n, dtype=torch.float32, device=dev)
    F32, F64, PTM = _lib.GLV_F32, _lib.GLV_F64, _lib.GLV_PTETAPHIM
    PLAIN, COMP = _lib.GLV_PLAIN, _lib.GLV_COMPENSATED
    # pointers marshalled once: host work between the events and the launch would be timed
    cSA, cSB, cSA64, cSB64 = ptr4(SA), ptr4(SB), ptr4(SA64), ptr4(SB64)
    pMC, pFB, p64, p32 = MC.data_ptr(), FB.data_ptr(), m64.data_ptr(), m32.data_ptr()
    runs = {
        "fp32_comp": (lambda: lib.glv_invariant_mass(F32, PTM, COMP, n, cSA, cSB, pMC, pFB, sp), MC, 36),
        "fp64_plain": (lambda: lib.glv_invariant_mass(F64, PTM, PLAIN, n, cSA64, cSB64, p64, None, sp), m64, 72),
        "fp32_plain": (lambda: lib.glv_invariant_mass(F32, PTM, PLAIN, n, cSA, cSB, p32, None, sp), m32, 36),
    }
    stream = torch.cuda.current_stream()
    out = {"pairs": n, "reference": None if ref_host is None else
           "oracle: accurate (cancellation-free) binary64 mass of the same FP32 inputs, host cores"}
    # the three variants in rotation, as kernels run within a step: the same
    # launch repeated back to back measures slower on this GPU than interleaved
    torch.cuda.synchronize()
    fb0 = int(FB.item())
    for _ in range(warmup):
        for call, _, _ in runs.values():
            call()
    evs = {name: [] for name in runs}
    for _ in range(steps):
        for name, (call, _, _) in runs.items():
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            if call() != 0:
                raise RuntimeError(f"{name}: launch failed")
            e1.record(stream)
            evs[name].append((e0, e1))
    torch.cuda.synchronize()
    out["fp32_comp_fp64_redo_per_launch"] = (int(FB.item()) - fb0) / (warmup + steps)
    ref = None if ref_host is None else torch.from_numpy(ref_host).to(dev)

    def p999(x):  # the 99.9th percentile: smallest of the largest 0.1 %
        k = max(1, x.numel() - int(np.ceil(0.999 * x.numel())) + 1)
        return float(torch.topk(x, k).values.min())

    for name, (call, res, bytes_per_pair) in runs.items():
        us = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs[name]])) * 1e3
        out[name] = {"avg_us": round(us, 2), "alg_GBps": round(bytes_per_pair * n / us / 1e3, 1)}
        if ref is None:
            continue
        err = (res.to(torch.float64) - ref).abs()
        rel = err / ref.abs().clamp_min(1e-300)
        out[name].update({"max_rel_err": float(rel.max()), "max_abs_err_GeV": float(err.max()),
                          "pairs_over_1e-5_rel": int((rel > 1e-5).sum()),
                          "pairs_over_tolerance": int((err > 4e-6 * ref.abs() + 1e-6).sum())})
        for sub_name, sel in (("collinear", collinear), ("generic", ~collinear)):
            r, a = rel[sel], err[sel]
            out[name][sub_name] = {"pairs": int(sel.sum()), "max_rel_err": float(r.max()),
                                   "p999_rel_err": p999(r), "max_abs_err_GeV": float(a.max()),
                                   "p999_abs_err_GeV": p999(a)}
        del err, rel
    return out


def cpu_baseline(a, b, gm, x, beta, gy, sa, sb, off, parts, parts32, g_tot, g_em, g_pair, min_seconds=10.0,
                 max_reps=20):
    """The oracle on the host cores over one step's workload (2^24 items per
    element-wise kernel in FP64 and in FP32, 2^26 stress pairs, 2^20 events),
    repeated until at least `min_seconds` have passed, in the benchmark's
    unit.  Returns the summary and the oracle's accurate masses of the stress
    pairs (the reference of the precision comparison)."""
    import oracle

    threads = len(os.sched_getaffinity(0))
    oracle.set_threads(threads)
    used = oracle.get_threads()
    r32 = lambda cols: tuple(np.asarray(c, dtype=np.float32) for c in cols)  # noqa: E731
    a32, b32, x32, beta32, gy32 = r32(a), r32(b), r32(x), r32(beta), r32(gy)
    gm32 = np.asarray(gm, dtype=np.float32)
    reps = 0
    ref = None
    t = time.perf_counter()
    while True:
        for xa, xb, xg, xx, xbeta, xgy in ((a, b, gm, x, beta, gy), (a32, b32, gm32, x32, beta32, gy32)):
            oracle.mass_plain("PtEtaPhiM", xa, xb)
            oracle.mass_vjp("PtEtaPhiM", xa, xb, xg)
            oracle.boost(xx, xbeta)
            oracle.boost_vjp(xx, xbeta, xgy)
        m_acc = oracle.mass_accurate(sa, sb)
        if ref is None:
            ref = m_acc
        oracle.event_reduce("PtEtaPhiM", off, parts)
        oracle.event_reduce("PtEtaPhiM", off, parts32, oracle.ACCURATE)
        oracle.event_reduce_vjp("PtEtaPhiM", off, parts, g_tot, g_em, g_pair)
        reps += 1
        dt = time.perf_counter() - t
        if dt >= min_seconds or reps >= max_reps:
            break
    items = reps * (8 * N_ITEMS + N_STRESS + 3 * N_EVENTS)
    # one thread (the paper's CPU baseline form) on 1/32 of a step: 2^19 items, 2^21 stress pairs, 2^15 events
    n1, s1, e1 = N_ITEMS // 32, N_STRESS // 32, N_EVENTS // 32
    cut = lambda cols, k=n1: tuple(c[:k] for c in cols)  # noqa: E731
    off1 = off[: e1 + 1]
    np1, nq1 = int(off1[-1]), int(np.sum((np.diff(off1) * (np.diff(off1) - 1)) // 2))
    p1, p32 = tuple(c[:np1] for c in parts), tuple(c[:np1] for c in parts32)
    oracle.set_threads(1)
    t1 = time.perf_counter()
    for xa, xb, xg, xx, xbeta, xgy in ((a, b, gm, x, beta, gy), (a32, b32, gm32, x32, beta32, gy32)):
        oracle.mass_plain("PtEtaPhiM", cut(xa), cut(xb))
        oracle.mass_vjp("PtEtaPhiM", cut(xa), cut(xb), xg[:n1])
        oracle.boost(cut(xx), cut(xbeta))
        oracle.boost_vjp(cut(xx), cut(xbeta), cut(xgy))
    oracle.mass_accurate(cut(sa, s1), cut(sb, s1))
    oracle.event_reduce("PtEtaPhiM", off1, p1)
    oracle.event_reduce("PtEtaPhiM", off1, p32, oracle.ACCURATE)
    oracle.event_reduce_vjp("PtEtaPhiM", off1, p1, tuple(c[:e1] for c in g_tot), g_em[:e1], g_pair[:nq1])
    dt1 = time.perf_counter() - t1
    oracle.set_threads(threads)
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), cpu)
    except OSError:
        pass
    return {"value": round(items / dt / 1e9, 5), "unit": "Gevents/s", "cores": used, "kind": "oracle", "cpu": cpu,
            "sample": f"{reps} x one step's workload: 2^24 pairs through mass fwd+bwd and 2^24 vectors through "
                      f"boost fwd+bwd, each on FP64 and on FP32 inputs, the accurate mass of 2^26 stress pairs, "
                      f"2^20 jagged events through the plain reduction, its VJP and the accurate reduction "
                      f"(binary64 oracle); {dt:.2f} s wall on {used} threads",
            "single_thread": {"value": round((8 * n1 + s1 + 3 * e1) / dt1 / 1e9, 6), "unit": "Gevents/s",
                              "sample": f"1/32 of a step on 1 thread, {dt1:.2f} s"}}, ref


if __name__ == "__main__":
    main()
