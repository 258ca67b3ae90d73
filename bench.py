#!/usr/bin/env python3
"""Scan / lookup benchmark on one MI355X.

Default workload (one step = the whole hot path over one synthetic column):
  one column of 500M rows, Zipf(1.0) over 2^20 values (20-bit codes), stored as
  PP-VBS, ByteSlice (3 slices) and Bit-Packed (20 bits); on each layout the
  scans '<', '=' and BETWEEN at selectivities 0.1, 1, 10, 50, 90 % into a
  result bitvector, then a lookup of 5M uniform random row IDs (1 %) returning
  uint32 values.

Printed: one JSON line.  ``value`` is the PP-VBS scan throughput in Gtuples/s
(rows scanned / kernel time, inputs resident in HBM); the line also carries
ByteSlice / Bit-Packed scan and lookup throughputs, the roofline of the PP-VBS
scan kernel (algorithmic bytes per launch over its HIP-event duration against
8 TB/s), the same step's scans as one batched launch, a serving run
(continuous batching vs one query at a time: saturation and p50/p99) and the
CPU oracle timed on a bounded sample.

Other workloads print their own line: ``--workload wide`` (16-column table:
layout advisor per column, pipelined conjunction, lookups),
``--workload batch`` (256 predicates over 64 columns in one launch),
``--workload serve`` (continuous batching over resident tables) and
``--workload sweep`` (skew, domain and Gaussian-variance sensitivity).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "scan Gtuples/s + % HBM peak (PP-VBS vs ByteSlice); lookup Mrows/s; p99"
HBM_PEAK_GBS = 8000.0
LAYOUTS = ("ppvbs", "byteslice", "bitpacked")
KERNEL_SOURCES = ("paper_2209_00220_amd/csrc/device_common.h", "paper_2209_00220_amd/csrc/slice_scan.h",
                  "paper_2209_00220_amd/csrc/scan_kernel.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "scan_lookup_500M_traffic.txt")
TRACE_CMD = "rocprofv3 --kernel-trace --stats -d rocprof_out/trace -o run --output-format csv -- python3 bench.py"
PMC_CMDS = ["rocprofv3 --pmc %s -d rocprof_out/%s -o run --output-format csv -- python3 bench.py --steps 1 "
            "--warmup 0 --no-batch --serve-queries 0 --no-cpu-baseline --copy-calibration" % (c, d)
            for c, d in (("FETCH_SIZE", "pmc_fetch"), ("WRITE_SIZE", "pmc_write"))]


def progress(msg: str):
    sys.stderr.write("[bench %7.1fs] %s\n" % (time.time() - T0, msg))
    sys.stderr.flush()


T0 = time.time()


def kernel_hash() -> str:
    """Hash of the scan kernel's source code with comments and blank lines
    removed (a comment edit does not change the kernel)."""
    import re

    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines()]
        h.update("\n".join(ln for ln in lines if ln.strip()).encode())
    return h.hexdigest()[:16]


def read_traffic(key: str = "hbm_bytes_per_launch"):
    """HBM bytes per PP-VBS launch (key: scan, or lookup_hbm_bytes_per_launch) from
    the committed rocprofv3 counter summary, only when it was taken on the current
    kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv, section, rows = {}, None, {}
    for line in open(TRAFFIC_FILE):
        if line.endswith("launches (fetch and write MB per launch, scaled):\n"):
            section = line.split()[0]
            rows[section] = []
            continue
        if section and line.startswith("  ") and " fetch " in line:
            f = line.split()
            rows[section].append((f[0], float(f[f.index("fetch") + 1]) + float(f[f.index("write") + 1])))
            continue
        section = None
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_hash") != kernel_hash():
        return None
    # the PP-VBS table must be whole (every benchmark predicate and the lookup, once)
    # and the stated figures must follow from its rows
    pp = rows.get("ppvbs", [])
    scans = [mb for op, mb in pp if op != "lookup"]
    looks = [mb for op, mb in pp if op == "lookup"]
    from datagen import workloads

    if len(scans) != 3 * len(workloads.SELECTIVITIES) or len(looks) != 1:
        return None
    try:
        want = float(kv[key])
    except (KeyError, ValueError):
        return None
    got = (sum(scans) / len(scans) if key == "hbm_bytes_per_launch" else looks[0]) * 1e6
    return want if abs(got - want) <= 1e5 else None


LINE_BYTES = 128   # a random access fills one L2 line of 128 bytes on this chip


def lookup_alg_bytes_per_id(info) -> float:
    """Algorithmic bytes of one lookup by row ID: the 4-byte ID and 4-byte value,
    plus one 128-byte line per random access the layout needs.  PP-VBS: BS_1;
    then, per later byte j <= L(r), the M_j word, the directory entry and the
    BS_j byte; and the M_{L+1} word that shows the code ends, for the rows whose
    length no decode-table leaf fixes (rows_end_by_mask).  ByteSlice: one line per slice.  Bit-Packed: one line, two when the code
    straddles two dwords.  Decode tables (trie, dictionary) are not counted."""
    K = int(info.k_max)
    if info.layout == 2:   # PP-VBS
        n = float(info.n_rows) or 1.0
        lines = 0.0
        for L in range(1, K + 1):
            lines += (info.rows_by_len[L] * (1 + 3 * (L - 1)) + info.rows_end_by_mask[L]) / n
    elif info.layout == 1:
        lines = float(K)
    else:
        w = int(info.width_bits)
        lines = 1.0 + sum(1 for k in range(32) if (k * w) % 32 + w > 32) / 32.0
    return 8.0 + LINE_BYTES * lines


# ---------------------------------------------------------------- profile summaries
# The committed files under profiles/ are made from rocprofv3's CSV output by the
# two functions below (CPU only): the commands that produced the CSVs and the
# command that summarised them are written into each file's header.
STEP_KERNELS = ("k_scan_slices", "k_scan_packed", "k_lookup", "k_fill")


def _kernel_rows(path):
    import csv

    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _short(name: str) -> str:
    return name.replace("void ", "").replace("bst::dev::", "").split("(")[0]


def _is_step_kernel(name: str) -> bool:
    s = _short(name)
    if not any(s.startswith(k) for k in STEP_KERNELS):
        return False
    return not (s.startswith("k_scan_slices") and s.rstrip(">").endswith("true"))   # instrumented counters run


def _step_launches(rows, n_steps: int, n_preds: int, layouts=LAYOUTS):
    """The launches of the first `n_steps` benchmark steps, in order: each step is,
    per layout, its scans and then one lookup.  The steps' lookups are the first
    lookups of the run (the counter runs and the launch tuner before the steps
    only scan), so the region ends at the step's last lookup and is counted back
    from there."""
    seq = [r for r in rows if _is_step_kernel(r["Kernel_Name"])]
    lk = [k for k, r in enumerate(seq) if _short(r["Kernel_Name"]).startswith("k_lookup")]
    per = len(layouts) * (n_preds + 1)
    need = n_steps * len(layouts)
    assert len(lk) >= need, "trace holds %d lookups, the steps need %d" % (len(lk), need)
    end = lk[need - 1] + 1
    region = seq[end - n_steps * per:end]
    assert all(_short(region[k]["Kernel_Name"]).startswith("k_lookup") for k in range(n_preds, len(region), n_preds + 1)), \
        "step launches out of order"
    return region


def _step_layout_order(n_preds: int, layouts):
    """(layout, predicate index or 'lookup') of each launch of one benchmark step."""
    order = []
    for lay in layouts:
        order += [(lay, i) for i in range(n_preds)] + [(lay, "lookup")]
    return order


def summarize_trace(trace_dir: str, steps: int, warmup: int, cmd: str, out_path: str, preds, layouts=LAYOUTS):
    """Per-launch durations of the timed steps from a rocprofv3 --kernel-trace run of
    the default benchmark, plus the --stats table of the whole run."""
    import numpy as np

    rows = sorted(_kernel_rows(os.path.join(trace_dir, "run_kernel_trace.csv")), key=lambda r: int(r["Start_Timestamp"]))
    seq = _step_launches(rows, warmup + steps, len(preds), layouts)
    order = _step_layout_order(len(preds), layouts)
    per = len(order)
    timed = seq[warmup * per:(warmup + steps) * per]
    assert len(timed) == steps * per, "trace holds %d step launches, expected %d" % (len(timed), steps * per)
    dur = {}
    names = {}
    for k, r in enumerate(timed):
        key = order[k % per]
        dur.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        names[key] = _short(r["Kernel_Name"])
    lines = ["rocprofv3 kernel trace of the default benchmark: 500M-row column, 20-bit Zipf(1.0) values,",
             "%d predicates x %d layouts + a 5M-ID lookup per layout per step; %d warmup and %d timed steps" % (
                 len(preds), len(layouts), warmup, steps),
             "after the launch-shape tuner, then the batched launch and the serving run (the tuner's, the",
             "batch's and the serving run's kernels appear in the stats table only).",
             "",
             "commands (repo root; TMPDIR=/tmp):",
             "  " + cmd,
             "  python3 bench.py --summarize-trace rocprof_out/trace --out profiles/scan_lookup_500M_kernel_trace.txt",
             "",
             "timed steps only (per launch, from the trace's start/end stamps, microseconds):",
             "  %-12s %6s %10s %10s %10s" % ("group", "calls", "avg_us", "min_us", "max_us")]
    for lay in layouts:
        for what in ("scan", "lookup"):
            v = [x for key, xs in dur.items() if key[0] == lay and ((key[1] == "lookup") == (what == "lookup"))
                 for x in xs]
            lines.append("  %-12s %6d %10.1f %10.1f %10.1f" % (lay + " " + what, len(v), np.mean(v), min(v), max(v)))
    lines += ["", "scan launches of the timed steps by predicate (average over steps, microseconds):"]
    for lay in layouts:
        for i, (op, lo, hi, sel) in enumerate(preds):
            lit = "%d..%d" % (lo, hi) if hi is not None else "%d" % lo
            lines.append("  %-9s %-8s %-16s sel %.4f  %-45s %7.1f" % (lay, op, lit, sel, names[(lay, i)],
                                                                     np.mean(dur[(lay, i)])))
    stats = _kernel_rows(os.path.join(trace_dir, "run_kernel_stats.csv"))
    lines += ["", "--stats of the whole run (top 25 by total time):",
              "  %-70s %6s %12s %10s" % ("kernel", "calls", "total_ms", "avg_us")]
    for r in stats[:25]:
        lines.append("  %-70s %6s %12.3f %10.1f" % (_short(r["Name"])[:70], r["Calls"], float(r["TotalDurationNs"]) / 1e6,
                                                    float(r["AverageNs"]) / 1e3))
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


BATCH_TRACE_CMD = ("rocprofv3 --kernel-trace --stats -d rocprof_out/batchtrace -o run --output-format csv -- "
                   "python3 bench.py --workload batch")


def summarize_batch_trace(trace_dir: str, bench_json: str, out_path: str, n_preds: int, passes: int = 5):
    """Device spans of the batched-scan workload from a rocprofv3 kernel trace of
    `bench.py --workload batch`: its last `passes` passes of single launches (the
    timed ones, right before the first batch launch) and its last `passes` batch
    replays (each starts with the counter reset; the result checks follow)."""
    import numpy as np

    rows = sorted(_kernel_rows(os.path.join(trace_dir, "run_kernel_trace.csv")), key=lambda r: int(r["Start_Timestamp"]))
    names = [_short(r["Kernel_Name"]) for r in rows]
    t0 = [int(r["Start_Timestamp"]) for r in rows]
    t1 = [int(r["End_Timestamp"]) for r in rows]
    first_batch = next(k for k, n in enumerate(names) if n.startswith("k_reset_counters") or n.startswith("k_batch"))
    single = [k for k in range(first_batch) if names[k].startswith("k_scan") or names[k].startswith("k_fill")]
    single = single[-passes * n_preds:]
    assert len(single) == passes * n_preds, "trace holds %d single launches before the batch" % len(single)
    resets = [k for k, n in enumerate(names) if n.startswith("k_reset_counters")]
    batch_kernels = ("k_reset_counters", "k_batch", "k_scan", "k_fill")
    tail = next((k for k in range(resets[-1], len(rows)) if not names[k].startswith(batch_kernels)), len(rows))
    marks = resets[-passes:] + [tail]

    def span(ks):
        return (max(t1[k] for k in ks) - min(t0[k] for k in ks)) / 1e6, sum(t1[k] - t0[k] for k in ks) / 1e6

    s_sp = [span(single[i * n_preds:(i + 1) * n_preds]) for i in range(passes)]
    b_ks = [list(range(marks[i], marks[i + 1])) for i in range(passes)]
    b_sp = [span(ks) for ks in b_ks]
    res = {}
    with open(bench_json) as f:
        for line in f:
            if line.startswith("{"):
                res = json.loads(line)
    lines = ["Kernel trace of the batched-scan workload: %d predicates (<, <=, =, BETWEEN; selectivity" % n_preds,
             "log-uniform 0.01-50 %) over 64 PP-VBS columns (n log-uniform in [1e6, 1e8], w in 8..32, Zipf s in",
             "[0, 1.5]), 4.66 G rows scanned per pass.",
             "",
             "commands (repo root; TMPDIR=/tmp):",
             "  " + BATCH_TRACE_CMD + " > rocprof_out/batchtrace.out",
             "  python3 bench.py --summarize-batch-trace rocprof_out/batchtrace rocprof_out/batchtrace.out "
             "--out profiles/batch_256preds_64cols_kernel_trace.txt",
             "",
             "%d single launches per pass (the tuned single-column launch shape), last %d passes; span = first" % (
                 n_preds, passes),
             "start to last end, busy = summed kernel time, ms:",
             "  spans " + " ".join("%6.3f" % a for a, _ in s_sp) + "   median %.3f" % np.median([a for a, _ in s_sp]),
             "  busy  " + " ".join("%6.3f" % b for _, b in s_sp) + "   median %.3f" % np.median([b for _, b in s_sp]),
             "",
             "one batch (graph replay with the autotuned shape: solo threshold %s tiles, grid %s, tiles per" % (
                 res.get("solo_tiles"), res.get("grid")),
             "grab %s, %s stream(s)), last %d replays, ms:" % (res.get("tiles_per_grab"), res.get("streams"), passes),
             "  spans " + " ".join("%6.3f" % a for a, _ in b_sp) + "   median %.3f" % np.median([a for a, _ in b_sp]),
             "  busy  " + " ".join("%6.3f" % b for _, b in b_sp) + "   median %.3f" % np.median([b for _, b in b_sp]),
             "",
             "kernels of the last replay (start relative to the replay's first kernel, duration, us):"]
    base = t0[b_ks[-1][0]]
    for k in b_ks[-1]:
        lines.append("  %-52s start %8.1f  dur %8.1f" % (names[k][:52], (t0[k] - base) / 1e3, (t1[k] - t0[k]) / 1e3))
    if res:
        lines += ["", "bench.py's own HIP-event figures in the same run: batch %s ms, single launches %s ms (speedup %s)" % (
            res.get("batch_ms"), res.get("single_launches_ms"), res.get("speedup")),
            "value %s Gtuples/s, algorithmic bytes %s per pass (%.1f %% of 8 TB/s)" % (
                res.get("value"), res.get("alg_bytes"), 100 * res.get("batch_hbm_frac", 0))]
    lines += ["", "The profiler widens the gaps between the %d single launches (span %.3f ms); their summed" % (
        n_preds, np.median([a for a, _ in s_sp])),
        "kernel time (%.3f ms) bounds what a run without it can reach. The batch replay's span (%.3f ms)" % (
            np.median([b for _, b in s_sp]), np.median([a for a, _ in b_sp])),
        "is %.2fx less device time than that bound." % (np.median([b for _, b in s_sp]) / np.median([a for a, _ in b_sp]))]
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def summarize_counters(fetch_dir: str, write_dir: str, cmds, out_path: str, preds, layouts=LAYOUTS):
    """HBM bytes per launch from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, in KiB per dispatch) of a one-step benchmark, each scaled by what
    the same counter reads for a 1 GiB device-to-device copy at the start."""
    import numpy as np

    def load(d, counter):
        rows = _kernel_rows(os.path.join(d, "run_counter_collection.csv"))
        rows = [r for r in rows if r["Counter_Name"] == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return rows

    fr, wr = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    # the counter run's own benchmark line (its stdout, beside the counter folder):
    # the in-kernel byte counters of each predicate
    counted = {}
    bench_out = fetch_dir.rstrip("/") + ".out"
    if os.path.exists(bench_out):
        for ln in open(bench_out):
            if ln.startswith("{"):
                lay_res = json.loads(ln).get("layouts", {})
                counted = {lay: v.get("counters_by_predicate") for lay, v in lay_res.items()}
    copy_f = [r for r in fr if "copyBuffer" in r["Kernel_Name"]][0]
    copy_w = [r for r in wr if "copyBuffer" in r["Kernel_Name"]][0]
    gib = float(1 << 30)
    f_scale = gib / (float(copy_f["Counter_Value"]) * 1024)   # the copy reads 1 GiB
    w_scale = gib / (float(copy_w["Counter_Value"]) * 1024)   # and writes 1 GiB
    fs, ws = _step_launches(fr, 1, len(preds), layouts), _step_launches(wr, 1, len(preds), layouts)
    order = _step_layout_order(len(preds), layouts)
    assert len(fs) == len(ws) == len(order), (len(fs), len(ws), len(order))
    lines = (["HBM traffic per launch of the benchmark step (500M-row column, 20-bit Zipf(1.0)), from",
             "two rocprofv3 counter runs of a one-step benchmark; kernel_hash names the scan kernel",
             "sources these counters were taken on (bench.py reports roofline.traffic only when it",
             "matches the current sources).",
             "",
             "commands (repo root; TMPDIR=/tmp; the first run's stdout goes to rocprof_out/pmc_fetch.out):"] +
             ["  " + c for c in cmds] + [
             "  python3 bench.py --summarize-pmc rocprof_out/pmc_fetch rocprof_out/pmc_write --out profiles/scan_lookup_500M_traffic.txt",
             "",
             "Per scan, beside the measured traffic, the kernel's own byte counters (bst_scan_stats, MB):",
             "alg128 = algorithmic bytes at 128-byte granularity, exact = the same bytes exactly,",
             "no-stop = what a scan without early stop would read, skipped = no-stop - exact.",
             "",
             "calibration: the 1 GiB device-to-device copy reads FETCH_SIZE = %.1f KiB and writes WRITE_SIZE = %.1f KiB;"
             % (float(copy_f["Counter_Value"]), float(copy_w["Counter_Value"])),
             "fetch is scaled x%.3f and write x%.3f below." % (f_scale, w_scale), ""])
    per_lay = {}
    for (lay, i), a, b in zip(order, fs, ws):
        assert a["Kernel_Name"] == b["Kernel_Name"]
        fb = float(a["Counter_Value"]) * 1024 * f_scale
        wb = float(b["Counter_Value"]) * 1024 * w_scale
        per_lay.setdefault(lay, []).append((i, _short(a["Kernel_Name"]), fb, wb))
    for lay in layouts:
        lines.append("%s launches (fetch and write MB per launch, scaled):" % lay)
        scans, ctrs = [], []
        for i, name, fb, wb in per_lay[lay]:
            if i == "lookup":
                lines.append("  %-8s %-16s %-45s fetch %8.1f  write %6.1f" % ("lookup", "5M ids", name, fb / 1e6, wb / 1e6))
                continue
            op, lo, hi, _ = preds[i]
            lit = "%d..%d" % (lo, hi) if hi is not None else "%d" % lo
            row = "  %-8s %-16s %-45s fetch %8.1f  write %6.1f" % (op, lit, name, fb / 1e6, wb / 1e6)
            c = (counted.get(lay) or [None] * len(preds))[i]
            if c is not None:
                exact, full, l128 = c
                row += "   alg128 %7.1f  exact %7.1f  no-stop %7.1f  skipped %7.1f" % (
                    l128 / 1e6, exact / 1e6, full / 1e6, (full - exact) / 1e6)
                ctrs.append(c)
            lines.append(row)
            scans.append(fb + wb)
        lines.append("  average HBM bytes per scan launch: %.0f" % np.mean(scans))
        if ctrs:
            m = np.mean(np.array(ctrs, dtype=np.float64), axis=0)
            lines.append("  average counted MB per scan launch: alg128 %.1f, exact %.1f, no-stop %.1f, skipped %.1f"
                         % (m[2] / 1e6, m[0] / 1e6, m[1] / 1e6, (m[1] - m[0]) / 1e6))
        lines.append("")
    pp = [fb + wb for i, _, fb, wb in per_lay.get("ppvbs", []) if i != "lookup"]
    lk = [fb + wb for i, _, fb, wb in per_lay.get("ppvbs", []) if i == "lookup"]
    lines += ["kernel_hash: %s" % kernel_hash(),
              "hbm_bytes_per_launch: %.0f" % np.mean(pp),
              "lookup_hbm_bytes_per_launch: %.0f" % (lk[0] if lk else float("nan"))]
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


WAIT_CMD = ("rocprofv3 --pmc SQ_WAIT_ANY SQ_WAVE_CYCLES -d rocprof_out/pmc_wait -o run --output-format csv -- "
            "python3 bench.py --steps 1 --warmup 0 --no-batch --serve-queries 0 --no-cpu-baseline")


def summarize_wait(wait_dir: str, out_path: str, preds, layouts=LAYOUTS):
    """The share of wave cycles spent waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES) of
    every launch of a one-step benchmark, from one rocprofv3 --pmc run."""
    import numpy as np

    rows = _kernel_rows(os.path.join(wait_dir, "run_counter_collection.csv"))
    by = {}
    for r in rows:
        d = by.setdefault(int(r["Dispatch_Id"]), {"Kernel_Name": r["Kernel_Name"], "Dispatch_Id": r["Dispatch_Id"]})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
    seq = [by[k] for k in sorted(by)]
    steps = _step_launches(seq, 1, len(preds), layouts)
    order = _step_layout_order(len(preds), layouts)
    lines = ["Share of wave cycles spent waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES) per launch of the",
             "benchmark step (500M-row column, 20-bit Zipf(1.0)), from one rocprofv3 counter run; kernel_hash",
             "names the scan kernel sources the counters were taken on.",
             "",
             "commands (repo root; TMPDIR=/tmp):",
             "  " + WAIT_CMD,
             "  python3 bench.py --summarize-wait rocprof_out/pmc_wait --out profiles/scan_lookup_500M_wait.txt",
             ""]
    cur = None
    for (lay, i), r in zip(order, steps):
        if lay != cur:
            if cur:
                lines.append("")
            lines.append("%s launches:" % lay)
            cur = lay
        share = r.get("SQ_WAIT_ANY", 0.0) / max(r.get("SQ_WAVE_CYCLES", 0.0), 1.0)
        if i == "lookup":
            lines.append("  %-8s %-16s %-45s wait %.3f" % ("lookup", "5M ids", _short(r["Kernel_Name"]), share))
        else:
            op, lo, hi, _ = preds[i]
            lit = "%d..%d" % (lo, hi) if hi is not None else "%d" % lo
            lines.append("  %-8s %-16s %-45s wait %.3f" % (op, lit, _short(r["Kernel_Name"]), share))
    lines += ["", "kernel_hash: %s" % kernel_hash()]
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_threads() -> int:
    """Worker threads for the CPU baseline: the host cores this process may use,
    at most 16 (a one-GPU share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_chunks(x, threads: int):
    """The oracle's own PP-VBS layout of x (dictionary, Algorithm 1, VBS), split into
    `threads` chunks of whole 64-row groups; each chunk's starting cursor into
    every BS_j comes from one popcount pass over M_j."""
    import numpy as np

    from oracle.dictionary import build_dictionary
    from oracle.layout import vbs_build
    from oracle.ppe import ppe_numerical
    from oracle.scan import CodeTable

    A, Q, rank = build_dictionary(x)
    C, Lc = ppe_numerical(Q)
    K = int(Lc.max())
    BS, M = vbs_build(C[rank], Lc[rank], K)
    table = CodeTable(A, C, Lc, K)
    n = x.shape[0]
    bounds = sorted(set([min(n, (n * k // threads + 63) // 64 * 64) for k in range(threads)] + [n]))
    cur = {j: np.concatenate([[0], np.cumsum(M[j], dtype=np.int64)])[bounds] for j in range(2, K + 1)}
    chunks = []
    for k in range(len(bounds) - 1):
        r0, r1 = bounds[k], bounds[k + 1]
        bs = [None, BS[1][r0:r1]] + [BS[j][cur[j][k]:cur[j][k + 1]] for j in range(2, K + 1)]
        m = [None, None] + [M[j][r0:r1] for j in range(2, K + 1)]
        chunks.append((r0, bs, m))
    return chunks, K, table


def _time_oracle(chunks, K, table, preds, ids, threads: int):
    """Seconds for every scan of `preds` and for the lookup of `ids`, the chunks
    spread over `threads` host threads (numpy releases the interpreter lock in its
    array operations)."""
    import concurrent.futures as cf

    import numpy as np

    from oracle.lookup import lookup_ids
    from oracle.scan import decode_vbs_values, scan_vbs

    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        t0 = time.perf_counter()
        for op, lo, hi, _ in preds:
            list(ex.map(lambda ch: scan_vbs(ch[1], ch[2], K, table, op, lo, hi), chunks))
        t_scan = time.perf_counter() - t0
        t0 = time.perf_counter()
        vals = list(ex.map(lambda ch: decode_vbs_values(ch[1], ch[2], K, table), chunks))
        lookup_ids(np.concatenate(vals), ids)
        t_lookup = time.perf_counter() - t0
    return t_scan, t_lookup


def cpu_baseline(x, preds, ids, sample_rows: int, threads: int):
    """The oracle (decode every code, compare, pack bits; lookups index the decoded
    values) timed on the host: every benchmark predicate on the first sample_rows
    rows of the column, and the benchmark's row IDs that fall in that range, at
    `threads` host threads and at one; then the small single-column workload
    (1M rows, one '<' scan, 10k lookups) in full."""
    import numpy as np

    from datagen import workloads

    xs = np.ascontiguousarray(x[:sample_rows])
    sid = ids[ids < sample_rows]
    chunks, K, table = _oracle_chunks(xs, threads)
    ts_t, tl_t = _time_oracle(chunks, K, table, preds, sid, threads)
    ts_1, tl_1 = _time_oracle(chunks, K, table, preds, sid, 1)
    c1 = workloads.config1()
    x1 = c1["x"]
    ch1, K1, tb1 = _oracle_chunks(x1, threads)
    p1 = [("lt", c1["lt_literal"], None, c1["lt_selectivity"])]
    c1_t = _time_oracle(ch1, K1, tb1, p1, c1["ids"], threads)
    c1_1 = _time_oracle(ch1, K1, tb1, p1, c1["ids"], 1)
    rate = lambda rows, t: round(rows / t / 1e9, 6)
    return {
        "value": rate(sample_rows * len(preds), ts_t),
        "unit": "Gtuples/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "PP-VBS scans (decode, compare, pack) of the first %d rows of the same column, all %d "
                  "predicates, %d host threads (%.1f s; one thread %.1f s); lookups of the %d benchmark row IDs "
                  "in that range (decode and index)" % (sample_rows, len(preds), threads, ts_t, ts_1, sid.shape[0]),
        "value_1thread": rate(sample_rows * len(preds), ts_1),
        "lookup_mrows": round(sid.shape[0] / tl_t / 1e6, 3),
        "lookup_mrows_1thread": round(sid.shape[0] / tl_1 / 1e6, 3),
        "cpu_model": _cpu_model(),
        "small_workload": {
            "rows": int(x1.shape[0]), "scan_gtuples": rate(x1.shape[0], c1_t[0]),
            "scan_gtuples_1thread": rate(x1.shape[0], c1_1[0]),
            "lookup_mrows": round(c1["ids"].shape[0] / c1_t[1] / 1e6, 3),
            "lookup_mrows_1thread": round(c1["ids"].shape[0] / c1_1[1] / 1e6, 3)},
    }


def serve_queries(x_counts, layouts, n_queries: int, seed: int):
    """Queries over the benchmark column seen as a table whose columns are its
    layouts: 1-3 predicates (selectivity log-uniform in [0.01 %, 50 %]) and a
    lookup of one column."""
    import numpy as np

    from datagen import workloads
    from paper_2209_00220_amd.serve import Query

    v, c = x_counts
    rng = np.random.default_rng(seed)
    qs = []
    for i in range(n_queries):
        preds = []
        for _ in range(int(rng.integers(1, 4))):
            sel = float(np.exp(rng.uniform(np.log(1e-4), np.log(0.5))))
            col = layouts[int(rng.integers(0, len(layouts)))]
            kind = int(rng.integers(0, 3))
            if kind == 0:
                lo, _ = workloads.lit_lt(v, c, sel)
                preds.append((col, "lt", lo, None))
            elif kind == 1:
                lo, _ = workloads.lit_lt(v, c, 1.0 - sel)
                preds.append((col, "ge", lo, None))
            else:
                lo, hi, _ = workloads.lit_between(v, c, sel)
                preds.append((col, "between", lo, hi))
        qs.append(Query(i, "t", preds, [layouts[int(rng.integers(0, len(layouts)))]]))
    return qs


def serve_bench(dev_cols, x_counts, n_queries: int, budget_bytes: int, **server_kw):
    """Saturation throughput (all queries at once) of the continuous-batching
    server and of one query at a time, then p50/p99 of both under Poisson
    arrivals at 25, 50 and 80 % of the one-at-a-time saturation."""
    from paper_2209_00220_amd.serve import GpuExecutor, Server, latency_summary, poisson_arrivals, run_serial

    layouts = list(dev_cols)
    ex = GpuExecutor({"t": dev_cols})
    warm = serve_queries(x_counts, layouts, 8, seed=99)
    Server(ex, budget_bytes, **server_kw).run(warm, keep_values=False)
    run_serial(ex, warm, keep_values=False)
    qs = serve_queries(x_counts, layouts, n_queries, seed=5)
    sat = latency_summary(Server(ex, budget_bytes, **server_kw).run(qs, keep_values=False))
    sat_serial = latency_summary(run_serial(ex, qs, keep_values=False))
    loads = []
    for frac in (0.25, 0.5, 0.8):
        qps = frac * sat_serial["qps"]
        for q, a in zip(qs, poisson_arrivals(n_queries, qps, seed=6)):
            q.arrival = float(a)
        srv = Server(ex, budget_bytes, **server_kw)
        served = latency_summary(srv.run(qs, keep_values=False))
        serial = latency_summary(run_serial(ex, qs, keep_values=False))
        loads.append({"load": frac, "offered_qps": round(qps, 1),
                      "p50_ms": round(served["p50_ms"], 3), "p99_ms": round(served["p99_ms"], 3),
                      "one_at_a_time_p50_ms": round(serial["p50_ms"], 3),
                      "one_at_a_time_p99_ms": round(serial["p99_ms"], 3),
                      "mean_batch": round(sum(srv.batch_sizes) / max(1, len(srv.batch_sizes)), 2)})
    mid = loads[1]
    for q in qs:
        q.arrival = 0.0
    return {
        "queries": n_queries,
        "budget_bytes": budget_bytes,
        "saturation_qps": round(sat["qps"], 1),
        "saturation_qps_one_at_a_time": round(sat_serial["qps"], 1),
        "offered_qps": mid["offered_qps"],
        "p50_ms": mid["p50_ms"],
        "p99_ms": mid["p99_ms"],
        "one_at_a_time_p50_ms": mid["one_at_a_time_p50_ms"],
        "one_at_a_time_p99_ms": mid["one_at_a_time_p99_ms"],
        "mean_batch": mid["mean_batch"],
        "loads": loads,
    }


def _ms_events(fn, repeats=5):
    """Median milliseconds of fn() between HIP events on the current stream."""
    import numpy as np
    import torch

    fn()
    ts = []
    for _ in range(repeats):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def wide_main(args):
    """Wide table: per-column layout advice (Algorithm 5), a pipelined four-column
    conjunction in the chosen layouts, and lookups of three columns on its rows."""
    import numpy as np
    import torch

    from datagen import workloads
    from paper_2209_00220_amd.advisor import advise_column
    from paper_2209_00220_amd.column import bv_compact, bv_popcount, bv_to_numpy, nwords, u32_to_numpy

    n = args.wide_rows
    torch.cuda.set_device(0)
    xs, adv = {}, {}
    t_adv = 0.0
    for c in range(16):
        x, w = workloads.config3_column(c, n)
        xs[c] = x
        progress("column %d: w=%d s=%.1f -- advisor over 3 layouts" % (c, w, workloads.WIDE_SKEWS[c % 4]))
        t0 = time.time()
        a = advise_column(x, numeric=True, width=w, layouts=("byteslice", "ppvbs", "bitpacked"), keep="all")
        t_adv += time.time() - t0
        adv[c] = a
        progress("  chose %s, AUC %s" % (a.chosen, {k: round(v, 4) for k, v in a.aucs.items()}))
    # the query: '<' at about 31.6 % on each filter column, pipelined
    lits = {}
    for c in workloads.WIDE_FILTER:
        v, k = workloads.value_counts(xs[c], workloads.WIDE_WIDTHS[c % 6])
        lits[c] = workloads.lit_lt(v, k, 0.316)[0]
    bvs = [torch.empty(nwords(n), dtype=torch.int64, device="cuda") for _ in range(2)]

    def conj(choice):
        cur = None
        for i, c in enumerate(workloads.WIDE_FILTER):
            col = adv[c].columns[choice(c)][1]
            col.scan("lt", lits[c], in_mask=cur, out=bvs[i % 2])
            cur = bvs[i % 2]
        return cur

    res = {}
    for name, choice in (("advised", lambda c: adv[c].chosen), ("ppvbs", lambda c: "ppvbs"),
                         ("byteslice", lambda c: "byteslice"), ("bitpacked", lambda c: "bitpacked")):
        ms = _ms_events(lambda: conj(choice))
        res[name] = {"conjunction_ms": round(ms, 3), "gtuples": round(4 * n / (ms * 1e-3) / 1e9, 1)}
    sel_bv = conj(lambda c: adv[c].chosen)
    count = int(bv_popcount(sel_bv, n).item())
    want = np.ones(n, dtype=bool)
    for c in workloads.WIDE_FILTER:
        want &= xs[c] < np.uint32(lits[c])
    assert count == int(want.sum()), "conjunction count differs from the plain one"
    ids, _ = bv_compact(sel_bv, n, max(count, 1))
    look = {}
    for c in workloads.WIDE_LOOKUP:
        col = adv[c].columns[adv[c].chosen][1]
        out_v = torch.empty(max(count, 1), dtype=torch.int32, device="cuda")
        ms = _ms_events(lambda: col.lookup(ids[:count], out=out_v[:count]))
        got = u32_to_numpy(out_v[:count])
        assert np.array_equal(got, xs[c][want]), "lookup differs from the raw values"
        look[c] = {"layout": adv[c].chosen, "ms": round(ms, 3), "mrows": round(count / (ms * 1e-3) / 1e6, 1)}
    out = {
        "metric": "wide-table conjunction Gtuples/s (advised layouts) and lookup Mrows/s",
        "value": res["advised"]["gtuples"], "unit": "Gtuples/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "16 columns x %d rows; '<' on columns 2,5,7,9 (~31.6%% each) pipelined; "
                               "lookup of columns 0,10,11 on the qualifying rows" % n, "rows": n},
        "advisor": {str(c): {"chosen": adv[c].chosen, "auc": {k: round(v, 5) for k, v in adv[c].aucs.items()},
                             "w": workloads.WIDE_WIDTHS[c % 6], "s": workloads.WIDE_SKEWS[c % 4]} for c in adv},
        "advisor_seconds": round(t_adv, 1),
        "conjunction": res, "qualifying_rows": count, "lookups": {str(k): v for k, v in look.items()},
    }
    print(json.dumps(out), flush=True)


def _grab_name(grab):
    """tiles_per_grab as reported: a number, or "round robin"."""
    from paper_2209_00220_amd import _lib as L

    return "round robin" if grab == L.BATCH_ROUND_ROBIN else grab


def batch_main(args):
    """Many scans over many columns: one persistent launch (HIP graph, autotuned
    shape) against one launch per predicate."""
    import numpy as np
    import torch

    import datagen
    from datagen import workloads
    from paper_2209_00220_amd import _lib as L
    from paper_2209_00220_amd.batch import autotune_batch, time_call
    from paper_2209_00220_amd.column import DeviceColumn, Dictionary, HostColumn, bv_popcount

    torch.cuda.set_device(0)
    specs = workloads.config4_columns(args.batch_cols)
    cols, counts, keep = [], [], []
    for i, (n, w, s, seed) in enumerate(specs):
        x = datagen.zipf_column(n, w, s, seed=seed)
        counts.append(workloads.value_counts(x, w))
        d = Dictionary(x)
        hc = HostColumn.encode(d, "ppvbs")
        d.close()
        cols.append(DeviceColumn(hc))
        keep.append(hc)
        del x
        if i % 8 == 7:
            progress("encoded %d / %d columns" % (i + 1, len(specs)))
    preds = workloads.config4_predicates(counts, args.batch_preds)
    outs = [cols[c].new_bv() for c, *_ in preds]
    rows = sum(int(cols[c].n_rows) for c, *_ in preds)
    alg = alg_lines = 0
    for (c, op, lo, hi, _), o in zip(preds, outs):
        _, ctr = cols[c].scan_stats(op, lo, hi, out=o)
        alg += int(ctr[0].item())
        alg_lines += int(ctr[4].item())

    def singles():
        for (c, op, lo, hi, _), o in zip(preds, outs):
            cols[c].scan(op, lo, hi, out=o)

    # the single launches at their own best launch shape (also used by the batch's items)
    from paper_2209_00220_amd.batch import autotune_scan

    tuned, _ = autotune_scan([(cols[c], op, lo, hi) for c, op, lo, hi, _ in preds])
    progress("scan launch tuned: grid %d, gather %d" % tuned)
    single_ms = _ms_events(singles)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    b, best, table = autotune_batch([(cols[c], op, lo, hi, None) for c, op, lo, hi, _ in preds], outs,
                                    grids=[cus * 2, cus * 3, cus * 4, cus * 8],
                                    grabs=(8, 16, 32, 64, L.BATCH_ROUND_ROBIN), streams=args.batch_streams, repeats=3)
    one_stream = min(v for k, v in table.items() if k[3] == 1) if 1 in args.batch_streams else None
    batch_ms = time_call(lambda: b.launch(best[1], best[2], True), repeats=5)
    torch.cuda.synchronize()
    # every result's popcount against the plain count from the value counts
    for (c, op, lo, hi, _), o in zip(preds, outs):
        v, k = counts[c]
        if op == "lt":
            want = int(k[v < lo].sum())
        elif op == "le":
            want = int(k[v <= lo].sum())
        elif op == "eq":
            want = int(k[v == lo].sum())
        else:
            want = int(k[(v >= lo) & (v <= hi)].sum())
        assert int(bv_popcount(o, int(cols[c].n_rows)).item()) == want, (c, op, lo, hi)
    out = {
        "metric": "batched scans Gtuples/s (one persistent launch vs one launch per predicate)",
        "value": round(rows / (batch_ms * 1e-3) / 1e9, 1), "unit": "Gtuples/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "%d PP-VBS columns (n log-uniform in [1e6, 1e8], w in 8..32, Zipf s in [0, 1.5]); "
                               "%d predicates (<, <=, =, BETWEEN; selectivity log-uniform 0.01-50%%)"
                               % (len(specs), len(preds)), "rows_scanned": rows},
        "batch_ms": round(batch_ms, 3), "single_launches_ms": round(single_ms, 3),
        "speedup": round(single_ms / batch_ms, 3), "solo_tiles": best[0], "grid": best[1],
        "tiles_per_grab": _grab_name(best[2]), "streams": best[3],
        "one_stream_ms": None if one_stream is None else round(one_stream, 3),
        "alg_bytes": alg_lines, "exact_alg_bytes": alg,
        "batch_hbm_frac": round(alg_lines / (batch_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
        "batch_hbm_frac_exact": round(alg / (batch_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
        "single_gtuples": round(rows / (single_ms * 1e-3) / 1e9, 1),
    }
    print(json.dumps(out), flush=True)


def serve_main(args):
    """Serving workload: tables of 4 resident PP-VBS columns (rows uniform in
    [--serve-rows-lo, --serve-rows-hi], 4e8..1e9 by default; w in 8..32, Zipf s in [0.5, 1.5]);
    queries of 1-4 predicates and a lookup of 1-2 columns.  Saturation
    throughput and p50/p99 under Poisson arrivals at 25/50/80 % of the
    one-query-at-a-time saturation, served with continuous batching and one
    query at a time."""
    import numpy as np
    import torch

    import datagen
    from datagen import workloads
    from paper_2209_00220_amd.column import DeviceColumn, Dictionary, HostColumn
    from paper_2209_00220_amd.serve import GpuExecutor, Query, Server, latency_summary, poisson_arrivals, run_serial

    torch.cuda.set_device(0)
    spec = workloads.config5_tables(args.serve_tables, 4, args.serve_rows_lo, args.serve_rows_hi,
                                    log_uniform=args.serve_log_uniform)
    tables, counts, keep = {}, [], []
    rows_total = 0
    for t, (n, cols) in enumerate(spec):
        tables["t%d" % t], cs = {}, []
        for c, (w, sk, seed) in enumerate(cols):
            # one column at a time: raw values are freed once encoded; the value
            # counts (for literal picking) come from the column's dictionary
            x = datagen.zipf_column(n, w, sk, seed=seed)
            d = Dictionary(x)
            del x
            cs.append(d.values_counts())
            hc = HostColumn.encode(d, "ppvbs")
            d.close()
            tables["t%d" % t]["c%d" % c] = DeviceColumn(hc)
            keep.append(hc)
            progress("table %d column %d: %d rows, w=%d, s=%.2f, %.2f bytes/row" % (
                t, c, n, w, sk, hc.info.layout_bytes / max(1, n)))
        counts.append(cs)
        rows_total += 4 * n
        progress("table %d / %d: %d rows x 4 columns" % (t + 1, len(spec), n))
    resident = sum(int(dc.device_bytes) for cols in tables.values() for dc in cols.values())
    raw = workloads.config5_queries(counts, args.serve_queries, seed=56)
    qs = [Query(i, "t%d" % t, [("c%d" % c, op, lo, hi) for c, op, lo, hi in preds], ["c%d" % c for c in look])
          for i, (t, preds, look) in enumerate(raw)]
    ex = GpuExecutor(tables)
    budget = int(args.serve_budget_gb * (1 << 30))
    warm = [Query(10_000 + q.qid, q.table, q.preds, q.lookups) for q in qs[:16]]
    Server(ex, budget).run(warm, keep_values=False)
    run_serial(ex, warm, keep_values=False)
    progress("saturation: all %d queries at once" % len(qs))
    srv = Server(ex, budget)
    served = srv.run(qs, keep_values=False)
    serial = run_serial(ex, qs, keep_values=False)
    for q in qs:   # the two schedules give every query the same rows
        assert served[q.qid].count == serial[q.qid].count, q
    sat, sat_serial = latency_summary(served), latency_summary(serial)
    loads = []
    for frac in (0.25, 0.5, 0.8):
        qps = frac * sat_serial["qps"]
        for q, a in zip(qs, poisson_arrivals(len(qs), qps, seed=57)):
            q.arrival = float(a)
        s_l = Server(ex, budget)
        a = latency_summary(s_l.run(qs, keep_values=False))
        b = latency_summary(run_serial(ex, qs, keep_values=False))
        loads.append({"load": frac, "offered_qps": round(qps, 1), "p50_ms": round(a["p50_ms"], 3),
                      "p99_ms": round(a["p99_ms"], 3), "one_at_a_time_p50_ms": round(b["p50_ms"], 3),
                      "one_at_a_time_p99_ms": round(b["p99_ms"], 3),
                      "mean_batch": round(sum(s_l.batch_sizes) / max(1, len(s_l.batch_sizes)), 2)})
        progress("load %.0f%%: %s" % (100 * frac, json.dumps(loads[-1])))
    out = {
        "metric": "served queries/s at saturation (continuous batching vs one query at a time); p50/p99 under load",
        "value": round(sat["qps"], 1), "unit": "queries/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "%d tables x 4 PP-VBS columns, rows %s in [%.0e, %.0e] per table, "
                               "w in 8..32, Zipf s in [0.5, 1.5]; %d queries of 1-4 predicates "
                               "(<, >=, BETWEEN; selectivity log-uniform 0.01-50%%) + lookup of 1-2 columns"
                               % (len(spec), "log-uniform" if args.serve_log_uniform else "uniform",
                                  args.serve_rows_lo, args.serve_rows_hi, len(qs)),
                   "rows_resident": rows_total, "resident_bytes": resident, "budget_bytes": budget},
        "saturation_qps_one_at_a_time": round(sat_serial["qps"], 1),
        "speedup": round(sat["qps"] / sat_serial["qps"], 3),
        "mean_batch": round(sum(srv.batch_sizes) / max(1, len(srv.batch_sizes)), 2),
        "loads": loads,
    }
    print(json.dumps(out), flush=True)


def sweep_main(args):
    """Skew, domain and distribution sensitivity: per (Zipf s, width w), and per
    (Gaussian sigma, width w), the bytes per row of each layout and its '<'
    (about 10 %) and '=' (most frequent value) scan rates."""
    import numpy as np
    import torch

    import datagen
    from datagen import workloads
    from paper_2209_00220_amd.column import DeviceColumn, Dictionary, HostColumn

    torch.cuda.set_device(0)
    n = args.sweep_rows
    rows = []

    def point(x, w, rec, label):
        v, k = workloads.value_counts(x, w)
        lt = workloads.lit_lt(v, k, 0.10)[0]
        eq = int(v[int(np.argmax(k))])
        d = Dictionary(x)
        rec["distinct"] = int(v.shape[0])
        for lay in LAYOUTS:
            hc = HostColumn.encode(d, lay, width=0 if lay == "ppvbs" else w)
            col = DeviceColumn(hc)
            out = col.new_bv()
            t_lt = _ms_events(lambda: col.scan("lt", lt, out=out))
            t_eq = _ms_events(lambda: col.scan("eq", eq, out=out))
            rec[lay] = {"bits_per_row": round(8 * hc.info.layout_bytes / n, 3),
                        "lt_gtuples": round(n / (t_lt * 1e-3) / 1e9, 1),
                        "eq_gtuples": round(n / (t_eq * 1e-3) / 1e9, 1)}
            col.close()
            hc.close()
        d.close()
        rows.append(rec)
        progress(label + "  " + "  ".join(
            "%s %.1f b/row lt %.0f eq %.0f" % (l, rec[l]["bits_per_row"], rec[l]["lt_gtuples"], rec[l]["eq_gtuples"])
            for l in LAYOUTS))

    for s in (0.0, 0.5, 1.0, 1.5, 2.0):
        for w in (4, 8, 12, 16, 20, 24):
            x = datagen.zipf_column(n, w, s, seed=1000 + int(10 * s) * 100 + w)
            point(x, w, {"dist": "zipf", "s": s, "w": w}, "zipf s=%.1f w=%d" % (s, w))
            del x
    # Gaussian columns of growing variance (sigma = 2^(w/4), 2^(w/2), 2^(3w/4))
    for w in (12, 20):
        for q in (1, 2, 3):
            sigma = 2.0 ** (q * w / 4.0)
            x = datagen.gaussian_column(n, w, sigma, seed=7000 + 10 * w + q)
            point(x, w, {"dist": "gaussian", "sigma": round(sigma, 1), "w": w},
                  "gaussian sigma=2^%.0f w=%d" % (q * w / 4.0, w))
            del x
    out = {"metric": "scan Gtuples/s and bits/row per layout across Zipf skew, domain width and Gaussian variance",
           "unit": "Gtuples/s", "n_gpus": 1, "dtype": "u8", "data": "synthetic",
           "config": {"workload": "%d rows per column; Zipf s in {0..2} x width w in {4..24}; Gaussian "
                                  "sigma in {2^(w/4), 2^(w/2), 2^(3w/4)} x w in {12, 20}" % n, "rows": n},
           "points": rows}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("scan", "wide", "batch", "serve", "sweep"), default="scan",
                    help="scan: the one-column benchmark (default); wide: 16-column table with the advisor, "
                         "a conjunction and lookups; batch: 256 predicates over 64 columns in one launch; "
                         "serve: continuous batching over resident tables; "
                         "sweep: skew x domain (and Gaussian variance) sensitivity of every layout")
    ap.add_argument("--serve-tables", type=int, default=8)
    ap.add_argument("--serve-rows-lo", type=float, default=4e8)
    ap.add_argument("--serve-rows-hi", type=float, default=1e9)
    ap.add_argument("--serve-log-uniform", action="store_true", help="table rows log-uniform (default uniform)")
    ap.add_argument("--sweep-rows", type=int, default=50_000_000)
    ap.add_argument("--wide-rows", type=int, default=100_000_000)
    ap.add_argument("--batch-cols", type=int, default=64)
    ap.add_argument("--batch-preds", type=int, default=256)
    ap.add_argument("--batch-streams", type=lambda v: tuple(int(x) for x in v.split(",")), default=(1, 2, 4),
                    help="stream counts the batch autotuner tries (comma-separated, each 1..4)")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rows", type=int, default=500_000_000)
    ap.add_argument("--cpu-sample", type=int, default=3_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--layouts", default=",".join(LAYOUTS))
    ap.add_argument("--no-lookup", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in scan launch shape")
    ap.add_argument("--preds", default="", help="comma-separated predicate indices to run (profiling)")
    ap.add_argument("--serve-queries", type=int, default=200, help="queries of the serving run (0: skip)")
    ap.add_argument("--no-batch", dest="batch", action="store_false", help="skip the batched-launch measurement")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device-to-device (a plain copy kernel to scale memory counters)")
    ap.add_argument("--summarize-trace", metavar="DIR", help="write a kernel-trace summary of DIR (CPU only)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write an HBM-traffic summary of two counter runs (CPU only)")
    ap.add_argument("--summarize-wait", metavar="DIR", help="write a wait-share summary of a counter run (CPU only)")
    ap.add_argument("--summarize-batch-trace", nargs=2, metavar=("DIR", "BENCH_OUT"),
                    help="write a kernel-trace summary of a --workload batch run (CPU only)")
    ap.add_argument("--out", help="summary file to write")
    args = ap.parse_args()
    if args.summarize_batch_trace:
        summarize_batch_trace(args.summarize_batch_trace[0], args.summarize_batch_trace[1], args.out, args.batch_preds)
        return
    if args.summarize_trace or args.summarize_pmc or args.summarize_wait:
        from datagen import workloads

        preds = workloads.config2_predicates(args.rows)
        if args.summarize_wait:
            summarize_wait(args.summarize_wait, args.out, preds)
        elif args.summarize_trace:
            summarize_trace(args.summarize_trace, args.steps, args.warmup, TRACE_CMD, args.out, preds)
        else:
            summarize_counters(args.summarize_pmc[0], args.summarize_pmc[1], PMC_CMDS, args.out, preds)
        return
    if args.workload != "scan":
        if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
            print("bench.py measures one GPU; run with --gpus 1", file=sys.stderr)
            sys.exit(2)
        {"wide": wide_main, "batch": batch_main, "serve": serve_main, "sweep": sweep_main}[args.workload](args)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the scan/lookup path has no multi-GPU form here "
              "(rows would shard by range with no exchange); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from datagen import workloads
    from paper_2209_00220_amd import _lib
    from paper_2209_00220_amd.column import DeviceColumn, Dictionary, HostColumn, u32_from_numpy

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    layouts = [l for l in args.layouts.split(",") if l]
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    n = args.rows
    progress("generating %d rows (Zipf 1.0 over 2^20)" % n)
    wl = workloads.config2(n)
    x, preds, ids = wl["x"], wl["preds"], wl["ids"]
    if args.preds:
        preds = [preds[int(i)] for i in args.preds.split(",")]
    progress("dictionary")
    d = Dictionary(x)
    cols = {}
    for lay in layouts:
        progress("encode + upload %s" % lay)
        hc = HostColumn.encode(d, lay, width=0 if lay == "ppvbs" else 20)
        cols[lay] = (hc, DeviceColumn(hc))
    d.close()
    torch.cuda.synchronize()
    ids_t = u32_from_numpy(ids)
    out_bv = cols[layouts[0]][1].new_bv()
    out_vals = torch.empty(ids.shape[0], dtype=torch.int32, device="cuda")

    # algorithmic bytes per scan launch (deterministic per predicate), untimed
    alg = {}
    for lay in layouts:
        col = cols[lay][1]
        for i, (op, lo, hi, _) in enumerate(preds):
            _, ctr = col.scan_stats(op, lo, hi, out=out_bv)
            torch.cuda.synchronize()
            c = ctr.cpu().numpy()
            alg[(lay, i)] = (int(c[0]), int(c[3]), int(c[4]))
    progress("counters done")
    tune_info = None
    if not args.no_tune:
        # launch shape of the single-column scans (grid, later-level gather limit),
        # timed on this step's own scans before the timed region
        from paper_2209_00220_amd.batch import autotune_scan

        tuned, table = autotune_scan([(cols[lay][1], op, lo, hi) for lay in layouts for op, lo, hi, _ in preds])
        tune_info = {"scan_grid": int(tuned[0]), "gather_rows": int(tuned[1]),
                     "candidates_ms": {"%d/%d" % k: round(v, 3) for k, v in sorted(table.items())}}
        progress("scan launch tuned: grid %d, gather %d (%s)" % (
            tuned[0], tuned[1], ", ".join("%d/%d: %.2f ms" % (g, r, t) for (g, r), t in sorted(table.items()))))

    stream = torch.cuda.current_stream()
    n_ev = len(layouts) * (len(preds) + 1)

    def new_events(k):
        return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k)]

    # Timed steps: per layout, one pair of events around its scans (launched back
    # to back) and one around its lookup; the steps themselves run back to back
    # with no host wait between them (a device left idle between steps starts the
    # next one slower, and an event pair around every launch adds its own gaps).
    timed_events = [new_events(2 * len(layouts)) for _ in range(max(1, args.steps))]
    # one more step with an event pair around every launch, for the per-predicate times
    launch_events = new_events(n_ev)

    def step(ev):
        e = 0
        for lay in layouts:
            col = cols[lay][1]
            ev[e][0].record(stream)
            for op, lo, hi, _ in preds:
                col.scan(op, lo, hi, out=out_bv)
            ev[e][1].record(stream)
            ev[e + 1][0].record(stream)
            if not args.no_lookup:
                col.lookup(ids_t, out=out_vals)
            ev[e + 1][1].record(stream)
            e += 2

    def step_by_launch(ev):
        e = 0
        for lay in layouts:
            col = cols[lay][1]
            for op, lo, hi, _ in preds:
                ev[e][0].record(stream)
                col.scan(op, lo, hi, out=out_bv)
                ev[e][1].record(stream)
                e += 1
            ev[e][0].record(stream)
            if not args.no_lookup:
                col.lookup(ids_t, out=out_vals)
            ev[e][1].record(stream)
            e += 1

    for _ in range(args.warmup):
        step(timed_events[0])
    torch.cuda.synchronize()
    progress("warmup done; timing %d steps" % args.steps)
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(timed_events[k])
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    acc = np.zeros(2 * len(layouts))
    for k in range(args.steps):
        acc += np.asarray([a.elapsed_time(b) for a, b in timed_events[k]])
    dur = acc / max(1, args.steps)   # ms per layout's scans and per lookup, averaged over steps
    ms_per_step = t_total / max(1, args.steps) * 1e3
    step_by_launch(launch_events)
    torch.cuda.synchronize()
    by_launch = [a.elapsed_time(b) for a, b in launch_events]

    # Outside the timed steps: the lookups with the same IDs in ascending order,
    # and each layout's scans cold -- one launch per predicate right after a
    # 1 GiB write, which evicts the last-level cache (256 MB) -- each launch
    # between its own pair of events.
    sorted_ids_t = u32_from_numpy(np.sort(ids))
    flush_buf = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    sorted_ms, cold_ms = {}, {}
    for lay in layouts:
        col = cols[lay][1]
        sorted_ms[lay] = None if args.no_lookup else _ms_events(lambda: col.lookup(sorted_ids_t, out=out_vals))
        cold_ms[lay] = 0.0
        for op, lo, hi, _ in preds:
            flush_buf.fill_(1)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            col.scan(op, lo, hi, out=out_bv)
            b.record(stream)
            b.synchronize()
            cold_ms[lay] += a.elapsed_time(b)
    del flush_buf, sorted_ids_t

    res = {}
    for li, lay in enumerate(layouts):
        scans_ms = float(dur[2 * li])            # the layout's scans, back to back
        lookup_ms = float(dur[2 * li + 1])
        alg_b = np.array([alg[(lay, i)][0] for i in range(len(preds))], dtype=np.float64)
        full_b = np.array([alg[(lay, i)][1] for i in range(len(preds))], dtype=np.float64)
        line_b = np.array([alg[(lay, i)][2] for i in range(len(preds))], dtype=np.float64)
        res[lay] = {
            "scan_gtuples": n * len(preds) / (scans_ms * 1e-3) / 1e9,
            "scan_ms_avg": scans_ms / len(preds),
            # per predicate, from the extra step with events around every launch
            "scan_ms": by_launch[li * (len(preds) + 1):li * (len(preds) + 1) + len(preds)],
            # algorithmic bytes at 128-byte granularity (the lines that hold them)
            # per second: the peak-equivalent rate; and the exact bytes' rate
            "alg_gbs": line_b.sum() / (scans_ms * 1e-3) / 1e9,
            "alg_bytes_per_launch": float(line_b.mean()),
            "exact_gbs": alg_b.sum() / (scans_ms * 1e-3) / 1e9,
            "exact_bytes_per_launch": float(alg_b.mean()),
            "full_bytes_per_launch": float(full_b.mean()),
            "lookup_ms": lookup_ms,
            "lookup_alg_bytes_per_id": lookup_alg_bytes_per_id(cols[lay][0].info),
            "lookup_mrows": (ids.shape[0] / (lookup_ms * 1e-3) / 1e6) if not args.no_lookup else None,
            "lookup_sorted_mrows": None if sorted_ms[lay] is None else ids.shape[0] / (sorted_ms[lay] * 1e-3) / 1e6,
            "cold_scan_gtuples": n * len(preds) / (cold_ms[lay] * 1e-3) / 1e9,
        }

    main_lay = "ppvbs" if "ppvbs" in res else layouts[0]
    r = res[main_lay]
    lay_name = {"ppvbs": "PP-VBS", "byteslice": "ByteSlice", "bitpacked": "Bit-Packed"}[main_lay]
    # the committed counter summary covers the PP-VBS launches
    traffic = read_traffic() if main_lay == "ppvbs" else None
    # the streaming probe on the same BS_1: the traffic of a scan settled by byte 1
    # without the compares, in the scans' launch shape -- the rate such a scan can
    # reach here (untimed steps; its own HIP events)
    bs1 = cols[main_lay][1].bufs[_lib.BUF_BS1]   # None for a Bit-Packed column
    probe_gbs = None
    if bs1 is not None:
        probe_out = torch.empty(bs1.numel() // 8, dtype=torch.uint8, device="cuda")
        probe_ms = _ms_events(lambda: _lib.bst_stream_probe(bs1, bs1.numel(), probe_out,
                                                            torch.cuda.current_stream().cuda_stream))
        probe_gbs = (bs1.numel() + probe_out.numel()) / (probe_ms * 1e-3) / 1e9
        del probe_out
    roofline = {
        "bound": "hbm",
        "achieved": round(r["alg_gbs"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(r["alg_gbs"] / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": "%s (%s)" % ("k_scan_packed" if main_lay == "bitpacked" else "k_scan_slices", lay_name),
        "alg_bytes_per_launch": r["alg_bytes_per_launch"],
        "granularity_bytes": 128,
        # the same algorithmic bytes counted exactly (not rounded to lines)
        "exact_alg_bytes_per_launch": r["exact_bytes_per_launch"],
        "exact_frac": round(r["exact_gbs"] / HBM_PEAK_GBS, 4),
        # bytes early stop saved: a scan without it reads every row's bytes up to
        # the literal's length and the masks past them
        "bytes_skipped_per_launch": round(r["full_bytes_per_launch"] - r["exact_bytes_per_launch"]),
        "avg_launch_ms": r["scan_ms_avg"],
        # HBM bytes moved per second (counter traffic / launch time), and the
        # streaming probe's rate on the same bytes' shape: how close the scan's
        # actual traffic runs to what this chip streams
        "traffic_gbs": None if traffic is None else round(traffic / (r["scan_ms_avg"] * 1e-3) / 1e9, 1),
        "probe_gbs": None if probe_gbs is None else round(probe_gbs, 1),
    }
    lookup_roofline = None
    if not args.no_lookup:
        lk_gbs = r["lookup_alg_bytes_per_id"] * ids.shape[0] / (r["lookup_ms"] * 1e-3) / 1e9
        lookup_roofline = {
            "bound": "hbm",
            "achieved": round(lk_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(lk_gbs / HBM_PEAK_GBS, 4),
            "traffic": read_traffic("lookup_hbm_bytes_per_launch") if main_lay == "ppvbs" else None,
            "kernel": "k_lookup (%s)" % lay_name,
            "alg_bytes_per_id": round(r["lookup_alg_bytes_per_id"], 1),
            "ids_per_launch": int(ids.shape[0]),
            "avg_launch_ms": r["lookup_ms"],
        }
    out = {
        "metric": METRIC,
        "value": round(r["scan_gtuples"], 3),
        "unit": "Gtuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": "1 column x %d rows, 20-bit Zipf(1.0) values; PP-VBS / ByteSlice / Bit-Packed; "
                        "<, =, BETWEEN at 0.1/1/10/50/90%% selectivity; lookup of %d random row IDs" % (n, ids.shape[0]),
            "rows": n,
            "predicates": [[op, lo, hi, round(sel, 6)] for op, lo, hi, sel in preds],
            "lookup_ids": int(ids.shape[0]),
            "layout_bytes": {lay: int(cols[lay][0].info.layout_bytes) for lay in layouts},
        },
        "roofline": roofline,
        "scan_tuning": tune_info,
        "lookup_roofline": lookup_roofline,
        "layouts": {lay: {
            "scan_gtuples": round(v["scan_gtuples"], 3),
            "scan_hbm_frac": round(v["alg_gbs"] / HBM_PEAK_GBS, 4),
            "scan_hbm_frac_exact": round(v["exact_gbs"] / HBM_PEAK_GBS, 4),
            "alg_bytes_per_launch": round(v["alg_bytes_per_launch"]),
            "exact_alg_bytes_per_launch": round(v["exact_bytes_per_launch"]),
            "full_bytes_per_launch": round(v["full_bytes_per_launch"]),
            # per predicate, from the instrumented scans: [exact algorithmic bytes,
            # bytes without early stop, algorithmic bytes at 128-byte granularity]
            "counters_by_predicate": [list(alg[(lay, i)]) for i in range(len(preds))],
            "lookup_mrows": None if v["lookup_mrows"] is None else round(v["lookup_mrows"], 1),
            "lookup_sorted_ids_mrows": None if v["lookup_sorted_mrows"] is None else round(v["lookup_sorted_mrows"], 1),
            "cold_scan_gtuples": round(v["cold_scan_gtuples"], 3),
            "lookup_hbm_frac": None if v["lookup_mrows"] is None else round(
                v["lookup_alg_bytes_per_id"] * ids.shape[0] / (v["lookup_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        } for lay, v in res.items()},
        "lookup_mrows": None if r["lookup_mrows"] is None else round(r["lookup_mrows"], 1),
        "p99_ms": None,
    }
    for lay in layouts:
        progress("%-9s scan us per predicate: %s" % (lay, " ".join("%.0f" % (1e3 * v) for v in res[lay]["scan_ms"])))
    for lay in layouts:
        progress("%-9s scan %.1f Gtuples/s  (%.0f GB/s algorithmic at 128 B, %.1f%% of 8 TB/s; exact bytes %.1f%%)"
                 "  lookup %s Mrows/s" % (
            lay, res[lay]["scan_gtuples"], res[lay]["alg_gbs"], 100 * res[lay]["alg_gbs"] / HBM_PEAK_GBS,
            100 * res[lay]["exact_gbs"] / HBM_PEAK_GBS,
            "-" if res[lay]["lookup_mrows"] is None else "%.0f" % res[lay]["lookup_mrows"]))
    for lay in layouts:
        progress("%-9s cold scans %.1f Gtuples/s; lookup of the IDs sorted %s Mrows/s" % (
            lay, res[lay]["cold_scan_gtuples"],
            "-" if res[lay]["lookup_sorted_mrows"] is None else "%.0f" % res[lay]["lookup_sorted_mrows"]))
    if args.batch:
        # the same step's scans as one persistent launch (replayed from a HIP graph)
        from paper_2209_00220_amd import _lib as L
        from paper_2209_00220_amd.batch import autotune_batch, time_call

        progress("batched form: %d scans in one launch" % (len(layouts) * len(preds)))
        specs = [(cols[lay][1], op, lo, hi, None) for lay in layouts for op, lo, hi, _ in preds]
        outs = [cols[layouts[0]][1].new_bv() for _ in specs]
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        # one stream: every one of these 500M-row scans fills the device alone (and
        # runs solo), so spreading them over streams has never paid here
        b, best, table = autotune_batch(specs, outs, grids=[cus * 2, cus * 3, cus * 4, cus * 8],
                                        grabs=(8, 16, 32, 64, L.BATCH_ROUND_ROBIN), streams=(1,), repeats=3)
        batch_ms = time_call(lambda: b.launch(best[1], best[2], True), repeats=5)
        # the timed steps' single launches, back to back
        single_ms = float(sum(res[lay]["scan_ms_avg"] * len(preds) for lay in layouts))
        out["batch"] = {"scans": len(specs), "solo_tiles": best[0], "grid": best[1],
                        "tiles_per_grab": _grab_name(best[2]), "streams": best[3],
                        "batch_ms": round(batch_ms, 3), "single_launches_ms": round(single_ms, 3),
                        "batch_gtuples": round(n * len(specs) / (batch_ms * 1e-3) / 1e9, 1)}
        progress("batch: %s" % json.dumps(out["batch"]))
        b.close()
        del outs
    if args.serve_queries > 0:
        progress("serving %d queries (continuous batching vs one at a time)" % args.serve_queries)
        out["serving"] = serve_bench({lay: cols[lay][1] for lay in layouts}, workloads.value_counts(x, 20),
                                     args.serve_queries, int(args.serve_budget_gb * (1 << 30)))
        out["p99_ms"] = out["serving"]["p99_ms"]
        progress("serving: %s" % json.dumps(out["serving"]))
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle) on %d rows" % args.cpu_sample)
        out["cpu_baseline"] = cpu_baseline(x, preds, ids, min(args.cpu_sample, n), _host_threads())
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
