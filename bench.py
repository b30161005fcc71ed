#!/usr/bin/env python3
"""Benchmark of the moment-pass least-squares fit on one MI355X.

One step = the whole single-fit hot path on one batch of synthetic input
resident in HBM: sampled range -> power-sum pass -> fixed-order combine ->
Hankel assembly and Gaussian elimination with partial pivoting -> (refinement
pass and correction for the compensated-float32 form) -> change back to the
x-basis, all through the C ABI on torch's current stream.

Workload of the line (default): one cubic fit of n = 1e8 float32 points,
x ~ U[-1, 1], coefficients N(0, 1), noise N(0, 0.01^2).  Both accumulation
forms are timed (float64 accumulation; compensated float32 with one float64
refinement pass); ``value`` is the points/s of the form named by --form
(default: the faster of the two that meets the 1e-6 coefficient bound).  The
streaming QR route (fit_qr) is timed on the same data as a third, reported
form ("qr").

Timing: W warm-up steps, then K steps between two events on the launch stream
with the library's kernel clock armed (each launch's main kernel stamps its
own start and end, lsefit_timing_*), so that ``ms_per_step`` and the kernel
durations of ``roofline`` come from the same launches; then K more steps with
nothing armed, reported as ``plain_ms_per_step``.

The line also carries compact blocks for the other workloads (``configs``):
the float64 linear fit of 1e6 points, the 65,536 ragged fits against one
fit_single call per fit, the 4,096-fit forward + adjoint against per-fit
forward + backward calls, and the shifted quintic of 1e7 points; each with its
points/s, the main kernel's rate and the error against the oracle.
--no-extra-configs leaves them out.

Prints one JSON line.  --gpus above 1 is refused: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
METRIC = "points/s & HBM GB/s (% peak) for moment pass+solve at ≤1e-6 rel coef err"
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ("paper_1512_08017_amd/csrc/kernels_impl.hpp", "paper_1512_08017_amd/csrc/device.hpp",
                  "paper_1512_08017_amd/csrc/kernels.hpp", "paper_1512_08017_amd/csrc/launchers.hpp",
                  "paper_1512_08017_amd/csrc/dispatch.hip", "paper_1512_08017_amd/csrc/api.hip")
HEADLINE_KERNEL = "k_moments<3, 0, float, 2>"   # float64 sums of float32 points, degree 3, two loads in flight
TRACE_FILE = os.path.join(PROFILES, "moments_cubic_f32_kernel_trace.txt")
TRAFFIC_FILE = os.path.join(PROFILES, "moments_cubic_f32_traffic.txt")
CEILING_FILE = os.path.join(PROFILES, "read_probe_ceiling.txt")
KIND_NAMES = ((0, "moments"), (1, "refine"), (2, "adjoint"), (3, "combine"), (4, "probe"), (5, "residual"),
              (6, "range"), (7, "plan"))


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--degree", type=int, default=3)
    ap.add_argument("--form", choices=("auto", "f64", "f32c"), default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-configs", action="store_true",
                    help="leave out the compact blocks of the other workloads")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target CPU time of the oracle baseline")
    ap.add_argument("--schedule", type=str, default=None, help="JSON schedule for the streaming kernels")
    ap.add_argument("--workload", choices=("cubic_f32", "ragged_batch", "grad_batch", "shifted_quintic",
                                           "linear_f64", "runge"), default="cubic_f32",
                    help="cubic_f32 is the benchmark; the others print their full measurement alone")
    ap.add_argument("--per-fit-limit", type=int, default=4096,
                    help="batched workloads: fits timed one call sequence at a time for the per-fit "
                         "baseline (0: no per-fit baseline)")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched workloads: plans keep the default schedule (or --schedule) instead of tuning")
    ap.add_argument("--lean", action="store_true",
                    help="with --workload: only the main form (no extra forms, no per-call cold/warm timings)")
    ap.add_argument("--read-probe", action="store_true", help="sweep the read and copy bandwidth probes instead")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="a few steps of each form plus one plain device copy of known size (for --pmc runs)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc output folders into the traffic summary")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("DIR", "TITLE", "COMMAND"),
                    help="turn a rocprofv3 --pmc --kernel-trace csv folder into a per-kernel counter summary")
    ap.add_argument("--out", type=str, default=None, help="where the --summarize-* commands write")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("DIR", "TITLE", "COMMAND"),
                    help="turn a rocprofv3 --kernel-trace --stats folder into a text summary (--out: where)")
    ap.add_argument("--summarize-probe", nargs=3, metavar=("JSON", "TRACE_DIR", "COMMAND"),
                    help="turn a --read-probe JSON line (and a kernel trace of that run) into the ceiling summary")
    ap.add_argument("--timed", nargs=3, metavar=("KERNEL", "SKIP", "TAKE"),
                    help="with --summarize-trace: also average dispatches SKIP .. SKIP+TAKE-1 of KERNEL "
                         "(the timed region of the command)")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# summaries of rocprofv3 output (text files under profiles/)
# ---------------------------------------------------------------------------
COPY_BYTES_NOTE = "plain copy: torch copy_ of the 1e8-point float32 x (400,000,000 bytes read, 400,000,000 written)"


def _read_counter_csv(folder, counter):
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    rows.append((r.get("Kernel_Name", ""), float(r["Counter_Value"])))
    return rows


def summarize_pmc(fetch_dir, write_dir, out_path=None):
    out = {}
    for counter, folder in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _read_counter_csv(folder, counter)
        mom = [v for k, v in rows if HEADLINE_KERNEL in k]
        ref = [v for k, v in rows if "k_refine" in k]
        cpy = [v for k, v in rows if ("copy" in k.lower() or "elementwise" in k.lower()) and "lsefit" not in k]
        out[counter] = {"moments_kib": sorted(mom), "refine_kib": sorted(ref), "copy_kib": sorted(cpy)}
    lines = ["# HBM traffic of the power-sum kernel (k_moments) and the refinement kernel (k_refine)",
             "# workload: cubic fit, n = 1e8 float32 points (800,000,000 algorithmic bytes per pass)",
             "# commands (two runs, one counter each; on the MI355X machine, from /tmp with TMPDIR=/tmp):",
             f"#   timeout -s KILL 180 rocprofv3 --pmc FETCH_SIZE -d {fetch_dir} -o run --output-format csv -- "
             "python3 /root/repo/bench.py --pmc-probe",
             f"#   timeout -s KILL 180 rocprofv3 --pmc WRITE_SIZE -d {write_dir} -o run --output-format csv -- "
             "python3 /root/repo/bench.py --pmc-probe",
             f"#   python3 /root/repo/bench.py --summarize-pmc {fetch_dir} {write_dir} "
             "--out /root/repo/profiles/moments_cubic_f32_traffic.txt",
             f"# {COPY_BYTES_NOTE}",
             f"kernel_hash {kernel_hash()}"]
    for counter, d in out.items():
        for key, vals in d.items():
            lines.append(f"{counter}.{key} " + " ".join(f"{v:.1f}" for v in vals))
    out_path = out_path or TRAFFIC_FILE
    os.makedirs(os.path.dirname(os.path.abspath(out_path)), exist_ok=True)
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_trace(folder, title, command, out_path=None, timed=None):
    """Per-kernel call count and duration (avg/min/max) of the library's kernels
    from a rocprofv3 --kernel-trace --stats output folder, as a short text
    summary; with timed = (kernel, skip, take) also the average over that
    kernel's dispatches skip .. skip+take-1 in launch order (the timed region
    of a bench.py run is dispatches W .. W+K-1 of its headline kernel)."""
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(folder, "**", "*kernel_stats.csv"), recursive=True):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if "lsefit" in r.get("Name", ""):
                    rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                                 float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3))
    lines = [f"# rocprofv3 kernel-trace summary: {title}",
             "# command (on the MI355X machine, from /tmp with TMPDIR=/tmp):",
             f"#   {command}",
             "# summarised by: python3 /root/repo/bench.py --summarize-trace DIR TITLE COMMAND "
             + (f"--timed '{timed[0]}' {timed[1]} {timed[2]} " if timed else "") + "--out FILE",
             f"#   (DIR = {folder}, TITLE and COMMAND = the two lines above, FILE = this file)",
             f"kernel_hash {kernel_hash()}"]
    for name, calls, avg, mn, mx in sorted(rows, key=lambda r: -r[1] * r[2]):
        short = name.split("(")[0]
        lines.append(f"{short:60s} calls {calls:6d}  avg {avg:10.2f} us  min {mn:10.2f} us  max {mx:10.2f} us")
    if timed:
        kname, skip, take = timed[0], int(timed[1]), int(timed[2])
        disp = []
        for path in glob.glob(os.path.join(folder, "**", "*kernel_trace.csv"), recursive=True):
            with open(path) as fh:
                for r in csv.DictReader(fh):
                    if kname in r["Kernel_Name"]:
                        disp.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
        disp.sort()
        sel = [(e - s) / 1e3 for s, e in disp[skip:skip + take]]
        if sel:
            lines.append(f"timed_region {kname} dispatches {skip}..{skip + len(sel) - 1} of {len(disp)}  "
                         f"avg {sum(sel) / len(sel):.2f} us  min {min(sel):.2f} us  max {max(sel):.2f} us")
    text = "\n".join(lines) + "\n"
    if out_path:
        os.makedirs(os.path.dirname(os.path.abspath(out_path)), exist_ok=True)
        with open(out_path, "w") as fh:
            fh.write(text)
    print(text, end="")


def summarize_counters(folder, title, command, out_path=None):
    """Per-kernel dispatch count, average duration and the average of every
    counter of a rocprofv3 --pmc --kernel-trace csv output folder (the
    library's kernels only), as a short text summary."""
    import csv
    import glob
    from collections import defaultdict
    vals = defaultdict(lambda: defaultdict(list))
    for path in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if "lsefit" in r["Kernel_Name"]:
                    vals[r["Kernel_Name"].split("(")[0]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    durs = defaultdict(list)
    for path in glob.glob(os.path.join(folder, "**", "*kernel_trace.csv"), recursive=True):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if "lsefit" in r["Kernel_Name"]:
                    durs[r["Kernel_Name"].split("(")[0]].append(
                        (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = [f"# rocprofv3 counter summary: {title}",
             "# command (on the MI355X machine, from /tmp with TMPDIR=/tmp):",
             f"#   {command}",
             "# summarised by: python3 /root/repo/bench.py --summarize-counters DIR TITLE COMMAND --out FILE",
             f"#   (DIR = {folder}, TITLE and COMMAND = the two lines above, FILE = this file)",
             "# per kernel: dispatches, average duration, then the average value of each counter per dispatch",
             f"kernel_hash {kernel_hash()}"]
    order = sorted(vals, key=lambda k: -sum(durs.get(k, [0.0])))
    for k in order:
        d = durs.get(k, [])
        avg = sum(d) / len(d) if d else float("nan")
        lines.append(f"{k}  dispatches {len(d)}  avg {avg:.2f} us")
        for c in sorted(vals[k]):
            v = vals[k][c]
            lines.append(f"    {c:28s} {sum(v) / len(v):18,.1f}")
    text = "\n".join(lines) + "\n"
    if out_path:
        os.makedirs(os.path.dirname(os.path.abspath(out_path)), exist_ok=True)
        with open(out_path, "w") as fh:
            fh.write(text)
    print(text, end="")


def summarize_probe(json_path, trace_dir, command, out_path=None):
    """The read and copy ceilings from a --read-probe run (its JSON line: each
    configuration timed by the kernel clock) and, from a rocprofv3 kernel trace
    of the same run, the fastest dispatch of each probe kernel as a cross-check."""
    import csv
    import glob
    with open(json_path) as fh:
        d = json.loads(fh.read().strip().splitlines()[-1])
    rows = d["rows"]
    lines = ["# read and copy bandwidth ceilings of the MI355X (lsefit_read_probe, lsefit_copy_probe)",
             "# two float32 arrays of 1e8 elements: 800,000,000 bytes read per launch (read probe), and as",
             "# many written (copy probe: 1,600,000,000 bytes per launch, the traffic shape of the adjoint pass)",
             "# 16-byte loads and stores, no arithmetic; every configuration launched 10 times, timed by the kernel",
             "# clock (lsefit_timing_*); pattern 0: each wave reads one contiguous share; pattern 1: the grid",
             "# strides over 16-byte vectors; pattern 2: each block reads one contiguous share, its waves take",
             "# turns; nt: non-temporal loads (and stores)",
             "# command (on the MI355X machine, from /tmp with TMPDIR=/tmp):",
             f"#   {command}",
             f"# summarised by: python3 /root/repo/bench.py --summarize-probe JSON TRACE_DIR COMMAND --out FILE",
             f"kernel_hash {kernel_hash()}"]
    for probe in ("read", "copy"):
        best = max((r for r in rows if r["probe"] == probe), key=lambda r: r["gbps"])
        lines.append(f"best_{probe}: {best['gbps']:.0f} GB/s ({best['gbps'] / HBM_PEAK_GBPS:.1%} of 8 TB/s)  "
                     + json.dumps({k: best[k] for k in ("waves_per_cu", "wpb", "unroll", "pattern", "nt")}))
    lines.append("")
    for probe in ("read", "copy"):
        for pat in (0, 1, 2):
            for nt in (0, 1):
                sel = [r for r in rows if r["probe"] == probe and r["pattern"] == pat and r["nt"] == nt]
                if not sel:
                    continue
                b = max(sel, key=lambda r: r["gbps"])
                lines.append(f"{probe} pattern {pat} nt {nt}: best {b['gbps']:7.0f} GB/s at waves/CU "
                             f"{b['waves_per_cu']}, waves/block {b['wpb']}, unroll {b['unroll']}")
    if trace_dir:
        best = {}
        for path in glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True):
            with open(path) as fh:
                for r in csv.DictReader(fh):
                    k = r["Kernel_Name"]
                    if "_probe<" not in k:
                        continue
                    us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
                    name = k.split("(")[0].replace("void lsefit::", "")
                    best[name] = min(best.get(name, us), us)
        lines.append("")
        lines.append("# rocprofv3 kernel trace of the same run: fastest dispatch of each probe kernel")
        for name in sorted(best):
            nbytes = 1.6e9 if "copy" in name else 0.8e9
            lines.append(f"{name:34s} {best[name]:8.2f} us  {nbytes / (best[name] * 1e-6) / 1e9:7.0f} GB/s")
    text = "\n".join(lines) + "\n"
    out_path = out_path or CEILING_FILE
    with open(out_path, "w") as fh:
        fh.write(text)
    print(text, end="")


def _summary_fields(path):
    """{first word: rest of the line} of a summary file, or None without a matching kernel hash."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        k, _, rest = line.strip().partition(" ")
        vals[k] = rest
    if vals.get("kernel_hash") != kernel_hash():
        return None
    return vals


def traffic_bytes(kernel="moments"):
    """Scaled HBM bytes per launch from the stored --pmc summary, or None if stale/missing."""
    vals = _summary_fields(TRAFFIC_FILE)
    if vals is None:
        return None
    try:
        fetch = sorted(float(v) for v in vals[f"FETCH_SIZE.{kernel}_kib"].split())
        write = sorted(float(v) for v in vals[f"WRITE_SIZE.{kernel}_kib"].split())
        cf = max(float(v) for v in vals["FETCH_SIZE.copy_kib"].split())
        cw = max(float(v) for v in vals["WRITE_SIZE.copy_kib"].split())
    except (KeyError, ValueError):
        return None
    # scale each counter by (known bytes of the plain copy) / (its reading of that copy)
    sf = 400_000_000 / (cf * 1024.0)
    sw = 400_000_000 / (cw * 1024.0)
    med = lambda a: a[len(a) // 2]
    return med(fetch) * 1024.0 * sf + med(write) * 1024.0 * sw


def profile_timed_avg_ms():
    """The rocprofv3 average of the headline kernel over the timed region of the
    committed trace summary (same kernel sources), in ms, or None."""
    vals = _summary_fields(TRACE_FILE)
    if vals is None or "timed_region" not in vals:
        return None
    words = vals["timed_region"].split()
    try:
        return float(words[words.index("avg") + 1]) / 1e3
    except (ValueError, IndexError):
        return None


def measured_ceiling_gbps(kind="read"):
    """Best rate of the project's read (or copy) probe from its stored summary (or None)."""
    if not os.path.exists(CEILING_FILE):
        return None
    for line in open(CEILING_FILE):
        if line.startswith(f"best_{kind}:"):
            return float(line.split()[1])
    return None


# ---------------------------------------------------------------------------
# GPU timing
# ---------------------------------------------------------------------------
def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _time(fn, steps, warmup):
    """ms per call of fn over `steps` back-to-back calls between two events on
    torch's current stream (the stream the library launches on)."""
    import torch
    for _ in range(warmup):
        fn()
    a, b = _events()
    torch.cuda.synchronize()
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def _kernel_avgs():
    from paper_1512_08017_amd import _lib
    L = _lib.load()
    out = {}
    for kind, name in KIND_NAMES:
        tot, cnt = ctypes.c_double(0.0), ctypes.c_int64(0)
        _lib.check(L.lsefit_timing_read(kind, ctypes.byref(tot), ctypes.byref(cnt)), "lsefit_timing_read")
        if cnt.value:
            out[name] = {"avg_ms": tot.value / cnt.value, "launches": int(cnt.value)}
    return out


def armed_region(fn, steps):
    """(ms per call, kernel durations) of `steps` calls of fn with the kernel
    clock armed: both figures describe the same launches."""
    from paper_1512_08017_amd import _lib
    L = _lib.load()
    _lib.check(L.lsefit_timing_reset(), "lsefit_timing_reset")
    _lib.check(L.lsefit_timing_enable(1), "lsefit_timing_enable")
    try:
        ms = _time(fn, steps, 0)
    finally:
        L.lsefit_timing_enable(0)
    return ms, _kernel_avgs()


def timed_form(fn, steps, warmup):
    """Warm-up, the timed region (kernel clock armed) and a plain region of the same length."""
    for _ in range(warmup):
        fn()
    ms, kern = armed_region(fn, steps)
    plain = _time(fn, steps, 0)
    return ms, plain, kern


def _both_forms(plan, fn, args):
    """A tuned plan's step in both replay forms: graph replays (after the capture),
    then eager launches (kernel clock armed, and a plain region).  Returns the
    form the tuning kept (True: graph), the graph time, the armed and plain
    eager times and the kernel times; the plan keeps its tuned form."""
    graph = plan.graph
    plan.set_graph(True)
    graph_ms = _time(fn, args.steps, args.warmup)
    plan.set_graph(False)
    ms, plain, kern = timed_form(fn, args.steps, 2)
    plan.set_graph(graph)
    return graph, graph_ms, ms, plain, kern


MALL_FLUSH_BYTES = 1 << 30   # > the 256 MB Infinity Cache


def _cold_warm(fn, reps):
    """Median and minimum per-call time of fn, warm (back to back) and cold
    (after writing a 1 GiB scratch buffer, which evicts the 256 MB MALL), each
    call between its own pair of events on the current stream."""
    import torch
    flush = torch.empty(MALL_FLUSH_BYTES // 4, dtype=torch.float32, device="cuda:0")
    out = {}
    for kind in ("warm", "cold"):
        ts = []
        for i in range(reps):
            if kind == "cold":
                flush.fill_(float(i))
            a, b = _events()
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        ts.sort()
        out[f"{kind}_median_ms"] = ts[len(ts) // 2]
        out[f"{kind}_min_ms"] = ts[0]
    del flush
    return out


def _r(v, nd=6):
    return float(f"{v:.{nd}g}")


class SingleFitRunner:
    """Pre-allocated buffers and one C-ABI step: fit_single (the fused single-fit
    call) or, with route="qr", fit_qr (the streaming QR route)."""

    def __init__(self, x, y, degree, precision, route="moments", **opts):
        import torch
        from paper_1512_08017_amd import _lib, api
        self.L = _lib.load()
        self.x, self.y, self.m, self.precision = x, y, degree, precision
        self.fn = self.L.fit_qr if route == "qr" else self.L.fit_single
        self.name = "fit_qr" if route == "qr" else "fit_single"
        self.opt = api.options(degree, precision, 1, **opts)
        nbytes = api.workspace_bytes(1, degree)
        self.ws = torch.zeros(nbytes, dtype=torch.uint8, device=x.device)
        self.coef = torch.empty(2 * (degree + 1), dtype=torch.float64, device=x.device)
        self.status = torch.empty(1, dtype=torch.int32, device=x.device)
        vp = ctypes.c_void_p
        dt = _lib.F32 if x.dtype == torch.float32 else _lib.F64
        self.args = (vp(x.data_ptr()), vp(y.data_ptr()), x.numel(), dt, ctypes.byref(self.opt),
                     vp(self.ws.data_ptr()), self.ws.numel(), vp(self.coef.data_ptr()), vp(self.status.data_ptr()),
                     None, ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream))
        self._check = _lib.check

    def step(self):
        self._check(self.fn(*self.args), self.name)


def residual_pass(runner, n, steps, warmup):
    """Times fit_residuals after the runner's fit (Table V pass): the sum of
    squared errors alone (8 B per float32 point read) and with every residual
    stored (8 B read + 4 B written), with the residual kernel's own duration."""
    import torch
    from paper_1512_08017_amd import _lib
    L = _lib.load()
    vp = ctypes.c_void_p
    x, y = runner.x, runner.y
    sse = torch.empty(1, dtype=torch.float64, device=x.device)
    res = torch.empty_like(x)
    st = vp(torch.cuda.current_stream(x.device).cuda_stream)
    out = {}
    for name, rptr, nbytes in (("sse_only", None, 8.0 * n), ("stored", vp(res.data_ptr()), 12.0 * n)):
        args_ = (vp(x.data_ptr()), vp(y.data_ptr()), None, None, 1, n, 0, ctypes.byref(runner.opt), None,
                 vp(runner.ws.data_ptr()), runner.ws.numel(), vp(sse.data_ptr()), rptr, st)
        fn = lambda: _lib.check(L.fit_residuals(*args_), "fit_residuals")
        for _ in range(warmup):
            fn()
        ms, kern = armed_region(fn, steps)
        kms = kern["residual"]["avg_ms"]
        out[name] = {"ms_per_call": _r(ms), "kernel_ms": _r(kms), "kernel_gbps": round(nbytes / (kms * 1e-3) / 1e9, 1),
                     "algorithmic_bytes": int(nbytes)}
    out["sse"] = float(sse.cpu()[0])
    return out


# ---------------------------------------------------------------------------
# CPU baseline legs: the oracle, timed on the host's cores; its results are
# also the reference the GPU forms are checked against (the oracle never runs
# on the measured GPU path)
# ---------------------------------------------------------------------------
def cpu_baseline(x_np, y_np, degree, target_s, timed=True):
    """(baseline record or None, oracle result); untimed: one oracle pass for the reference only."""
    from oracle import c_oracle
    if not timed:
        return None, c_oracle.fit(x_np, y_np, degree)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    t0 = time.perf_counter()
    reps = 0
    res = None
    while True:
        res = c_oracle.fit(x_np, y_np, degree, threads=threads)
        reps += 1
        el = time.perf_counter() - t0
        if el >= target_s or reps >= 1000:
            break
    used = c_oracle.max_threads()
    # one thread (the paper's sequential execution), on a bounded prefix of the same points
    n1 = min(x_np.shape[0], 20_000_000)
    t1 = time.perf_counter()
    reps1 = 0
    while True:
        c_oracle.fit(x_np[:n1], y_np[:n1], degree, threads=1)
        reps1 += 1
        el1 = time.perf_counter() - t1
        if el1 >= target_s / 3 or reps1 >= 100:
            break
    c_oracle.fit(x_np[:1000], y_np[:1000], degree, threads=threads)   # back to all threads
    return {"value": x_np.shape[0] * reps / el, "unit": "points/s", "cores": int(used), "kind": "oracle",
            "sample": f"{reps} full pass(es) of the plain-C float64 oracle over the same {x_np.shape[0]:,} points "
                      f"(compensated sums + partial-pivoting elimination), {el:.1f} s on {used} host threads",
            "build": c_oracle.BUILD_NOTE,
            "single_thread": {"value": n1 * reps1 / el1, "unit": "points/s",
                              "sample": f"{reps1} pass(es) over the first {n1:,} points on 1 thread, {el1:.1f} s"}}, res


def single_cpu_leg(wl, m, center=None, scale=None):
    """One timed pass of the plain-C float64 oracle over a single-fit workload
    (the reference and a CPU rate); (result, record)."""
    from oracle import c_oracle
    t0 = time.perf_counter()
    if center is None:
        ref = c_oracle.fit(wl.x, wl.y, m)
    else:
        ref = c_oracle.fit(wl.x, wl.y, m, center, scale)
    s = time.perf_counter() - t0
    return ref, {"value": wl.n / s, "unit": "points/s", "cores": c_oracle.max_threads(), "kind": "oracle",
                 "sample": f"one pass over the {wl.n:,} points, {s:.3f} s"}


def ragged_cpu_leg(bf):
    """The plain-C float64 oracle over the whole ragged batch on the host's
    threads: the reference coefficients and a CPU rate."""
    from oracle import c_oracle
    t0 = time.perf_counter()
    ref, rst = c_oracle.fit_batched(bf.x, bf.y, bf.offsets, bf.degrees, stride=4)
    cpu_s = time.perf_counter() - t0
    return ref, rst, {"value": bf.total_points / cpu_s, "unit": "points/s", "cores": c_oracle.max_threads(),
                      "kind": "oracle",
                      "sample": f"one pass of the plain-C float64 oracle over all {bf.batch} fits, {cpu_s:.2f} s"}


def grad_cpu_leg(bf, gbar, sample):
    """The float64 adjoint oracle (NumPy, one thread): forward fit + adjoint of
    the sampled fits of the gradient batch with upstream gbar; (per-fit
    results, record)."""
    from oracle import adjoint
    t0 = time.perf_counter()
    res = {}
    for f in sample:
        lo, hi = int(bf.offsets[f]), int(bf.offsets[f + 1])
        res[f] = adjoint.gradients(bf.x[lo:hi], bf.y[lo:hi], int(bf.degrees[f]), gbar[f, : int(bf.degrees[f]) + 1])
    cpu_s = time.perf_counter() - t0
    npts = sum(int(bf.offsets[f + 1] - bf.offsets[f]) for f in sample)
    return res, {"value": npts / cpu_s, "unit": "points/s", "cores": 1, "kind": "oracle",
                 "sample": f"forward fit + adjoint of the float64 oracle on {len(sample)} sampled fits, "
                           f"{cpu_s:.2f} s"}


def quintic_cpu_leg(wl):
    """The exact minimiser of the shifted quintic (integer power sums over its
    2^-14 grid of x, rational elimination) and one timed pass of the plain-C
    oracle in the shifted variable."""
    import numpy as np
    from oracle import exact
    a_ex, b_ex = exact.fit_exact_grid(wl.x, wl.y, 5, 1000.5, 0.5, 2.0 ** -14)
    _, rec = single_cpu_leg(wl, 5, 1000.5, 0.5)
    return (np.array([float(v) for v in a_ex]), np.array([float(v) for v in b_ex])), rec


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def _dev():
    import torch
    return torch.device("cuda:0")


def _normwise(got, ref):
    import numpy as np
    got, ref = np.asarray(got, float), np.asarray(ref, float)
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def _batched_err(bf, coef, ref):
    """max over fits of the normwise coefficient error (only each fit's own degree counts)."""
    import numpy as np
    m = bf.degrees.astype(np.int64)
    mask = np.arange(coef.shape[1])[None, :] <= m[:, None]
    diff = np.where(mask, np.abs(coef - ref[:, : coef.shape[1]]), 0.0).max(axis=1)
    scale = np.where(mask, np.abs(ref[:, : coef.shape[1]]), 0.0).max(axis=1)
    return float(np.max(diff / scale))


def bench_linear(args):
    """Plain linear fit, 1e6 float64 points (launch-latency bound: 16 MB)."""
    import torch
    from paper_1512_08017_amd import workloads as W
    wl = W.linear_f64()
    x, y = torch.from_numpy(wl.x).to(_dev()), torch.from_numpy(wl.y).to(_dev())
    r = SingleFitRunner(x, y, 1, "f64")
    ms, plain, kern = timed_form(r.step, args.steps, args.warmup)
    ref, cpu = single_cpu_leg(wl, 1)
    km = kern["moments"]["avg_ms"]
    return {"workload": f"linear_f64: one degree-1 fit of n={wl.n} float64 points, x~U[0,10], y=2+3x+N(0,0.5^2)",
            "ms_per_step": _r(ms), "plain_ms_per_step": _r(plain), "points_per_s": _r(wl.n / (ms * 1e-3)),
            "us_per_fit": _r(ms * 1e3), "kernel": "k_moments", "kernel_ms": _r(km),
            "kernel_gbps": round(16.0 * wl.n / (km * 1e-3) / 1e9, 1), "kernels": kern,
            "status": int(r.status.cpu()[0]),
            "max_rel_coef_err": _normwise(r.coef[:2].cpu().numpy(), ref["a"]), "cpu_baseline": cpu}


def bench_quintic(args, full=False):
    """Ill-conditioned stress: degree 5, 1e7 float32 x in [1000, 1001]; the
    compensated float32 form with refinement (and the float64 form) against the
    exact minimiser, error per coefficient in the t- and x-basis."""
    import numpy as np
    import torch
    from paper_1512_08017_amd import workloads as W
    wl = W.shifted_quintic()
    x, y = torch.from_numpy(wl.x).to(_dev()), torch.from_numpy(wl.y).to(_dev())
    (a_ex, b_ex), cpu = quintic_cpu_leg(wl)
    out = {"workload": f"shifted_quintic: one degree-5 fit of n={wl.n} float32 points, x~U[1000,1001]",
           "cpu_baseline": cpu}
    for prec in ("f32c", "f64"):
        r = SingleFitRunner(x, y, 5, prec)
        ms, plain, kern = timed_form(r.step, args.steps, args.warmup)
        a = r.coef[:6].cpu().numpy()
        b = r.coef[6:12].cpu().numpy()
        km = kern["moments"]["avg_ms"]
        out[prec] = {"ms_per_step": _r(ms), "plain_ms_per_step": _r(plain), "points_per_s": _r(wl.n / (ms * 1e-3)),
                     "kernel_ms": _r(km), "kernel_gbps": round(8.0 * wl.n / (km * 1e-3) / 1e9, 1),
                     "kernels": kern, "status": int(r.status.cpu()[0]),
                     "max_rel_err_per_coef_t": float(np.max(np.abs(b - b_ex) / np.abs(b_ex))),
                     "max_rel_err_per_coef_x": float(np.max(np.abs(a - a_ex) / np.abs(a_ex)))}
        if full:
            out[prec]["per_call"] = _cold_warm(r.step, 20)
    return out


def _per_fit_single_calls(L, x, y, bf, nfit, dev):
    """Raw fit_single calls, one per fit, on preallocated buffers, each return
    code checked: (callable, points)."""
    import torch
    from paper_1512_08017_amd import _lib, api
    ws = torch.zeros(api.workspace_bytes(1, 3), dtype=torch.uint8, device=dev)
    cbuf = torch.zeros(nfit, 8, dtype=torch.float64, device=dev)
    sbuf = torch.zeros(nfit, dtype=torch.int32, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    opts = [api.options(int(m)) for m in range(1, 4)]
    calls = []
    pts = 0
    for f in range(nfit):
        lo, hi = int(bf.offsets[f]), int(bf.offsets[f + 1])
        m = int(bf.degrees[f])
        pts += hi - lo
        calls.append((ctypes.c_void_p(x.data_ptr() + 4 * lo), ctypes.c_void_p(y.data_ptr() + 4 * lo), hi - lo,
                      _lib.F32, ctypes.byref(opts[m - 1]), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                      ctypes.c_void_p(cbuf.data_ptr() + 64 * f), ctypes.c_void_p(sbuf.data_ptr() + 4 * f), None,
                      stream))
    fs = L.fit_single

    def run():
        for c in calls:
            rc = fs(*c)
            if rc:
                _lib.check(rc, "fit_single")

    return run, pts, (cbuf, sbuf, ws)


def _per_fit_record(run, pts, nfit, kinds):
    """Per-fit baseline: wall time of the call loop (events around it, which also
    bound the GPU time) and the summed kernel durations of its launches."""
    ms = _time(run, 1, 1)
    _, kern = armed_region(run, 1)
    gpu_ms = sum(kern[k]["avg_ms"] * kern[k]["launches"] for k in kinds if k in kern)
    return {"fits": nfit, "points": pts, "ms": _r(ms), "ms_per_fit": _r(ms / nfit),
            "points_per_s": _r(pts / (ms * 1e-3)), "kernel_ms_sum": _r(gpu_ms),
            "kernel_points_per_s": _r(pts / (gpu_ms * 1e-3))}


def bench_ragged(args, full=False):
    """65,536 ragged fits (log-uniform lengths in [16, 65536], degree 1..3): one
    persistent batched launch sequence (tuned plan, graph replay) against one
    fit_single call per fit on the same GPU; with full, also the compensated
    float32 form, the streaming QR route and the Chebyshev basis."""
    import numpy as np
    import torch
    import paper_1512_08017_amd as lf
    from paper_1512_08017_amd import _lib, api, workloads as W
    dev = _dev()
    log("generating ragged_batch (65,536 fits)")
    bf = W.ragged_batch()
    x, y = torch.from_numpy(bf.x).to(dev), torch.from_numpy(bf.y).to(dev)
    off, dg = torch.from_numpy(bf.offsets).to(dev), torch.from_numpy(bf.degrees).to(dev)
    P = bf.total_points
    ref, rst, cpu = ragged_cpu_leg(bf)
    out = {"workload": f"ragged_batch: {bf.batch} fits, lengths log-uniform in [16, 65536], degree 1..3, "
                       f"{P} float32 points", "points": P, "cpu_baseline": cpu}
    for prec in (("f64", "f32c") if full else ("f64",)):
        coef = torch.zeros(bf.batch, 4, dtype=torch.float64, device=dev)
        status = torch.zeros(bf.batch, dtype=torch.int32, device=dev)
        plan = lf.Plan(bf.batch, 3, precision=prec)
        if not args.no_tune:
            plan.tune(x, y, off, dg, precision=prec, reps=3)
        step = lambda: lf.fit_batched(x, y, off, dg, 3, precision=prec, plan=plan, out=(coef, status))
        graph, graph_ms, ms, plain, kern = _both_forms(plan, step, args)
        tuned_ms = graph_ms if graph else plain
        passes = 2 if prec == "f32c" else 1
        km = kern["moments"]["avg_ms"]
        out[prec] = {"ms_per_step": _r(tuned_ms), "replay_form": "graph" if graph else "eager",
                     "graph_ms_per_step": _r(graph_ms), "eager_ms_per_step": _r(ms),
                     "eager_plain_ms_per_step": _r(plain),
                     "points_per_s": _r(P / (tuned_ms * 1e-3)), "tuned_schedule": plan.schedule,
                     "step_gbps": round(8.0 * P * passes / (tuned_ms * 1e-3) / 1e9, 1),
                     "kernel": "k_moments", "kernel_ms": _r(km), "kernel_gbps": round(8.0 * P / (km * 1e-3) / 1e9, 1),
                     "kernels": kern, "all_ok": bool((status.cpu().numpy() == 0).all()),
                     "max_rel_coef_err": _batched_err(bf, coef.cpu().numpy(), ref)}
        plan.close()
        log(f"ragged {prec}: {out[prec]}")
    if full:
        coef = torch.zeros(bf.batch, 4, dtype=torch.float64, device=dev)
        status = torch.zeros(bf.batch, dtype=torch.int32, device=dev)
        sse = torch.zeros(bf.batch, dtype=torch.float64, device=dev)
        wsq = torch.zeros(api.workspace_bytes(bf.batch, 3), dtype=torch.uint8, device=dev)
        qr_fn = lambda: lf.fit_qr_batched(x, y, off, dg, 3, ws=wsq, out=(coef, status, sse))
        ms, plain, kern = timed_form(qr_fn, args.steps, args.warmup)
        out["qr"] = {"ms_per_step": _r(ms), "points_per_s": _r(P / (ms * 1e-3)), "kernels": kern,
                     "all_ok": bool((status.cpu().numpy() == 0).all()),
                     "max_rel_coef_err": _batched_err(bf, coef.cpu().numpy(), ref),
                     "kernel_gbps": round(8.0 * P / (kern["moments"]["avg_ms"] * 1e-3) / 1e9, 1)}
        log(f"ragged qr: {out['qr']}")
        cplan = lf.Plan(bf.batch, 3)
        if not args.no_tune:
            cplan.tune(x, y, off, dg, reps=3, basis="chebyshev")
        cfn = lambda: lf.fit_batched(x, y, off, dg, 3, plan=cplan, out=(coef, status), basis="chebyshev")
        graph, cgraph_ms, ms, plain, kern = _both_forms(cplan, cfn, args)
        tuned_ms = cgraph_ms if graph else plain
        out["chebyshev"] = {"ms_per_step": _r(tuned_ms), "replay_form": "graph" if graph else "eager",
                            "graph_ms_per_step": _r(cgraph_ms), "eager_ms_per_step": _r(ms),
                            "points_per_s": _r(P / (tuned_ms * 1e-3)), "tuned_schedule": cplan.schedule,
                            "kernels": kern, "all_ok": bool((status.cpu().numpy() == 0).all()),
                            "kernel_gbps": round(8.0 * P / (kern["moments"]["avg_ms"] * 1e-3) / 1e9, 1)}
        cplan.close()
        log(f"ragged chebyshev: {out['chebyshev']}")
    nfit = min(args.per_fit_limit, bf.batch)
    if nfit > 0:
        L = _lib.load()
        run, pts, keep = _per_fit_single_calls(L, x, y, bf, nfit, dev)
        out["per_fit_launches"] = _per_fit_record(run, pts, nfit, ("moments", "combine"))
        cb, sb = keep[0].cpu().numpy(), keep[1].cpu().numpy()
        out["per_fit_launches"]["all_ok"] = bool((sb == 0).all())
        pf = out["per_fit_launches"]
        out["speedup_vs_per_fit"] = _r(out["f64"]["points_per_s"] / pf["points_per_s"])
        out["speedup_vs_per_fit_kernels"] = _r(out["f64"]["points_per_s"] / pf["kernel_points_per_s"])
        del cb
    return out


def bench_grad(args, full=False):
    """4,096 fits x 4,096 float32 points, m = 2, loss sum ||a - a_target||^2:
    batched forward + hand-written adjoint (one tuned plan drives both) against
    per-fit forward + backward calls on the same GPU; gradients checked
    against the float64 adjoint oracle on 64 sampled fits."""
    import numpy as np
    import torch
    import paper_1512_08017_amd as lf
    from paper_1512_08017_amd import _lib, api, workloads as W
    dev = _dev()
    bf = W.grad_batch()
    x, y = torch.from_numpy(bf.x).to(dev), torch.from_numpy(bf.y).to(dev)
    off, dg = torch.from_numpy(bf.offsets).to(dev), torch.from_numpy(bf.degrees).to(dev)
    target = torch.from_numpy(bf.target).to(dev)
    P, B = bf.total_points, bf.batch
    coef = torch.zeros(B, 3, dtype=torch.float64, device=dev)
    status = torch.zeros(B, dtype=torch.int32, device=dev)
    gx, gy = torch.empty_like(x), torch.empty_like(y)
    plan = lf.Plan(B, 2)
    if not args.no_tune:
        plan.tune(x, y, off, dg, reps=3)
    L = _lib.load()
    o = api.options(2)
    vp = ctypes.c_void_p
    stream = vp(torch.cuda.current_stream(dev).cuda_stream)
    g = torch.empty(B, 3, dtype=torch.float64, device=dev)
    neg2t = -2.0 * target

    def fwd_bwd():
        lf.fit_batched(x, y, off, dg, 2, plan=plan, out=(coef, status))
        torch.add(neg2t, coef, alpha=2.0, out=g)   # dL/da = 2 (a - target), one kernel
        _lib.check(L.fit_backward(vp(x.data_ptr()), vp(y.data_ptr()), vp(off.data_ptr()), vp(dg.data_ptr()), B,
                                  _lib.F32, ctypes.byref(o), plan.handle, None, 0, vp(g.data_ptr()), 3,
                                  vp(gx.data_ptr()), vp(gy.data_ptr()), stream), "fit_backward")

    graph, graph_ms, ms, plain, kern = _both_forms(plan, fwd_bwd, args)
    tuned_ms = graph_ms if graph else plain
    torch.cuda.synchronize()
    rng = np.random.default_rng(4064)
    sample = np.sort(rng.choice(B, 64, replace=False))
    gbar = g.cpu().numpy()
    ores, cpu = grad_cpu_leg(bf, gbar, sample)
    gxn, gyn = gx.cpu().numpy(), gy.cpu().numpy()
    edx = max(_normwise(gxn[f * 4096:(f + 1) * 4096], ores[f]["dx"]) for f in sample)
    edy = max(_normwise(gyn[f * 4096:(f + 1) * 4096], ores[f]["dy"]) for f in sample)
    eco = max(_normwise(coef[f].cpu().numpy(), ores[f]["a"]) for f in sample)
    fwd_bytes, bwd_bytes = 8.0 * P, 16.0 * P
    out = {"workload": f"grad_batch: {B} fits x 4096 float32 points, m=2, loss sum ||a - a_target||^2, "
                       "forward + adjoint", "points": P,
           "ms_per_step": _r(tuned_ms), "replay_form": "graph" if graph else "eager",
           "graph_ms_per_step": _r(graph_ms), "eager_ms_per_step": _r(ms), "eager_plain_ms_per_step": _r(plain),
           "points_per_s": _r(P / (tuned_ms * 1e-3)), "tuned_schedule": plan.schedule,
           "step_gbps": round((fwd_bytes + bwd_bytes) / (tuned_ms * 1e-3) / 1e9, 1), "kernels": kern,
           "moments_gbps": round(fwd_bytes / (kern["moments"]["avg_ms"] * 1e-3) / 1e9, 1),
           "adjoint_gbps": round(bwd_bytes / (kern["adjoint"]["avg_ms"] * 1e-3) / 1e9, 1),
           "all_ok": bool((status.cpu().numpy() == 0).all()),
           "sampled_fits": 64, "max_rel_err_dx": edx, "max_rel_err_dy": edy, "max_rel_coef_err": eco,
           "cpu_baseline": cpu}
    if full:
        out["per_call"] = _cold_warm(fwd_bwd, 20)
    nfit = min(args.per_fit_limit, B)
    if nfit > 0:
        # per fit: fit_batched and fit_backward on a one-fit batch, raw C-ABI calls on
        # preallocated buffers, with the same upstream gradient as the batched step
        off1 = torch.tensor([0, 4096], dtype=torch.int64, device=dev)
        dg1 = torch.tensor([2], dtype=torch.int32, device=dev)
        ws1 = torch.zeros(api.workspace_bytes(1, 2), dtype=torch.uint8, device=dev)
        c1 = torch.zeros(nfit, 3, dtype=torch.float64, device=dev)
        s1 = torch.zeros(nfit, dtype=torch.int32, device=dev)
        g1 = g.clone()
        calls = []
        for f in range(nfit):
            xp, yp = vp(x.data_ptr() + 4 * 4096 * f), vp(y.data_ptr() + 4 * 4096 * f)
            calls.append(((xp, yp, vp(off1.data_ptr()), vp(dg1.data_ptr()), 1, _lib.F32, ctypes.byref(o), None,
                           vp(ws1.data_ptr()), ws1.numel(), vp(c1.data_ptr() + 24 * f), 3, vp(s1.data_ptr() + 4 * f),
                           stream),
                          (xp, yp, vp(off1.data_ptr()), vp(dg1.data_ptr()), 1, _lib.F32, ctypes.byref(o), None,
                           vp(ws1.data_ptr()), ws1.numel(), vp(g1.data_ptr() + 24 * f), 3,
                           vp(gx.data_ptr() + 4 * 4096 * f), vp(gy.data_ptr() + 4 * 4096 * f), stream)))
        fb, bw = L.fit_batched, L.fit_backward

        def run():
            for a, b in calls:
                rc = fb(*a) or bw(*b)
                if rc:
                    _lib.check(rc, "per-fit forward/backward")

        pf = _per_fit_record(run, nfit * 4096, nfit, ("moments", "combine", "adjoint"))
        pf["all_ok"] = bool((s1.cpu().numpy() == 0).all())
        out["per_fit"] = pf
        out["speedup_vs_per_fit"] = _r(out["points_per_s"] / pf["points_per_s"])
        out["speedup_vs_per_fit_kernels"] = _r(out["points_per_s"] / pf["kernel_points_per_s"])
    if full:
        cstate = {}

        def fwd_bwd_cheb():
            c, _, ws = lf.fit_batched(x, y, off, dg, 2, ws=cstate.get("ws"), center=0.0, scale=1.0,
                                      basis="chebyshev")
            cstate["ws"] = ws
            lf.fit_backward(x, y, off, dg, 2, 2.0 * (c - target), ws=ws, center=0.0, scale=1.0, basis="chebyshev")

        cms, cplain, ckern = timed_form(fwd_bwd_cheb, args.steps, args.warmup)
        out["chebyshev"] = {"ms_per_step": _r(cms), "points_per_s": _r(P / (cms * 1e-3)), "kernels": ckern,
                            "adjoint_gbps": round(bwd_bytes / (ckern["adjoint"]["avg_ms"] * 1e-3) / 1e9, 1)}
    plan.close()
    return out


def cheb_cpu_baseline(x_np, y_np, m, given):
    """One Chebyshev-basis oracle fit on [-1, 1] (given) or on the exact extent
    of x (automatic): (oracle result, seconds, threads it used)."""
    from oracle import c_oracle, cheb
    c0, s0 = (0.0, 1.0) if given else cheb.cheb_range(x_np)
    t0 = time.perf_counter()
    ref = c_oracle.cheb_fit(x_np, y_np, m, c0, s0)
    return ref, time.perf_counter() - t0, c_oracle.max_threads()


def cheb_flops_per_point(m: int) -> int:
    """float64 flops of one point of the Chebyshev streaming pass (fma = 2):
    t (fma), 2t (add), T_2..T_m by T_(k+1) = 2t T_k - T_(k-1) (m-1 fma), the
    sums C_1..C_m and D_0 (m+1 adds), D_1..D_m and E_1..E_m = sum T_m T_j
    (2m fma)."""
    fma = 1 + (m - 1) + 2 * m
    add = 1 + m + 1
    return 2 * fma + add


def bench_runge(args):
    """Chebyshev basis, the higher degrees Sec. V leaves open: one fit of
    n = 1e8 float32 points of the Runge function on [-1, 1], m = 12, with the
    range given (one streaming pass) and automatic (an extra pass over x for
    the exact extent).  Reports points/s, the moment kernel against both the
    HBM and the float64 vector roofline, and the error against the C oracle."""
    import numpy as np
    import torch
    from paper_1512_08017_amd import workloads as W
    wl = W.runge()
    m, n = wl.degree, wl.n
    x, y = torch.from_numpy(wl.x).to(_dev()), torch.from_numpy(wl.y).to(_dev())
    out = {"workload": f"runge: one degree-{m} Chebyshev-basis fit of n={n} float32 points, x~U[-1,1], "
                       "y=1/(1+25x^2)+N(0,1e-3^2)", "n": n, "degree": m,
           "flops_per_point": cheb_flops_per_point(m), "bytes_per_point": 8}
    for mode, kw in (("given", {"center": 0.0, "scale": 1.0}), ("auto", {})):
        r = SingleFitRunner(x, y, m, "f64", basis="chebyshev", **kw)
        ms, plain, kern = timed_form(r.step, args.steps, args.warmup)
        c_gpu = r.coef[: m + 1].cpu().numpy()
        ref, cpu_s, cpu_threads = cheb_cpu_baseline(wl.x, wl.y, m, given=(mode == "given"))
        mk = kern["moments"]["avg_ms"] * 1e-3
        gbps = 8.0 * n / mk / 1e9
        tflops = cheb_flops_per_point(m) * n / mk / 1e12
        out[mode] = {"ms_per_step": ms, "plain_ms_per_step": plain, "points_per_s": n / (ms * 1e-3), "kernels": kern,
                     "moments_gbps": gbps, "moments_hbm_frac": gbps / HBM_PEAK_GBPS,
                     "moments_fp64_tflops": tflops, "moments_fp64_frac": tflops / FP64_VECTOR_PEAK_TFLOPS,
                     "status": int(r.status.cpu()[0]),
                     "max_rel_coef_err": float(np.max(np.abs(c_gpu - ref["c"])) / np.max(np.abs(ref["c"]))),
                     "cpu_oracle_points_per_s": n / cpu_s, "cpu_oracle_threads": cpu_threads}
        log(f"runge {mode}: {json.dumps(out[mode])}")
    return out


def probe_sweep(args):
    """Read and copy bandwidth probes over the benchmark's 800 MB of x and y
    (and, for the copy, 800 MB written), per schedule, load pattern and load
    kind: the attainable ceilings of the power-sum pass (read) and of the
    adjoint pass (read + write).  Each launch is timed by its own kernel clock."""
    import torch
    import paper_1512_08017_amd as lf
    from paper_1512_08017_amd import _lib
    L = _lib.load()
    dev = _dev()
    n = args.n
    x = torch.rand(n, device=dev)
    y = torch.rand(n, device=dev)
    ox, oy = torch.empty_like(x), torch.empty_like(y)
    out = torch.zeros(1 << 16, dtype=torch.float32, device=dev)
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    cus = lf.device_cus()
    vp = ctypes.c_void_p
    rows = []
    for probe in ("read", "copy"):
        for wpc in (4, 8, 16):
            for wpb in (2, 4):
                for unroll in (1, 2, 4):
                    sch = _lib.Schedule(cus * wpc, wpb, 256, unroll)
                    for pattern in (0, 1, 2):
                        for nt in (0, 1):
                            if probe == "read":
                                a_ = (vp(x.data_ptr()), vp(y.data_ptr()), n, ctypes.byref(sch), pattern, nt,
                                      vp(out.data_ptr()), out.numel(), st)
                                fn = lambda: _lib.check(L.lsefit_read_probe(*a_), "lsefit_read_probe")
                            else:
                                a_ = (vp(x.data_ptr()), vp(y.data_ptr()), vp(ox.data_ptr()), vp(oy.data_ptr()), n,
                                      ctypes.byref(sch), pattern, nt, st)
                                fn = lambda: _lib.check(L.lsefit_copy_probe(*a_), "lsefit_copy_probe")
                            _time(fn, 3, 2)
                            _, kern = armed_region(fn, args.steps)
                            ms = kern["probe"]["avg_ms"]
                            nbytes = (8.0 if probe == "read" else 16.0) * n
                            rows.append({"probe": probe, "waves_per_cu": wpc, "wpb": wpb, "unroll": unroll,
                                         "pattern": pattern, "nt": nt, "ms": ms,
                                         "gbps": nbytes / (ms * 1e-3) / 1e9})
                            log(json.dumps(rows[-1]))
    best = {p: max((r for r in rows if r["probe"] == p), key=lambda r: r["gbps"]) for p in ("read", "copy")}
    return {"probe": "read and copy ceilings, two float32 arrays of n elements", "n": n, "best": best, "rows": rows}


# ---------------------------------------------------------------------------
# the benchmark line
# ---------------------------------------------------------------------------
def bench_cubic(args):
    import numpy as np
    import torch
    from paper_1512_08017_amd import workloads as W
    dev = _dev()
    log(f"generating cubic_f32 workload n={args.n:,}")
    t0 = time.perf_counter()
    wl = W.cubic_f32(n=args.n)
    log(f"generated in {time.perf_counter() - t0:.1f}s; copying to {torch.cuda.get_device_name(dev)}")
    x = torch.from_numpy(wl.x).to(dev)
    y = torch.from_numpy(wl.y).to(dev)
    torch.cuda.synchronize()

    if args.pmc_probe:
        for prec in ("f64", "f32c"):
            r = SingleFitRunner(x, y, args.degree, prec)
            for _ in range(3):
                r.step()
        buf = torch.empty_like(x)
        buf.copy_(x)
        torch.cuda.synchronize()
        log("pmc probe done")
        return None

    forms = {}
    resid = None
    for prec, route in (("f64", "moments"), ("f32c", "moments"), ("qr", "qr")):
        r = SingleFitRunner(x, y, args.degree, "f64" if prec == "qr" else prec, route=route)
        ms, plain, kern = timed_form(r.step, args.steps, args.warmup)
        if prec == "f64":
            resid = residual_pass(r, args.n, min(args.steps, 50), 3)
            log(f"residual pass: {resid}")
        forms[prec] = {"ms_per_step": ms, "plain_ms_per_step": plain, "points_per_s": args.n / (ms * 1e-3),
                       "step_gbps": (8.0 * args.n * (2 if prec == "f32c" else 1)) / (ms * 1e-3) / 1e9,
                       "kernels": kern, "status": int(r.status.cpu()[0]),
                       "coef": r.coef[: args.degree + 1].cpu().numpy()}
        log(f"{prec}: {ms:.4f} ms/step (plain {plain:.4f}), {forms[prec]['points_per_s']:.3e} points/s, "
            f"kernels {kern}")

    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
    cpu, ref = cpu_baseline(wl.x, wl.y, args.degree, args.cpu_seconds, timed=not args.no_cpu_baseline)
    if cpu is not None:
        log(f"cpu oracle {cpu['value']:.3e} points/s on {cpu['cores']} threads")
    for prec, f in forms.items():
        a = f.pop("coef")
        f["max_rel_coef_err"] = float(np.max(np.abs(a - ref["a"])) / np.max(np.abs(ref["a"])))

    ok = {p: f for p, f in forms.items() if f["status"] == 0 and f["max_rel_coef_err"] <= 1e-6 and p != "qr"}
    if args.form == "auto":
        head = max(ok, key=lambda p: ok[p]["points_per_s"]) if ok else "f64"
    else:
        head = args.form
    hf = forms[head]
    mk = hf["kernels"].get("moments")
    bytes_per_launch = 8.0 * args.n
    roof = None
    if mk:
        kms = mk["avg_ms"]
        achieved = bytes_per_launch / (kms * 1e-3) / 1e9
        traffic = traffic_bytes("moments")
        ceiling = measured_ceiling_gbps("read")
        prof = profile_timed_avg_ms()
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": None if traffic is None else round(traffic / 1e9, 4), "traffic_unit": "GB per launch",
                "kernel": HEADLINE_KERNEL if head == "f64" else "k_moments", "avg_launch_ms": round(kms, 5),
                "launches": mk["launches"],
                "timing": "kernel clock of each launch in the timed region (first block start to last wave end)",
                "algorithmic_bytes_per_launch": int(bytes_per_launch),
                "rocprof_timed_region_avg_ms": None if prof is None else round(prof, 5),
                "measured_read_ceiling": ceiling,
                "frac_of_measured_ceiling": None if ceiling is None else round(achieved / ceiling, 4)}
        if kms > hf["ms_per_step"]:
            roof = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": None,
                    "traffic": None,
                    "reason": f"kernel time {kms:.5f} ms exceeds the step {hf['ms_per_step']:.5f} ms it is part of"}
    line = {
        "metric": METRIC,
        "value": round(hf["points_per_s"], 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(hf["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "f64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"cubic_f32: one degree-{args.degree} fit of n={args.n} float32 points, "
                               "x~U[-1,1], a~N(0,1), noise N(0,0.01^2)",
                   "n": args.n, "degree": args.degree, "form": head,
                   "hbm_gbps_step": round(hf["step_gbps"], 1),
                   "hbm_frac_step": round(hf["step_gbps"] / HBM_PEAK_GBPS, 4)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": {p: {k: (_r(v) if isinstance(v, float) else v) for k, v in f.items()} for p, f in forms.items()},
        "residual_pass": resid,
    }
    return line


def main():
    args = parse()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, out_path=args.out)
        return 0
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace, out_path=args.out, timed=args.timed)
        return 0
    if args.summarize_probe:
        summarize_probe(*args.summarize_probe, out_path=args.out)
        return 0
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, out_path=args.out)
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}): "
              "it measures one GPU's share; sharding across GPUs is not implemented", file=sys.stderr)
        return 2

    import torch  # noqa: F401
    import paper_1512_08017_amd as lf

    if args.schedule:
        lf.set_default_schedule(json.loads(args.schedule))
    if args.read_probe:
        print(json.dumps(probe_sweep(args)), flush=True)
        return 0
    if args.workload != "cubic_f32":
        fn = {"ragged_batch": bench_ragged, "grad_batch": bench_grad, "shifted_quintic": bench_quintic,
              "linear_f64": lambda a, full=True: bench_linear(a), "runge": lambda a, full=True: bench_runge(a)}
        print(json.dumps(fn[args.workload](args, full=not args.lean)), flush=True)
        return 0
    line = bench_cubic(args)
    if line is None:
        return 0
    if not args.no_extra_configs:
        configs = {}
        for name, fn in (("linear_f64", bench_linear), ("shifted_quintic", bench_quintic),
                         ("grad_batch", bench_grad), ("ragged_batch", bench_ragged)):
            log(f"config {name}")
            configs[name] = fn(args)
            log(f"config {name}: {json.dumps(configs[name])}")
        line["configs"] = configs
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
