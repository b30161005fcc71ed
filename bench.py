#!/usr/bin/env python3
"""Benchmark of the moment-pass least-squares fit on one MI355X.

One step = the whole single-fit hot path on one batch of synthetic input
resident in HBM: sampled range -> power-sum pass -> fixed-order combine ->
Hankel assembly and Gaussian elimination with partial pivoting -> (refinement
pass and correction for the compensated-float32 form) -> change back to the
x-basis, all through the C ABI on torch's current stream.

Workload (default): one cubic fit of n = 1e8 float32 points, x ~ U[-1, 1],
coefficients N(0, 1), noise N(0, 0.01^2).  Both accumulation forms are timed
(float64 accumulation; compensated float32 with one float64 refinement pass);
``value`` is the points/s of the form named by --form (default: the faster of
the two that meets the 1e-6 coefficient bound).

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
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
METRIC = "points/s & HBM GB/s (% peak) for moment pass+solve at ≤1e-6 rel coef err"
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ("paper_1512_08017_amd/csrc/kernels_impl.hpp", "paper_1512_08017_amd/csrc/device.hpp",
                  "paper_1512_08017_amd/csrc/dispatch.hip", "paper_1512_08017_amd/csrc/api.hip")


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
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--degree", type=int, default=3)
    ap.add_argument("--form", choices=("auto", "f64", "f32c"), default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target CPU time of the oracle baseline")
    ap.add_argument("--schedule", type=str, default=None, help="JSON schedule for the streaming kernels")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="a few steps of each form plus one plain device copy of known size (for --pmc runs)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc output folders into the traffic summary in profiles/")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# traffic summary from rocprofv3 --pmc runs
# ---------------------------------------------------------------------------
TRAFFIC_FILE = os.path.join(PROFILES, "moments_cubic_f32_traffic.txt")
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


def summarize_pmc(fetch_dir, write_dir):
    out = {}
    for counter, folder in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _read_counter_csv(folder, counter)
        mom = [v for k, v in rows if "k_moments" in k]
        ref = [v for k, v in rows if "k_refine" in k]
        cpy = [v for k, v in rows if ("copy" in k.lower() or "elementwise" in k.lower()) and "lsefit" not in k]
        out[counter] = {"moments_kib": sorted(mom), "refine_kib": sorted(ref), "copy_kib": sorted(cpy)}
    lines = ["# HBM traffic of the power-sum kernel (k_moments) and the refinement kernel (k_refine)",
             "# workload: cubic fit, n = 1e8 float32 points (800,000,000 algorithmic bytes per pass)",
             "# commands (two runs, one counter each):",
             "#   rocprofv3 --pmc FETCH_SIZE -d gpurun_out/pmc_fetch -o run --output-format csv -- "
             "python3 bench.py --pmc-probe",
             "#   rocprofv3 --pmc WRITE_SIZE -d gpurun_out/pmc_write -o run --output-format csv -- "
             "python3 bench.py --pmc-probe",
             "#   python3 bench.py --summarize-pmc gpurun_out/pmc_fetch gpurun_out/pmc_write",
             f"# {COPY_BYTES_NOTE}",
             f"kernel_hash {kernel_hash()}"]
    for counter, d in out.items():
        for key, vals in d.items():
            lines.append(f"{counter}.{key} " + " ".join(f"{v:.1f}" for v in vals))
    os.makedirs(PROFILES, exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def traffic_bytes(kernel="moments"):
    """Scaled HBM bytes per launch from the stored --pmc summary, or None if stale/missing."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        vals[k] = v
    if vals.get("kernel_hash", [None])[0] != kernel_hash():
        return None
    try:
        fetch = sorted(float(v) for v in vals[f"FETCH_SIZE.{kernel}_kib"])
        write = sorted(float(v) for v in vals[f"WRITE_SIZE.{kernel}_kib"])
        cf = max(float(v) for v in vals["FETCH_SIZE.copy_kib"])
        cw = max(float(v) for v in vals["WRITE_SIZE.copy_kib"])
    except (KeyError, ValueError):
        return None
    # scale each counter by (known bytes of the plain copy) / (its reading of that copy)
    sf = 400_000_000 / (cf * 1024.0)
    sw = 400_000_000 / (cw * 1024.0)
    med = lambda a: a[len(a) // 2]
    return med(fetch) * 1024.0 * sf + med(write) * 1024.0 * sw


# ---------------------------------------------------------------------------
# GPU timing
# ---------------------------------------------------------------------------
class SingleFitRunner:
    """Pre-allocated buffers and one C-ABI step (fit_single: the fused single-fit call)."""

    def __init__(self, x, y, degree, precision):
        import torch
        from paper_1512_08017_amd import _lib, api
        self.L = _lib.load()
        self.x, self.y, self.m, self.precision = x, y, degree, precision
        self.opt = api.options(degree, precision, 1)
        nbytes = api.workspace_bytes(1, degree)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
        self.mom = torch.empty(3 * degree + 4, dtype=torch.float64, device=x.device)
        self.coef = torch.empty(2 * (degree + 1), dtype=torch.float64, device=x.device)
        self.status = torch.empty(1, dtype=torch.int32, device=x.device)
        vp = ctypes.c_void_p
        dt = _lib.F32 if x.dtype == torch.float32 else _lib.F64
        self.args = (vp(x.data_ptr()), vp(y.data_ptr()), x.numel(), dt, ctypes.byref(self.opt),
                     vp(self.ws.data_ptr()), self.ws.numel(), vp(self.coef.data_ptr()), vp(self.status.data_ptr()),
                     None, ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream))
        self._check = _lib.check

    def step(self):
        self._check(self.L.fit_single(*self.args), "fit_single")


def _region(runner, steps):
    import torch
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        runner.step()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps, (time.perf_counter() - t0) / steps * 1e3


def time_steps(runner, steps, warmup):
    """Two timed regions of `steps` steps each: the first plain (ms/step), the
    second with the library's per-kernel HIP events on the launch stream (kernel
    durations; the events themselves add a little time to that region's steps)."""
    from paper_1512_08017_amd import _lib
    L = _lib.load()
    for _ in range(warmup):
        runner.step()
    ms, wall_ms = _region(runner, steps)
    L.lsefit_timing_reset()
    L.lsefit_timing_enable(1)
    ms_inst, _ = _region(runner, steps)
    L.lsefit_timing_enable(0)
    kern = {}
    for kind, name in ((0, "moments"), (1, "refine"), (3, "combine")):
        tot, cnt = ctypes.c_double(0.0), ctypes.c_int64(0)
        _lib.check(L.lsefit_timing_read(kind, ctypes.byref(tot), ctypes.byref(cnt)), "lsefit_timing_read")
        if cnt.value:
            kern[name] = {"avg_ms": tot.value / cnt.value, "launches": int(cnt.value)}
    return ms, wall_ms, ms_inst, kern


def cpu_baseline(x_np, y_np, degree, target_s):
    from oracle import c_oracle
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
    return {"value": x_np.shape[0] * reps / el, "unit": "points/s", "cores": int(used), "kind": "oracle",
            "sample": f"{reps} full pass(es) of the plain-C float64 oracle over the same {x_np.shape[0]:,} points "
                      f"(compensated sums + partial-pivoting elimination), {el:.1f} s on {used} host threads"}, res


def main():
    args = parse()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}): "
              "this build measures one GPU's share; sharding across GPUs is not built", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1512_08017_amd as lf
    from paper_1512_08017_amd import workloads as W

    dev = torch.device("cuda:0")
    if args.schedule:
        lf.set_default_schedule(json.loads(args.schedule))
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
        return 0

    forms = {}
    for prec in ("f64", "f32c"):
        r = SingleFitRunner(x, y, args.degree, prec)
        ms, wall_ms, ms_inst, kern = time_steps(r, args.steps, args.warmup)
        st = int(r.status.cpu()[0])
        forms[prec] = {"ms_per_step": ms, "wall_ms_per_step": wall_ms, "instrumented_ms_per_step": ms_inst,
                       "points_per_s": args.n / (ms * 1e-3),
                       "step_gbps": (8.0 * args.n * (2 if prec == "f32c" else 1)) / (ms * 1e-3) / 1e9,
                       "kernels": kern, "status": st, "coef": r.coef[: args.degree + 1].cpu().numpy()}
        log(f"{prec}: {ms:.4f} ms/step, {forms[prec]['points_per_s']:.3e} points/s, kernels {kern}")

    cpu = None
    ref = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu, ref = cpu_baseline(wl.x, wl.y, args.degree, args.cpu_seconds)
        log(f"cpu oracle {cpu['value']:.3e} points/s on {cpu['cores']} threads")
    else:
        from oracle import c_oracle
        ref = c_oracle.fit(wl.x, wl.y, args.degree)
    for prec, f in forms.items():
        a = f.pop("coef")
        f["max_rel_coef_err"] = float(np.max(np.abs(a - ref["a"])) / np.max(np.abs(ref["a"])))

    ok = {p: f for p, f in forms.items() if f["status"] == 0 and f["max_rel_coef_err"] <= 1e-6}
    if args.form == "auto":
        head = max(ok, key=lambda p: ok[p]["points_per_s"]) if ok else "f64"
    else:
        head = args.form
    hf = forms[head]
    mk = hf["kernels"].get("moments")
    bytes_per_launch = 8.0 * args.n
    roof = None
    if mk:
        achieved = bytes_per_launch / (mk["avg_ms"] * 1e-3) / 1e9
        traffic = traffic_bytes("moments")
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": None if traffic is None else round(traffic / 1e9, 4),
                "kernel": "k_moments", "avg_launch_ms": round(mk["avg_ms"], 5),
                "algorithmic_bytes_per_launch": int(bytes_per_launch)}
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
        "forms": {p: {k: (float(f"{v:.6g}") if isinstance(v, float) else v) for k, v in f.items()}
                  for p, f in forms.items()},
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
