"""Benchmark: SGP4 propagation of the 9,341-satellite x 1,000-time grid on one MI355X.

A step is one pass of the hot path over the batch: initialisation of the
per-satellite constants plus the dense propagation (the paper's jaxsgp4
timing includes initialisation too, section 3.1).  The headline `value` is
the FP32-mixed path's whole-job throughput in satellite-time points per
second; the FP64 and plain-FP32 paths are timed the same way and reported
under "paths".  Inputs are resident in device memory before timing starts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-c2] [--ragged] [--vjp]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks: HBM 8 TB/s; vector FP64 78.6 TFLOP/s (256 CUs x
# 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz) and vector FP32 157.3 TFLOP/s.  The
# FP32 and mixed kernels are priced against the FP32 figure: their measured
# issue rate (VALU instructions per wave x waves / SIMDs / duration) is above
# 16 lanes per clock, so the FP64 figure is no ceiling for them.
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "mixed": 157.3}
# Operations the model performs per point (oracle operation count, simplified
# drag off, 3 Kepler iterations): 76 add/sub + 120 mul + 14 div + 4 sqrt +
# 18 sin/cos + 1 atan2, each counted once.
ALG_FLOP_PER_POINT = 233
BYTES_PER_POINT = {"fp64": 49, "fp32": 25, "mixed": 25}
PAPER_POINTS_PER_S = 9341 * 1000 / 3.8e-3   # A100, FP32, init included (section 3.3): context only


def log(msg):
    print(msg, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dense_9341x1000_hbm_traffic.md")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "dense_9341x1000_instruction_mix.md")
KERNEL_SOURCES = ("sgp4mi_common.h", "sgp4mi_math.h", "sgp4mi_point.h", "sgp4mi_out.h", "sgp4mi_prop.hip")


def profile_values(path):
    """The 'name: value' lines of a committed rocprofv3 summary, or None when the
    dense kernel's sources changed after the counters were taken (the summary
    records the hash of the sources it was measured with)."""
    import hashlib
    try:
        text = open(path).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        parts = line.strip().split(":")
        if len(parts) == 2 and parts[0].strip().replace("_", "").isalnum():
            vals[parts[0].strip()] = parts[1].strip()
    blob = b"".join(open(os.path.join(ROOT, "paper_2603_27830_amd", "csrc", f), "rb").read() for f in KERNEL_SOURCES)
    if hashlib.sha256(blob).hexdigest()[:16] != vals.get("kernel_sources_sha256_16"):
        return None
    return vals


def measured_traffic(path_name):
    """HBM bytes per launch of the dense kernel from the FETCH_SIZE / WRITE_SIZE
    summary (copy-calibrated), or None when stale."""
    vals = profile_values(TRAFFIC_FILE)
    try:
        return float(vals[f"{path_name}_fetch_bytes"]) + float(vals[f"{path_name}_write_bytes"])
    except (KeyError, TypeError):
        return None


def valu_quads_per_wave(path_name):
    """(SQ_ACTIVE_INST_VALU, SQ_ACTIVE_INST_VALU2) per wavefront of the dense
    kernel: quad-cycles in which the wavefront's SIMD issued a VALU instruction
    of it, and those in which it issued two (dual issue), or None when stale."""
    vals = profile_values(COUNTERS_FILE)
    try:
        return float(vals[f"{path_name}_active_inst_valu_per_wave"]), float(vals[f"{path_name}_active_inst_valu2_per_wave"])
    except (KeyError, TypeError):
        return None


class ClockSampler:
    """The GPU's graphics clock under a load: a host thread reads the driver's
    current clock of every XCD (amdsmi GPU metrics) every 20 ms; the first
    `settle` seconds are not counted (the driver refreshes the metric about
    once a second, so early samples still show the clock before the load).
    Reports mean/min/max in MHz, or None where amdsmi is not available."""

    def __init__(self, settle=1.0):
        self.samples, self.stop, self.thread, self.handle = [], False, None, None
        self.settle = settle
        try:
            import amdsmi
            amdsmi.amdsmi_init()
            self.amdsmi = amdsmi
            self.handle = amdsmi.amdsmi_get_processor_handles()[0]
        except Exception:  # noqa: BLE001 - the clock is reported as unavailable
            self.amdsmi = None

    def _read(self):
        m = self.amdsmi.amdsmi_get_gpu_metrics_info(self.handle)
        clks = [c for c in m.get("current_gfxclks", []) if isinstance(c, (int, float)) and c > 0]
        return sum(clks) / len(clks) if clks else float(m["current_gfxclk"])

    def _run(self):
        t0 = time.perf_counter()
        while not self.stop:
            try:
                x = self._read()
            except Exception:  # noqa: BLE001
                return
            if time.perf_counter() - t0 >= self.settle:
                self.samples.append(x)
            time.sleep(0.02)

    def __enter__(self):
        if self.amdsmi is not None:
            import threading
            self.thread = threading.Thread(target=self._run, daemon=True)
            self.thread.start()
        return self

    def __exit__(self, *exc):
        self.stop = True
        if self.thread is not None:
            self.thread.join()

    def summary(self):
        if not self.samples:
            return None
        return {"mean_mhz": sum(self.samples) / len(self.samples), "min_mhz": min(self.samples),
                "max_mhz": max(self.samples), "samples": len(self.samples),
                "source": "amdsmi GPU metrics current_gfxclks (mean over XCDs), every 20 ms"}


def executed_flop_per_point(path_name):
    """FP32 + FP64 VALU flops the dense kernel executes per point (rocprofv3
    SQ_INSTS_VALU_FLOPS_FP32 / _FP64 per wavefront of 64 points, FMA counted
    twice), or None when stale."""
    vals = profile_values(COUNTERS_FILE)
    try:
        return float(vals[f"{path_name}_flops_fp32_per_point"]) + float(vals[f"{path_name}_flops_fp64_per_point"])
    except (KeyError, TypeError):
        return None


class LaunchTimer:
    """HIP events recorded on the launch stream around one kernel launch of every
    `every`-th timed step; mean() is that launch's average duration over the
    sampled steps of the timed region.  Sampling keeps the event packets from
    stretching every step (events around every launch add ~3 us per step)."""

    def __init__(self, torch, every=5):
        self.torch, self.on, self.pairs, self.every, self.count = torch, False, [], every, 0

    def __call__(self, launch):
        if not self.on:
            return launch()
        self.count += 1
        if (self.count - 1) % self.every:
            return launch()
        s = self.torch.cuda.current_stream()
        a, b = self.torch.cuda.Event(enable_timing=True), self.torch.cuda.Event(enable_timing=True)
        a.record(s)
        r = launch()
        b.record(s)
        self.pairs.append((a, b))
        return r

    def mean(self):
        return sum(a.elapsed_time(b) for a, b in self.pairs) / len(self.pairs) * 1e-3


def time_steps(fn, steps, warmup, torch, timer=None):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if timer is not None:
        timer.on = True
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    if timer is not None:
        timer.on = False
    return dt


def paper_protocol(fn, torch, min_total=0.2, trials=5):
    """Adaptive repeats until a trial exceeds min_total seconds; minimum of 5 trials (section 3.1)."""
    fn()
    torch.cuda.synchronize()
    reps = 1
    while True:
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if dt >= min_total:
            break
        reps *= 2
    best = dt / reps
    for _ in range(trials - 1):
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        best = min(best, (time.perf_counter() - t0) / reps)
    return best


def kernel_time(launch, torch, reps=20):
    """Average duration of one propagate launch, from HIP events on the launch stream."""
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    launch()
    e0.record(s)
    for _ in range(reps):
        launch()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cat, trials=5, big_trials=3):
    """The oracle (serial FP64 C++, untuned) on the host, built -O3 -march=native
    -ffp-contract=off for this machine: all cores on the full 9,341 x 1,000 grid
    (the headline figure), on the full 100,000 x 1,440 grid and on the full
    1,000,000-satellite ragged catalogue (in satellite chunks that reuse their
    output buffers), and one core on a 1% satellite sample of each, extrapolated
    linearly to the whole batch.  Paper protocol: repeat until >= 0.2 s, report
    the minimum and the median of the trials."""
    import statistics
    import tempfile
    import synth
    from oracle import build as oracle_build
    cores = max(1, min(os.cpu_count() or 1, 64))
    native = os.path.join(tempfile.mkdtemp(prefix="sgp4_oracle_"), "liboracle_native.so")
    build_flags = " ".join(oracle_build.flags(native=True))
    try:
        oracle_build.build(native=True, out=native)
        os.environ["SGP4_ORACLE_LIB"] = native
    except Exception as e:  # noqa: BLE001 - fall back to the portable build, and say so
        build_flags = " ".join(oracle_build.flags(native=False)) + f" (native build failed: {e})"
    import oracle

    def timed(fn, npts, n_trials, warm=True):
        if warm:
            fn()
        reps = 1
        while True:
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            dt = time.perf_counter() - t0
            if dt >= 0.2:
                break
            reps *= 2
        runs = [dt / reps]
        for _ in range(n_trials - 1):
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            runs.append((time.perf_counter() - t0) / reps)
        return {"min_s": min(runs), "median_s": statistics.median(runs), "value": npts / min(runs),
                "median_value": npts / statistics.median(runs), "trials": n_trials}

    out = {"unit": "sat-time points/s", "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
           "build": f"g++ {build_flags}"}
    c1 = timed(lambda: oracle.propagate(cat.elem, cat.t, nthreads=cores), cat.n * cat.T, trials)
    k = max(1, cat.n // 100)
    sub = np.ascontiguousarray(cat.elem[:, :k])
    c1_one = timed(lambda: oracle.propagate(sub, cat.t, nthreads=1), k * cat.T, trials)
    out.update(value=c1["value"], median=c1["median_value"],
               sample=f"full {cat.n} x {cat.T} grid on {cores} threads (init included); min (and median) of "
                      f"{trials} trials of >= 0.2 s",
               single_core_value=c1_one["value"],
               single_core_sample=f"first {k} satellites x {cat.T} times on 1 thread (1% sample)")
    log(f"[bench] cpu oracle c1: {c1['value']:.3e} pts/s on {cores} threads, {c1_one['value']:.3e} on one")

    # 100,000 x 1,440 in chunks of 10,000 satellites
    c2 = synth.config2("1d")
    chunks = [np.ascontiguousarray(c2.elem[:, i:i + 10000]) for i in range(0, c2.n, 10000)]
    r2 = timed(lambda: [oracle.propagate(ch, c2.t, nthreads=cores) for ch in chunks], c2.n * c2.T, big_trials,
               warm=False)
    k2 = c2.n // 100
    s2 = np.ascontiguousarray(c2.elem[:, :k2])
    r2_one = timed(lambda: oracle.propagate(s2, c2.t, nthreads=1), k2 * c2.T, big_trials)
    out["c2_100k_x_1440"] = {"all_cores": r2, "single_core_1pct": r2_one,
                             "single_core_extrapolated_s": c2.n * c2.T / r2_one["value"],
                             "note": "single-core time extrapolated linearly from the first 1% of satellites"}
    log(f"[bench] cpu oracle c2: {r2['value']:.3e} pts/s on {cores} threads, {r2_one['value']:.3e} on one")
    del chunks

    # 1M-satellite ragged catalogue in chunks of 100,000 satellites
    c3 = synth.config3()
    pieces = []
    for i in range(0, c3.n, 100000):
        j = min(c3.n, i + 100000)
        lo, hi = int(c3.offsets[i]), int(c3.offsets[j])
        pieces.append((np.ascontiguousarray(c3.elem[:, i:j]), c3.offsets[i:j + 1] - lo, c3.t[lo:hi]))
    r3 = timed(lambda: [oracle.propagate_ragged(e, o, t, nthreads=cores) for e, o, t in pieces], c3.nnz, big_trials,
               warm=False)
    k3 = c3.n // 100
    e3s, o3s = np.ascontiguousarray(c3.elem[:, :k3]), c3.offsets[:k3 + 1]
    t3s = c3.t[:int(o3s[-1])]
    r3_one = timed(lambda: oracle.propagate_ragged(e3s, o3s, t3s, nthreads=1), int(o3s[-1]), big_trials)
    out["c3_ragged_1M"] = {"all_cores": r3, "single_core_1pct": r3_one,
                           "single_core_extrapolated_s": c3.nnz / r3_one["value"],
                           "note": "single-core time extrapolated linearly from the first 1% of satellites"}
    log(f"[bench] cpu oracle c3: {r3['value']:.3e} pts/s on {cores} threads, {r3_one['value']:.3e} on one")
    return out


def calibrate(torch):
    """Achievable rates on this GPU: unpacked FP64 and FP32 FMA (8 independent
    chains per lane; FP32 with all operands in vector registers and with one in a
    scalar register) and a non-temporal store stream."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2603_27830_amd", "libsgp4mi_calib.so"))
    lib.sgp4mi_calib_fma.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    lib.sgp4mi_calib_store.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    stream = torch.cuda.current_stream().cuda_stream
    blocks, iters = 256 * 64, 4096
    res = {}
    names = {0: "fma_f64_tflops", 1: "fma_f32_vgpr_tflops", 2: "fma_f32_sgpr_operand_tflops"}
    for prec, dt in ((0, torch.float64), (1, torch.float32), (2, torch.float32)):
        out = torch.empty(blocks * 256, dtype=dt, device="cuda")
        launch = lambda: lib.sgp4mi_calib_fma(prec, ctypes.c_void_p(out.data_ptr()), blocks, iters, stream)
        sec = kernel_time(launch, torch, reps=5)
        res[names[prec]] = blocks * 256 * iters * 8 * 2 / sec / 1e12
    lib.sgp4mi_calib_rate.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    kinds = ["v_fma_f32 (vector operands)", "v_fma_f32 (one scalar operand)", "v_mul_f32", "v_fma_f64", "v_sin_f32",
             "v_rcp_f32", "v_rcp_f64", "v_cvt_f32_f64"]
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    simds = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    res["clocks_per_wave_instruction_per_simd_at_2.4GHz"] = {}
    for kind, name in enumerate(kinds):
        launch = lambda: lib.sgp4mi_calib_rate(kind, ctypes.c_void_p(out.data_ptr()), blocks, 1024, stream)
        sec = kernel_time(launch, torch, reps=5)
        per_simd = blocks * 4 * 1024 * 8 / simds
        res["clocks_per_wave_instruction_per_simd_at_2.4GHz"][name] = round(sec * 2.4e9 / per_simd, 2)
    n = 1 << 30  # 8 GiB of doubles
    buf = torch.empty(n, dtype=torch.float64, device="cuda")
    launch = lambda: lib.sgp4mi_calib_store(ctypes.c_void_p(buf.data_ptr()), n, 256 * 64, stream)
    sec = kernel_time(launch, torch, reps=5)
    res["store_nt_gbs"] = n * 8 / sec / 1e9
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-c2", action="store_true", help="skip the 100k x 1440 comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-ragged", action="store_true", help="skip the 1M-satellite ragged catalogue")
    ap.add_argument("--no-vjp", action="store_true", help="skip the VJP on the 9341 x 1000 grid")
    ap.add_argument("--no-short", action="store_true",
                    help="skip the short-list (1M satellites x 1-32 times) elements-to-states comparison")
    ap.add_argument("--only", default=None, help="time one path only (fp64, fp32, mixed) for profiling")
    ap.add_argument("--ragged-only", default=None, metavar="PREC",
                    help="profiling mode: only the 1M-satellite ragged catalogue in one precision (fp64, mixed)")
    ap.add_argument("--ragged-config", default=None, metavar="MODE,BLOCK,PER_CU[;...]",
                    help="with --ragged-only: fixed plan configurations (';'-separated) instead of the autotuner's")
    ap.add_argument("--sweep", action="store_true",
                    help="time every dense launch configuration (workgroup size x constant residency) per precision")
    ap.add_argument("--calibrate", action="store_true",
                    help="run only the calibration microbenchmarks (FMA issue rates, non-temporal store bandwidth)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (3 launches), the reference for HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: one GPU only; --gpus {args.gpus} is not supported (propagation would shard by blocks of "
              "satellites with no exchange step, each GPU running this same single-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2603_27830_amd as sg
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate:
        print(json.dumps(calibrate(torch)), flush=True)
        return
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": src.numel() * 4, "launches": 3}))
        return
    cat = synth.config1()
    elem = torch.from_numpy(cat.elem).to(dev)
    t = torch.from_numpy(cat.t).to(dev)
    P = cat.n * cat.T
    if args.sweep:
        rec = sg.init(elem)
        table = {}
        for name in ("fp64", "fp32", "mixed"):
            dt = torch.float64 if name == "fp64" else torch.float32
            out = (torch.empty((3, cat.n, cat.T), dtype=dt, device=dev),
                   torch.empty((3, cat.n, cat.T), dtype=dt, device=dev),
                   torch.empty((cat.n, cat.T), dtype=torch.uint8, device=dev))
            cfgs = [(b, sc, 0) for b in (256, 512) for sc in (False, True)]
            cfgs += [(b, True, -1) for b in (64, 128, 256, 512)]
            cfgs += [(b, True, k) for b in (256, 512) for k in (4, 8)]
            for block, scalar, per_cu in cfgs:
                cfg = block | (0x10000 if scalar else 0)
                cfg |= 0x40000 if per_cu < 0 else ((0x20000 | (per_cu << 20)) if per_cu else 0)
                us = kernel_time(lambda: sg.propagate(rec, t, name, out=out, block=cfg), torch) * 1e6
                mapping = "tiles" if per_cu < 0 else ("persist" + str(per_cu) if per_cu else "grid")
                key = f"{name}/b{block}/{'scalar' if scalar else 'vector'}/{mapping}"
                table[key] = round(us, 2)
                log(f"[sweep] {key}: {us:.1f} us")
        print(json.dumps({"dense_sweep_us": table}), flush=True)
        return
    if args.ragged_only:
        c3 = synth.config3()
        rec3 = sg.init(torch.from_numpy(c3.elem).to(dev))
        off3 = torch.from_numpy(c3.offsets).to(dev)
        t3 = torch.from_numpy(c3.t).to(dev)
        cfgs = ([tuple(int(x) for x in c.split(",")) for c in args.ragged_config.split(";")]
                if args.ragged_config else [None])
        for cfg in cfgs:
            plan = sg.RaggedPlan(rec3, off3, t3, args.ragged_only, autotune=cfg is None, graph=False, config=cfg)
            k3 = kernel_time(plan.launch, torch, reps=3)
            log(f"[ragged] {args.ragged_only}: {c3.nnz / k3:.3e} pts/s, {k3 * 1e3:.3f} ms ({plan.describe()})")
            print(json.dumps({"ragged": args.ragged_only, "nnz": c3.nnz, "launch_ms": k3 * 1e3,
                              "plan": json.loads(plan.describe())}), flush=True)
            plan.close()
        return
    paths = {}
    names = [args.only] if args.only else ["fp64", "fp32", "mixed"]
    for name in names:
        rec = sg.init(elem)
        dt = torch.float64 if name == "fp64" else torch.float32
        out = (torch.empty((3, cat.n, cat.T), dtype=dt, device=dev), torch.empty((3, cat.n, cat.T), dtype=dt, device=dev),
               torch.empty((cat.n, cat.T), dtype=torch.uint8, device=dev))

        timer = LaunchTimer(torch)

        def step():
            r = sg.init(elem)
            timer(lambda: sg.propagate(r, t, name, out=out))

        def prop_only():
            sg.propagate(rec, t, name, out=out)

        s = time_steps(step, args.steps, args.warmup, torch, timer)
        k = timer.mean()
        # the clock under the same load: the step repeated for a second while
        # the driver's clock is sampled (the timed region is too short for it)
        with ClockSampler(settle=0.3 if args.only else 1.0) as clock:
            t_end = time.perf_counter() + (0.6 if args.only else 2.0)
            while time.perf_counter() < t_end:
                for _ in range(50):
                    step()
                torch.cuda.synchronize()
        # --only is the profiling mode: a handful of launches, no adaptive repeats
        kb = kernel_time(prop_only, torch, reps=2 if args.only else 20)
        pp = paper_protocol(step, torch) if not args.only else float("nan")
        paths[name] = {
            "points_per_s": P / s, "ms_per_step": s * 1e3, "propagate_kernel_us": k * 1e6,
            "propagate_back_to_back_us": kb * 1e6,
            "propagate_only_points_per_s": P / k, "paper_protocol_min_ms": pp * 1e3,
            "hbm_gbs": BYTES_PER_POINT[name] * P / k / 1e9,
            "alg_tflops": ALG_FLOP_PER_POINT * P / k / 1e12,
            "gpu_clock": clock.summary(),
        }
        log(f"[bench] {name}: {P / s:.3e} pts/s, step {s * 1e3:.3f} ms, kernel {k * 1e6:.1f} us")

    if not args.no_c2 and not args.only:
        c2 = synth.config2("1d")
        e2 = torch.from_numpy(c2.elem).to(dev)
        t2 = torch.from_numpy(c2.t).to(dev)
        P2 = c2.n * c2.T
        paths["c2_100k_x_1440"] = {}
        for name in ("fp64", "mixed"):
            rec2 = sg.init(e2)
            dt = torch.float64 if name == "fp64" else torch.float32
            out2 = (torch.empty((3, c2.n, c2.T), dtype=dt, device=dev),
                    torch.empty((3, c2.n, c2.T), dtype=dt, device=dev),
                    torch.empty((c2.n, c2.T), dtype=torch.uint8, device=dev))
            k2 = kernel_time(lambda: sg.propagate(rec2, t2, name, out=out2), torch, reps=5)
            paths["c2_100k_x_1440"][name] = {"propagate_only_points_per_s": P2 / k2, "kernel_ms": k2 * 1e3,
                                             "hbm_gbs": BYTES_PER_POINT[name] * P2 / k2 / 1e9}
            log(f"[bench] c2 {name}: {P2 / k2:.3e} pts/s, kernel {k2 * 1e3:.3f} ms")
            if name == "mixed":
                # Conjunction screening of the whole 100k x 1,440 output at 10 km
                # (device-memory buckets: beyond the on-chip size).
                import ctypes
                from paper_2603_27830_amd import _native
                L = _native.lib()
                wsb = int(L.sgp4_screen_workspace_bytes(c2.n, c2.T))
                ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
                cap = 1 << 22
                pairs = torch.empty((cap, 3), dtype=torch.int32, device=dev)
                dist = torch.empty(cap, dtype=torch.float64, device=dev)
                cnt = torch.empty(1, dtype=torch.int64, device=dev)
                vp = lambda x: ctypes.c_void_p(x.data_ptr())  # noqa: E731
                st = lambda: ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)  # noqa: E731
                ksc = kernel_time(lambda: _native.check(L.sgp4_screen(
                    vp(out2[0]), _native.SGP4_FP32_MIXED, vp(out2[2]), c2.n, c2.T, 10.0, cap, vp(pairs), vp(dist),
                    vp(cnt), vp(ws), wsb, st()), "sgp4_screen"), torch, reps=3)
                events = int(cnt.item())
                paths["c2_100k_x_1440"]["screen_10km"] = {"ms": ksc * 1e3, "events": events,
                                                         "satellite_times_per_s": P2 / ksc}
                log(f"[bench] screen 100k x 1440 (10 km): {ksc * 1e3:.3f} ms, {events} events")
                del ws, pairs, dist
            del out2, rec2
        # 7-day variant: 1,008 times at 10-minute steps
        t7 = torch.from_numpy(synth.config2("7d").t).to(dev)
        P7 = c2.n * int(t7.numel())
        paths["c2_100k_x_1008_7d"] = {}
        for name in ("fp64", "mixed"):
            rec2 = sg.init(e2)
            dt = torch.float64 if name == "fp64" else torch.float32
            out7 = (torch.empty((3, c2.n, P7 // c2.n), dtype=dt, device=dev),
                    torch.empty((3, c2.n, P7 // c2.n), dtype=dt, device=dev),
                    torch.empty((c2.n, P7 // c2.n), dtype=torch.uint8, device=dev))
            k7 = kernel_time(lambda: sg.propagate(rec2, t7, name, out=out7), torch, reps=5)
            paths["c2_100k_x_1008_7d"][name] = {"propagate_only_points_per_s": P7 / k7, "kernel_ms": k7 * 1e3}
            log(f"[bench] c2 7-day {name}: {P7 / k7:.3e} pts/s, kernel {k7 * 1e3:.3f} ms")
            del out7, rec2
        torch.cuda.empty_cache()

    if not args.no_vjp and not args.only:
        # Differentiation workload: g_r = 2 (r - r_obs), observations from the
        # perturbed truth elements propagated by the FP64 kernel plus 10 m noise
        # (the oracle is not used outside the CPU-baseline leg).
        c4, truth, noise = synth.config4()
        rec = sg.init(elem)
        r_obs, _, _ = sg.propagate(sg.init(torch.from_numpy(truth).to(dev)), t, "fp64")
        r_obs += torch.from_numpy(noise).to(dev)
        paths["vjp_9341x1000"] = {}
        for name in ("fp64", "mixed"):
            r, _, _ = sg.propagate(rec, t, name)
            gr = (2.0 * (r.double() - r_obs)).to(r.dtype).contiguous()
            kv = kernel_time(lambda: sg.vjp(rec, t, gr, None, name), torch, reps=5)
            paths["vjp_9341x1000"][name] = {"points_per_s": P / kv, "kernel_ms": kv * 1e3}
            log(f"[bench] vjp {name}: {P / kv:.3e} pts/s, {kv * 1e3:.3f} ms")
            del r, gr
        del r_obs
        # Full Jacobian d(r, v)/d(elements) at every point: 42 doubles per point.
        paths["jacobian_9341x1000"] = {}
        jac = torch.empty((6, 7, cat.n, cat.T), dtype=torch.float64, device=dev)
        for name in ("fp64", "mixed"):
            kj = kernel_time(lambda: sg.jacobian(rec, t, name, out=jac), torch, reps=3)
            paths["jacobian_9341x1000"][name] = {"points_per_s": P / kj, "kernel_ms": kj * 1e3,
                                                 "hbm_gbs": 336 * P / kj / 1e9}
            log(f"[bench] jacobian {name}: {P / kj:.3e} pts/s, {kj * 1e3:.3f} ms")
        del jac
        torch.cuda.empty_cache()

    if not args.no_vjp and not args.only:
        # Deep-space catalogue (4,096 satellites x 1,008 times over 7 days; every
        # set takes the lunar-solar terms, the 15% in the resonant classes the
        # resonance integrator as well).
        c5 = synth.config5()
        e5, t5 = torch.from_numpy(c5.elem).to(dev), torch.from_numpy(c5.t).to(dev)
        P5 = c5.n * c5.T
        paths["deep_4096x1008"] = {}
        for name in ("fp64", "mixed"):
            rec5 = sg.init(e5, ref_jd=synth.DEEP_REF_JD)
            dt = torch.float64 if name == "fp64" else torch.float32
            out5 = (torch.empty((3, c5.n, c5.T), dtype=dt, device=dev), torch.empty((3, c5.n, c5.T), dtype=dt, device=dev),
                    torch.empty((c5.n, c5.T), dtype=torch.uint8, device=dev))
            k5 = kernel_time(lambda: sg.propagate(rec5, t5, name, out=out5), torch, reps=10)
            paths["deep_4096x1008"][name] = {"points_per_s": P5 / k5, "kernel_ms": k5 * 1e3}
            log(f"[bench] deep space 4096x1008 {name}: {P5 / k5:.3e} pts/s, {k5 * 1e3:.3f} ms")
            del out5, rec5
        torch.cuda.empty_cache()

    if not args.no_vjp and not args.only:
        # Conjunction screening of the 9,341 x 1,000 mixed output (float positions,
        # codes given), D = 10 km: one workgroup per sample time.
        import ctypes
        from paper_2603_27830_amd import _native
        rec = sg.init(elem)
        r_s, _, e_s = sg.propagate(rec, t, "mixed")
        cap = 1 << 20
        pairs = torch.empty((cap, 3), dtype=torch.int32, device=dev)
        dist = torch.empty(cap, dtype=torch.float64, device=dev)
        cnt = torch.empty(1, dtype=torch.int64, device=dev)
        wsb = int(_native.lib().sgp4_screen_workspace_bytes(cat.n, cat.T))
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        vp = lambda x: ctypes.c_void_p(x.data_ptr())  # noqa: E731

        def screen_launch():
            _native.check(_native.lib().sgp4_screen(
                vp(r_s), _native.SGP4_FP32_MIXED, vp(e_s), cat.n, cat.T, 10.0, cap, vp(pairs), vp(dist), vp(cnt),
                vp(ws), wsb, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), "sgp4_screen")

        ks = kernel_time(screen_launch, torch, reps=10)
        events = int(cnt.item())
        paths["screen_9341x1000"] = {"dist_km": 10.0, "events": events, "ms": ks * 1e3,
                                     "satellite_times_per_s": P / ks,
                                     "pairs_per_s_brute_force_equivalent": cat.n * (cat.n - 1) / 2 * cat.T / ks}
        log(f"[bench] screen 9341 x 1000 (10 km): {ks * 1e3:.3f} ms, {events} events")
        del r_s, e_s, pairs, dist, ws
        torch.cuda.empty_cache()

    if not args.no_short and not args.only:
        # Short time lists over the 1M-satellite catalogue's elements: the fused
        # elements-to-states launch against the two-stage path's parts (init;
        # the flat and the 64-time tile dense mappings).
        n5 = 1_000_000
        el5 = synth.shell_elements(n5, 3)
        el5[6, np.random.default_rng(1003).random(n5) < 0.05] *= 100.0
        e5 = torch.from_numpy(el5).to(dev)
        paths["short_lists_1M"] = {}
        rec5 = sg.init(e5)
        ki = kernel_time(lambda: sg.init(e5), torch, reps=5)
        paths["short_lists_1M"]["init_ms"] = ki * 1e3
        log(f"[bench] 1M init {ki * 1e3:.3f} ms")
        for T5 in (1, 8, 16, 32, 48):
            t5 = torch.from_numpy(np.linspace(0.0, 1440.0, T5)).to(dev)
            row = {}
            for name in ("fp64", "mixed"):
                dt = torch.float64 if name == "fp64" else torch.float32
                out5 = (torch.empty((3, n5, T5), dtype=dt, device=dev), torch.empty((3, n5, T5), dtype=dt, device=dev),
                        torch.empty((n5, T5), dtype=torch.uint8, device=dev))
                kf = kernel_time(lambda: sg.propagate_elements(e5, t5, name, out=out5), torch, reps=5)
                kl = kernel_time(lambda: sg.propagate(rec5, t5, name, out=out5, block=256 | 0x80000), torch, reps=5)
                kt = kernel_time(lambda: sg.propagate(rec5, t5, name, out=out5,
                                                      block=(256 if name == "fp64" else 512) | 0x50000), torch, reps=5)
                row[name] = {"fused_ms": kf * 1e3, "flat_ms": kl * 1e3, "tiles_ms": kt * 1e3,
                             "fused_points_per_s": n5 * T5 / kf}
                log(f"[bench] 1M x {T5} {name}: fused {kf * 1e3:.3f} ms; propagate flat {kl * 1e3:.3f} ms, "
                    f"tiles {kt * 1e3:.3f} ms")
                del out5
            paths["short_lists_1M"][f"T{T5}"] = row
        del rec5
        del e5
        torch.cuda.empty_cache()

    if not args.no_short and not args.only:
        # Ingestion: 200,000 synthetic two-line element sets (3LE, 32 MB of
        # text) parsed on the host by the library's native parser.
        from synth import text as stx
        el6 = synth.shell_elements(200_000, 6)
        txt = stx.tle_text(el6, three_line=True).encode()
        best = float("inf")
        for _ in range(3):
            t0 = time.perf_counter()
            sg.parse_text(txt, "tle", ref_jd=stx.REF_JD, threads=16)
            best = min(best, time.perf_counter() - t0)
        paths["ingest_tle_200k"] = {"parse_ms": best * 1e3, "records_per_s": 200_000 / best, "threads": 16,
                                    "text_mb": len(txt) / 1e6}
        log(f"[bench] parse 200k TLE ({len(txt) / 1e6:.0f} MB): {best * 1e3:.1f} ms, {200_000 / best:.3e} rec/s")

    if not args.no_ragged and not args.only:
        c3 = synth.config3()
        rec3 = sg.init(torch.from_numpy(c3.elem).to(dev))
        off3 = torch.from_numpy(c3.offsets).to(dev)
        t3 = torch.from_numpy(c3.t).to(dev)
        paths["c3_ragged_1M"] = {"nnz": c3.nnz}
        for name in ("fp64", "mixed"):
            plan = sg.RaggedPlan(rec3, off3, t3, name, autotune=True, graph=True)
            k3 = kernel_time(plan.launch, torch, reps=3)
            paths["c3_ragged_1M"][name] = {"points_per_s": c3.nnz / k3, "launch_ms": k3 * 1e3,
                                           "plan": json.loads(plan.describe())}
            log(f"[bench] c3 {name}: {c3.nnz / k3:.3e} pts/s ({plan.describe()})")
            plan.close()
            torch.cuda.empty_cache()
        # Gradient over the same lists: the ragged VJP for a unit cotangent on r
        # (every point's forward pass recomputed and swept in reverse).
        for name in ("fp64", "mixed"):
            gdt = torch.float64 if name == "fp64" else torch.float32
            gr3 = torch.ones((3, c3.nnz), dtype=gdt, device=dev)
            kv = kernel_time(lambda: sg.vjp_ragged(rec3, off3, t3, gr3, None, name), torch, reps=3)
            paths["c3_ragged_1M"][f"vjp_{name}"] = {"points_per_s": c3.nnz / kv, "kernel_ms": kv * 1e3}
            log(f"[bench] c3 vjp {name}: {c3.nnz / kv:.3e} pts/s, {kv * 1e3:.2f} ms")
            del gr3
            torch.cuda.empty_cache()

    head = paths.get("mixed") or paths[names[0]]
    head_name = "mixed" if "mixed" in paths else names[0]
    # Roofline of the dominant kernel (the headline path's propagate launch):
    # attainable = min(ALU peak, intensity x HBM peak), so the fraction of it
    # reached is the larger of the HBM (output bytes) and ALU (algorithmic ops)
    # fractions, and that one names the bound.
    k_s = head["propagate_kernel_us"] * 1e-6
    gbs = BYTES_PER_POINT[head_name] * P / k_s / 1e9
    tfl = ALG_FLOP_PER_POINT * P / k_s / 1e12
    traffic = measured_traffic(head_name)
    hbm = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
           "traffic": traffic}
    peak = VALU_PEAK_TFLOPS[head_name]
    alu = {"bound": "alu", "achieved": tfl, "peak": peak, "unit": "TFLOP/s", "frac": tfl / peak,
           "traffic": traffic}
    roof, other = (hbm, alu) if hbm["frac"] >= alu["frac"] else (alu, hbm)
    # The same launch priced by what the VALU executes (counter-based flops, the
    # elementary functions' expansions included) instead of the algorithmic count.
    xf = executed_flop_per_point(head_name)
    counters = None if xf is None else {
        "bound": "alu", "executed_flop_per_point": xf, "achieved": xf * P / k_s / 1e12, "peak": peak,
        "unit": "TFLOP/s", "frac": xf * P / k_s / 1e12 / peak}

    # The bound the counters show: the fraction of the launch's SIMD quad-cycles
    # (at the clock sampled during the timed steps) in which the VALU issued
    # this kernel's instructions, a dual-issued pair counted once.
    quads = valu_quads_per_wave(head_name)
    clk = head.get("gpu_clock")
    issue = None
    if quads is not None and clk is not None:
        waves = cat.n * ((cat.T + 63) // 64)
        busy = waves * (quads[0] - quads[1]) / 1024.0          # quad-cycles per SIMD
        avail = clk["mean_mhz"] * 1e6 / 4.0 * k_s                # quad-cycles per SIMD in the launch
        issue = {"bound": "valu_issue", "achieved": busy / k_s / 1e9, "peak": clk["mean_mhz"] * 1e6 / 4.0 / 1e9,
                 "unit": "G VALU quad-cycles/s per SIMD", "frac": busy / avail,
                 "valu_quads_per_wave": quads[0], "dual_issue_quads_per_wave": quads[1],
                 "clock_mhz": clk["mean_mhz"]}
    calib = None
    if not args.only:
        try:
            c = calibrate(torch)
            calib = {k: c[k] for k in ("fma_f64_tflops", "fma_f32_vgpr_tflops", "fma_f32_sgpr_operand_tflops",
                                       "store_nt_gbs") if k in c}
        except Exception as e:  # noqa: BLE001 - reported, not fatal
            calib = {"error": repr(e)}

    line = {
        "metric": "sat-time propagations/s at 9341x1000: FP32-mixed vs FP64 GPU; % of VALU peak",
        "value": head["points_per_s"], "unit": "sat-time points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": head["points_per_s"] / PAPER_POINTS_PER_S,
        "vs_baseline_note": "paper: 9,341 x 1,000 in 3.8 ms on one A100, FP32, init included (context)",
        "dtype": "fp32+fp64 (mixed)" if head_name == "mixed" else head_name,
        "data": "synthetic (seeded Starlink-shaped catalogue)",
        "config": {"workload": "9341 satellites x 1000 times over 0-1440 min, init + dense propagate",
                   "satellites": cat.n, "times": cat.T, "precision": head_name},
        "roofline": roof, "roofline_other": other, "roofline_executed": counters, "roofline_issue": issue,
        "gpu_clock": clk, "calibration": calib,
        "paths": paths,
    }
    if not args.no_cpu and not args.only:
        line["cpu_baseline"] = cpu_baseline(cat)
        log(f"[bench] cpu oracle: {line['cpu_baseline']['value']:.3e} pts/s on {line['cpu_baseline']['cores']} cores")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
