"""Benchmark of the PW advection hot path on one MI355X.

One step = one pass of the whole hot path over the 4096x4096x64 FP64 grid
(1.07e9 cells, halo 2): forward source terms (su, sv, sw) and the gather
adjoint (gu, gv, gw) for multipliers (lu, lv, lw), in one fused launch.
Inputs are generated on the device by the library's counter-based generator
and halo-filled before the timed region, so the timed region holds only the
advection kernel.

Printed: one JSON line with the headline value (FP64 fused fwd+adj Gcells/s),
the roofline of that kernel (algorithmic bytes / measured average launch time
against 8 TB/s HBM), per-path figures (fwd / adj / fused in FP64, FP32,
FP32 storage with FP64 arithmetic, binary16 and bfloat16 storage; the fused
Euler step and its unfused equivalent),
and the CPU oracle timed on a bounded sample of the same workload.

Also printed, as context: the host-resident offload (fields in pinned host
memory, pipelined x-slab transfers, pw_advect_fwd_host) at 4096x1024x64.

Also printed: the library's plain streaming copy over the headline's own
arrays (the achievable-bandwidth reference, timed interleaved with the
kernels), the paths at 1024x1024x64 (the precision workload), and the
cache-resident 256x256x64 forward and fused pass.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload NAME]
       [--kernel auto|direct|march] [--no-cpu-baseline] [--no-offload]
       [--paths-reps R] [--no-paths] [--no-medium] [--only PATH:DTYPE|copy|copy3|copy6]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL = {  # algorithmic: each input read once, each output written once
    ("fwd", 8): 48, ("adj", 8): 72, ("fused", 8): 96,
    ("fwd", 4): 24, ("adj", 4): 36, ("fused", 4): 48,
    # Euler step u + dt*su fused into the forward: reads u, v, w, writes the
    # new fields (the same streams as the forward); unfused it is the forward
    # plus a pass reading u and su and writing the new field (+72 B FP64)
    ("update", 8): 48, ("update", 4): 24, ("fwd+axpy", 8): 120, ("fwd+axpy", 4): 60,
    ("fwd", 2): 12, ("adj", 2): 18, ("fused", 2): 24,
}
DT = 0.5   # timestep of the update path (any value: the timing does not depend on it)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _code_only(text):
    """Source text without comments and whitespace (a comment edit leaves the
    kernels, and so their measured traffic, unchanged)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return re.sub(r"\s+", "", text)


# the sources that define the x-marching kernels (whose HBM traffic the
# counter records hold): a change elsewhere leaves their code unchanged
KERNEL_SOURCES = ("pw_march.hip", "pw_stencil.h", "pw_half.h")


def kernel_source_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2010_01545_amd", "csrc", name), "r") as f:
            h.update(name.encode())
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel_name, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    e = rec.get("kernels", {}).get(kernel_name)
    if not e or e.get("workload") != workload or rec.get("source_hash") != kernel_source_hash():
        return None
    return e.get("hbm_bytes_per_launch")


class Grid:
    """The arrays of one grid: u, v, w [, lu, lv, lw], su, sv, sw [, gu, gv,
    gw].  pooled: views into one allocation (pwadvect.alloc_fields, the
    layout the headline uses); else one allocation per array."""

    def __init__(self, pw, torch, nx, ny, nz, h, dtype, seed, with_lambda, compute=None, pooled=True):
        self.nx, self.ny, self.nz, self.h = nx, ny, nz, h
        self.compute = compute
        self.cells = nx * ny * nz
        shape = (nx + 2 * h, ny + 2 * h, nz + 2 * h)
        dev = torch.device("cuda:0")
        n = 12 if with_lambda else 6
        if pooled:
            arrs = pw.alloc_fields(n, shape, dtype, device=dev)
        else:
            arrs = [torch.empty(shape, dtype=dtype, device=dev) for _ in range(n)]
        self.f = arrs[0:3]
        self.l = arrs[3:6] if with_lambda else []
        self.s = arrs[6:9] if with_lambda else arrs[3:6]
        self.g = arrs[9:12] if with_lambda else []
        for fid, t in enumerate(self.f):
            pw.fill_uniform(t, h, seed, fid, 10.0, zero_lids=(fid == 2))
            pw.halo_periodic(t, h)
        for q, t in enumerate(self.l):
            pw.fill_uniform(t, h, seed, 3 + q, 1.0, False)
            pw.halo_periodic(t, h)
        from paper_2010_01545_amd import inputs
        tzc1, tzc2, self.tcx, self.tcy = inputs.coefficients(nz)
        self.t1 = torch.from_numpy(tzc1).to(dev)
        self.t2 = torch.from_numpy(tzc2).to(dev)

    def launch(self, pw, path):
        c = self.compute
        if path == "update":
            pw.fwd_update(*self.f, self.t1, self.t2, self.tcx, self.tcy, self.h, *self.f, DT, *self.s, compute=c)
        elif path == "fwd+axpy":
            import torch
            pw.fwd(*self.f, self.t1, self.t2, self.tcx, self.tcy, self.h, *self.s, compute=c)
            for f, sq in zip(self.f, self.s):
                torch.add(f, sq, alpha=DT, out=sq)
        elif path == "fwd":
            pw.fwd(*self.f, self.t1, self.t2, self.tcx, self.tcy, self.h, *self.s, compute=c)
        elif path == "adj":
            pw.adj(*self.f, *self.l, self.t1, self.t2, self.tcx, self.tcy, self.h, *self.g, compute=c)
        else:
            pw.fwd_adj(*self.f, *self.l, self.t1, self.t2, self.tcx, self.tcy, self.h,
                       out=self.s + self.g, compute=c)


def time_launches(torch, fn, reps):
    """Per-launch durations (ms) from HIP events recorded on the stream the
    kernels are launched on (torch's current stream)."""
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for r in range(reps):
        fn()
        ev[r + 1].record(stream)
    torch.cuda.synchronize()
    return [ev[r].elapsed_time(ev[r + 1]) for r in range(reps)]


def settle(torch, fn, seconds=None):
    """Untimed launches of fn for `seconds` (default CLOCK_SETTLE_S): after
    an idle period (allocating and filling a new grid) the GPU runs these
    kernels near 1.5 GHz and ramps its clock up over their first launches
    (about 0.1 s), which would otherwise fall into a short timed run."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < (CLOCK_SETTLE_S if seconds is None else seconds):
        fn()
        torch.cuda.synchronize()


def path_record(path, esize, cells, times_ms):
    ts = sorted(times_ms)
    avg = sum(times_ms) / len(times_ms)
    bpc = BYTES_PER_CELL[(path, esize)]
    return {
        "gcells_per_s": cells / (avg * 1e-3) / 1e9,
        "ms_avg": avg, "ms_min": ts[0], "ms_median": ts[len(ts) // 2],
        "ms_p90": ts[min(len(ts) - 1, int(0.9 * len(ts)))],
        "alg_bytes_per_cell": bpc,
        "alg_GBps": bpc * cells / (avg * 1e-3) / 1e9,
        "hbm_frac": bpc * cells / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "reps": len(times_ms),
    }


# untimed launches of the headline kernel before its warm-up (seconds)
CLOCK_SETTLE_S = 0.3

# launch shapes of the streaming copy: (bytes per thread and array, workgroups (0 = one pass),
# cache hints: 1 non-temporal loads, 2 non-temporal stores)
COPY_SHAPES = ((4, 0, 0), (4, 0, 1), (4, 0, 2), (4, 0, 3), (8, 0, 0), (16, 0, 0), (16, 0, 3), (16, 2048, 0))


def copy_reference(pw, torch, g, reps=5):
    """The library's plain streaming copy (pw_stream_copy) over the very
    arrays the headline kernel uses (same placement in HBM): 6 arrays read and
    6 written (the fused pass's streams: u, v, w, lu, lv, lw -> su .. gw) and
    3 + 3 (the forward's).  Each launch shape and cache policy is timed; the
    fastest is the achievable-bandwidth reference.  Timed interleaved with the FP64 fused and
    forward kernels on the same arrays, so that their ratio compares like with
    like."""
    nbytes = g.f[0].numel() * g.f[0].element_size()
    rec = {"kernel": "pw_stream_copy: every thread reads its unit of each source then writes each destination; "
                     "storage arrays of %d bytes" % nbytes}
    for tag, src, dst, path in (("6R6W", g.f + g.l, g.s + g.g, "fused"), ("3R3W", g.f, g.s, "fwd")):
        shapes = {}
        for unit, b, hints in COPY_SHAPES:
            pw.stream_copy(src, dst, b, unit, hints)
            ms = time_launches(torch, lambda: pw.stream_copy(src, dst, b, unit, hints), reps)
            shapes["unit_%d_blocks_%d_hints_%d" % (unit, b, hints)] = {
                "ms": sum(ms) / len(ms), "GBps": 2 * len(src) * nbytes / (sum(ms) / len(ms) * 1e-3) / 1e9}
        best = min(shapes, key=lambda k: shapes[k]["ms"])
        unit, b, hints = (int(x) for x in best.split("_")[1::2])
        # interleaved: copy, kernel, copy, kernel ...
        tc, tk = [], []
        for _ in range(reps):
            tc += time_launches(torch, lambda: pw.stream_copy(src, dst, b, unit, hints), 1)
            tk += time_launches(torch, lambda: g.launch(pw, path), 1)
        mc, mk = sum(tc) / len(tc), sum(tk) / len(tk)
        rec[tag] = {"ms": mc, "GBps": 2 * len(src) * nbytes / (mc * 1e-3) / 1e9, "unit": unit, "blocks": b,
                    "hints": hints, "launch_shapes": shapes,
                    "interleaved_%s_f64_ms" % path: mk,
                    "%s_f64_time_fraction_of_copy" % path: mc / mk}
        # torch's device copy of the same arrays, for comparison
        step = lambda: [d.copy_(x) for d, x in zip(dst, src)]
        step()
        t = time_launches(torch, step, reps)
        rec[tag]["torch_copy_GBps"] = 2 * len(src) * nbytes / (sum(t) / len(t) * 1e-3) / 1e9
    return rec


def host_threads():
    """Host threads for the CPU baseline: OMP_NUM_THREADS when set, else the
    usable cores, at most 16 (one GPU's share of its host)."""
    usable = os.cpu_count() or 1
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    n = int(os.environ.get("OMP_NUM_THREADS", usable))
    return max(1, min(n, usable, 16)), usable


def cpu_baseline(nx, ny, nz, seed, budget_s=8.0, planes=32, slab_planes=8):
    """The oracle (FP64 C, unmodified) timed on the host on bounded samples of
    the workload:
      * value: forward + scatter adjoint (the fused step's work) on all host
        threads at once, each running the single-threaded oracle on its own
        x-slab of slab_planes planes (slab t starts at plane t * slab_planes;
        its x halo planes are the true neighbour planes, y is periodic), for
        about budget_s of wall time; ctypes releases the GIL during each call;
      * single_thread: the same on x-planes 0..planes-1 on one thread;
      * fwd_openmp: the OpenMP build of the oracle's forward on that slab."""
    import threading
    import numpy as np
    import oracle
    from paper_2010_01545_amd import inputs
    h = 2
    tzc1, tzc2, tcx, tcy = inputs.coefficients(nz)

    def slab(a):  # x halo from the true neighbour planes, y periodic, z pad 0
        s = np.pad(a, ((0, 0), (h, h), (0, 0)), mode="wrap")
        return np.ascontiguousarray(np.pad(s, ((0, 0), (0, 0), (h, h))))

    def make(x0, n):
        f = [slab(a) for a in inputs.winds(seed, nx, ny, nz, x0=x0 - h, x1=x0 + n + h)]
        lam = [slab(a) for a in inputs.multipliers_uniform(seed, nx, ny, nz, x0=x0 - h, x1=x0 + n + h)]
        return f, lam

    def step(f, lam):
        oracle.fwd(*f, tzc1, tzc2, tcx, tcy, h)
        oracle.adj(*f, *lam, tzc1, tzc2, tcx, tcy, h)

    threads, usable = host_threads()
    # all threads at once, each on its own slab
    data = [None] * threads
    reps = [0] * threads
    gate = threading.Barrier(threads + 1)
    deadline = [0.0]

    def worker(t):
        data[t] = make(t * slab_planes, slab_planes)
        gate.wait()
        while True:
            step(*data[t])
            reps[t] += 1
            if time.perf_counter() >= deadline[0]:
                break

    pool = [threading.Thread(target=worker, args=(t,)) for t in range(threads)]
    for th in pool:
        th.start()
    t0 = time.perf_counter()
    deadline[0] = t0 + 1e9
    gate.wait()
    t0 = time.perf_counter()
    deadline[0] = t0 + budget_s
    for th in pool:
        th.join()
    wall = time.perf_counter() - t0
    slab_cells = slab_planes * ny * nz
    multi = sum(reps) * slab_cells / wall / 1e9
    del data

    # one thread
    f, lam = make(0, planes)
    cells = planes * ny * nz
    spent, n1 = 0.0, 0
    while spent < budget_s:
        t1 = time.perf_counter()
        step(f, lam)
        spent += time.perf_counter() - t1
        n1 += 1
    single = cells * n1 / spent / 1e9
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    t1 = time.perf_counter()
    nrep = 0
    while time.perf_counter() - t1 < 2.0:
        oracle.fwd(*f, tzc1, tzc2, tcx, tcy, h, threaded=True)
        nrep += 1
    fwd_omp = cells * nrep / (time.perf_counter() - t1) / 1e9
    return {
        "value": multi, "unit": "Gcells/s", "cores": threads, "kind": "oracle",
        "sample": "oracle fwd + scatter adjoint, FP64, unmodified single-threaded C, run concurrently by %d "
                  "threads, each on its own %d-plane x-slab of the %dx%dx%d grid (slabs at planes 0, %d, ...; "
                  "%d cells each), %d slab steps in %.1f s"
                  % (threads, slab_planes, nx, ny, nz, slab_planes, slab_cells, sum(reps), wall),
        "single_thread": {"value": single, "unit": "Gcells/s", "cores": 1,
                          "sample": "the same on x-planes 0..%d (%d cells), %d steps in %.1f s"
                                    % (planes - 1, cells, n1, spent)},
        "fwd_openmp": {"value": fwd_omp, "unit": "Gcells/s", "threads": threads,
                       "sample": "oracle forward only, OpenMP build, x-planes 0..%d" % (planes - 1)},
        "host": {"cpu_model": model, "usable_cores": usable},
    }


def offload_measure(pw, torch, reps=4, chunk=64):
    """Host-resident fields (pinned) at the paper's largest grid, 2^28 cells:
    pipelined pw_advect_fwd_host against its parts measured alone."""
    from paper_2010_01545_amd import inputs
    nx, ny, nz, h, seed = 4096, 1024, 64, 2, 4
    cells = nx * ny * nz
    dt = torch.float64
    shape = (nx + 2 * h, ny + 2 * h, nz + 2 * h)
    dev = torch.device("cuda:0")
    g = Grid(pw, torch, nx, ny, nz, h, dt, seed, False)        # device copies of the winds
    host_in = [torch.empty(shape, dtype=dt, pin_memory=True) for _ in range(3)]
    host_out = [torch.empty(shape, dtype=dt, pin_memory=True) for _ in range(3)]
    for hsrc, d in zip(host_in, g.f):
        hsrc.copy_(d)
    ws = torch.empty(pw.offload_workspace_bytes(shape, h, dt, chunk), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def timed(fn, n):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        fn()
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(n):
            fn()
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / n

    run = lambda: pw.fwd_host(*host_in, g.t1, g.t2, g.tcx, g.tcy, h, *host_out, chunk, ws)
    # copy-out modes: the runtime's copies, the library's copy kernel and
    # direct writes by the advection kernel, warmed, then timed call by call
    # in alternation so that none profits from another's warm-up; then the
    # automatic choice among them (the default; it learns from every call's
    # time)
    calls = {"runtime": [], "kernel": [], "direct": []}
    for _ in range(2):      # (the first call of each mode carries one-time costs)
        for mode in calls:
            with pw.tuning(copy_out=mode):
                run()
            torch.cuda.synchronize()
    for _ in range(reps):
        for mode in calls:
            with pw.tuning(copy_out=mode):
                calls[mode].append(timed(run, 1))
    # the automatic mode as a caller uses it: consecutive calls, after the
    # calls above taught it each mode's time on this device
    calls["auto"] = []
    with pw.tuning(copy_out="auto"):
        for _ in range(2 * reps):
            calls["auto"].append(timed(run, 1))
    med = lambda v: sorted(v)[len(v) // 2]
    by_mode = {m: med(v) for m, v in calls.items()}
    default_mode = {v: k for k, v in pw.COPY_OUT.items()}[pw.get_tuning(pw.TUNE_COPY_OUT)]
    t_off = by_mode[default_mode]
    t_h2d = timed(lambda: [d.copy_(hsrc, non_blocking=True) for d, hsrc in zip(g.f, host_in)], reps)
    t_d2h = timed(lambda: [o.copy_(d, non_blocking=True) for o, d in zip(host_out, g.s)], reps)
    t_k = timed(lambda: g.launch(pw, "fwd"), reps)
    nbytes = 3 * shape[0] * shape[1] * shape[2] * 8
    rec = {
        "workload": "%dx%dx%d FP64 forward, fields and source terms in pinned host memory, halo %d, "
                    "x-slabs of %d planes" % (nx, ny, nz, h, chunk),
        "cells": cells,
        "gcells_per_s_incl_transfers": cells / (t_off * 1e-3) / 1e9,
        "ms_pipelined": t_off,
        "copy_out_default": default_mode,
        "ms_pipelined_by_copy_out": by_mode,
        "ms_per_call": {k: [round(x, 2) for x in v] for k, v in calls.items()},
        "ms_copy_in_alone": t_h2d, "ms_copy_out_alone": t_d2h, "ms_kernel_alone": t_k,
        "copy_in_GBps": nbytes / (t_h2d * 1e-3) / 1e9, "copy_out_GBps": nbytes / (t_d2h * 1e-3) / 1e9,
        "ms_serial_sum": t_h2d + t_d2h + t_k,
        "overlap": (t_h2d + t_d2h + t_k) / t_off,
        "ideal_ms": max(t_h2d, t_d2h),
        "bytes_each_way": nbytes,
    }
    del g, host_in, host_out, ws
    torch.cuda.empty_cache()
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper_scale")
    ap.add_argument("--kernel", default="auto", choices=["auto", "direct", "march"])
    ap.add_argument("--paths-reps", type=int, default=10)
    ap.add_argument("--no-paths", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-offload", action="store_true")
    ap.add_argument("--no-separate", action="store_true",
                    help="skip the FP64 record over separately allocated arrays (same kernels, same grid)")
    ap.add_argument("--no-medium", action="store_true",
                    help="skip the cache-resident 256x256x64 record (its launches share the kernels' names)")
    ap.add_argument("--only", default=None, help="profile helper: run only this path/dtype, e.g. fused:f64, "
                    "or the streaming copy of 3 or 6 storage arrays (copy3, copy6)")
    ap.add_argument("--copy-blocks", type=int, default=0, help="launch shape of --only copy3/copy6")
    ap.add_argument("--copy-unit", type=int, default=4, help="bytes per thread and array of --only copy3/copy6")
    ap.add_argument("--copy-hints", type=int, default=0,
                    help="cache hints of --only copy3/copy6: 1 non-temporal loads, 2 stores, 3 both")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the PW advection path is measured on one "
              "GPU's grid; the library has no multi-GPU path (x-slab decomposition with halo "
              "exchange).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2010_01545_amd import inputs, pwadvect as pw

    wl = inputs.WORKLOADS[args.workload]
    nx, ny, nz, seed = wl["nx"], wl["ny"], wl["nz"], wl["seed"]
    h = inputs.HALO
    cells = nx * ny * nz
    pw.set_kernel(args.kernel)
    torch.cuda.init()
    log("bench: %s %dx%dx%d, kernel=%s" % (args.workload, nx, ny, nz, args.kernel))

    if args.only == "copy":
        # calibration for the HBM byte counters: a plain device copy of a
        # known size (4 GiB read + 4 GiB written per launch)
        n = 4 << 30
        src = torch.empty(n // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(args.warmup + args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copy calibration done (%d bytes per launch each way)" % n)
        return
    if args.only in ("copy3", "copy6"):
        # the streaming copy reference over the headline's storage arrays
        g = Grid(pw, torch, nx, ny, nz, h, torch.float64, seed, True)
        n = int(args.only[-1])
        src, dst = (g.f + g.l)[:n], (g.s + g.g)[:n]
        torch.cuda.synchronize()
        for _ in range(args.warmup + args.steps):
            pw.stream_copy(src, dst, args.copy_blocks, args.copy_unit, args.copy_hints)
        torch.cuda.synchronize()
        log("bench: profile run of %s done" % args.only)
        return
    if args.only:
        path, dt = args.only.split(":")
        st_dt = {"f64": torch.float64, "f16": torch.float16, "bf16": torch.bfloat16}.get(dt, torch.float32)
        g = Grid(pw, torch, nx, ny, nz, h, st_dt, seed, path != "fwd",
                 compute=torch.float64 if dt == "f32f64" else None)
        torch.cuda.synchronize()
        for _ in range(args.warmup + args.steps):
            g.launch(pw, path)
        torch.cuda.synchronize()
        log("bench: profile run of %s done" % args.only)
        return

    # ---- headline: FP64 fused forward + adjoint
    g = Grid(pw, torch, nx, ny, nz, h, torch.float64, seed, True)
    torch.cuda.synchronize()
    log("bench: inputs ready")
    # After an idle period the GPU starts these kernels near 1.5 GHz and ramps
    # its clock up over their first 5-8 launches (about 0.1 s); let it settle
    # before the warm-up launches, so that the timed launches all see the
    # clock the workload holds.
    settle(torch, lambda: g.launch(pw, "fused"))
    for _ in range(args.warmup):
        g.launch(pw, "fused")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    times = time_launches(torch, lambda: g.launch(pw, "fused"), args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    head = path_record("fused", 8, cells, times)
    log("bench: fused f64 %.2f ms/launch, %.1f Gcells/s" % (head["ms_avg"], head["gcells_per_s"]))

    # achievable-bandwidth reference on the same arrays
    copy_ref = copy_reference(pw, torch, g)
    log("bench: stream copy 6R6W %.0f GB/s (fused at %.3f of its speed), 3R3W %.0f GB/s (fwd at %.3f)" % (
        copy_ref["6R6W"]["GBps"], copy_ref["6R6W"]["fused_f64_time_fraction_of_copy"],
        copy_ref["3R3W"]["GBps"], copy_ref["3R3W"]["fwd_f64_time_fraction_of_copy"]))

    paths = {"fused_f64": head}
    if not args.no_paths:
        for p in ("fwd", "adj", "update", "fwd+axpy"):
            g.launch(pw, p)
            paths[p + "_f64"] = path_record(p, 8, cells, time_launches(torch, lambda: g.launch(pw, p),
                                                                       args.paths_reps))
            log("bench: %s f64 %.2f ms" % (p, paths[p + "_f64"]["ms_avg"]))
    del g
    torch.cuda.empty_cache()

    if not args.no_paths:
        g = Grid(pw, torch, nx, ny, nz, h, torch.float32, seed, True)
        settle(torch, lambda: g.launch(pw, "fused"))
        for p in ("fwd", "adj", "fused"):
            g.launch(pw, p)
            paths[p + "_f32"] = path_record(p, 4, cells, time_launches(torch, lambda: g.launch(pw, p),
                                                                       args.paths_reps))
            log("bench: %s f32 %.2f ms" % (p, paths[p + "_f32"]["ms_avg"]))
        del g
        torch.cuda.empty_cache()
        # FP32 storage with FP64 arithmetic
        g = Grid(pw, torch, nx, ny, nz, h, torch.float32, seed, True, compute=torch.float64)
        settle(torch, lambda: g.launch(pw, "fused"))
        for p in ("fwd", "adj", "fused"):
            g.launch(pw, p)
            paths[p + "_f32f64"] = path_record(p, 4, cells, time_launches(torch, lambda: g.launch(pw, p),
                                                                          args.paths_reps))
            log("bench: %s f32-storage/f64-arithmetic %.2f ms" % (p, paths[p + "_f32f64"]["ms_avg"]))
        del g
        torch.cuda.empty_cache()
        # 16-bit storage, float arithmetic
        for tag, dt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
            g = Grid(pw, torch, nx, ny, nz, h, dt, seed, True)
            settle(torch, lambda: g.launch(pw, "fused"))
            for p in ("fwd", "adj", "fused"):
                g.launch(pw, p)
                paths[p + "_" + tag] = path_record(p, 2, cells, time_launches(torch, lambda: g.launch(pw, p),
                                                                               args.paths_reps))
                log("bench: %s %s %.2f ms" % (p, tag, paths[p + "_" + tag]["ms_avg"]))
            del g
            torch.cuda.empty_cache()
        for p in ("fwd", "adj", "fused"):
            for v in ("_f32", "_f32f64", "_f16", "_bf16"):
                paths[p + v]["speedup_vs_f64"] = paths[p + "_f64"]["ms_avg"] / paths[p + v]["ms_avg"]

    # the same FP64 launches over twelve separately allocated arrays: their
    # speed depends on where each allocation lands in HBM
    separate = None
    if not args.no_paths and not args.no_separate:
        g = Grid(pw, torch, nx, ny, nz, h, torch.float64, seed, True, pooled=False)
        separate = {"layout": "one allocation per array"}
        settle(torch, lambda: g.launch(pw, "fused"))
        for p in ("fused", "fwd"):
            g.launch(pw, p)
            separate[p + "_f64"] = path_record(p, 8, cells, time_launches(torch, lambda: g.launch(pw, p),
                                                                          args.paths_reps))
            separate[p + "_f64"]["time_vs_pooled"] = separate[p + "_f64"]["ms_avg"] / paths[p + "_f64"]["ms_avg"]
        log("bench: separately allocated arrays: fused f64 %.2f ms, fwd f64 %.2f ms" % (
            separate["fused_f64"]["ms_avg"], separate["fwd_f64"]["ms_avg"]))
        del g
        torch.cuda.empty_cache()

    # 256x256x64 (the medium workload): the forward's six FP64 arrays (221 MB)
    # fit the 256 MB Infinity Cache, so its rate is not an HBM figure
    medium = None
    if not args.no_medium:
        wm = inputs.WORKLOADS["medium"]
        g = Grid(pw, torch, wm["nx"], wm["ny"], wm["nz"], h, torch.float64, wm["seed"], True)
        cm = wm["nx"] * wm["ny"] * wm["nz"]
        medium = {"workload": "medium %dx%dx%d FP64, 100 launches each" % (wm["nx"], wm["ny"], wm["nz"]),
                  "note": "fwd working set 221 MB fits the 256 MB Infinity Cache: not an HBM rate"}
        settle(torch, lambda: [g.launch(pw, "fused") for _ in range(20)])
        for p in ("fwd", "fused"):
            g.launch(pw, p)
            medium[p] = path_record(p, 8, cm, time_launches(torch, lambda: g.launch(pw, p), 100))
        del g
        torch.cuda.empty_cache()

    # 1024x1024x64 (the precision workload): GB/s of the FP64 and FP32 paths
    precision = None
    if not args.no_paths:
        wp = inputs.WORKLOADS["precision"]
        cp = wp["nx"] * wp["ny"] * wp["nz"]
        precision = {"workload": "precision %dx%dx%d, 20 launches each" % (wp["nx"], wp["ny"], wp["nz"])}
        for tag, dt, esz in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
            g = Grid(pw, torch, wp["nx"], wp["ny"], wp["nz"], h, dt, wp["seed"], True)
            settle(torch, lambda: [g.launch(pw, "fused") for _ in range(4)])
            for p in ("fwd", "adj", "fused"):
                g.launch(pw, p)
                precision[p + "_" + tag] = path_record(p, esz, cp, time_launches(torch, lambda: g.launch(pw, p), 20))
            del g
            torch.cuda.empty_cache()
        for p in ("fwd", "adj", "fused"):
            precision[p + "_f32"]["speedup_vs_f64"] = precision[p + "_f64"]["ms_avg"] / precision[p + "_f32"]["ms_avg"]
        log("bench: 1024^2 fwd f64 %.0f GB/s, f32 %.0f GB/s" % (precision["fwd_f64"]["alg_GBps"],
                                                             precision["fwd_f32"]["alg_GBps"]))

    # taller columns, FP64 and FP32: 128 levels at 2048 x 2048 (two
    # wavefronts per column in the marching kernels; the same cells per plane
    # as the headline grid's quarter, twice the levels) and 400 levels at
    # 2048 x 1024 (two z-chunks of 254 levels, four wavefronts each)
    def tall_record(tnx, tny, tnz, tseed):
        ct = tnx * tny * tnz
        rec = {"workload": "tall columns %dx%dx%d, 10 launches each" % (tnx, tny, tnz)}
        for tag, dt, esz in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
            g = Grid(pw, torch, tnx, tny, tnz, h, dt, tseed, True)
            settle(torch, lambda: g.launch(pw, "fused"))
            for p in ("fwd", "adj", "fused"):
                g.launch(pw, p)
                rec[p + "_" + tag] = path_record(p, esz, ct, time_launches(torch, lambda: g.launch(pw, p), 10))
            del g
            torch.cuda.empty_cache()
        log("bench: %dx%dx%d fwd f64 %.2f ms (%.0f GB/s), fused f64 %.2f ms" % (
            tnx, tny, tnz, rec["fwd_f64"]["ms_avg"], rec["fwd_f64"]["alg_GBps"], rec["fused_f64"]["ms_avg"]))
        return rec

    tall = tall_chunked = None
    if not args.no_paths:
        tall = tall_record(2048, 2048, 128, 5)
        tall_chunked = tall_record(2048, 1024, 400, 6)

    kname = "fused_f64"
    traffic = measured_traffic(kname, args.workload)
    achieved = head["alg_GBps"]
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "pw_advect_fwd_adj FP64 (%s)" % pw.get_kernel(),
                "alg_bytes_per_launch": 96 * cells}

    out = {
        "metric": "Gcells/s PW advection fwd & fwd+adj, FP64 vs FP32, % of HBM roofline",
        "value": head["gcells_per_s"], "unit": "Gcells/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (counter-based U(-10,10) winds, U(-1,1) multipliers)",
        "config": {"workload": "%s %dx%dx%d halo %d, FP64 fused forward + adjoint"
                   % (args.workload, nx, ny, nz, h), "nx": nx, "ny": ny, "nz": nz, "halo": h,
                   "cells": cells, "kernel": args.kernel,
                   "layout": "pooled: each grid's arrays are views into one allocation"},
        "roofline": roofline,
        "paths": paths,
        "copy_reference": copy_ref,
        "separate_allocations": separate,
        "precision_workload": precision,
        "tall_columns": tall,
        "tall_columns_chunked": tall_chunked,
        "medium_cache_resident": medium,
        "source_hash": kernel_source_hash(),
        "clock_settle_s": CLOCK_SETTLE_S,
    }
    if not args.no_offload:
        log("bench: host-resident offload at 4096x1024x64")
        out["offload"] = offload_measure(pw, torch)
        o = out["offload"]
        log("bench: offload %.1f ms pipelined (%s); by copy-out mode %s (in %.1f, kernel %.1f, out %.1f)" % (
            o["ms_pipelined"], o["copy_out_default"],
            ", ".join("%s %.1f" % kv for kv in o["ms_pipelined_by_copy_out"].items()),
            o["ms_copy_in_alone"], o["ms_kernel_alone"], o["ms_copy_out_alone"]))
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(nx, ny, nz, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
