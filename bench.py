"""Throughput of the fused D2Q9 kinetic step with local kinetic sensors on one
MI355X, against the unfused passes, the HBM roofline and the FP64 CPU oracle.

Workload: smooth random field (seed 0, 16 Fourier modes), D2Q9 BGK, 4096x4096
periodic, tau = 0.52, FP32 deviation storage in the row-interleaved layout
([ny][9][nx]; --layout planes for [9][ny][nx]); one step = pull streaming +
moments + equilibrium + S_KL, S_NEQ, S_PI + refinement flags + BGK collision +
FP64 global sums, all in one kernel (plus one small reduction kernel per
batch of steps).  Inputs are resident in HBM before the timed region starts.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--cpu-full] [--forms]
                    [--ext] [--ddf] [--q25] [--regrid] [--no-two-step]
    python bench.py --mode kernel --steps 5      # short run for profilers
    python bench.py --mode copy                  # copy-kernel yardstick only

Prints ONE JSON line (the last line of stdout).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, vendor figure
BYTES_F32_FUSED = 85            # 9 x 4 read + 9 x 4 written + 3 x 4 sensors + 1 flag
BYTES_F32_PLAIN = 193           # stream 36 + 36, sensors 36 + 13, collide 36 + 36
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_d2q9_fused_f32_4096.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2603_13618_amd", "csrc", "d2q9.hip")
# the fused FP32 step at the default launch shape (4 cells per thread)
# (non-temporal stores: the two 604 MB state buffers exceed the last-level cache)
FUSED_KERNEL = "d2q9_fused_lds<float,4,false,true>"
FUSED_KERNEL_PREFIX = "d2q9_fused_lds"     # rocprofv3 prints the bare name
# the double-distribution step (FP32): 50 x 4 read + 50 x 4 written + 5 x 4
# sensors + 1 flag per cell (the method's bytes; the two kernels of the step
# also hand 6 values per cell over and read g's own cell twice: 569 B)
BYTES_F32_DDF = 421
DDF_KERNEL = "d2q25_ddf_kernel<float,32,4,false,false,true> + d2q25_ddf_g_kernel<float,64,4,false,true>"
# the single-distribution D2Q25 step (FP32): 25 x 4 read + 25 x 4 written + 4 x 4
# sensors + 1 flag per cell
BYTES_F32_Q25 = 217
Q25_KERNEL = "d2q25_kernel<float,32,4,false,false,true>"
LAYOUT = "rows"                 # population layout of every lattice (--layout)


RUNS = 5                        # timed runs per measurement; the median is reported


def warm_up(torch, work, seconds=0.04):
    """Sustained load before a timed leg: the chip's clocks dip a few
    milliseconds into a burst of work and settle some 20 ms later (see
    profiles/d2q9_fused_f32_4096_clock_ramp.md), so each leg runs its own
    step for 40 ms first."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        work()
        torch.cuda.synchronize()


def median_time(torch, ev, runs, work, out=None):
    """Median over `runs` of the time of work() (seconds), each run bracketed
    by HIP events on torch's current stream (the library's stream) and a
    synchronisation.  The individual times are appended to `out` if given."""
    times = []
    for _ in range(runs):
        s, e = ev(), ev()
        s.record()
        work()
        e.record()
        torch.cuda.synchronize()
        times.append(s.elapsed_time(e) * 1e-3)
    if out is not None:
        out.extend(times)
    return sorted(times)[len(times) // 2]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    # untimed steps first: under sustained load the chip's clocks dip a few
    # milliseconds in and settle some 15 ms later (about 60 steps here)
    p.add_argument("--warmup", type=int, default=60)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-steps", type=int, default=40)
    p.add_argument("--cpu-full", action="store_true",
                   help="time the FP64 oracle alone on every workload (all cores and one thread, "
                        "bounded samples of each) and print that JSON line; no GPU is used")
    p.add_argument("--headline-only", action="store_true",
                   help="skip the legs of the other forms (16-bit storage, D2Q25 single and "
                        "double distribution, adjoint, two steps per launch)")
    p.add_argument("--forms", action="store_true",
                   help="time the BF16/FP16 storage forms on the 8192^2 workload (the default)")
    p.add_argument("--ext", action="store_true",
                   help="also time the fused steps with every extension sensor on")
    p.add_argument("--ddf", action="store_true",
                   help="time the D2Q25 double-distribution step on the 2048^2 Riemann problem "
                        "(the default)")
    p.add_argument("--q25", action="store_true",
                   help="time the D2Q25 single-distribution step on the 2048^2 Riemann problem "
                        "(the default)")
    p.add_argument("--adjoint", action="store_true",
                   help="time the differentiation workload, forward and hand-written adjoint "
                        "(the default)")
    p.add_argument("--two-step", action="store_true",
                   help="time two fused steps per launch (launch_steps = 2) against one, FP32 on "
                        "the 4096^2 and 8192^2 smooth fields (the default; kept for explicit use)")
    p.add_argument("--no-two-step", action="store_true", help="skip the two-steps-per-launch leg")
    p.add_argument("--fp64", action="store_true",
                   help="also time the FP64 forms: D2Q9 on the 4096^2 smooth field and the D2Q25 "
                        "double distribution on the 2048^2 Riemann quadrants")
    p.add_argument("--case3", action="store_true",
                   help="also run the modified 2D Riemann problem No. 3 at the paper's 1024^2 "
                        "to t = 0.85 (double distribution, FP32; about 196k steps)")
    p.add_argument("--regrid", action="store_true",
                   help="also time the regridding hand-off on the final flag map")
    p.add_argument("--layout", choices=["planes", "rows"], default="rows",
                   help="population layout of every lattice: plane-major [Q][ny][nx] or "
                        "row-interleaved [ny][Q][nx]")
    p.add_argument("--mode", choices=["bench", "kernel", "copy"], default="bench")
    p.add_argument("--workload", choices=["smooth4096", "riemann2048", "smooth8192-bf16",
                                          "smooth8192-f16", "adjoint1024", "smooth4096-ext",
                                          "riemann2048-ext", "riemann2048-ddf", "riemann2048-ddf-ext",
                                          "smooth4096-two", "smooth8192-two"],
                   default="smooth4096", help="workload of --mode kernel (profiling runs)")
    p.add_argument("--traffic-from", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                   help="assemble the traffic summary from four rocprofv3 --pmc output "
                        "directories (FETCH_SIZE and WRITE_SIZE of '--mode kernel', then of "
                        "'--mode copy') and write it under profiles/")
    return p.parse_args()


def kernel_hash():
    # the kernel source and the launch-shape and layout code around it
    h = hashlib.sha256()
    for name in ("d2q9.hip", "lks_device.h", "lks_internal.h", "lks_api.hip"):
        with open(os.path.join(ROOT, "paper_2603_13618_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_entry(n_cells):
    """HBM bytes per launch of the fused kernel from the committed counter
    summary, or None if absent or taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if (t.get("kernel_hash") != kernel_hash() or t.get("cells") != n_cells
            or t.get("layout", "planes") != LAYOUT):
        return None
    return t.get("bytes_per_launch")


def _pmc_mean(directory, counter, kernel_prefix):
    """Mean per-dispatch value of a counter for kernels whose name starts with
    kernel_prefix, from a rocprofv3 counter_collection.csv."""
    import csv
    import glob
    vals = []
    for path in glob.glob(os.path.join(directory, "*counter_collection.csv")):
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter and r["Kernel_Name"].startswith(kernel_prefix):
                    vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no {counter} samples for {kernel_prefix} under {directory}")
    return sum(vals) / len(vals), len(vals)


def assemble_traffic(dirs):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the fused kernel, each
    scaled by the ratio of the copy kernel's known bytes to what the same
    counter reads for it."""
    from paper_2603_13618_amd import workloads
    n = workloads.SMOOTH_4096["nx"]
    copy_bytes = 9 * n * n * 4
    lay = [] if LAYOUT == "rows" else ["--layout", LAYOUT]
    fetch, nf = _pmc_mean(dirs[0], "FETCH_SIZE", FUSED_KERNEL_PREFIX)
    write, nw = _pmc_mean(dirs[1], "WRITE_SIZE", FUSED_KERNEL_PREFIX)
    cfetch, _ = _pmc_mean(dirs[2], "FETCH_SIZE", "copy_kernel")
    cwrite, _ = _pmc_mean(dirs[3], "WRITE_SIZE", "copy_kernel")
    kf = copy_bytes / (cfetch * 1024.0)
    kw = copy_bytes / (cwrite * 1024.0)
    read_b = fetch * 1024.0 * kf
    write_b = write * 1024.0 * kw
    out = {
        "kernel": FUSED_KERNEL, "cells": n * n, "kernel_hash": kernel_hash(), "layout": LAYOUT,
        "fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write, "dispatches": [nf, nw],
        "copy_fetch_kib": cfetch, "copy_write_kib": cwrite, "copy_bytes_each_way": copy_bytes,
        "fetch_scale": kf, "write_scale": kw,
        "read_bytes_per_launch": read_b, "write_bytes_per_launch": write_b,
        "bytes_per_launch": read_b + write_b,
        "algorithmic_bytes_per_launch": BYTES_F32_FUSED * n * n,
        "commands": [
            " ".join(["rocprofv3 --pmc FETCH_SIZE -T -d <dir> -o fetch --output-format csv --",
                      "python bench.py --mode kernel --steps 3"] + lay),
            " ".join(["rocprofv3 --pmc WRITE_SIZE -T -d <dir> -o write --output-format csv --",
                      "python bench.py --mode kernel --steps 3"] + lay),
            "rocprofv3 --pmc FETCH_SIZE -T -d <dir> -o cfetch --output-format csv -- "
            "python bench.py --mode copy",
            "rocprofv3 --pmc WRITE_SIZE -T -d <dir> -o cwrite --output-format csv -- "
            "python bench.py --mode copy",
            " ".join(["python bench.py --traffic-from <fetch dir> <write dir> <copy fetch dir>",
                      "<copy write dir>"] + lay),
        ],
    }
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def main():
    global LAYOUT
    args = parse()
    LAYOUT = args.layout
    if args.traffic_from:
        assemble_traffic(args.traffic_from)
        return
    if args.cpu_full:
        print(json.dumps(cpu_full()), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design note, not a measured configuration.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_13618_amd import inputs, lks, workloads

    wl = workloads.SMOOTH_4096
    n = wl["nx"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    if args.mode == "copy":
        nbytes = 9 * n * n * 4
        a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        lks.copy_probe(b, a)
        torch.cuda.synchronize()
        s, e = ev(), ev()
        reps = 10
        s.record()
        for _ in range(reps):
            lks.copy_probe(b, a)
        e.record()
        torch.cuda.synchronize()
        t = s.elapsed_time(e) / reps * 1e-3
        print(json.dumps({"mode": "copy", "bytes_read": nbytes, "bytes_written": nbytes,
                          "GBps": 2 * nbytes / t / 1e9, "us": t * 1e6}))
        return

    rho, ux, uy = inputs.smooth_random(n, seed=wl["seed"], cutoff=wl["cutoff"])
    lat = lks.Lattice(9, n, n, "f32", tau=wl["tau"], thr=wl["thr"], flag_mask=wl["flag_mask"],
                      max_steps=max(args.steps, 1), layout=LAYOUT, device=dev)
    # the initial fields stay on the device: re-initialising the headline
    # state then needs no host transfer (no idle gap before the timed steps)
    fields = [torch.as_tensor(a, dtype=torch.float64).to(dev).contiguous() for a in (rho, ux, uy)]
    lat.init(*fields)

    if args.mode == "kernel":
        if args.workload != "smooth4096":
            del lat
            kernel_only(args, torch, lks, inputs, workloads, dev)
            return
        lat.step(args.steps)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "kernel", "steps": args.steps}))
        return

    # ---- the yardsticks first: the copy ceiling and the unfused passes (both
    #      part of the line) run before the headline.  A kernel trace from
    #      process start shows why: the first few launches run at full speed,
    #      then the chip's clocks dip (the fused step slows from 241 to
    #      ~315 us about 4 ms into sustained load) and recover over the next
    #      ~20 ms.  The two legs keep the GPU busy for ~35 ms, and the headline
    #      state is re-initialised on the device right after them, so its
    #      warm-up and timed steps run at the settled clock.
    copy_gbps = copy_ceiling(torch, lks, dev, ev, 9 * n * n * 4)
    lat.step(2, fused=False)
    torch.cuda.synchronize()
    ps = max(args.steps // 2, 10)
    t_plain = median_time(torch, ev, RUNS, lambda: lat.step(ps, fused=False)) / ps

    # ---- warmup, then the timed region: RUNS runs of exactly K fused steps on
    #      the library's stream (torch's current stream), the median reported
    lat.init(*fields)
    lat.step(args.warmup)
    torch.cuda.synchronize()
    run_times = []
    t_step = median_time(torch, ev, RUNS, lambda: lat.step(args.steps), out=run_times) / args.steps
    faults = lat.check()
    mlups = n * n / t_step / 1e6

    # ---- the fused kernel alone: back-to-back launches between the two
    #      state buffers, bracketed by events on the same stream, median of RUNS
    reps = max(args.steps, 10)
    src, dst = lat.pop[lat.current()[0]], lat.pop[1 - lat.current()[0]]
    lat.step_from(src, dst)
    torch.cuda.synchronize()

    def alone():
        for r in range(reps):
            lat.step_from(src, dst) if r % 2 == 0 else lat.step_from(dst, src)
    t_kernel = median_time(torch, ev, RUNS, alone) / reps
    achieved = BYTES_F32_FUSED * n * n / t_kernel / 1e9
    traffic = traffic_entry(n * n)

    regrid = time_regrid(torch, lks, lat, ev) if args.regrid else None

    out = {
        "metric": "MLUPS incl. sensor + achieved HBM GB/s (% roofline), fused FP32 vs plain",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 4),
        "ms_per_step_runs": [round(t / args.steps * 1e3, 4) for t in run_times],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "D2Q9 BGK 4096x4096 periodic, FP32 deviation storage, fused pull-stream "
                        "+ collide + S_KL/S_NEQ/S_PI + flags + FP64 sums, tau=0.52, smooth "
                        "random field (seed 0, 16 modes)",
            "grid": [n, n], "tau": wl["tau"], "lattice": "D2Q9", "layout": LAYOUT,
        },
        "achieved_GBps": round(BYTES_F32_FUSED * n * n / t_step / 1e9, 1),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "kernel": FUSED_KERNEL,
            "bytes_per_launch": BYTES_F32_FUSED * n * n,
            "kernel_us": round(t_kernel * 1e6, 2),
            "copy_GBps": round(copy_gbps, 1),
            "frac_of_copy": round(achieved / copy_gbps, 4),
        },
        "plain": {
            "MLUPS": round(n * n / t_plain / 1e6, 1),
            "ms_per_step": round(t_plain * 1e3, 4),
            "GBps_model": round(BYTES_F32_PLAIN * n * n / t_plain / 1e9, 1),
            "fused_speedup": round(t_plain / t_step, 3),
        },
        "positivity_faults": faults,
    }

    # the other forms: reported beside the headline on the same GPU
    legs = not args.headline_only
    del lat
    torch.cuda.empty_cache()
    if legs or args.forms:
        out["forms"] = time_forms(torch, lks, inputs, workloads, dev, ev)
    if legs or args.q25:
        out["q25"] = time_q25(torch, lks, inputs, workloads, dev, ev)
    if legs or args.ddf:
        out["ddf"] = time_ddf(torch, lks, inputs, workloads, dev, ev)
    if legs or args.adjoint:
        out["adjoint"] = time_adjoint(torch, lks, inputs, workloads, dev, ev)
    if args.ext:
        out["ext"] = time_ext(torch, lks, inputs, workloads, dev, ev)
    if args.fp64:
        out["fp64"] = time_fp64(torch, lks, inputs, workloads, dev, ev)
    if args.case3:
        out["case3"] = run_case3(torch, lks, inputs, dev, ev)
    if legs and not args.no_two_step:
        out["two_step"] = time_two_step(torch, lks, inputs, workloads, dev, ev)
    if regrid is not None:
        out["regrid"] = regrid

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps, rho, ux, uy, wl)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def time_regrid(torch, lks, lat, ev, b=2, ts=8, eff=0.98):
    """The regridding hand-off on the current flag map: buffer layer of b cells
    and tile counts on the device (HIP events on the library's stream), then
    the host clustering of the counts (wall clock), 2 buffer cells and 98 %
    efficiency as in the paper."""
    lv = lat.tag_buffer(b)
    counts = lat.tag_tiles(lv, 1, ts)
    torch.cuda.synchronize()
    reps = 20
    s, e = ev(), ev()
    s.record()
    for _ in range(reps):
        lat.tag_buffer(b, out=lv)
    e.record()
    torch.cuda.synchronize()
    t_buf = s.elapsed_time(e) / reps * 1e-3
    s.record()
    for _ in range(reps):
        lat.tag_tiles(lv, 1, ts, out=counts)
    e.record()
    torch.cuda.synchronize()
    t_tiles = s.elapsed_time(e) / reps * 1e-3
    c = counts.cpu().numpy()
    t0 = time.perf_counter()
    boxes = lks.cluster(c, lat.nx, lat.ny, ts, eff)
    t_cl = time.perf_counter() - t0
    cells = lat.nx * lat.ny
    area = sum((x1 - x0) * (y1 - y0) for x0, y0, x1, y1 in boxes)
    return {"buffer_us": round(t_buf * 1e6, 2), "buffer_GBps": round(2 * cells / t_buf / 1e9, 1),
            "tiles_us": round(t_tiles * 1e6, 2), "tiles_GBps": round(cells / t_tiles / 1e9, 1),
            "cluster_ms": round(t_cl * 1e3, 2), "boxes": len(boxes),
            "efficiency": round(float(c.sum()) / max(area, 1), 4), "b": b, "ts": ts, "eff": eff}


def copy_ceiling(torch, lks, dev, ev, nbytes):
    """Rate of the library's plain copy kernel over one population buffer's
    worth of bytes (read + write), GB/s."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    lks.copy_probe(b, a)
    torch.cuda.synchronize()
    s, e = ev(), ev()
    reps = 20
    s.record()
    for _ in range(reps):
        lks.copy_probe(b, a)
    e.record()
    torch.cuda.synchronize()
    t = s.elapsed_time(e) / reps * 1e-3
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / t / 1e9


EXT9 = ("kn", "hr", "sigma_h", "sigma_hkl", "alpha", "shear", "qh", "comp", "strain")
EXT25 = ("kn", "hr", "sigma_h", "sigma_hkl", "alpha", "shear", "qh", "qf")
EXTDDF = EXT25 + ("comp", "strain")


def ext_lattices(lks, inputs, workloads, dev, steps):
    """The two extension-sensor workloads, initialised: D2Q9 4096^2 FP32 with
    every D2Q9 extension sensor, D2Q25 2048^2 FP32 Riemann with every D2Q25
    one (thresholds as the base workloads, extension sensors not flagged)."""
    wl = workloads.SMOOTH_4096
    n = wl["nx"]
    rho, ux, uy = inputs.smooth_random(n, seed=wl["seed"], cutoff=wl["cutoff"])
    a = lks.Lattice(9, n, n, "f32", tau=wl["tau"], thr=wl["thr"], flag_mask=wl["flag_mask"],
                    max_steps=max(steps, 1), ext=EXT9, layout=LAYOUT, device=dev)
    a.init(rho, ux, uy)
    wq = workloads.RIEMANN_2048
    m = wq["nx"]
    rho, ux, uy, T, states = inputs.riemann_quadrants(m, seed=wq["seed"])
    dx = 1.0 / m
    b = lks.Lattice(25, m, m, "f32", mu=wq["mu"], dt=inputs.riemann_dt(states, dx), dx=dx,
                    bc=(1, 1), thr=wq["thr"], flag_mask=wq["flag_mask"], max_steps=max(steps, 1),
                    ext=EXT25, layout=LAYOUT, device=dev)
    b.init(rho, ux, uy, T)
    return a, b


def time_ext(torch, lks, inputs, workloads, dev, ev):
    """Fused steps with every extension sensor on (timing only): D2Q9, the
    single and the double distribution on D2Q25."""
    k = 40
    a, b = ext_lattices(lks, inputs, workloads, dev, k)
    c = ddf_lattice(lks, inputs, workloads, dev, k, ext=EXTDDF)
    res = {}
    for name, lat, nbytes in (("d2q9_4096_f32_ext9", a, 85 + 4 * len(EXT9)),
                              ("d2q25_2048_f32_ext8", b, 217 + 4 * len(EXT25)),
                              ("d2q25_ddf_2048_f32_ext10", c, BYTES_F32_DDF + 4 * len(EXTDDF))):
        warm_up(torch, lambda: lat.step(1))
        t = median_time(torch, ev, RUNS, lambda: lat.step(k)) / k
        cells = lat.nx * lat.ny
        res[name] = {"MLUPS": round(cells / t / 1e6, 1), "us_per_step": round(t * 1e6, 1),
                     "GBps_model": round(nbytes * cells / t / 1e9, 1), "bytes_per_lup": nbytes,
                     "faults": lat.check()}
    del a, b, c
    torch.cuda.empty_cache()
    return res


def ddf_lattice(lks, inputs, workloads, dev, steps, ext=None):
    """The double-distribution workload, initialised (FP32 storage), with the
    extension sensors `ext` if given."""
    wl = workloads.RIEMANN_2048_DDF
    n = wl["nx"]
    rho, ux, uy, T, states = inputs.riemann_quadrants(n, seed=wl["seed"])
    dx = 1.0 / n
    lat = lks.Lattice(25, n, n, "f32", mu=wl["mu"], dt=inputs.riemann_dt(states, dx, gamma=wl["gamma"]),
                      dx=dx, bc=(1, 1), thr=wl["thr"], flag_mask=wl["flag_mask"],
                      max_steps=max(steps, 1), model="ddf", gamma=wl["gamma"],
                      prandtl=wl["prandtl"], thr_qe=wl["thr_qe"], ext=ext, layout=LAYOUT, device=dev)
    lat.init(rho, ux, uy, T)
    return lat


def q25_lattice(lks, inputs, workloads, dev, steps):
    """The single-distribution D2Q25 Riemann workload, initialised (FP32)."""
    wl = workloads.RIEMANN_2048
    n = wl["nx"]
    rho, ux, uy, T, states = inputs.riemann_quadrants(n, seed=wl["seed"])
    dx = 1.0 / n
    lat = lks.Lattice(25, n, n, "f32", mu=wl["mu"], dt=inputs.riemann_dt(states, dx), dx=dx,
                      bc=(1, 1), thr=wl["thr"], flag_mask=wl["flag_mask"], max_steps=max(steps, 1),
                      layout=LAYOUT, device=dev)
    lat.init(rho, ux, uy, T)
    return lat


def time_ddf(torch, lks, inputs, workloads, dev, ev):
    """Fused double-distribution steps (timing only)."""
    k = 40
    return time_d2q25(torch, ev, ddf_lattice(lks, inputs, workloads, dev, k), k,
                      workloads.RIEMANN_2048_DDF["name"], DDF_KERNEL, BYTES_F32_DDF)


def time_q25(torch, lks, inputs, workloads, dev, ev):
    """Fused single-distribution D2Q25 steps (timing only)."""
    k = 40
    return time_d2q25(torch, ev, q25_lattice(lks, inputs, workloads, dev, k), k,
                      workloads.RIEMANN_2048["name"], Q25_KERNEL, BYTES_F32_Q25)


def time_d2q25(torch, ev, lat, k, name, kernel, bpl):
    """Whole steps, then the step kernel(s) alone between the two state buffers
    (after untimed steps that let the clocks settle)."""
    warm_up(torch, lambda: lat.step(1))
    t = median_time(torch, ev, RUNS, lambda: lat.step(k)) / k
    src, dst = lat.pop[lat.current()[0]], lat.pop[1 - lat.current()[0]]

    def alone():
        for r in range(k):
            lat.step_from(src, dst) if r % 2 == 0 else lat.step_from(dst, src)
    tk = median_time(torch, ev, RUNS, alone) / k
    cells = lat.nx * lat.ny
    res = {"workload": name, "MLUPS": round(cells / t / 1e6, 1),
           "us_per_step": round(t * 1e6, 1), "kernel": kernel, "kernel_us": round(tk * 1e6, 1),
           "bytes_per_lup": bpl,
           "GBps_model": round(bpl * cells / tk / 1e9, 1),
           "frac_hbm": round(bpl * cells / tk / 1e9 / HBM_PEAK_GBPS, 4),
           "faults": lat.check()}
    del lat
    torch.cuda.empty_cache()
    return res


def kernel_only(args, torch, lks, inputs, workloads, dev):
    """A short run of one of the other workloads (for profilers)."""
    if args.workload == "riemann2048-ddf-ext":
        ddf_lattice(lks, inputs, workloads, dev, args.steps, ext=EXTDDF).step(args.steps)
    elif args.workload.endswith("-ext"):
        a, b = ext_lattices(lks, inputs, workloads, dev, args.steps)
        (a if args.workload.startswith("smooth") else b).step(args.steps)
    elif args.workload == "riemann2048-ddf":
        ddf_lattice(lks, inputs, workloads, dev, args.steps).step(args.steps)
    elif args.workload == "riemann2048":
        wl = workloads.RIEMANN_2048
        n = wl["nx"]
        rho, ux, uy, T, states = inputs.riemann_quadrants(n, seed=wl["seed"])
        dx = 1.0 / n
        lat = lks.Lattice(25, n, n, "f32", mu=wl["mu"], dt=inputs.riemann_dt(states, dx), dx=dx,
                          bc=(1, 1), thr=wl["thr"], flag_mask=wl["flag_mask"],
                          max_steps=max(args.steps, 1), layout=LAYOUT, device=dev)
        lat.init(rho, ux, uy, T)
        lat.step(args.steps)
    elif args.workload.endswith("-two"):
        wl = workloads.SMOOTH_4096 if args.workload.startswith("smooth4096") else workloads.SMOOTH_8192
        n = wl["nx"]
        rho, ux, uy = inputs.smooth_random(n, seed=wl["seed"], cutoff=wl["cutoff"])
        lat = lks.Lattice(9, n, n, "f32", tau=wl["tau"], thr=wl["thr"] or workloads.SMOOTH_4096["thr"],
                          flag_mask=wl["flag_mask"], max_steps=max(args.steps, 1), layout=LAYOUT,
                          launch_steps=2, device=dev)
        lat.init(rho, ux, uy)
        lat.step(args.steps)
    elif args.workload.startswith("smooth8192"):
        wl = workloads.SMOOTH_8192
        n = wl["nx"]
        rho, ux, uy = inputs.smooth_random(n, seed=wl["seed"], cutoff=wl["cutoff"])
        lat = lks.Lattice(9, n, n, args.workload.split("-")[1], tau=wl["tau"], thr=wl["thr"],
                          flag_mask=wl["flag_mask"], max_steps=max(args.steps, 1), layout=LAYOUT, device=dev)
        lat.init(rho, ux, uy)
        lat.step(args.steps)
    else:
        from paper_2603_13618_amd import adjoint
        wl = workloads.ADJOINT_1024
        n = wl["nx"]
        rho, ux, uy = inputs.smooth_random(n, seed=wl["seed"], cutoff=wl["cutoff"])
        u = torch.tensor(ux, device=dev, requires_grad=True)
        v = torch.tensor(uy, device=dev, requires_grad=True)
        L = adjoint.kl_sensor_loss(u, v, torch.tensor(rho, device=dev), tau=wl["tau"],
                                   nsteps=args.steps, checkpoint=wl["checkpoint"], dtype="f32",
                                   layout=LAYOUT)
        L.backward()
    torch.cuda.synchronize()
    print(json.dumps({"mode": "kernel", "workload": args.workload, "steps": args.steps}))


def time_two_step(torch, lks, inputs, workloads, dev, ev, k=32, rounds=RUNS):
    """Two fused steps per launch (launch_steps = 2) against one, FP32 on the
    smooth 4096^2 and 8192^2 fields: each form warmed up, then timed in
    alternating runs of k steps, median run of each (the headline's
    statistic)."""
    res = {}
    for wl in (workloads.SMOOTH_4096, workloads.SMOOTH_8192):
        n = wl["nx"]
        rho, ux, uy = inputs.smooth_random(n, seed=wl["seed"], cutoff=wl["cutoff"])
        lats = {}
        for ls in (0, 2):
            lat = lks.Lattice(9, n, n, "f32", tau=wl["tau"], thr=wl["thr"] or workloads.SMOOTH_4096["thr"],
                              flag_mask=wl["flag_mask"], max_steps=64, layout=LAYOUT, launch_steps=ls,
                              device=dev)
            lat.init(rho, ux, uy)
            lat.step(60)
            lats[ls] = lat
        torch.cuda.synchronize()
        times = {0: [], 2: []}
        for _ in range(rounds):
            for ls, lat in lats.items():
                median_time(torch, ev, 1, lambda: lat.step(k), out=times[ls])
        med = {ls: sorted(t)[len(t) // 2] / k for ls, t in times.items()}
        res[f"f32_{n}"] = {"grid": [n, n],
                           "one_step": {"MLUPS": round(n * n / med[0] / 1e6, 1),
                                        "us_per_step": round(med[0] * 1e6, 1)},
                           "two_step": {"MLUPS": round(n * n / med[2] / 1e6, 1),
                                        "us_per_step": round(med[2] * 1e6, 1)},
                           "speedup": round(med[0] / med[2], 3)}
        del lats, lat
        torch.cuda.empty_cache()
    return res


def time_fp64(torch, lks, inputs, workloads, dev, ev):
    """FP64 storage and arithmetic: the fused D2Q9 step on the 4096^2 smooth
    field (whole steps and the kernel alone) and the double distribution on
    the 2048^2 Riemann quadrants (whole steps), medians of RUNS."""
    res = {}
    wl = workloads.SMOOTH_4096
    n = wl["nx"]
    rho, ux, uy = inputs.smooth_random(n, seed=wl["seed"], cutoff=wl["cutoff"])
    lat = lks.Lattice(9, n, n, "f64", tau=wl["tau"], thr=wl["thr"], flag_mask=wl["flag_mask"], max_steps=32,
                      layout=LAYOUT, device=dev)
    lat.init(rho, ux, uy)
    warm_up(torch, lambda: lat.step(1))
    k = 16
    t = median_time(torch, ev, RUNS, lambda: lat.step(k)) / k
    src, dst = lat.pop[lat.current()[0]], lat.pop[1 - lat.current()[0]]

    def alone():
        for r in range(k):
            lat.step_from(src, dst) if r % 2 == 0 else lat.step_from(dst, src)
    tk = median_time(torch, ev, RUNS, alone) / k
    res["d2q9_f64_4096"] = {"MLUPS": round(n * n / t / 1e6, 1), "us_per_step": round(t * 1e6, 1),
                            "kernel_us": round(tk * 1e6, 1), "bytes_per_lup": 169,
                            "GBps_model": round(169 * n * n / tk / 1e9, 1)}
    del lat
    torch.cuda.empty_cache()
    wq = workloads.RIEMANN_2048_DDF
    n = wq["nx"]
    r, u, v, T, states = inputs.riemann_quadrants(n, seed=wq["seed"])
    dx = 1.0 / n
    lat = lks.Lattice(25, n, n, "f64", mu=wq["mu"], dt=inputs.riemann_dt(states, dx, gamma=wq["gamma"]), dx=dx,
                      bc=(1, 1), max_steps=32, model="ddf", gamma=wq["gamma"], prandtl=wq["prandtl"],
                      layout=LAYOUT, device=dev)
    lat.init(r, u, v, T)
    warm_up(torch, lambda: lat.step(1))
    k = 8
    t = median_time(torch, ev, RUNS, lambda: lat.step(k)) / k
    res["ddf_f64_2048"] = {"MLUPS": round(n * n / t / 1e6, 1), "us_per_step": round(t * 1e6, 1),
                           "bytes_per_lup": 841, "GBps_model": round(841 * n * n / t / 1e9, 1)}
    del lat
    torch.cuda.empty_cache()
    return res


def run_case3(torch, lks, inputs, dev, ev, n=1024, mu=1e-3, gamma=1.4, prandtl=0.71, t_end=0.85):
    """The paper's modified Riemann problem No. 3 (Sec. IV): air, mu = 1e-3,
    CFL 0.01, outflow edges, from the initial quadrants to t_end, FP32 double
    distribution.  Whole run timed with HIP events (sums reduced every 64
    steps); the final state summarised: ranges, positivity faults, x <-> y
    asymmetry, and the kinetic class-1 sensors against the macroscopic ones."""
    import numpy as np
    fields = inputs.riemann_case3(n)
    dx = 1.0 / n
    dt = inputs.cfl_dt(fields, dx, gamma)
    steps = int(round(t_end / dt))
    lat = lks.Lattice(25, n, n, "f32", mu=mu, dt=dt, dx=dx, bc=(1, 1), max_steps=64, model="ddf",
                      gamma=gamma, prandtl=prandtl, layout=LAYOUT, device=dev)
    lat.init(*fields)
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record()
    lat.step(steps - 1)
    b.record()
    torch.cuda.synchronize()
    t = a.elapsed_time(b) * 1e-3
    m = [x.clone() for x in lat.moments()]
    lat.step(1)
    mac = lat.macro_sensors(*m, mu=mu, lam=-(gamma - 1.0) * mu, kappa=gamma / (gamma - 1.0) * mu / prandtl,
                            which=("tau", "qnsf"))
    r, ux, uy, T = (x.double().cpu().numpy() for x in m)
    s = lat.sensors.double().cpu().numpy()

    def med(k, name):
        q = mac[name].cpu().numpy()
        keep = q > 1e-3 * q.max()
        return round(float(np.median(s[k][keep] / q[keep])), 4)
    res = {"workload": "modified 2D Riemann problem No. 3, D2Q25 double distribution FP32, air "
                       f"(gamma={gamma}, Pr={prandtl}), mu={mu}, {n}x{n} outflow, CFL 0.01, t_end={t_end}",
           "steps": steps, "s": round(t, 3), "MLUPS": round(n * n * (steps - 1) / t / 1e6, 1),
           "us_per_step": round(t / (steps - 1) * 1e6, 2),
           "rho": [round(float(r.min()), 4), round(float(r.max()), 4)],
           "T": [round(float(T.min()), 4), round(float(T.max()), 4)],
           "fault_cells_last_step": int((lat.flags >= 128).sum()),
           "asymmetry_rho": float(np.abs(r - r.T).max() / r.max()),
           "S_PI_over_tau_NS_median": med(2, "tau"), "S_Q_over_q_NSF_median": med(3, "qnsf"),
           "sensor_p50_p99": {nm: [float(np.percentile(s[k][np.isfinite(s[k])], p)) for p in (50, 99)]
                              for k, nm in enumerate(("S_KL", "S_NEQ", "S_PI", "S_Q", "S_QE"))}}
    del lat
    torch.cuda.empty_cache()
    return res


def time_adjoint(torch, lks, inputs, workloads, dev, ev):
    """The differentiation workload (D2Q9 1024^2 FP32, 200 steps, checkpoint
    every 20): the forward run keeping checkpoints plus the backward pass
    (segment recompute and the hand-written adjoint kernels) behind
    torch.autograd, median of RUNS after one untimed pass."""
    from paper_2603_13618_amd import adjoint
    wl = workloads.ADJOINT_1024
    n, steps, K = wl["nx"], wl["steps"], wl["checkpoint"]
    rho, ux, uy = inputs.smooth_random(n, seed=wl["seed"], cutoff=wl["cutoff"])
    r = torch.tensor(rho, device=dev)
    u0, v0 = torch.tensor(ux, device=dev), torch.tensor(uy, device=dev)

    def run():
        u, v = u0.clone().requires_grad_(True), v0.clone().requires_grad_(True)
        L = adjoint.kl_sensor_loss(u, v, r, tau=wl["tau"], nsteps=steps, checkpoint=K, dtype="f32",
                                   layout=LAYOUT)
        L.backward()
    warm_up(torch, run)
    t = median_time(torch, ev, RUNS, run)
    return {"workload": wl["name"], "ms_forward_backward": round(t * 1e3, 3),
            "steps": steps, "checkpoint": K,
            "MLUPS_forward_equivalent": round(n * n * steps / t / 1e6, 1)}


def time_forms(torch, lks, inputs, workloads, dev, ev):
    """BF16 / FP16 deviation storage on the 8192^2 smooth field (timing only)."""
    wl = workloads.SMOOTH_8192
    n = wl["nx"]
    rho, ux, uy = inputs.smooth_random(n, seed=wl["seed"], cutoff=wl["cutoff"])
    res = {}
    for dtype, nbytes in (("bf16", 49), ("f16", 49), ("f32", 85)):
        lat = lks.Lattice(9, n, n, dtype, tau=wl["tau"], thr=wl["thr"] or workloads.SMOOTH_4096["thr"],
                          flag_mask=wl["flag_mask"], max_steps=64, layout=LAYOUT, device=dev)
        lat.init(rho, ux, uy)
        warm_up(torch, lambda: lat.step(1))
        k = 40
        t = median_time(torch, ev, RUNS, lambda: lat.step(k)) / k
        res[dtype] = {"MLUPS": round(n * n / t / 1e6, 1), "GBps_model": round(nbytes * n * n / t / 1e9, 1),
                      "bytes_per_lup": nbytes, "grid": [n, n]}
        del lat
        torch.cuda.empty_cache()
    return res


def host_threads():
    """Cores this process may use (affinity mask, capped by OMP_NUM_THREADS)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cap = os.environ.get("OMP_NUM_THREADS", "")
    if cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(n, 1)


def cpu_model():
    """The host CPU's model name (/proc/cpuinfo), or the platform string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(steps, rho, ux, uy, wl, steps_1thread=2):
    """The FP64 oracle on the host cores: the full 4096^2 grid for a few steps
    on every core this process may use, then on one thread, plus the whole
    128^2 double-shear-layer run (500 steps) on every core."""
    import oracle
    from paper_2603_13618_amd import inputs
    threads = host_threads()
    f0 = oracle.equilibrium(9, rho, ux, uy)
    oracle.run(9, f0, 1, tau=wl["tau"], nthreads=threads)          # page-in
    t0 = time.perf_counter()
    oracle.run(9, f0, steps, tau=wl["tau"], thr=wl["thr"], mask=wl["flag_mask"], nthreads=threads)
    t = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.run(9, f0, steps_1thread, tau=wl["tau"], thr=wl["thr"], mask=wl["flag_mask"], nthreads=1)
    t1 = time.perf_counter() - t0
    del f0
    r1, u1, v1 = inputs.double_shear_layer(128)
    g0 = oracle.equilibrium(9, r1, u1, v1)
    t0 = time.perf_counter()
    oracle.run(9, g0, 500, tau=0.55, nthreads=threads)
    tc1 = time.perf_counter() - t0
    n = rho.size
    return {"value": round(n * steps / t / 1e6, 2), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"FP64 C oracle (OpenMP), full {rho.shape[1]}x{rho.shape[0]} grid, {steps} "
                      f"steps of the same workload, {t:.1f} s",
            "cpu_model": cpu_model(),
            "value_1thread": round(n * steps_1thread / t1 / 1e6, 2),
            "sample_1thread": f"the same grid, {steps_1thread} steps on one thread, {t1:.1f} s",
            "double_shear_128": {"MLUPS": round(128 * 128 * 500 / tc1 / 1e6, 2), "cores": threads,
                                 "sample": f"128x128 D2Q9 FP64, tau 0.55, all 500 steps, {tc1:.2f} s"}}


def cpu_full():
    """The FP64 oracle on each workload, on every core this process may use
    and on one thread: the whole double shear layer (128^2, 500 steps) and
    bounded samples of the others (the full grid for a few steps)."""
    import oracle
    from paper_2603_13618_amd import inputs, workloads
    threads = host_threads()
    res = {"cpu_model": cpu_model(), "cores": threads, "kind": "oracle", "unit": "MLUPS"}

    def rate(name, cells, runs):
        out = {}
        for label, nthr, steps, fn in runs:
            fn(1, nthr)                                  # page-in
            t0 = time.perf_counter()
            fn(steps, nthr)
            t = time.perf_counter() - t0
            out[label] = {"MLUPS": round(cells * steps / t / 1e6, 3), "steps": steps, "s": round(t, 2)}
        res[name] = out

    r, u, v = inputs.double_shear_layer(128)
    f1 = oracle.equilibrium(9, r, u, v)
    rate("double_shear_128_d2q9", 128 * 128,
         [(f"{threads}_threads", threads, 500, lambda k, t: oracle.run(9, f1, k, tau=0.55, nthreads=t)),
          ("1_thread", 1, 500, lambda k, t: oracle.run(9, f1, k, tau=0.55, nthreads=t))])
    for wl, k_all, k_one in ((workloads.SMOOTH_4096, 20, 2), (workloads.SMOOTH_8192, 5, 1)):
        n = wl["nx"]
        r, u, v = inputs.smooth_random(n, seed=wl["seed"], cutoff=wl["cutoff"])
        f = oracle.equilibrium(9, r, u, v)
        del r, u, v
        rate(f"smooth_{n}_d2q9", n * n,
             [(f"{threads}_threads", threads, k_all, lambda k, t: oracle.run(9, f, k, tau=wl["tau"], nthreads=t)),
              ("1_thread", 1, k_one, lambda k, t: oracle.run(9, f, k, tau=wl["tau"], nthreads=t))])
        del f
    wq = workloads.RIEMANN_2048
    n = wq["nx"]
    r, u, v, T, states = inputs.riemann_quadrants(n, seed=wq["seed"])
    dx = 1.0 / n
    dt = inputs.riemann_dt(states, dx)
    f = oracle.equilibrium(25, r, u, v, T)
    rate(f"riemann_{n}_d2q25", n * n,
         [(f"{threads}_threads", threads, 4,
           lambda k, t: oracle.run(25, f, k, mu=wq["mu"], dt=dt, dx=dx, bc=(1, 1), nthreads=t)),
          ("1_thread", 1, 1, lambda k, t: oracle.run(25, f, k, mu=wq["mu"], dt=dt, dx=dx, bc=(1, 1), nthreads=t))])
    return res


if __name__ == "__main__":
    main()
