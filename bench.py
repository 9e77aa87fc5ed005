#!/usr/bin/env python3
"""Throughput of the photon-package life cycle on one MI355X.

Workload: the edge-on spiral -- stellar exponential disk (h_R 4, h_z 0.4
kpc) in a dust exponential disk (h_R 6, h_z 0.25 kpc, face-on V-band tau 1)
on 256x256x64 cells over +-20 x +-20 x +-2 kpc, albedo 0.6, g 0.6, three
512x512 frames at 0/60/90 degrees, 1e7 packages, FP32 traversal with FP64
package state and tallies.  One step is the whole hot path once: the
forward run (emission, peel-off, continuous absorption, forced scattering,
HG scattering, tallies) and the path-replay adjoint of an L2 image loss
against a fixed target image (rendered once, before timing, from a
perturbed density).  Inputs are resident on the device before timing.

Prints one JSON line.  `value` is packages per second of whole steps;
`roofline` describes the life-cycle kernel (forward or adjoint) that takes
the larger share of the step, per launch (HIP events around it on the
stream it runs on, recorded by the library); `rooflines` gives both;
`traversal` is the walk alone (trace_path on random rays in the same grid);
`fp64_path` times one step of the plain FP64 GPU path and compares the two
precisions against the Monte Carlo noise; `powcub_grid` and `kdtree_grid`
time one step of the same model on a PowCub grid (rectilinear, cells graded
towards the centre) and on a k-d tree grid adapted to the dust;
`panchromatic` times one panchromatic step of the multiwavelength disk (the
stellar run over 100 wavelengths with the absorbed tally, the dust's
equilibrium temperatures and re-emission, the dust run from the cells);
`cpu_baseline` times the FP64 CPU oracle on a bounded package sample of the
same workload.

`--collect-profiles DIR` runs this script under rocprofv3 (a kernel-trace
summary, then FETCH_SIZE and WRITE_SIZE counter passes with a 1 GiB copy
for calibration) as child processes and writes the summaries to profiles/.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "photon packages/sec (with peel-off) and cell-crossings/s vs HBM/L2 roofline"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes (what the method moves, not what line-granular hardware
# moves): one density value per cell crossing that reads it, one FP64
# read-modify-write (8 B read + 8 B written) per tally deposit and per
# forward peel-off contribution into a frame, one FP64 read of dL/dI per
# adjoint peel-off contribution; a traversal ray reads its origin and
# direction (48 B) and writes its optical depth (8 B).
BYTES_PER_CROSSING = {0: 8, 1: 4}
BYTES_PER_DEPOSIT = 16
BYTES_PER_PEEL_FORWARD = 16
BYTES_PER_PEEL_ADJOINT = 8
BYTES_PER_RAY = 56
COPY_BYTES = 1 << 30
# kernel names as rocprofv3 prints them -> keys of profiles/traffic.json
KERNELS = {
    "forward": "void mcrt::k_life<float, false, 0, false>(mcrt::RunParams)",
    "adjoint": "void mcrt::k_life<float, true, 0, false>(mcrt::RunParams)",
    "peel_tau_forward": "void mcrt::k_peeltau<float, false, 0, false>(mcrt::PeelJobParams)",
    "peel_tau_adjoint": "void mcrt::k_peeltau<float, true, 0, false>(mcrt::PeelJobParams)",
    "peel_deposit": "void mcrt::k_peeldep<float, 0, false>(mcrt::PeelJobParams)",
    "trace": "void mcrt::k_trace<float, 0>(mcrt::TraceParams)",
}


def source_hash():
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1410_1629_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(key):
    """Hardware HBM bytes per launch of a kernel from the committed counter
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
    except ValueError:
        return None
    k = rec.get("kernels", {}).get(key)
    if not k or rec.get("source_hash") != source_hash():
        return None
    return k.get("hbm_bytes_per_launch")


def life_bytes(st, prec, adjoint):
    """Algorithmic bytes of the life-cycle kernel of one call (the queued
    peel-ray walks of the adjoint run in their own kernels and are excluded)."""
    x = st["x_path"] + st["x_locate"] + st["x_peel"] - st["x_queue"]
    peel = BYTES_PER_PEEL_ADJOINT if adjoint else BYTES_PER_PEEL_FORWARD
    return x * BYTES_PER_CROSSING[prec] + (st["deposits"] - st["d_queue"]) * BYTES_PER_DEPOSIT + st["peels"] * peel


def rel_l1(a, b):
    den = b.abs().sum().item()
    return (a - b).abs().sum().item() / den if den > 0 else float("nan")


def cpu_baseline(prob, seconds):
    """FP64 oracle (forward run + gradient) on the first packages of the
    workload, sized to take about `seconds` on the host cores."""
    import numpy as np

    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS") or 0) or len(os.sched_getaffinity(0))
    adj = np.random.default_rng(0).standard_normal((1, 1, sum(d["nx"] * d["ny"] for d in prob["detectors"])))

    def timed(n):
        p = dict(prob, n_packages=n, first_package=0)
        t0 = time.perf_counter()
        oracle.run(p, threads=threads)
        oracle.grad(p, adj, threads=threads)
        return time.perf_counter() - t0

    n, t = max(200, 50 * threads), 0.0
    while True:  # grow the sample until it takes a second, then size it to the target
        t = timed(n)
        if t >= 1.0 or n >= 2_000_000:
            break
        n *= 4
    if t < seconds and n < 2_000_000:
        n = int(min(n * seconds / max(t, 1e-3), 2_000_000))
        t = timed(n)
    return {"value": n / t, "unit": "packages/s", "cores": threads, "kind": "oracle",
            "sample": "first %d packages of the same workload, FP64 forward run + gradient, %.1f s" % (n, t)}


def traversal(B, prob, n_rays, dev):
    """trace_path over random rays in the workload's grid: origins uniform in
    the box, isotropic directions, optical depth only."""
    import torch
    g = torch.Generator(device=dev)
    g.manual_seed(11)
    box = prob["box"]
    lo = torch.tensor([box[0], box[2], box[4]], dtype=torch.float64, device=dev)
    hi = torch.tensor([box[1], box[3], box[5]], dtype=torch.float64, device=dev)
    o = lo + (hi - lo) * torch.rand((n_rays, 3), generator=g, dtype=torch.float64, device=dev)
    k = torch.randn((n_rays, 3), generator=g, dtype=torch.float64, device=dev)
    k /= k.norm(dim=1, keepdim=True)
    rho = B.density_tensor(prob, dev)
    tau = torch.empty(n_rays, dtype=torch.float64, device=dev)
    x = B.trace_path(prob, rho, 1.0, prob["precision"], o, k, tau)
    reps = 5
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        B.trace_path(prob, rho, 1.0, prob["precision"], o, k, tau, crossings=False)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    alg = x * BYTES_PER_CROSSING[prob["precision"]] + n_rays * BYTES_PER_RAY
    achieved = alg / (ms / 1e3) / 1e9
    hw = traffic_for("trace")
    out = {"kernel": KERNELS["trace"], "rays": n_rays, "ms": ms, "crossings": x,
           "crossings_per_s": x / (ms / 1e3), "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": hw,
           "note": "ms covers the call (bricking the densities plus the walk kernel)"}
    if hw:
        out["hardware_gbs"] = hw / (ms / 1e3) / 1e9
        out["hardware_frac"] = out["hardware_gbs"] / HBM_PEAK_GBS
    return out


def fp64_comparison(B, prob, step_fn, images32, grad32, dev):
    """One step of the plain FP64 GPU path on the same packages; its
    difference from the FP32 path next to the Monte Carlo noise of the
    images (half the relative L1 difference of the two halves of the
    package range, about the noise of the full run)."""
    import torch
    p64 = dict(prob, precision=0)
    rho64 = B.density_tensor(p64, dev)
    images = torch.empty_like(images32)
    grad = torch.empty_like(grad32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sf, sb = step_fn(p64, rho64, images, grad)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    half = prob["n_packages"] // 2
    ia = torch.empty_like(images32)
    ib = torch.empty_like(images32)
    rho32 = B.density_tensor(prob, dev)
    B.run_photons(dict(prob, n_packages=half), rho32, ia, None, flags=prob["flags"] & ~B.ABSORB)
    B.run_photons(dict(prob, n_packages=prob["n_packages"] - half, first_package=half), rho32, ib, None,
                  flags=prob["flags"] & ~B.ABSORB)
    return {"packages_per_s": prob["n_packages"] / wall, "ms_per_step": wall * 1e3,
            "forward_ms": sf["kernel_ms"], "adjoint_ms": sb["kernel_ms"],
            "images_rel_l1_fp32_vs_fp64": rel_l1(images32, images),
            "gradient_rel_l1_fp32_vs_fp64": rel_l1(grad32, grad),
            "images_mc_noise_rel_l1": 0.5 * rel_l1(ia, ib)}


def grid_leg(B, prob, target, dev, note):
    """One step (forward + adjoint against the benchmark's target image) of
    the same model on another grid kind, after one untimed step: the
    rectilinear- or tree-grid kernels at the benchmark's package count."""
    import torch
    rho = B.density_tensor(prob, dev)
    images = torch.empty_like(target)
    adj = torch.empty_like(target)
    absorbed = torch.empty((1, rho.numel()), dtype=torch.float64, device=dev)
    grad = torch.empty(rho.numel(), dtype=torch.float64, device=dev)

    def step():
        sf = B.run_photons(prob, rho, images, absorbed)
        torch.sub(images, target, out=adj)
        adj.mul_(2.0)
        sb = B.backward_density(prob, rho, adj, grad)
        return sf, sb

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sf, sb = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_pkg = prob["n_packages"]
    x = sf["x_path"] + sf["x_locate"] + sf["x_peel"] + sb["x_path"] + sb["x_locate"] + sb["x_peel"]
    return {"workload": "%s, %s, %d packages" % (prob["name"], note, n_pkg), "cells": int(rho.numel()),
            "packages_per_s": n_pkg / wall, "ms_per_step": wall * 1e3, "forward_ms": sf["kernel_ms"],
            "adjoint_ms": sb["kernel_ms"], "crossings_per_s": x / wall}


def panchromatic_leg(B, dev, n_per_lambda=1_000_000):
    """One panchromatic step, after one untimed step: stellar run with the
    absorbed tally -> dust_emission -> dust run from the cells, all 100
    wavelengths, n_per_lambda packages per wavelength in each run."""
    import numpy as np
    import torch
    from paper_1410_1629_amd import workloads as W
    prob, dust = W.panchromatic(n_packages=n_per_lambda)
    rho = B.density_tensor(prob, dev)
    ncell, nl = rho.numel(), len(prob["kappa"])
    images = torch.empty(B.image_shape(prob), dtype=torch.float64, device=dev)
    absorbed = torch.empty((nl, ncell), dtype=torch.float64, device=dev)
    em = torch.empty((nl, ncell), dtype=torch.float64, device=dev)
    T = torch.empty(ncell, dtype=torch.float64, device=dev)
    dprob = W.dust_problem(prob, em)
    dimages = torch.empty(B.image_shape(dprob), dtype=torch.float64, device=dev)
    dabs = torch.empty((nl, ncell), dtype=torch.float64, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def step():
        s1 = B.run_photons(prob, rho, images, absorbed)
        ev[0].record()
        B.dust_emission(prob, rho, prob["precision"], absorbed, dust["lambda"], dust["dlambda"], dust["kappa_abs"],
                        dust["emissivity"], em, T)
        ev[1].record()
        s2 = B.run_photons(dprob, rho, dimages, dabs)
        return s1, s2

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s1, s2 = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    Tn = T.cpu().numpy()
    tally = absorbed.sum().item()
    items = s1["packages"] + s2["packages"]
    return {"workload": "%s: stellar run, dust emission (modified black bodies), dust run; %d wavelengths, %d packages "
                        "per wavelength per run" % (prob["name"], nl, n_per_lambda),
            "cells": int(ncell), "packages_per_s": items / wall, "ms_per_step": wall * 1e3,
            "stellar_ms": s1["kernel_ms"], "dust_emission_ms": ev[0].elapsed_time(ev[1]), "dust_run_ms": s2["kernel_ms"],
            "absorbed_fraction": s1["absorbed"] / s1["emitted"],
            "reemitted_over_absorbed_tally": s2["emitted"] / tally,
            "dust_T_median_K": float(np.median(Tn[Tn > 0])), "dust_T_max_K": float(Tn.max())}


def collect_profiles(out_dir, prof, run=True):
    """Runs this script under rocprofv3 as child processes (this process
    never touches the GPU) and writes the summaries to `prof` (profiles/);
    run=False only summarizes the raw output already in out_dir."""
    os.makedirs(out_dir, exist_ok=True)
    me = os.path.abspath(__file__)
    child = [sys.executable, me, "--steps", "2", "--warmup", "1", "--no-cpu-baseline", "--no-fp64", "--no-powcub",
             "--no-panchromatic"]
    runs = {
        "trace": ["rocprofv3", "--kernel-trace", "--stats", "--output-format", "csv"],
        "fetch": ["rocprofv3", "--kernel-trace", "--output-format", "csv", "--pmc", "FETCH_SIZE"],
        "write": ["rocprofv3", "--kernel-trace", "--output-format", "csv", "--pmc", "WRITE_SIZE"],
    }
    for name, cmd in (runs.items() if run else ()):
        extra = ["--calibrate-copy"] if name != "trace" else []
        full = cmd + ["-d", os.path.join(out_dir, name), "-o", name, "--"] + child + extra
        print("[profile] " + " ".join(full), flush=True)
        r = subprocess.run(["timeout", "-k", "10", "300"] + full)
        if r.returncode != 0:
            print("[profile] %s pass failed with status %d" % (name, r.returncode), flush=True)
            sys.exit(r.returncode)

    def dispatches(name):
        f = glob.glob(os.path.join(out_dir, name, "**", "*counter_collection.csv"), recursive=True)[0]
        agg = {}
        for r in csv.DictReader(open(f)):
            key = int(r["Dispatch_Id"])
            a = agg.setdefault(key, {"kernel": r["Kernel_Name"], "value": 0.0})
            a["value"] += float(r["Counter_Value"])
        return [agg[k] for k in sorted(agg)]

    factors = {}
    per_kernel = {}
    for name, counter in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        ds = dispatches(name)
        copy = ds[0]  # the calibration copy is the first kernel of the child process
        # the copy reads and writes COPY_BYTES once; counters are in KiB
        factors[counter] = COPY_BYTES / (copy["value"] * 1024.0)
        for key, kname in KERNELS.items():
            vals = [d["value"] for d in ds if d["kernel"] == kname]
            if vals:
                per_kernel.setdefault(key, {})[counter + "_kib_per_dispatch"] = sum(vals) / len(vals)
    kernels = {}
    for key, v in per_kernel.items():
        if "FETCH_SIZE_kib_per_dispatch" in v and "WRITE_SIZE_kib_per_dispatch" in v:
            b = 1024.0 * (v["FETCH_SIZE_kib_per_dispatch"] * factors["FETCH_SIZE"] +
                          v["WRITE_SIZE_kib_per_dispatch"] * factors["WRITE_SIZE"])
            kernels[key] = dict(v, hbm_bytes_per_launch=b)
    stats_f = glob.glob(os.path.join(out_dir, "trace", "**", "*kernel_stats.csv"), recursive=True)[0]
    stats = list(csv.DictReader(open(stats_f)))
    os.makedirs(prof, exist_ok=True)
    with open(os.path.join(prof, "traffic.json"), "w") as f:
        json.dump({"source_hash": source_hash(), "workload": "edge_on_spiral_256x256x64, 1e7 packages, FP32",
                   "copy_calibration_bytes": COPY_BYTES, "factors": factors, "kernels": kernels,
                   "command": "python bench.py --collect-profiles " + out_dir}, f, indent=1)
    with open(os.path.join(prof, "life_kernels_spiral_1e7_fp32.md"), "w") as f:
        f.write("# Kernel trace and HBM counters: edge-on spiral, 1e7 packages, FP32 path\n\n")
        f.write("Command (writes this file and traffic.json): `python bench.py --collect-profiles %s`\n\n" % out_dir)
        f.write("Each pass runs `python bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-fp64 --no-powcub "
                "--no-panchromatic` under rocprofv3: `--kernel-trace --stats`, then `--pmc FETCH_SIZE` and `--pmc WRITE_SIZE` (the "
                "counter passes add `--calibrate-copy`: a 1 GiB device copy first, whose counter values give "
                "the scale factors below).\n\n")
        f.write("## Kernel durations (rocprofv3 --stats)\n\n| kernel | calls | average ms | total ms |\n|---|---|---|---|\n")
        for r in stats:
            n = r.get("Name") or r.get("KernelName") or ""
            if "mcrt" not in n:
                continue
            f.write("| `%s` | %s | %.3f | %.3f |\n" % (n, r["Calls"], float(r["AverageNs"]) / 1e6,
                                                      float(r["TotalDurationNs"]) / 1e6))
        f.write("\n## HBM traffic per dispatch (counter KiB x calibration factor)\n\n")
        f.write("Factors: FETCH_SIZE x %.3f, WRITE_SIZE x %.3f (1 GiB copy).\n\n" % (factors["FETCH_SIZE"],
                                                                                   factors["WRITE_SIZE"]))
        f.write("| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes per launch |\n|---|---|---|---|\n")
        for key, v in kernels.items():
            f.write("| `%s` | %.0f | %.0f | %.4g |\n" % (KERNELS[key], v["FETCH_SIZE_kib_per_dispatch"],
                                                       v["WRITE_SIZE_kib_per_dispatch"], v["hbm_bytes_per_launch"]))
    print("[profile] wrote %s/traffic.json and life_kernels_spiral_1e7_fp32.md" % prof, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packages", type=int, default=10_000_000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing (profiling runs)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-path comparison")
    ap.add_argument("--no-powcub", action="store_true", help="skip the PowCub- and k-d-tree-grid steps")
    ap.add_argument("--no-panchromatic", action="store_true", help="skip the panchromatic step")
    ap.add_argument("--calibrate-copy", action="store_true", help="run a 1 GiB device copy first (counter scale)")
    ap.add_argument("--collect-profiles", metavar="DIR", help="run the rocprofv3 passes (raw output in DIR)")
    ap.add_argument("--summarize-profiles", metavar="DIR", help="only rewrite the summaries from the raw output in DIR")
    ap.add_argument("--profiles-dir", default=os.path.join(ROOT, "profiles"), help="where the summaries go")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.collect_profiles or args.summarize_profiles:
        collect_profiles(args.collect_profiles or args.summarize_profiles, args.profiles_dir,
                         run=bool(args.collect_profiles))
        return

    import numpy as np
    import torch

    from paper_1410_1629_amd import binding as B
    from paper_1410_1629_amd import workloads as W

    B.load()
    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.add(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    prob = W.spiral(n_packages=args.packages, precision=1)
    prec = prob["precision"]
    rho = B.density_tensor(prob, dev)
    shape = B.image_shape(prob)
    images = torch.empty(shape, dtype=torch.float64, device=dev)
    absorbed = torch.empty((1, rho.numel()), dtype=torch.float64, device=dev)
    grad = torch.empty(rho.numel(), dtype=torch.float64, device=dev)
    adj = torch.empty(shape, dtype=torch.float64, device=dev)
    # target image of the L2 loss: the same model at a perturbed density
    zt = np.random.default_rng(3).standard_normal(prob["rho"].shape)
    rho_t = torch.as_tensor(W.as_f32_values(prob["rho"] * np.exp(0.1 * zt)).reshape(-1), dtype=rho.dtype,
                            device=dev)
    target = torch.empty(shape, dtype=torch.float64, device=dev)
    B.run_photons(dict(prob, seed=4358), rho_t, target, absorbed)
    del rho_t

    def step_fn(p, r, img, g):
        sf = B.run_photons(p, r, img, absorbed)
        torch.sub(img, target, out=adj)
        adj.mul_(2.0)
        sb = B.backward_density(p, r, adj, g)
        return sf, sb

    for _ in range(args.warmup):
        step_fn(prob, rho, images, grad)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fw, bw = [], []
    for _ in range(args.steps):
        sf, sb = step_fn(prob, rho, images, grad)
        fw.append(sf)
        bw.append(sb)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    ms_step = 1e3 * wall / args.steps
    n_pkg = prob["n_packages"]

    def summary(sts, adjoint):
        ms = float(np.mean([s["kernel_ms"] for s in sts]))
        life_ms = float(np.mean([s["life_ms"] for s in sts]))
        s0 = sts[-1]
        x = s0["x_path"] + s0["x_locate"] + s0["x_peel"]
        out = {"kernel_ms": ms, "life_ms": life_ms, "packages_per_s": n_pkg / (ms / 1e3), "crossings": x,
               "crossings_per_s": x / (ms / 1e3), "life_launches": s0["life_launches"]}
        for k in ("x_path", "x_locate", "x_peel", "x_queue", "events", "peels", "deposits"):
            out[k] = s0[k]
        out["life_algorithmic_bytes"] = life_bytes(s0, prec, adjoint)
        if adjoint:
            out["queue_ms"] = float(np.mean([s["queue_ms"] for s in sts]))
        return out

    fsum, bsum = summary(fw, False), summary(bw, True)

    def life_roofline(sm, key):
        # per launch of the life kernel: the call's bytes and time over its launches
        launch_s = sm["life_ms"] / 1e3 / sm["life_launches"]
        achieved = sm["life_algorithmic_bytes"] / sm["life_launches"] / launch_s / 1e9
        traffic = traffic_for(key)
        r = {"kernel": KERNELS[key], "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "launch_ms": launch_s * 1e3,
             "step_share": sm["life_ms"] / ms_step}
        if traffic:
            r["hardware_frac"] = traffic / launch_s / 1e9 / HBM_PEAK_GBS
        return r

    # the dominant kernel: the life kernel with the larger share of the step
    # (forward and adjoint are close; both are reported)
    rooflines = {"forward": life_roofline(fsum, "forward"), "adjoint": life_roofline(bsum, "adjoint")}
    key = "adjoint" if bsum["life_ms"] > fsum["life_ms"] else "forward"
    st_f = fw[-1]
    closure = (st_f["absorbed"] + st_f["escaped"] + st_f["truncated"] - st_f["emitted"]) / st_f["emitted"]
    out = {
        "metric": METRIC,
        "value": n_pkg / (ms_step / 1e3),
        "unit": "packages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "edge_on_spiral_256x256x64: exp-disk stars in exp-disk dust (face-on tau_V 1), "
                               "albedo 0.6, g 0.6, three 512x512 frames at 0/60/90 deg, %d packages; step = "
                               "forward run + path-replay adjoint of an L2 image loss" % n_pkg,
                   "grid": list(prob["n"]), "packages": n_pkg, "frames": [[d["nx"], d["ny"], d["incl"]] for d in
                                                                          prob["detectors"]],
                   "precision": "fp32 traversal, fp64 package state and tallies"},
        "crossings_per_s": (fsum["crossings"] + bsum["crossings"]) / (ms_step / 1e3),
        "forward": fsum,
        "adjoint": bsum,
        "energy_closure": closure,
        "roofline": rooflines[key],
        "rooflines": rooflines,
    }
    out["traversal"] = traversal(B, prob, 4_000_000, dev)
    if not args.no_fp64:
        out["fp64_path"] = fp64_comparison(B, prob, step_fn, images, grad, dev)
    if not args.no_powcub:
        out["powcub_grid"] = grid_leg(B, W.powcub_spiral(n_packages=n_pkg, precision=1), target, dev,
                                      "power-law cell widths (outermost/innermost 8, 8, 16)")
        out["kdtree_grid"] = grid_leg(B, W.kdtree_spiral(n_packages=n_pkg, precision=1), target, dev,
                                      "leaves halved along their longest side while their dust mass exceeds 3e-4")
    if not args.no_panchromatic:
        out["panchromatic"] = panchromatic_leg(B, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
