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
`roofline` describes the kernel with the longer average duration, from HIP
events around its launches on the stream it runs on; `cpu_baseline` times
the FP64 CPU oracle on a bounded package sample of the same workload.
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "photon packages/sec (with peel-off) and cell-crossings/s vs HBM/L2 roofline"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes: one density value per cell crossing, one FP64
# read-modify-write (8 B read + 8 B written) per tally deposit and per
# peel-off contribution landing in a frame.
BYTES_PER_CROSSING = {0: 8, 1: 4}
BYTES_PER_DEPOSIT = 16
BYTES_PER_PEEL = 16


def source_hash():
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1410_1629_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel, launches_bytes):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
    except ValueError:
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k or rec.get("source_hash") != source_hash():
        return None
    return k.get("hbm_bytes_per_launch")


def algorithmic_bytes(st, prec):
    x = st["x_path"] + st["x_locate"] + st["x_peel"]
    return x * BYTES_PER_CROSSING[prec] + st["deposits"] * BYTES_PER_DEPOSIT + st["peels"] * BYTES_PER_PEEL


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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packages", type=int, default=10_000_000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1410_1629_amd import binding as B
    from paper_1410_1629_amd import workloads as W

    B.load()
    dev = "cuda:0"
    torch.cuda.set_device(0)
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

    def step():
        sf = B.run_photons(prob, rho, images, absorbed)
        torch.sub(images, target, out=adj)
        adj.mul_(2.0)
        sb = B.backward_density(prob, rho, adj, grad)
        return sf, sb

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fw, bw = [], []
    for _ in range(args.steps):
        sf, sb = step()
        fw.append(sf)
        bw.append(sb)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    ms_step = 1e3 * wall / args.steps
    n_pkg = prob["n_packages"]

    def summary(sts):
        ms = float(np.mean([s["kernel_ms"] for s in sts]))
        s0 = sts[-1]
        x = s0["x_path"] + s0["x_locate"] + s0["x_peel"]
        return {"kernel_ms": ms, "packages_per_s": n_pkg / (ms / 1e3), "crossings": x,
                "crossings_per_s": x / (ms / 1e3), "x_path": s0["x_path"], "x_locate": s0["x_locate"],
                "x_peel": s0["x_peel"], "events": s0["events"], "peels": s0["peels"], "deposits": s0["deposits"],
                "algorithmic_bytes": algorithmic_bytes(s0, prec)}

    fsum, bsum = summary(fw), summary(bw)
    kname = {True: "k_life<float, true> (adjoint)", False: "k_life<float, false> (forward)"}
    dominant_adj = bsum["kernel_ms"] > fsum["kernel_ms"]
    dom = bsum if dominant_adj else fsum
    achieved = dom["algorithmic_bytes"] / (dom["kernel_ms"] / 1e3) / 1e9
    traffic = traffic_for("adjoint" if dominant_adj else "forward", None)
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
        "roofline": {"kernel": kname[dominant_adj], "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
