#!/usr/bin/env python3
"""Throughput of the photon-package life cycle on one MI355X.

Headline workload: the clumpy disk -- the edge-on spiral's stellar
exponential disk (h_R 4, h_z 0.4 kpc) in a dust disk (h_R 6, h_z 0.25 kpc)
carrying half the dust mass plus 2e4 Gaussian clumps at uniform random
positions carrying the other half (sigma lognormal, median 0.1 kpc), total
mass that of the face-on V-band tau 1 disk, on 512^3 cells over +-20 x +-20
x +-2 kpc (FP32 densities, 512 MiB: larger than the 256 MB MALL, so the
grid lives in HBM), albedo 0.6, g 0.6, two 1024x1024 frames at 0 and 90
degrees, 1e8 packages, FP32 traversal with FP64 package state and tallies.
One step is one forward run of the whole life cycle over the 1e8 packages:
emission, peel-off at emission and scattering, the pass-1 walk with
continuous absorption, forced scattering, Henyey-Greenstein scattering and
the FP64 image tallies.  Inputs are resident on the device before timing.

Prints one JSON line.  `value` is packages per second of whole steps.
`roofline` describes the kernel with the larger share of the step (the
life-cycle kernel or the queue's optical-depth walk), per launch: the
algorithmic bytes the method moves (4 B per density gather in FP32, 8 B per
FP64 tally read-modify-write and per pixel add) over the launch's duration
from HIP events on the call's stream (recorded by the library);
`rooflines` gives every kernel.  Extra keys: `spiral_step` (the edge-on
spiral on 256x256x64 cells with three 512x512 frames, 1e7 packages: one
forward run plus the path-replay adjoint of an L2 image loss, with the
plain FP64 GPU path beside it at the same dL/dI and the Monte Carlo noise
of two independent keys), `traversal` (trace_path on random rays through
the spiral's and the clumpy grid), `powcub_grid` and `kdtree_grid` (the
spiral step on a PowCub and on a k-d tree grid), `panchromatic` (stellar
run, dust emission, dust run on 100 wavelengths) and `cpu_baseline` (the
FP64 CPU oracle on the first packages of the headline workload, all host
cores and one core, with the GPU's result on the same packages compared
with it).

Modes: `--probes` runs the memory-system probes (streaming read, random
4-byte gathers over 1/16/512 MiB and 4 GiB, scattered and coalesced FP64
atomics) and prints their rates; `--collect-profiles DIR` runs this script
under rocprofv3 (a kernel-trace summary, then FETCH_SIZE and WRITE_SIZE
counter passes with a 1 GiB copy for calibration) as child processes, per
workload, and writes the summaries to profiles/; `--cpu-baselines` times the
oracle on every workload's package subset at all host cores and at one
core and writes profiles/cpu_baseline_oracle.md.
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
# Algorithmic bytes per unit of work: what the method must move, not what
# the line-granular hardware moves.  One density value per positive-length
# crossing that reads it; one FP64 read-modify-write per tally deposit
# (absorbed luminosity, gradient); one FP64 pixel add per forward peel-off
# contribution, one FP64 read of dL/dI per adjoint contribution; a trace
# ray reads its origin and direction and writes its optical depth.
BYTES_PER_CROSSING = {0: 8, 1: 4}
BYTES_PER_DEPOSIT = 8
BYTES_PER_PIXEL = 8
BYTES_PER_RAY = 56
COPY_BYTES = 1 << 30
# kernels as rocprofv3 names them (FP32 path, regular grid, frames only; the
# peel-ray walk with its LDS table of address terms)
KERNELS = {
    "life_forward": "void mcrt::k_life<float, false, 0, false>(mcrt::RunParams)",
    "peel_tau_forward": "void mcrt::k_peeltau<float, false, 0, false, true>(mcrt::PeelJobParams)",
    "life_adjoint": "void mcrt::k_life<float, true, 0, false>(mcrt::RunParams)",
    "peel_tau_adjoint": "void mcrt::k_peeltau<float, true, 0, false, true>(mcrt::PeelJobParams)",
    "peel_deposit": "void mcrt::k_peeldep<float, 0, false>(mcrt::PeelJobParams)",
    "trace": "void mcrt::k_trace<float, 0>(mcrt::TraceParams)",
    "attached": "void mcrt::k_attached<float, 0>(mcrt::RunParams)",
}
# the attached gradient's workspace: 11 FP64 values per event, written in the
# forward sweep and read back in the reverse sweep
BYTES_PER_ATTACHED_EVENT = 2 * 11 * 8
HEADLINE = "clumpy"
PROFILE_FILES = {"clumpy": "life_and_peel_kernels_clumpy_512cubed_1e8_fp32.md",
                 "spiral": "life_and_peel_kernels_spiral_256x256x64_1e7_fp32.md"}


def source_hash():
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1410_1629_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(workload, key):
    """Hardware bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) of a
    kernel on a workload from the committed counter summary, if it was
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
    except ValueError:
        return None
    if rec.get("source_hash") != source_hash():
        return None
    k = rec.get("workloads", {}).get(workload, {}).get(key)
    return k.get("bytes_per_launch") if k else None


def kernel_work(st, prec, adjoint):
    """Per kernel of one call: (algorithmic bytes, crossings, launches,
    milliseconds).  The life kernel walks paths, locate legs and the peel
    rays the queue could not take; the optical-depth walk every queued
    peel ray, adding its contribution to a pixel (forward) or reading its
    dL/dI (adjoint); the adjoint's deposit walk each queued ray again with
    one gradient deposit per crossing and no density loads."""
    cb = BYTES_PER_CROSSING[prec]
    # the adjoint launches the life kernel twice per chunk, once when it reads the forward run's tape (then its
    # queue has no optical-depth walks: peel_ms is 0)
    chunks = st["life_launches"] // (2 if adjoint and st["peel_ms"] > 0 else 1)
    x_life = st["x_path"] + st["x_locate"] + st["x_peel"] - st["x_queue"]
    x_tau = st["x_queue"] - st["d_queue"]
    out = {"life": (x_life * cb + (st["deposits"] - st["d_queue"]) * BYTES_PER_DEPOSIT, x_life, st["life_launches"],
                    st["life_ms"]),
           "peel_tau": (x_tau * cb + st["peels"] * BYTES_PER_PIXEL, x_tau, chunks, st["peel_ms"])}
    if adjoint:
        out["peel_deposit"] = (st["d_queue"] * BYTES_PER_DEPOSIT, st["d_queue"], chunks, st["dep_ms"])
    return out


def rooflines(st, prec, adjoint, workload, step_ms, level):
    """Roofline records of every kernel of a call (per launch)."""
    res = {}
    for name, (alg, x, launches, ms) in kernel_work(st, prec, adjoint).items():
        if launches == 0 or ms <= 0:
            continue
        key = "%s_%s" % (name, "adjoint" if adjoint else "forward") if name != "peel_deposit" else name
        launch_s = ms / 1e3 / launches
        achieved = alg / launches / launch_s / 1e9
        traffic = traffic_for(workload, key)
        r = {"kernel": KERNELS[key], "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "launch_ms": launch_s * 1e3,
             "launches_per_step": launches, "step_share": ms / step_ms,
             "crossings_per_s": x / (ms / 1e3), "algorithmic_bytes_per_launch": alg / launches,
             "level": level}
        if traffic:
            r["hardware_gbs"] = traffic / launch_s / 1e9
            r["hardware_frac"] = r["hardware_gbs"] / HBM_PEAK_GBS
            r["hardware_bytes_per_algorithmic_byte"] = traffic / (alg / launches)
        res[key] = r
    return res


def rel_l1(a, b):
    den = b.abs().sum().item()
    return (a - b).abs().sum().item() / den if den > 0 else float("nan")


def max_rel(a, b):
    """Largest relative difference over the elements above 1e-3 of the
    largest reference value."""
    import numpy as np
    a, b = np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()
    big = np.abs(b) > 1e-3 * np.abs(b).max()
    return float((np.abs(a - b)[big] / np.abs(b)[big]).max()) if big.any() else 0.0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    return int(os.environ.get("OMP_NUM_THREADS") or 0) or len(os.sched_getaffinity(0))


def oracle_rate(prob, seconds, threads, forward_only=True, adj=None, n0=None):
    """The FP64 oracle on the first packages of prob, the sample grown until
    it takes about `seconds`: (packages, seconds, images, stats)."""
    import oracle

    def timed(n):
        p = dict(prob, n_packages=n, first_package=0)
        t0 = time.perf_counter()
        img, _, st = oracle.run(p, threads=threads)
        if not forward_only:
            oracle.grad(p, adj, threads=threads)
        return time.perf_counter() - t0, img, st

    n = n0 or max(100, 25 * threads)
    t, img, st = timed(n)
    while t < 0.6 * seconds and n < 50_000_000:  # the last sample takes 0.6-1.5x `seconds`
        n = int(n * min(max(seconds / max(t, 1e-3), 1.5), 16))
        t, img, st = timed(n)
    return n, t, img, st


def cpu_baseline(B, prob, seconds, dev):
    """The FP64 oracle on the first packages of the headline workload, at
    all host cores and at one core (forward run, as the step), with the
    FP32 GPU path's images of the same packages compared with its own."""
    import torch
    threads = host_threads()
    n, t, img_o, st_o = oracle_rate(prob, seconds, threads)
    n1, t1, _, st1 = oracle_rate(prob, seconds / 3, 1, n0=max(50, n // (4 * threads)))
    rho = B.density_tensor(prob, dev)
    images = torch.empty(B.image_shape(prob), dtype=torch.float64, device=dev)
    B.run_photons(dict(prob, n_packages=n, first_package=0), rho, images, None)
    got = images.cpu().numpy()
    ia = torch.empty_like(images)
    B.run_photons(dict(prob, n_packages=n, first_package=0, seed=prob.get("seed", 4357) + 1000), rho, ia, None)
    x = lambda s: s["x_path"] + s["x_locate"] + s["x_peel"]
    import numpy as np
    return {"value": n / t, "unit": "packages/s", "cores": threads, "kind": "oracle",
            "sample": "first %d packages of the headline workload, FP64 oracle forward run, %.1f s on %d threads"
                      % (n, t, threads),
            "crossings_per_s": x(st_o) / t, "cpu_model": cpu_model(),
            "one_core": {"value": n1 / t1, "unit": "packages/s", "crossings_per_s": x(st1) / t1,
                         "sample": "first %d packages, %.1f s on 1 thread" % (n1, t1)},
            "gpu_on_sample": {"packages": n, "images_rel_l1_fp32_gpu_vs_oracle":
                              float(np.abs(got - img_o).sum() / np.abs(img_o).sum()),
                              "images_max_rel_fp32_gpu_vs_oracle": max_rel(got, img_o),
                              "images_mc_noise_rel_l1": rel_l1(images, ia) / 2 ** 0.5}}


def traversal(B, prob, n_rays, dev, workload):
    """trace_path over random rays in the workload's grid: origins uniform in
    the box, isotropic directions, optical depth only (4 B gathered per
    crossing, 56 B per ray); timed over 5 calls after one untimed call."""
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
    hw = traffic_for(workload, "trace")
    out = {"kernel": KERNELS["trace"], "rays": n_rays, "ms": ms, "crossings": x,
           "crossings_per_s": x / (ms / 1e3), "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": hw,
           "note": "ms covers the call (bricking the densities plus the walk kernel)"}
    if hw:
        out["hardware_gbs"] = hw / (ms / 1e3) / 1e9
        out["hardware_frac"] = out["hardware_gbs"] / HBM_PEAK_GBS
    return out


def summary(sts, n_pkg):
    import numpy as np
    s0 = sts[-1]
    out = {k: float(np.mean([s[k] for s in sts])) for k in ("kernel_ms", "life_ms", "queue_ms", "sort_ms", "peel_ms",
                                                              "dep_ms")}
    x = s0["x_path"] + s0["x_locate"] + s0["x_peel"]
    out.update(packages_per_s=n_pkg / (out["kernel_ms"] / 1e3), crossings=x,
               crossings_per_s=x / (out["kernel_ms"] / 1e3))
    for k in ("x_path", "x_locate", "x_peel", "x_queue", "events", "peels", "deposits", "d_queue", "life_launches"):
        out[k] = s0[k]
    return out


def spiral_step(B, W, dev, steps):
    """The edge-on spiral, 1e7 packages: one step is the forward run (which
    keeps the adjoint tape: T per leg, C per peel ray) plus the path-replay
    adjoint of an L2 image loss against a fixed target (rendered once from a
    perturbed density with another key), which reads the tape and replays
    each package once.  Beside it: the adjoint without the tape (two replays
    and the peel rays' optical-depth walks), the plain FP64 GPU path on the
    same step with the FP32 step's dL/dI, and the Monte Carlo noise of images
    and gradient from two more keys."""
    import numpy as np
    import torch
    prob = W.spiral(n_packages=10_000_000, precision=1)
    rho = B.density_tensor(prob, dev)
    shape = B.image_shape(prob)
    images = torch.empty(shape, dtype=torch.float64, device=dev)
    absorbed = torch.empty((1, rho.numel()), dtype=torch.float64, device=dev)
    grad = torch.empty(rho.numel(), dtype=torch.float64, device=dev)
    adj = torch.empty(shape, dtype=torch.float64, device=dev)
    zt = np.random.default_rng(3).standard_normal(prob["rho"].shape)
    rho_t = torch.as_tensor(W.as_f32_values(prob["rho"] * np.exp(0.1 * zt)).reshape(-1), dtype=rho.dtype,
                            device=dev)
    target = torch.empty(shape, dtype=torch.float64, device=dev)
    B.run_photons(dict(prob, seed=4358), rho_t, target, absorbed)
    del rho_t

    tape = B.new_tape(prob, dev)

    def step_fn(p, r, img, g, a, t):
        sf = B.run_photons(p, r, img, absorbed, tape=t)
        torch.sub(img, target, out=a)
        a.mul_(2.0)
        sb = B.backward_density(p, r, a, g, tape=t)
        return sf, sb

    step_fn(prob, rho, images, grad, adj, tape)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fw, bw = [], []
    for _ in range(steps):
        sf, sb = step_fn(prob, rho, images, grad, adj, tape)
        fw.append(sf)
        bw.append(sb)
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.perf_counter() - t0) / steps
    # the same adjoint without the tape (for comparison; same dL/dI)
    g_replay = torch.empty_like(grad)
    sb_replay = B.backward_density(prob, rho, adj, g_replay)
    n_pkg = prob["n_packages"]
    fsum, bsum = summary(fw, n_pkg), summary(bw, n_pkg)
    level = "MALL: the 16 MiB grid and 32 MiB tally fit in the 256 MB MALL behind the 4 MB L2 of each XCD"
    roof = rooflines(fw[-1], 1, False, "spiral", ms_step, level)
    roof.update(rooflines(bw[-1], 1, True, "spiral", ms_step, level))
    st_f = fw[-1]
    out = {"workload": "edge_on_spiral_256x256x64: exp-disk stars in exp-disk dust (face-on tau_V 1), albedo 0.6, "
                       "g 0.6, three 512x512 frames at 0/60/90 deg, %d packages, FP32 traversal; step = forward run "
                       "+ path-replay adjoint of an L2 image loss" % n_pkg,
           "packages_per_s": n_pkg / (ms_step / 1e3), "ms_per_step": ms_step,
           "crossings_per_s": (fsum["crossings"] + bsum["crossings"]) / (ms_step / 1e3),
           "forward": fsum, "adjoint": bsum, "rooflines": roof,
           "tape_gb": (tape.numel() / 1e9) if tape is not None else 0.0,
           "adjoint_without_tape": {"kernel_ms": sb_replay["kernel_ms"], "life_ms": sb_replay["life_ms"],
                                    "life_launches": sb_replay["life_launches"], "queue_ms": sb_replay["queue_ms"],
                                    "gradient_rel_l1_vs_tape": rel_l1(g_replay, grad)},
           "energy_closure": (st_f["absorbed"] + st_f["escaped"] + st_f["truncated"] - st_f["emitted"]) /
                             st_f["emitted"]}
    # the plain FP64 GPU path: the same step, the FP32 step's dL/dI
    img32, grad32, adj32 = images.clone(), grad.clone(), adj.clone()
    p64 = dict(prob, precision=0)
    rho64 = B.density_tensor(p64, dev)
    img64 = torch.empty_like(images)
    grad64 = torch.empty_like(grad)
    del tape
    tape64 = B.new_tape(p64, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sf64 = B.run_photons(p64, rho64, img64, absorbed, tape=tape64)
    sb64 = B.backward_density(p64, rho64, adj32, grad64, tape=tape64)
    torch.cuda.synchronize()
    wall64 = time.perf_counter() - t0
    # Monte Carlo noise: two more Philox keys, the same dL/dI
    ia, ib = torch.empty_like(images), torch.empty_like(images)
    ga, gb = torch.empty_like(grad), torch.empty_like(grad)
    for key, im_, g_ in ((5357, ia, ga), (6357, ib, gb)):
        B.run_photons(dict(prob, seed=key), rho, im_, absorbed)
        B.backward_density(dict(prob, seed=key), rho, adj32, g_)
    out["fp64_path"] = {"packages_per_s": n_pkg / wall64, "ms_per_step": wall64 * 1e3,
                        "forward_ms": sf64["kernel_ms"], "adjoint_ms": sb64["kernel_ms"],
                        "images_rel_l1_fp32_vs_fp64": rel_l1(img32, img64),
                        "images_max_rel_fp32_vs_fp64": max_rel(img32.cpu().numpy(), img64.cpu().numpy()),
                        "gradient_rel_l1_fp32_vs_fp64": rel_l1(grad32, grad64),
                        "gradient_max_rel_fp32_vs_fp64": max_rel(grad32.cpu().numpy(), grad64.cpu().numpy()),
                        "images_mc_noise_rel_l1": rel_l1(ia, ib) / 2 ** 0.5,
                        "gradient_mc_noise_rel_l1": rel_l1(ga, gb) / 2 ** 0.5,
                        "images_mc_noise_max_rel": max_rel(ia.cpu().numpy(), ib.cpu().numpy()),
                        "gradient_mc_noise_max_rel": max_rel(ga.cpu().numpy(), gb.cpu().numpy()),
                        "note": "both gradients take the FP32 step's dL/dI; noise = rel_L1 of two independent "
                                "keys / sqrt(2); the noise max_rel is that of the two keys' arrays"}
    return out


def grid_leg(B, prob, dev, note):
    """One step (forward + adjoint of an L2 loss against the image of a
    perturbed density) of the spiral model on another grid kind, after one
    untimed step: the rectilinear- or tree-grid kernels at 1e7 packages."""
    import numpy as np
    import torch
    rho = B.density_tensor(prob, dev)
    shape = B.image_shape(prob)
    images = torch.empty(shape, dtype=torch.float64, device=dev)
    target = torch.empty(shape, dtype=torch.float64, device=dev)
    adj = torch.empty(shape, dtype=torch.float64, device=dev)
    absorbed = torch.empty((1, rho.numel()), dtype=torch.float64, device=dev)
    grad = torch.empty(rho.numel(), dtype=torch.float64, device=dev)
    zt = np.random.default_rng(3).standard_normal(rho.numel())
    rho_t = torch.as_tensor(W_f32(prob["rho"].reshape(-1) * np.exp(0.1 * zt)), dtype=rho.dtype, device=dev)
    B.run_photons(dict(prob, seed=4358), rho_t, target, absorbed)

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


def attached_leg(B, W, dev):
    """The attached (pathwise) density gradient of the adjoint workload (64^3
    lognormal grid, 128^2 face-on frame, 1e7 packages; FP32 densities, FP64
    sweeps), after one untimed call, beside the detached adjoint of the same
    dL/dI with and without the forward run's tape.  The peel rays' deposit
    walks go through the peel-job queue (sort, k_peeldep).  Roofline of
    k_attached: 4 B per crossing that reads a density (every walk but the
    deposit walks), 8 B per gradient deposit it makes itself and per dL/dI
    read, and the workspace's 2 x 88 B per event (emission and
    scatterings)."""
    import torch
    prob = W.adjoint(n_packages=10_000_000, precision=1)
    rho = B.density_tensor(prob, dev)
    images = torch.empty(B.image_shape(prob), dtype=torch.float64, device=dev)
    tape = B.new_tape(prob, dev)
    B.run_photons(prob, rho, images, None, tape=tape)
    adj = 2.0 * (images - 0.9 * images)
    grad = torch.empty(rho.numel(), dtype=torch.float64, device=dev)
    out = {"workload": "adjoint_lognormal_64: 64^3 i.i.d. lognormal densities, 128x128 face-on frame, "
                       "10000000 packages; the attached gradient of an image loss"}
    for name, kw in (("attached", dict(attached=True)), ("detached_replay", {}), ("detached_tape", dict(tape=tape))):
        B.backward_density(prob, rho, adj, grad, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = B.backward_density(prob, rho, adj, grad, **kw)
        torch.cuda.synchronize()
        out[name + "_ms"] = (time.perf_counter() - t0) * 1e3
        out[name + "_kernel_ms"] = st["kernel_ms"]  # HIP events on the call's stream (the wall clock includes the host)
        if name == "attached":
            # k_attached's own work: every walk but the deposit walks reads densities (d_queue counts all
            # deposit-walk crossings); its deposits exclude those of the queued deposit walks (x_queue,
            # one deposit per crossing), which the peel-job kernels make
            x_all = st["x_path"] + st["x_locate"] + st["x_peel"]
            alg = ((x_all - st["d_queue"]) * BYTES_PER_CROSSING[1] + (st["deposits"] - st["x_queue"]) * BYTES_PER_DEPOSIT +
                   st["peels"] * BYTES_PER_PIXEL + (st["events"] + st["packages"]) * BYTES_PER_ATTACHED_EVENT)
            launches = st["life_launches"]
            launch_s = st["life_ms"] / 1e3 / launches
            achieved = alg / launches / launch_s / 1e9
            out["packages_per_s"] = prob["n_packages"] / (st["kernel_ms"] / 1e3)
            out["crossings_per_s"] = x_all / (st["kernel_ms"] / 1e3)
            out["queue_ms"] = st["queue_ms"]  # the queued deposit walks and their sort
            out["roofline"] = {"kernel": KERNELS["attached"], "bound": "hbm", "achieved": achieved,
                               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                               "traffic": None, "launch_ms": launch_s * 1e3, "launches_per_step": launches,
                               "algorithmic_bytes_per_launch": alg / launches,
                               "level": "MALL: the 1 MiB grid fits in the 256 MB MALL"}
    return out


def W_f32(a):
    from paper_1410_1629_amd import workloads as W
    return W.as_f32_values(a)


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
            # the two runs' kernels alone (the wall clock and the dust-emission events also hold
            # host time, which varies between processes and boxes)
            "runs_kernel_ms": s1["kernel_ms"] + s2["kernel_ms"],
            "runs_packages_per_s": items / ((s1["kernel_ms"] + s2["kernel_ms"]) / 1e3),
            "absorbed_fraction": s1["absorbed"] / s1["emitted"],
            "reemitted_over_absorbed_tally": s2["emitted"] / tally,
            "dust_T_median_K": float(np.median(Tn[Tn > 0])), "dust_T_max_K": float(Tn.max())}


# ---------------------------------------------------------------------------
# Probes of the memory system, and the oracle on every workload.

def probes(dev):
    """Streaming read, random 4-byte gathers over tables of 1, 16 and 512
    MiB and 4 GiB, and FP64 atomic adds (scattered over 1 MiB and 512 MiB,
    coalesced), each timed with HIP events (libmcrt_probes.so)."""
    import torch
    from paper_1410_1629_amd import binding as B
    out = {}
    big = torch.zeros((4 << 30) // 4, dtype=torch.float32, device=dev)
    r = B.probe("stream_read", big, n_ops=big.numel(), reps=5)
    out["stream_read"] = dict(r, gbs=big.numel() * 4 / (r["ms"] / 1e3) / 1e9, bytes=big.numel() * 4)
    n_g = 1 << 28
    for mib in (1, 16, 512, 4096):
        t = big[: (mib << 20) // 4]
        r = B.probe("gather", t, n_ops=n_g, reps=3)
        out["gather_%d_MiB" % mib] = dict(r, gathers_per_s=n_g / (r["ms"] / 1e3),
                                          algorithmic_gbs=4 * n_g / (r["ms"] / 1e3) / 1e9)
    del big
    n_a = 1 << 27
    for name, mib, kind in (("atomic_f64_scattered_1_MiB", 1, "atomic_scattered"),
                            ("atomic_f64_scattered_512_MiB", 512, "atomic_scattered"),
                            ("atomic_f64_coalesced_512_MiB", 512, "atomic_coalesced")):
        t = torch.zeros((mib << 20) // 8, dtype=torch.float64, device=dev)
        r = B.probe(kind, t, n_ops=n_a, reps=3)
        out[name] = dict(r, atomics_per_s=n_a / (r["ms"] / 1e3))
        del t
    return out


def cpu_baselines(seconds, prof_dir):
    """The oracle on every workload's first packages, all host cores and one
    core; writes profiles/cpu_baseline_oracle.md and returns the rows."""
    import numpy as np
    from paper_1410_1629_amd import workloads as W
    threads = host_threads()
    rows = []
    cases = [("uniform cube 32^3, FP64", W.cube(n_packages=100_000, precision=0)),
             ("edge-on spiral 256x256x64, 3 x 512^2 frames", W.spiral(precision=1)),
             ("multiwavelength 128^3, wavelengths 0, 50, 99 of 100", W.multiwavelength(lambdas=[0, 50, 99])),
             ("clumpy 512^3, 2 x 1024^2 frames", W.clumpy(precision=1)),
             ("adjoint 64^3 lognormal, 128^2 frame (forward + gradient)", W.adjoint(precision=1))]
    for name, prob in cases:
        fwd = not name.startswith("adjoint")
        adj = None
        if not fwd:
            adj = np.random.default_rng(0).standard_normal((1, 1, 128 * 128))
        nl = len(np.atleast_1d(prob["kappa"]))  # packages per wavelength: items = packages x wavelengths
        n, t, _, st = oracle_rate(prob, seconds, threads, forward_only=fwd, adj=adj)
        n1, t1, _, st1 = oracle_rate(prob, seconds / 3, 1, forward_only=fwd, adj=adj, n0=max(20, n // (4 * threads)))
        x = lambda s: s["x_path"] + s["x_locate"] + s["x_peel"]
        full = prob["n_packages"] * (100 if nl == 3 else nl)  # the multiwavelength disk has 100 wavelengths
        rows.append({"workload": name, "threads": threads, "packages": n * nl, "seconds": t,
                     "packages_per_s": n * nl / t, "crossings_per_s": x(st) / t,
                     "one_core_packages": n1 * nl, "one_core_seconds": t1, "one_core_packages_per_s": n1 * nl / t1,
                     "one_core_crossings_per_s": x(st1) / t1, "full_n_packages": full,
                     "extrapolated_full_s": full * t / (n * nl)})
        print("[cpu] %s: %d packages in %.1f s on %d threads; %d in %.1f s on one" % (name, n, t, threads, n1, t1),
              flush=True)
    os.makedirs(prof_dir, exist_ok=True)
    with open(os.path.join(prof_dir, "cpu_baseline_oracle.md"), "w") as f:
        f.write("# FP64 CPU oracle on the host cores of the GPU machine\n\n")
        f.write("Command: `python bench.py --cpu-baselines`.  CPU: %s; %d threads (all host cores given to the "
                "process) and 1 thread.  Each workload runs its first packages (package indices 0, 1, ...; the "
                "multiwavelength disk three of its wavelengths), the sample grown until it takes about %.0f s "
                "(one core: a third of that); full-size times are extrapolated linearly.  Forward runs; the "
                "adjoint workload times the forward run plus the gradient.\n\n" % (cpu_model(), threads, seconds))
        f.write("| workload | packages | s | packages/s | crossings/s | 1 core: packages | s | packages/s | "
                "crossings/s | full run (extrapolated, all cores) |\n|---|---|---|---|---|---|---|---|---|---|\n")
        for r in rows:
            f.write("| %s | %d | %.1f | %.4g | %.4g | %d | %.1f | %.4g | %.4g | %.0f s for %.3g packages |\n" % (
                r["workload"], r["packages"], r["seconds"], r["packages_per_s"], r["crossings_per_s"],
                r["one_core_packages"], r["one_core_seconds"], r["one_core_packages_per_s"],
                r["one_core_crossings_per_s"], r["extrapolated_full_s"], r["full_n_packages"]))
    return rows


# ---------------------------------------------------------------------------
# rocprofv3 summaries.

def collect_profiles(out_dir, prof, run=True):
    """Runs this script under rocprofv3 as child processes (this process
    never touches the GPU), one workload per child, and writes the
    summaries to `prof` (profiles/); run=False only summarizes the raw
    output already in out_dir."""
    os.makedirs(out_dir, exist_ok=True)
    me = os.path.abspath(__file__)
    passes = {
        "trace": ["rocprofv3", "--kernel-trace", "--stats", "--output-format", "csv"],
        "fetch": ["rocprofv3", "--kernel-trace", "--output-format", "csv", "--pmc", "FETCH_SIZE"],
        "write": ["rocprofv3", "--kernel-trace", "--output-format", "csv", "--pmc", "WRITE_SIZE"],
    }
    children = {"clumpy": [sys.executable, me, "--only", "clumpy", "--steps", "1", "--warmup", "0",
                           "--no-cpu-baseline"],
                "spiral": [sys.executable, me, "--only", "spiral", "--steps", "1", "--warmup", "0",
                           "--no-cpu-baseline"]}
    for wl, child in (children.items() if run else ()):
        for name, cmd in passes.items():
            extra = ["--calibrate-copy"] if name != "trace" else []
            d = os.path.join(out_dir, wl, name)
            full = cmd + ["-d", d, "-o", name, "--"] + child + extra
            print("[profile] " + " ".join(full), flush=True)
            r = subprocess.run(["timeout", "-k", "10", "420"] + full)
            if r.returncode != 0:
                print("[profile] %s %s pass failed with status %d" % (wl, name, r.returncode), flush=True)
                sys.exit(r.returncode)

    def dispatches(wl, name):
        f = glob.glob(os.path.join(out_dir, wl, name, "**", "*counter_collection.csv"), recursive=True)[0]
        agg = {}
        for r in csv.DictReader(open(f)):
            key = int(r["Dispatch_Id"])
            a = agg.setdefault(key, {"kernel": r["Kernel_Name"], "value": 0.0})
            a["value"] += float(r["Counter_Value"])
        return [agg[k] for k in sorted(agg)]

    record = {"source_hash": source_hash(), "copy_calibration_bytes": COPY_BYTES, "workloads": {},
              "command": "python bench.py --collect-profiles " + out_dir}
    for wl in children:
        factors, per_kernel = {}, {}
        for name, counter in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
            ds = dispatches(wl, name)
            copy = ds[0]  # the calibration copy is the first kernel of the child process
            factors[counter] = COPY_BYTES / (copy["value"] * 1024.0)
            for key, kname in KERNELS.items():
                vals = [d["value"] for d in ds if d["kernel"] == kname]
                if vals:
                    per_kernel.setdefault(key, {})[counter + "_kib_per_dispatch"] = sum(vals) / len(vals)
                    per_kernel[key]["dispatches"] = len(vals)
        kernels = {}
        for key, v in per_kernel.items():
            if "FETCH_SIZE_kib_per_dispatch" in v and "WRITE_SIZE_kib_per_dispatch" in v:
                b = 1024.0 * (v["FETCH_SIZE_kib_per_dispatch"] * factors["FETCH_SIZE"] +
                              v["WRITE_SIZE_kib_per_dispatch"] * factors["WRITE_SIZE"])
                kernels[key] = dict(v, bytes_per_launch=b)
        stats_f = glob.glob(os.path.join(out_dir, wl, "trace", "**", "*kernel_stats.csv"), recursive=True)[0]
        stats = list(csv.DictReader(open(stats_f)))
        record["workloads"][wl] = {k: v for k, v in kernels.items()}
        record["workloads"][wl]["_factors"] = factors
        os.makedirs(prof, exist_ok=True)
        title = {"clumpy": "clumpy disk, 512^3 cells (512 MiB of FP32 densities), two 1024^2 frames, 1e8 packages, "
                           "FP32 path: one forward run",
                 "spiral": "edge-on spiral, 256x256x64 cells, three 512^2 frames, 1e7 packages, FP32 path: one "
                           "forward run and one adjoint"}[wl]
        with open(os.path.join(prof, PROFILE_FILES[wl]), "w") as f:
            f.write("# Kernel trace and memory counters: %s\n\n" % title)
            f.write("Command (writes this file and traffic.json): `python bench.py --collect-profiles %s`\n\n"
                    % out_dir)
            f.write("Each pass runs `%s` under rocprofv3: `--kernel-trace --stats`, then `--pmc FETCH_SIZE` and "
                    "`--pmc WRITE_SIZE` (the counter passes add `--calibrate-copy`: a 1 GiB device copy first, whose "
                    "counter values give the scale factors below).\n\n" % " ".join(
                        ["python", "bench.py"] + children[wl][2:]))
            f.write("## Kernel durations (rocprofv3 --stats)\n\n| kernel | calls | average ms | total ms |\n"
                    "|---|---|---|---|\n")
            for r in stats:
                n = r.get("Name") or r.get("KernelName") or ""
                if "mcrt" not in n:
                    continue
                f.write("| `%s` | %s | %.3f | %.3f |\n" % (n, r["Calls"], float(r["AverageNs"]) / 1e6,
                                                          float(r["TotalDurationNs"]) / 1e6))
            f.write("\n## Bytes leaving the L2 per dispatch (counter KiB x calibration factor)\n\n")
            f.write("FETCH_SIZE and WRITE_SIZE count what each XCD's 4 MB L2 reads from and writes to the fabric: "
                    "the 256 MB MALL or HBM behind it.  Factors: FETCH_SIZE x %.3f, WRITE_SIZE x %.3f (1 GiB copy)."
                    "\n\n" % (factors["FETCH_SIZE"], factors["WRITE_SIZE"]))
            f.write("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | bytes per launch |\n"
                    "|---|---|---|---|---|\n")
            for key, v in kernels.items():
                f.write("| `%s` | %d | %.0f | %.0f | %.4g |\n" % (KERNELS[key], v["dispatches"],
                                                                v["FETCH_SIZE_kib_per_dispatch"],
                                                                v["WRITE_SIZE_kib_per_dispatch"],
                                                                v["bytes_per_launch"]))
    with open(os.path.join(prof, "traffic.json"), "w") as f:
        json.dump(record, f, indent=1)
    probe_profiles(out_dir, prof, run)
    print("[profile] wrote %s/traffic.json and the kernel summaries" % prof, flush=True)


PROBE_KERNELS = {"k_stream_read": "stream_read", "k_gather": "gather", "k_atomic_scattered": "atomic_scattered",
                 "k_atomic_coalesced": "atomic_coalesced"}


def probe_profiles(out_dir, prof, run=True):
    """The memory probes (--probes) under rocprofv3: kernel durations and the
    bytes each dispatch moves past the L2 (FETCH_SIZE, WRITE_SIZE), written
    to profiles/memory_probes.md."""
    me = os.path.abspath(__file__)
    child = [sys.executable, me, "--probes"]
    passes = {"trace": ["rocprofv3", "--kernel-trace", "--stats", "--output-format", "csv"],
              "fetch": ["rocprofv3", "--kernel-trace", "--output-format", "csv", "--pmc", "FETCH_SIZE"],
              "write": ["rocprofv3", "--kernel-trace", "--output-format", "csv", "--pmc", "WRITE_SIZE"]}
    outs = {}
    for name, cmd in passes.items():
        d = os.path.join(out_dir, "probes", name)
        full = cmd + ["-d", d, "-o", name, "--"] + child + (["--calibrate-copy"] if name != "trace" else [])
        if run:
            print("[profile] " + " ".join(full), flush=True)
            r = subprocess.run(["timeout", "-k", "10", "300"] + full, capture_output=(name == "trace"), text=True)
            if r.returncode != 0:
                print("[profile] probes %s pass failed with status %d" % (name, r.returncode), flush=True)
                sys.exit(r.returncode)
            if name == "trace":
                outs["json"] = [ln for ln in r.stdout.splitlines() if ln.startswith("{")][-1]
                with open(os.path.join(out_dir, "probes", "probes.json"), "w") as f:
                    f.write(outs["json"])
    with open(os.path.join(out_dir, "probes", "probes.json")) as f:
        rates = json.load(f)["probes"]
    stats_f = glob.glob(os.path.join(out_dir, "probes", "trace", "**", "*kernel_stats.csv"), recursive=True)[0]
    stats = {r["Name"]: r for r in csv.DictReader(open(stats_f))}
    counters = {}
    factors = {}
    for name, counter in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        f = glob.glob(os.path.join(out_dir, "probes", name, "**", "*counter_collection.csv"), recursive=True)[0]
        agg = {}
        for r in csv.DictReader(open(f)):
            a = agg.setdefault(int(r["Dispatch_Id"]), {"kernel": r["Kernel_Name"], "value": 0.0})
            a["value"] += float(r["Counter_Value"])
        ds = [agg[k] for k in sorted(agg)]
        factors[counter] = COPY_BYTES / (ds[0]["value"] * 1024.0)
        for d in ds[1:]:
            counters.setdefault(d["kernel"], {}).setdefault(counter, []).append(d["value"] * 1024.0 * factors[counter])
    with open(os.path.join(prof, "memory_probes.md"), "w") as f:
        f.write("# Memory-system probes on MI355X (include/mcrt_probes.h)\n\n")
        f.write("Command: `python bench.py --collect-profiles %s` (the probe passes run `python bench.py --probes` "
                "under `rocprofv3 --kernel-trace --stats`, then `--pmc FETCH_SIZE` and `--pmc WRITE_SIZE` with a "
                "1 GiB calibration copy first: factors %.3f and %.3f).\n\n" % (out_dir, factors["FETCH_SIZE"],
                                                                            factors["WRITE_SIZE"]))
        f.write("Rates from HIP events inside the probe (average of the timed runs):\n\n| probe | buffer | ops | ms "
                "| rate |\n|---|---|---|---|---|\n")
        for key, r in rates.items():
            rate = (("%.0f GB/s" % r["gbs"]) if "gbs" in r else ("%.3g gathers/s (%.0f GB/s of 4-byte values)" % (
                r["gathers_per_s"], r["algorithmic_gbs"]) if "gathers_per_s" in r else "%.3g atomics/s" %
                r["atomics_per_s"]))
            f.write("| %s | %.0f MiB | %.3g | %.3f | %s |\n" % (key, r["buffer_bytes"] / 2 ** 20, r["n_ops"], r["ms"],
                                                             rate))
        f.write("\n## Bytes past the L2 per dispatch, per probe\n\n| probe | kernel | dispatches | average ms "
                "(trace) | FETCH bytes per op | WRITE bytes per op |\n|---|---|---|---|---|---|\n")
        # dispatches per probe in launch order: one untimed run, then the timed runs
        order = [("stream_read", "k_stream_read", 6)] + [(k, "k_gather", 4) for k in rates if k.startswith("gather")] \
            + [(k, "k_atomic_scattered", 4) for k in rates if "scattered" in k] \
            + [(k, "k_atomic_coalesced", 4) for k in rates if "coalesced" in k]
        used = {}
        for key, short, nd in order:
            kname = [k for k in stats if short in k][0]
            i0 = used.get(kname, 0)
            used[kname] = i0 + nd
            c = counters.get(kname, {})
            fb = c.get("FETCH_SIZE", [])[i0:i0 + nd]
            wb = c.get("WRITE_SIZE", [])[i0:i0 + nd]
            ops = rates[key]["n_ops"] * (4 if short == "k_stream_read" else 1)  # stream: per byte read
            f.write("| %s | `%s` | %d | %.3f | %.3g | %.3g |\n" % (
                key, short, nd, float(stats[kname]["AverageNs"]) / 1e6,
                (sum(fb) / len(fb) / ops) if fb else float("nan"), (sum(wb) / len(wb) / ops) if wb else float("nan")))
        f.write("\nA trace row averages all dispatches of that kernel (every buffer size).  The streaming read's "
                "bytes are per byte read.  Bytes per op: a random "
                "4-byte gather moves a whole line once the table exceeds the L2; a scattered FP64 atomic is "
                "executed past the L2 as one request.\n")


# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packages", type=int, default=100_000_000, help="headline packages per step")
    ap.add_argument("--spiral-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--only", choices=["clumpy", "spiral"], help="one workload (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-extras", action="store_true", help="headline only")
    ap.add_argument("--calibrate-copy", action="store_true", help="run a 1 GiB device copy first (counter scale)")
    ap.add_argument("--collect-profiles", metavar="DIR", help="run the rocprofv3 passes (raw output in DIR)")
    ap.add_argument("--summarize-profiles", metavar="DIR", help="only rewrite the summaries from the raw output in DIR")
    ap.add_argument("--profiles-dir", default=os.path.join(ROOT, "profiles"), help="where the summaries go")
    ap.add_argument("--probes", action="store_true", help="memory-system probes only")
    ap.add_argument("--cpu-baselines", action="store_true", help="the oracle on every workload (CPU only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.collect_profiles or args.summarize_profiles:
        collect_profiles(args.collect_profiles or args.summarize_profiles, args.profiles_dir,
                         run=bool(args.collect_profiles))
        return
    if args.cpu_baselines:
        print(json.dumps({"cpu_baselines": cpu_baselines(args.cpu_seconds, args.profiles_dir)}), flush=True)
        return

    import numpy as np
    import torch

    from paper_1410_1629_amd import binding as B
    from paper_1410_1629_amd import workloads as W

    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.add(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    if args.probes:
        print(json.dumps({"probes": probes(dev)}), flush=True)
        return
    B.load()
    if args.only == "spiral":
        out = {"spiral_step": spiral_step(B, W, dev, args.steps),
               "traversal": {"spiral": traversal(B, W.spiral(n_packages=1, precision=1), 4_000_000, dev, "spiral")}}
        print(json.dumps(out), flush=True)
        return

    # headline: the clumpy disk, one forward run of 1e8 packages per step
    prob = W.clumpy(n_packages=args.packages, precision=1)
    rho = B.density_tensor(prob, dev)
    images = torch.empty(B.image_shape(prob), dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        B.run_photons(prob, rho, images, None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts = [B.run_photons(prob, rho, images, None) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    n_pkg = prob["n_packages"]
    fsum = summary(sts, n_pkg)
    level = "HBM: the 512 MiB grid exceeds the 256 MB MALL"
    roof = rooflines(sts[-1], 1, False, HEADLINE, ms_step, level)
    dom = max(roof, key=lambda k: roof[k]["step_share"])
    st = sts[-1]
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
        "config": {"workload": "clumpy_disk_512x512x512: exp-disk stars (h_R 4, h_z 0.4 kpc) in a dust disk (h_R 6, "
                               "h_z 0.25 kpc) with half the mass plus 2e4 Gaussian clumps (sigma lognormal, median 0.1 "
                               "kpc) with the other half, face-on tau_V 1, albedo 0.6, g 0.6, two 1024x1024 frames at "
                               "0 and 90 deg, %d packages; step = one forward run of the life cycle" % n_pkg,
                   "grid": list(prob["n"]), "packages": n_pkg,
                   "frames": [[d["nx"], d["ny"], d["incl"]] for d in prob["detectors"]],
                   "precision": "fp32 densities, optical depths and exponentials; fp64 package state, crossing "
                                "times of the life-cycle walks and tallies"},
        "crossings_per_s": fsum["crossings"] / (ms_step / 1e3),
        "crossings": {"x_path": st["x_path"], "x_locate": st["x_locate"], "x_peel": st["x_peel"]},
        "forward": fsum,
        "energy_closure": (st["absorbed"] + st["escaped"] + st["truncated"] - st["emitted"]) / st["emitted"],
        "roofline": roof[dom],
        "rooflines": roof,
    }
    if not args.no_extras:
        out["traversal"] = {"clumpy": traversal(B, prob, 4_000_000, dev, "clumpy")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(B, prob, args.cpu_seconds, dev)
    del rho, images
    if not args.no_extras and args.only is None:
        out["spiral_step"] = spiral_step(B, W, dev, args.spiral_steps)
        out["traversal"]["spiral"] = traversal(B, W.spiral(n_packages=1, precision=1), 4_000_000, dev, "spiral")
        out["powcub_grid"] = grid_leg(B, W.powcub_spiral(precision=1), dev,
                                      "power-law cell widths (outermost/innermost 8, 8, 16)")
        out["kdtree_grid"] = grid_leg(B, W.kdtree_spiral(precision=1), dev,
                                      "leaves halved along their longest side while their dust mass exceeds 3e-4")
        out["panchromatic"] = panchromatic_leg(B, dev)
        out["attached_gradient"] = attached_leg(B, W, dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
