"""Builds the gfx950 HIP library libmcrt.so in-tree with hipcc.

Flags: gfx950 only; -ffp-contract=off so FP64 event arithmetic rounds like
the plain expressions (the walk uses explicit fma); -munsafe-fp-atomics so
FP64 tallies use the hardware global atomic add; packed FP32 instructions
disabled.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmcrt.so")
SOURCES = [os.path.join(CSRC, "mcrt_kernels.hip")]
DEPENDS = SOURCES + [os.path.join(CSRC, h) for h in ("mcrt_device.hpp", "mcrt_lane.hpp", "mcrt_host.hpp", "mcrt_attached.hpp")] + [
    os.path.join(INCLUDE, "mcrt.h")]
# the memory-system probes the roofline is measured against (not the transport path)
PROBES_LIB = os.path.join(HERE, "libmcrt_probes.so")
PROBES_SOURCES = [os.path.join(CSRC, "mcrt_probes.hip")]
ARCH = "gfx950"


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return exe


def flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
            "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-I" + INCLUDE, "-I" + CSRC]


def _compile(sources, lib, verbose, extra=()):
    cmd = [hipcc()] + flags() + list(extra) + sources + ["-o", lib + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the packed-fp32 target feature; that warning is expected
    msg = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + msg)
    if verbose and msg.strip():
        print(msg)
    os.replace(lib + ".tmp", lib)
    return lib


def build(verbose=False, extra=()):
    """Builds libmcrt.so and libmcrt_probes.so; returns the former's path."""
    _compile(PROBES_SOURCES, PROBES_LIB, verbose, extra)
    return _compile(SOURCES, LIB, verbose, extra)


def needs_build():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in DEPENDS)


if __name__ == "__main__":
    print(build(verbose=True))
