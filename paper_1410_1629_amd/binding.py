"""Python binding of the C ABI in include/mcrt.h (argument marshalling only).

Every function here converts Python/torch arguments to the C structs and
device pointers the library expects and calls the entry point of the same
name; all work runs in the HIP kernels of libmcrt.so.  Loading fails loudly
when the library has not been built: there is no fallback.

Problems are the dicts built by `paper_1410_1629_amd.workloads`; device
buffers are torch tensors on a ROCm device.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcrt.so")

PEEL_EMIT, PEEL_SCAT, ABSORB, SPLIT, ATTACHED = 1, 2, 4, 8, 16
PREC_FP64, PREC_FP32 = 0, 1
OK, EINVAL, EOVERFLOW, EHIP = 0, -1, -2, -3


class McrtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mcrt error %d: %s" % (code, msg))
        self.code = code


class Grid(C.Structure):
    _fields_ = [("xmin", C.c_double), ("xmax", C.c_double), ("ymin", C.c_double), ("ymax", C.c_double),
                ("zmin", C.c_double), ("zmax", C.c_double), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("planes", C.POINTER(C.c_double)), ("tree_nodes", C.c_int32),
                ("tree_axis", C.POINTER(C.c_int32)), ("tree_split", C.POINTER(C.c_double)),
                ("tree_child", C.POINTER(C.c_int32))]


class Optics(C.Structure):
    _fields_ = [("n_lambda", C.c_int32), ("kappa", C.POINTER(C.c_double)), ("albedo", C.POINTER(C.c_double)),
                ("g", C.POINTER(C.c_double))]


class Source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("x", C.c_double), ("y", C.c_double), ("z", C.c_double),
                ("h_r", C.c_double), ("h_z", C.c_double), ("lum", C.POINTER(C.c_double)),
                ("cell_lum", C.c_void_p)]


class Detector(C.Structure):
    _fields_ = [("distance", C.c_double), ("incl_deg", C.c_double), ("azim_deg", C.c_double),
                ("pa_deg", C.c_double), ("nx", C.c_int32), ("ny", C.c_int32), ("half_x", C.c_double),
                ("half_y", C.c_double), ("kind", C.c_int32), ("eye", C.c_double * 3), ("target", C.c_double * 3),
                ("up", C.c_double * 3)]


DETECTOR_KINDS = {"frame": 0, "sed": 1, "perspective": 2}


class Opts(C.Structure):
    _fields_ = [("n_packages", C.c_uint64), ("first_package", C.c_uint64), ("seed", C.c_uint64),
                ("precision", C.c_int32), ("w_min", C.c_double), ("max_scatter", C.c_int32),
                ("flags", C.c_uint32), ("launch_blocks", C.c_int32), ("event_batch", C.c_int32),
                ("brick_shape", C.c_int32), ("peel_queue", C.c_int64), ("max_chunk", C.c_int64),
                ("tape", C.c_void_p), ("tape_bytes", C.c_uint64)]


def brick(lx, ly, lz):
    """Value of mcrt_opts.brick_shape for bricks of 2^lx x 2^ly x 2^lz cells."""
    return 0x1000 | lx | (ly << 4) | (lz << 8)


class Grads(C.Structure):
    _fields_ = [("rho", C.c_void_p), ("albedo", C.c_void_p), ("g", C.c_void_p), ("lum", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("emitted", C.c_double), ("absorbed", C.c_double), ("escaped", C.c_double),
                ("truncated", C.c_double), ("x_path", C.c_uint64), ("x_locate", C.c_uint64),
                ("x_peel", C.c_uint64), ("events", C.c_uint64), ("packages", C.c_uint64),
                ("peels", C.c_uint64), ("deposits", C.c_uint64), ("kernel_ms", C.c_double),
                ("x_queue", C.c_uint64), ("life_ms", C.c_double), ("queue_ms", C.c_double),
                ("d_queue", C.c_uint64), ("life_launches", C.c_uint64), ("sort_ms", C.c_double),
                ("peel_ms", C.c_double), ("dep_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

# Exported symbols of include/mcrt.h.
ABI_VERSION = 18  # MCRT_ABI_VERSION of the header these structs follow
SYMBOLS = ("run_photons", "trace_path", "trace_path_noalloc", "peel_off", "backward_density", "backward",
           "dust_emission", "mcrt_tape_bytes", "mcrt_last_error", "mcrt_abi_version")
NOALLOC_SCRATCH_BYTES = 96 << 20  # MCRT_NOALLOC_SCRATCH_BYTES


def load():
    """Loads libmcrt.so (raises if it is missing: build it with build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmcrt.so is not built (%s); run `python -m paper_1410_1629_amd.build` or "
                           "__graft_entry__.build()" % LIB_PATH)
    # torch first: the library then binds to the HIP runtime torch has loaded,
    # one runtime in the process (loaded the other way round, the library's
    # first HIP call found no device)
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.run_photons.argtypes = [C.POINTER(Grid), P, C.POINTER(Optics), C.c_int, C.POINTER(Source), C.c_int,
                                C.POINTER(Detector), C.POINTER(Opts), P, P, C.POINTER(Stats), P]
    lib.run_photons.restype = C.c_int
    lib.backward_density.argtypes = [C.POINTER(Grid), P, C.POINTER(Optics), C.c_int, C.POINTER(Source), C.c_int,
                                     C.POINTER(Detector), C.POINTER(Opts), P, P, C.POINTER(Stats), P]
    lib.backward_density.restype = C.c_int
    lib.trace_path.argtypes = [C.POINTER(Grid), P, d, C.c_int, i64, P, P, P, i32, P, P, P,
                               C.POINTER(C.c_uint64), P]
    lib.trace_path.restype = C.c_int
    lib.trace_path_noalloc.argtypes = lib.trace_path.argtypes
    lib.trace_path_noalloc.restype = C.c_int
    lib.peel_off.argtypes = [C.POINTER(Grid), P, d, d, C.c_int, i64, P, P, P, C.c_int, C.POINTER(Detector), P, P]
    lib.peel_off.restype = C.c_int
    lib.backward.argtypes = [C.POINTER(Grid), P, C.POINTER(Optics), C.c_int, C.POINTER(Source), C.c_int,
                             C.POINTER(Detector), C.POINTER(Opts), P, P, C.POINTER(Grads), C.POINTER(Stats), P]
    lib.backward.restype = C.c_int
    lib.dust_emission.argtypes = [C.POINTER(Grid), P, C.c_int, C.c_int, P, C.c_int, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double), d, P, P, P]
    lib.dust_emission.restype = C.c_int
    lib.mcrt_last_error.argtypes = []
    lib.mcrt_last_error.restype = C.c_char_p
    lib.mcrt_tape_bytes.argtypes = [C.POINTER(Optics), C.c_int, C.POINTER(Opts)]
    lib.mcrt_tape_bytes.restype = C.c_uint64
    lib.mcrt_abi_version.argtypes = []
    lib.mcrt_abi_version.restype = C.c_int
    if lib.mcrt_abi_version() != ABI_VERSION:
        raise RuntimeError("libmcrt.so has ABI version %d, the binding expects %d; rebuild it" % (
            lib.mcrt_abi_version(), ABI_VERSION))
    _lib = lib
    return lib


PROBES_PATH = os.path.join(HERE, "libmcrt_probes.so")
PROBE_KINDS = {"stream_read": 0, "gather": 1, "atomic_scattered": 2, "atomic_coalesced": 3}
_probes = None


def probe(kind, buf, n_ops, reps=3, stream=None):
    """mcrt_probe (include/mcrt_probes.h) on the device tensor buf: the
    average milliseconds of one run of the memory-system probe `kind`
    (stream_read, gather, atomic_scattered, atomic_coalesced) over n_ops
    operations."""
    global _probes
    if _probes is None:
        if not os.path.exists(PROBES_PATH):
            raise RuntimeError("libmcrt_probes.so is not built (%s)" % PROBES_PATH)
        lib = C.CDLL(PROBES_PATH)
        lib.mcrt_probe.argtypes = [C.c_int, C.c_void_p, C.c_uint64, C.c_uint64, C.c_int, C.POINTER(C.c_double),
                                   C.c_void_p]
        lib.mcrt_probe.restype = C.c_int
        _probes = lib
    ms = C.c_double(0.0)
    rc = _probes.mcrt_probe(PROBE_KINDS[kind], _ptr(buf), buf.numel() * buf.element_size(), int(n_ops), int(reps),
                            C.byref(ms), _stream(stream))
    if rc != 0:
        raise McrtError(rc, "mcrt_probe %s rejected its arguments or failed" % kind)
    return {"kind": kind, "ms": ms.value, "n_ops": int(n_ops), "buffer_bytes": buf.numel() * buf.element_size()}


def _check(rc):
    if rc != OK:
        raise McrtError(rc, load().mcrt_last_error().decode())


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _need(t, what, numel, dtype=None):
    """Checks a device tensor before its pointer reaches a kernel: the
    element count the layout needs and the element type (FP64 unless given).
    A kernel trusts these, so a mismatch is an error here, before any call."""
    import torch
    if t is None:
        return
    dt = torch.float64 if dtype is None else dtype
    if t.dtype != dt:
        raise ValueError("%s must be %s, got %s" % (what, dt, t.dtype))
    if t.numel() != numel:
        raise ValueError("%s has %d elements, the layout needs %d" % (what, t.numel(), numel))


def _density_dtype(precision):
    import torch
    return torch.float32 if int(precision) == PREC_FP32 else torch.float64


def _check_life(prob, rho, images=None, absorbed=None, adj=None, grad=None, overrides=None):
    """Sizes and types of a life-cycle call's device tensors (run_photons,
    backward_density, backward): rho float32 for the FP32 path and float64
    for the FP64 path with one value per cell; images and dL/dI in the image
    layout; the absorbed tally and dL/dA [n_lambda][ncell]; the density
    gradient [ncell]; all FP64."""
    prec = (overrides or {}).get("precision", prob.get("precision", 0))
    ncell = n_cells(prob)
    nl = len(np.atleast_1d(prob["kappa"]))
    _need(rho, "rho", ncell, _density_dtype(prec))
    npix = int(np.prod(image_shape(prob)))
    _need(images, "images", npix)
    _need(adj, "adj_images", npix)
    _need(absorbed, "absorbed", nl * ncell)
    _need(grad, "grad_rho", ncell)


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def make_grid(prob):
    """The grid of a problem dict: box, cells per axis and, for a
    rectilinear grid, prob["planes"] = (x planes, y planes, z planes), for a
    tree grid prob["tree"] = {"axis", "split", "child"} per node."""
    b, n = prob["box"], prob["n"]
    g = Grid(b[0], b[1], b[2], b[3], b[4], b[5], n[0], n[1], n[2], None, 0, None, None, None)
    planes = prob.get("planes")
    if planes is not None:
        arr = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1) for p in planes]))
        g._planes = arr  # kept alive with the struct
        g.planes = arr.ctypes.data_as(C.POINTER(C.c_double))
    tree = prob.get("tree")
    if tree is not None:
        ax = np.ascontiguousarray(tree["axis"], dtype=np.int32)
        sp = np.ascontiguousarray(tree["split"], dtype=np.float64)
        ch = np.ascontiguousarray(tree["child"], dtype=np.int32)
        g._tree = (ax, sp, ch)
        g.tree_nodes = ax.size
        g.tree_axis = ax.ctypes.data_as(C.POINTER(C.c_int32))
        g.tree_split = sp.ctypes.data_as(C.POINTER(C.c_double))
        g.tree_child = ch.ctypes.data_as(C.POINTER(C.c_int32))
    return g


def make_detectors(dets):
    """Instrument structs of detector dicts (kind "frame" by default, "sed"
    or "perspective" with eye, target and up)."""
    arr = (Detector * max(len(dets), 1))()
    v3 = C.c_double * 3
    for i, d in enumerate(dets):
        arr[i] = Detector(d.get("distance", 1.0), d.get("incl", 0.0), d.get("azim", 0.0), d.get("pa", 0.0), d["nx"],
                          d["ny"], d.get("half_x", 1.0), d.get("half_y", 1.0), DETECTOR_KINDS[d.get("kind", "frame")],
                          v3(*d.get("eye", (0.0, 0.0, 0.0))), v3(*d.get("target", (0.0, 0.0, 0.0))),
                          v3(*d.get("up", (0.0, 0.0, 0.0))))
    return arr


SOURCE_KINDS = {"point": 0, "expdisk": 1, "cells": 2}


def n_cells(prob):
    """Cells of the problem's grid (a tree grid's problem has n = (cells, 1, 1))."""
    return int(np.prod(prob["n"]))


def _cell_lum(src, nl, ncell, on_device):
    """The cell source's luminosities [n_lambda][ncell] FP64 as the call
    takes them: a device tensor (library) or a host array (CPU harness)."""
    a = src["cell_lum"]
    if on_device:
        import torch
        t = a if isinstance(a, torch.Tensor) else torch.as_tensor(np.asarray(a, dtype=np.float64))
        t = t.to(device="cuda", dtype=torch.float64).contiguous()
        if t.numel() != nl * ncell:
            raise ValueError("cell_lum has %d values, expected n_lambda x cells = %d" % (t.numel(), nl * ncell))
        return t, C.c_void_p(t.data_ptr())
    if not isinstance(a, np.ndarray):
        a = a.detach().cpu().numpy()
    h = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if h.size != nl * ncell:
        raise ValueError("cell_lum has %d values, expected n_lambda x cells = %d" % (h.size, nl * ncell))
    return h, h.ctypes.data_as(C.c_void_p)


class _Problem:
    """C views of a problem dict; keeps the host arrays alive.  A cell
    source's luminosities go to the device unless cells_on_device is False
    (the CPU harness)."""

    def __init__(self, prob, cells_on_device=True, **overrides):
        self.grid = make_grid(prob)
        self.kappa = np.ascontiguousarray(prob["kappa"], dtype=np.float64)
        self.albedo = np.ascontiguousarray(prob["albedo"], dtype=np.float64)
        self.g = np.ascontiguousarray(prob["g"], dtype=np.float64)
        dp = C.POINTER(C.c_double)
        self.optics = Optics(self.kappa.size, self.kappa.ctypes.data_as(dp), self.albedo.ctypes.data_as(dp),
                             self.g.ctypes.data_as(dp))
        srcs = prob["sources"]
        self.lums = [np.ascontiguousarray(np.broadcast_to(np.asarray(s["lum"], dtype=np.float64),
                                                          (self.kappa.size,))) for s in srcs]
        self.sources = (Source * len(srcs))()
        self.keep = []
        for i, s in enumerate(srcs):
            cell = None
            if s["kind"] == "cells":
                arr, cell = _cell_lum(s, self.kappa.size, n_cells(prob), cells_on_device)
                self.keep.append(arr)
            pos = s.get("pos", (0.0, 0.0, 0.0))
            self.sources[i] = Source(SOURCE_KINDS[s["kind"]], pos[0], pos[1], pos[2], s.get("h_r", 0.0),
                                     s.get("h_z", 0.0), self.lums[i].ctypes.data_as(dp), cell)
        self.n_src = len(srcs)
        self.detectors = make_detectors(prob["detectors"])
        self.n_det = len(prob["detectors"])
        o = dict(n_packages=prob["n_packages"], first_package=prob.get("first_package", 0),
                 seed=prob.get("seed", 4357), precision=prob.get("precision", 0), w_min=prob.get("w_min", 1e-4),
                 max_scatter=prob.get("max_scatter", 1000), flags=prob.get("flags", 7), launch_blocks=0,
                 event_batch=0, brick_shape=0, peel_queue=0, max_chunk=0, tape=None, tape_bytes=0)
        o.update(overrides)
        self.opts = Opts(int(o["n_packages"]), int(o["first_package"]), int(o["seed"]), int(o["precision"]),
                         float(o["w_min"]), int(o["max_scatter"]), int(o["flags"]), int(o["launch_blocks"]),
                         int(o["event_batch"]), int(o["brick_shape"]), int(o["peel_queue"]), int(o["max_chunk"]),
                         o["tape"], int(o["tape_bytes"]))


def tape_bytes(prob, **overrides):
    """mcrt_tape_bytes: the size of the adjoint tape of a run of the problem
    (0: the run cannot keep one)."""
    lib = load()
    pr = _Problem(prob, cells_on_device=False, **overrides)
    return int(lib.mcrt_tape_bytes(C.byref(pr.optics), pr.n_det, C.byref(pr.opts)))


def new_tape(prob, device="cuda", **overrides):
    """A device byte tensor of the problem's tape size, or None when the run
    cannot keep a tape."""
    import torch
    n = tape_bytes(prob, **overrides)
    return torch.empty(n, dtype=torch.uint8, device=device) if n else None


def _tape_args(prob, tape, overrides):
    """The tape's pointer and size for the options (after checking it)."""
    if tape is None:
        return overrides
    import torch
    _need(tape, "tape", tape.numel(), torch.uint8)
    need = tape_bytes(prob, **overrides)
    if need == 0 or tape.numel() < need:
        raise ValueError("tape has %d bytes, the run needs %d (0: it cannot keep one)" % (tape.numel(), need))
    return dict(overrides, tape=_ptr(tape).value, tape_bytes=tape.numel())


def image_shape(prob):
    comps = 2 if prob.get("flags", 7) & SPLIT else 1
    npix = int(sum(d["nx"] * d["ny"] for d in prob["detectors"]))
    return (comps, len(np.atleast_1d(prob["kappa"])), npix)


def density_tensor(prob, device="cuda"):
    """The problem's density as a device tensor of the precision's type."""
    import torch
    dt = torch.float32 if prob.get("precision", 0) == PREC_FP32 else torch.float64
    return torch.as_tensor(np.ascontiguousarray(prob["rho"]).reshape(-1), dtype=dt).to(device)


def run_photons(prob, rho, images, absorbed=None, stats=True, stream=None, tape=None, **overrides):
    """run_photons over the problem dict.  rho, images, absorbed: device
    tensors (images [comps][n_lambda][pixels] FP64, absorbed [n_lambda][ncell]
    FP64); tape: a device byte tensor (new_tape) the run fills for its
    adjoint, or None.  Returns the statistics dict (stats=True waits for the
    kernel)."""
    lib = load()
    _check_life(prob, rho, images=images, absorbed=absorbed, overrides=overrides)
    overrides = _tape_args(prob, tape, overrides)
    pr = _Problem(prob, **overrides)
    st = Stats()
    _check(lib.run_photons(C.byref(pr.grid), _ptr(rho), C.byref(pr.optics), pr.n_src, pr.sources, pr.n_det,
                           pr.detectors, C.byref(pr.opts), _ptr(images), _ptr(absorbed),
                           C.byref(st) if stats else None, _stream(stream)))
    return st.as_dict() if stats else None


def _attached(prob, attached, overrides):
    """The options with MCRT_ATTACHED set when the attached gradient is asked for."""
    if not attached:
        return overrides
    return dict(overrides, flags=int(overrides.get("flags", prob.get("flags", 7))) | ATTACHED)


def backward_density(prob, rho, adj_images, grad_rho, stats=True, stream=None, tape=None, attached=False,
                     **overrides):
    """backward_density: grad_rho (device FP64 [ncell]) = dL/drho for
    dL/dI = adj_images (device FP64, image layout of run_photons); tape: the
    forward run's tape (same problem and densities), or None; attached=True:
    the attached (pathwise) derivative (MCRT_ATTACHED; the tape is not
    used)."""
    lib = load()
    _check_life(prob, rho, adj=adj_images, grad=grad_rho, overrides=overrides)
    overrides = _attached(prob, attached, _tape_args(prob, tape, overrides))
    pr = _Problem(prob, **overrides)
    st = Stats()
    _check(lib.backward_density(C.byref(pr.grid), _ptr(rho), C.byref(pr.optics), pr.n_src, pr.sources, pr.n_det,
                                pr.detectors, C.byref(pr.opts), _ptr(adj_images), _ptr(grad_rho),
                                C.byref(st) if stats else None, _stream(stream)))
    return st.as_dict() if stats else None


def backward(prob, rho, adj_images, grad_rho=None, grad_albedo=None, grad_g=None, grad_lum=None, stats=True,
             stream=None, adj_absorbed=None, tape=None, attached=False, **overrides):
    """backward: the gradients of the loss with dL/dI = adj_images (and dL/dA
    = adj_absorbed [n_lambda][ncell] on the absorbed tally, if given) with
    respect to the densities (device FP64 [ncell]), the albedo and g
    ([n_lambda]) and the source luminosities ([n_src][n_lambda]); each
    output is a device FP64 tensor or None (not computed).  attached=True:
    the attached density gradient (grad_rho alone)."""
    lib = load()
    _check_life(prob, rho, adj=adj_images, absorbed=adj_absorbed, grad=grad_rho, overrides=overrides)
    nl = len(np.atleast_1d(prob["kappa"]))
    _need(grad_albedo, "grad_albedo", nl)
    _need(grad_g, "grad_g", nl)
    _need(grad_lum, "grad_lum", len(prob["sources"]) * nl)
    overrides = _attached(prob, attached, _tape_args(prob, tape, overrides))
    pr = _Problem(prob, **overrides)
    st = Stats()
    g = Grads(_ptr(grad_rho), _ptr(grad_albedo), _ptr(grad_g), _ptr(grad_lum))
    _check(lib.backward(C.byref(pr.grid), _ptr(rho), C.byref(pr.optics), pr.n_src, pr.sources, pr.n_det,
                        pr.detectors, C.byref(pr.opts), _ptr(adj_images), _ptr(adj_absorbed), C.byref(g),
                        C.byref(st) if stats else None, _stream(stream)))
    return st.as_dict() if stats else None


def trace_path(grid, rho, kappa, precision, origins, dirs, tau, max_seg=0, seg_cell=None, seg_len=None,
               n_seg=None, crossings=True, stream=None, noalloc=False):
    """trace_path for device tensors origins/dirs [n][3] FP64 and tau [n]
    FP64; optional segment lists.  Returns the total crossing count (or
    None).  `grid` is a problem dict or a Grid.  noalloc=True calls
    trace_path_noalloc instead (the library's per-device scratch array, no
    device allocation; grids up to NOALLOC_SCRATCH_BYTES)."""
    lib = load()
    entry = lib.trace_path_noalloc if noalloc else lib.trace_path
    g = grid if isinstance(grid, Grid) else make_grid(grid)
    n = int(origins.shape[0]) if origins is not None else 0
    _need(rho, "rho", g.nx * g.ny * g.nz, _density_dtype(precision))
    _need(origins, "origins", 3 * n)
    _need(dirs, "dirs", 3 * n)
    _need(tau, "tau", n)
    if seg_cell is not None:
        import torch
        _need(seg_cell, "seg_cell", n * int(max_seg), torch.int32)
        _need(seg_len, "seg_len", n * int(max_seg))
    if n_seg is not None:
        import torch
        _need(n_seg, "n_seg", n, torch.int32)
    c = C.c_uint64(0)
    _check(entry(C.byref(g), _ptr(rho), float(kappa), int(precision), n, _ptr(origins), _ptr(dirs),
                          _ptr(tau), int(max_seg), _ptr(seg_cell), _ptr(seg_len), _ptr(n_seg),
                          C.byref(c) if crossings else None, _stream(stream)))
    return c.value if crossings else None


def trace_path_noalloc(grid, rho, kappa, precision, origins, dirs, tau, max_seg=0, seg_cell=None, seg_len=None,
                       n_seg=None, crossings=True, stream=None):
    """trace_path_noalloc: trace_path without device allocation (the same
    arguments and results)."""
    return trace_path(grid, rho, kappa, precision, origins, dirs, tau, max_seg, seg_cell, seg_len, n_seg, crossings,
                      stream, noalloc=True)


def peel_off(grid, rho, kappa, g, precision, pos, dir_in, w, detectors, images, stream=None):
    """peel_off of events (device pos [n][3], dir_in [n][3] or None, w [n])
    into images (device FP64, frames of one wavelength, accumulated)."""
    lib = load()
    gr = grid if isinstance(grid, Grid) else make_grid(grid)
    dets = make_detectors(detectors)
    n = int(pos.shape[0]) if pos is not None else 0
    _need(rho, "rho", gr.nx * gr.ny * gr.nz, _density_dtype(precision))
    _need(pos, "pos", 3 * n)
    _need(dir_in, "dir_in", 3 * n)
    _need(w, "w", n)
    _need(images, "images", int(sum(d["nx"] * d["ny"] for d in detectors)))
    _check(lib.peel_off(C.byref(gr), _ptr(rho), float(kappa), float(g), int(precision), n, _ptr(pos),
                        _ptr(dir_in), _ptr(w), len(detectors), dets, _ptr(images), _stream(stream)))


def render(prob, device="cuda", rho=None, **overrides):
    """Allocates outputs and runs the problem: (images, absorbed or None, stats)."""
    import torch
    rho = density_tensor(prob, device) if rho is None else rho
    images = torch.empty(image_shape(prob), dtype=torch.float64, device=device)
    absorbed = None
    if prob.get("flags", 7) & ABSORB:
        absorbed = torch.empty((len(np.atleast_1d(prob["kappa"])), rho.numel()), dtype=torch.float64, device=device)
    st = run_photons(prob, rho, images, absorbed, **overrides)
    return images, absorbed, st


def dust_emission(grid, rho, precision, absorbed, lam, dlam, kappa_abs, emissivity, emission, temperature=None,
                  stream=None):
    """dust_emission: per cell the equilibrium temperature (device FP64
    [ncell], optional) and the emission spectrum (device FP64 [n_lambda]
    [ncell]) of the luminosity in absorbed (device FP64 [n_abs][ncell]);
    lam, dlam, kappa_abs: host arrays [n_lambda].  `grid` is a problem dict
    or a Grid."""
    lib = load()
    g = grid if isinstance(grid, Grid) else make_grid(grid)
    lam, dlam, ka = (np.ascontiguousarray(np.atleast_1d(v), dtype=np.float64) for v in (lam, dlam, kappa_abs))
    dp = C.POINTER(C.c_double)
    n_abs = int(absorbed.shape[0]) if absorbed is not None and absorbed.dim() == 2 else 1
    ncell = g.nx * g.ny * g.nz
    _need(rho, "rho", ncell, _density_dtype(precision))
    _need(absorbed, "absorbed", n_abs * ncell)
    _need(emission, "emission", lam.size * ncell)
    _need(temperature, "temperature", ncell)
    _check(lib.dust_emission(C.byref(g), _ptr(rho), int(precision), n_abs, _ptr(absorbed), lam.size,
                             lam.ctypes.data_as(dp), dlam.ctypes.data_as(dp), ka.ctypes.data_as(dp),
                             float(emissivity), _ptr(temperature), _ptr(emission), _stream(stream)))
