"""The C ABI of include/mcrt.h on the CPU: the built library exports every
function the header declares, the Python binding's struct layouts match the
C compiler's, and invalid arguments are rejected with MCRT_EINVAL and a
message before anything touches a GPU (argument checks run first, so these
calls are safe on a machine without one)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcrt.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\([^;{]*\)\s*;", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1410_1629_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libmcrt.so is not built")
    return binding.load()


@pytest.fixture(scope="module")
def B():
    from paper_1410_1629_amd import binding
    return binding


def test_header_declares_the_four_calls():
    names = _declared_functions()
    for n in ("run_photons", "trace_path", "peel_off", "backward_density", "mcrt_last_error", "mcrt_abi_version"):
        assert n in names, names


def test_library_exports_every_declared_function(lib, B):
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], check=True, capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    for n in _declared_functions():
        assert n in exported, n
        assert getattr(lib, n) is not None
    assert set(B.SYMBOLS) == set(_declared_functions())


def test_abi_version(lib, B):
    m = re.search(r"#define\s+MCRT_ABI_VERSION\s+(\d+)", open(HEADER).read())
    assert lib.mcrt_abi_version() == int(m.group(1)) == B.ABI_VERSION


def test_struct_layouts_match_the_c_compiler(B, tmp_path):
    structs = {"mcrt_grid": B.Grid, "mcrt_optics": B.Optics, "mcrt_source": B.Source, "mcrt_detector": B.Detector,
               "mcrt_opts": B.Opts, "mcrt_stats": B.Stats, "mcrt_grads": B.Grads}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mcrt.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(ln.split() for ln in subprocess.run([str(exe)], check=True, capture_output=True,
                                                    text=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[cname + "." + f]) == getattr(py, f).offset, (cname, f)


def _call_run(lib, B, prob, **over):
    pr = B._Problem(prob, **over)
    st = B.Stats()
    fake = C.c_void_p(0x1000)  # never dereferenced: the checks fail first
    return lib.run_photons(C.byref(pr.grid), fake, C.byref(pr.optics), pr.n_src, pr.sources, pr.n_det,
                           pr.detectors, C.byref(pr.opts), fake, fake, C.byref(st), None)


@pytest.mark.parametrize("case", ["n_packages", "precision", "flags", "w_min", "max_scatter", "launch_blocks",
                                  "event_batch", "brick_shape", "peel_queue", "max_chunk", "grid_cells", "grid_extent",
                                  "planes_order", "planes_ends", "planes_nan", "tree_unreached", "tree_twice",
                                  "tree_split_outside", "tree_cell_twice", "tree_and_planes", "tree_leaf_count",
                                  "albedo", "g", "kappa", "lum", "n_det", "det_pixels", "det_distance",
                                  "n_src", "src_kind", "src_scale", "fp32_axis"])
def test_invalid_arguments_are_rejected(lib, B, W, case):
    prob = W.small_problem(n=(4, 4, 4), n_packages=100)
    over = {}
    if case == "n_packages":
        over["n_packages"] = 0
    elif case == "precision":
        over["precision"] = 7
    elif case == "flags":
        over["flags"] = 64
    elif case == "w_min":
        over["w_min"] = -1.0
    elif case == "max_scatter":
        over["max_scatter"] = 0
    elif case == "launch_blocks":
        over["launch_blocks"] = 100
    elif case == "event_batch":
        over["event_batch"] = 65
    elif case == "brick_shape":
        over["brick_shape"] = B.brick(9, 0, 0)
    elif case == "peel_queue":
        over["peel_queue"] = -2
    elif case == "max_chunk":
        over["max_chunk"] = -1
    elif case == "grid_cells":
        prob["n"] = (0, 4, 4)
    elif case == "grid_extent":
        prob["box"] = (1.0, -1.0, -1, 1, -1, 1)
    elif case in ("planes_order", "planes_ends", "planes_nan"):
        pl = [np.linspace(-1.0, 1.0, 5) for _ in range(3)]
        if case == "planes_order":
            pl[1][2] = pl[1][1]  # not strictly increasing
        elif case == "planes_ends":
            pl[2][-1] = 1.5  # does not end at the box maximum
        else:
            pl[0][3] = np.nan
        prob["planes"] = tuple(pl)
    elif case.startswith("tree"):
        # x halved, then its upper half halved: 3 leaves -> cells 0, 1, 2
        tree = {"axis": np.array([0, -1, 0, -1, -1]), "split": np.array([0.0, 0, 0.5, 0, 0]),
                "child": np.array([1, 0, 3, 1, 2])}
        prob["n"] = (3, 1, 1)
        prob["rho"] = np.ones((1, 1, 3))
        if case == "tree_unreached":
            tree = {k: np.concatenate([v, v[-1:]]) for k, v in tree.items()}  # node 5 hangs loose
        elif case == "tree_twice":
            tree["child"][2] = 1  # node 2's children are nodes 1 and 2
        elif case == "tree_split_outside":
            tree["split"][2] = -0.5  # outside node 2, which is x in [0, 1]
        elif case == "tree_cell_twice":
            tree["child"][4] = 1
        elif case == "tree_and_planes":
            prob["planes"] = tuple(np.linspace(-1.0, 1.0, m + 1) for m in (3, 1, 1))
        else:
            prob["n"] = (4, 1, 1)
            prob["rho"] = np.ones((1, 1, 4))
        prob["tree"] = tree
    elif case == "albedo":
        prob["albedo"] = np.array([1.5])
    elif case == "g":
        prob["g"] = np.array([1.0])
    elif case == "kappa":
        prob["kappa"] = np.array([np.nan])
    elif case == "lum":
        prob["sources"] = [W.point(lum=-1.0)]
    elif case == "n_det":
        prob["detectors"] = [W.frame(10.0, 0.0, 4, 4, 1.0, 1.0)] * 9
    elif case == "det_pixels":
        prob["detectors"] = [W.frame(10.0, 0.0, 0, 4, 1.0, 1.0)]
    elif case == "det_distance":
        prob["detectors"] = [W.frame(0.0, 0.0, 4, 4, 1.0, 1.0)]
    elif case == "n_src":
        prob["sources"] = [W.point()] * 9
    elif case == "src_kind":
        prob["sources"] = [dict(W.point(), kind="ring")]
    elif case == "src_scale":
        prob["sources"] = [W.expdisk(0.0, 0.1)]
    elif case == "fp32_axis":
        # FP32 walks count crossed planes in FP32: 2^24 cells along an axis are refused
        prob["n"] = (1, 1, 1 << 24)
        over["precision"] = 1
    if case == "src_kind":
        # the binding maps kinds to the enum; pass an unknown value directly
        pr = B._Problem(dict(prob, sources=[W.point()]))
        pr.sources[0].kind = 5
        st = B.Stats()
        fake = C.c_void_p(0x1000)
        rc = lib.run_photons(C.byref(pr.grid), fake, C.byref(pr.optics), pr.n_src, pr.sources, pr.n_det,
                             pr.detectors, C.byref(pr.opts), fake, fake, C.byref(st), None)
    else:
        rc = _call_run(lib, B, prob, **over)
    assert rc == B.EINVAL, (case, rc)
    assert lib.mcrt_last_error().decode(), case
    if case == "fp32_axis":
        assert "2^24" in lib.mcrt_last_error().decode()


def test_backward_rejects_missing_gradients(lib, B, W):
    prob = W.small_problem(n=(4, 4, 4), n_packages=100)
    pr = B._Problem(prob)
    fake = C.c_void_p(0x1000)
    st = B.Stats()
    none = B.Grads(None, None, None, None)
    for grads in (None, C.byref(none)):
        rc = lib.backward(C.byref(pr.grid), fake, C.byref(pr.optics), pr.n_src, pr.sources, pr.n_det, pr.detectors,
                          C.byref(pr.opts), fake, None, grads, C.byref(st), None)
        assert rc == B.EINVAL
        assert lib.mcrt_last_error().decode()
    # a loss on the absorbed tally needs the density gradient
    only_albedo = B.Grads(None, fake, None, None)
    rc = lib.backward(C.byref(pr.grid), fake, C.byref(pr.optics), pr.n_src, pr.sources, pr.n_det, pr.detectors,
                      C.byref(pr.opts), fake, fake, C.byref(only_albedo), C.byref(st), None)
    assert rc == B.EINVAL and "adj_absorbed" in lib.mcrt_last_error().decode()


@pytest.mark.parametrize("case", ["kind", "sed_pixels", "eye_is_target", "up_along_view", "eye_nan", "persp_extent"])
def test_invalid_instruments_are_rejected(lib, B, W, case):
    prob = W.small_problem(n=(4, 4, 4), n_packages=100)
    if case == "sed_pixels":
        prob["detectors"] = [dict(W.sed(10.0, 30.0), nx=2)]
    elif case == "eye_is_target":
        prob["detectors"] = [W.perspective((0.5, 0.5, 0.5), (0.5, 0.5, 0.5), (0, 0, 1), 4, 4, 1.0, 1.0)]
    elif case == "up_along_view":
        prob["detectors"] = [W.perspective((0, 0, 3), (0, 0, 0), (0, 0, 2), 4, 4, 1.0, 1.0)]
    elif case == "eye_nan":
        prob["detectors"] = [W.perspective((0, np.nan, 3), (0, 0, 0), (0, 1, 0), 4, 4, 1.0, 1.0)]
    elif case == "persp_extent":
        prob["detectors"] = [W.perspective((0, 0, 3), (0, 0, 0), (0, 1, 0), 4, 4, 0.0, 1.0)]
    pr = B._Problem(prob)
    if case == "kind":
        pr.detectors[0].kind = 7
    st = B.Stats()
    fake = C.c_void_p(0x1000)
    rc = lib.run_photons(C.byref(pr.grid), fake, C.byref(pr.optics), pr.n_src, pr.sources, pr.n_det,
                         pr.detectors, C.byref(pr.opts), fake, fake, C.byref(st), None)
    assert rc == B.EINVAL, case
    assert "detector 0" in lib.mcrt_last_error().decode(), case


@pytest.mark.parametrize("case", ["cell_lum_null", "two_cell_sources"])
def test_invalid_cell_sources_are_rejected(lib, B, W, case):
    prob = W.small_problem(n=(4, 4, 4), n_packages=100)
    pr = B._Problem(prob)
    fake = C.c_void_p(0x1000)
    srcs = (B.Source * 2)()
    srcs[0] = pr.sources[0]
    srcs[0].kind = 2
    srcs[0].cell_lum = None if case == "cell_lum_null" else fake
    srcs[1] = srcs[0]
    st = B.Stats()
    rc = lib.run_photons(C.byref(pr.grid), fake, C.byref(pr.optics), 1 if case == "cell_lum_null" else 2, srcs,
                         pr.n_det, pr.detectors, C.byref(pr.opts), fake, fake, C.byref(st), None)
    assert rc == B.EINVAL
    assert "cell" in lib.mcrt_last_error().decode()


@pytest.mark.parametrize("case", ["n_abs", "absorbed", "n_lambda", "lambda", "dlambda", "kappa_abs", "emissivity",
                                  "emission", "precision", "rho", "grid"])
def test_invalid_dust_emission_arguments_are_rejected(lib, B, case):
    g = B.make_grid({"box": (-1, 1, -1, 1, -1, 1), "n": (4, 4, 4)})
    fake = C.c_void_p(0x1000)
    lam, dlam, ka = np.array([10.0, 100.0]), np.array([1.0, 10.0]), np.array([1.0, 0.1])
    args = dict(grid=C.byref(g), rho=fake, precision=0, n_abs=1, absorbed=fake, n_lambda=2, lam=lam, dlam=dlam,
                ka=ka, eps=1.0, temp=None, emission=fake)
    if case == "n_abs":
        args["n_abs"] = 0
    elif case == "absorbed":
        args["absorbed"] = None
    elif case == "n_lambda":
        args["n_lambda"] = 0
    elif case == "lambda":
        args["lam"] = np.array([10.0, -1.0])
    elif case == "dlambda":
        args["dlam"] = np.array([0.0, 1.0])
    elif case == "kappa_abs":
        args["ka"] = np.array([1.0, np.nan])
    elif case == "emissivity":
        args["eps"] = 0.0
    elif case == "emission":
        args["emission"] = None
    elif case == "precision":
        args["precision"] = 3
    elif case == "rho":
        args["rho"] = None
    elif case == "grid":
        g.nx = 0
    dp = C.POINTER(C.c_double)
    rc = lib.dust_emission(args["grid"], args["rho"], args["precision"], args["n_abs"], args["absorbed"],
                           args["n_lambda"], args["lam"].ctypes.data_as(dp), args["dlam"].ctypes.data_as(dp),
                           args["ka"].ctypes.data_as(dp), args["eps"], args["temp"], args["emission"], None)
    assert rc == B.EINVAL, case
    assert lib.mcrt_last_error().decode(), case


def test_well_formed_tree_is_accepted_before_any_device_work(lib, B, W):
    # the tree of the rejection cases, unchanged, passes the argument checks:
    # the call then fails only on the fake device pointers' stream work, not
    # with MCRT_EINVAL -- checked through the host-side preparation alone
    prob = W.small_problem(n=(3, 1, 1), n_packages=10)
    prob["rho"] = np.ones((1, 1, 3))
    prob["tree"] = {"axis": np.array([0, -1, 0, -1, -1]), "split": np.array([0.0, 0, 0.5, 0, 0]),
                    "child": np.array([1, 0, 3, 1, 2])}
    g = B.make_grid(prob)
    assert g.tree_nodes == 5


def test_null_pointers_are_rejected(lib, B, W):
    prob = W.small_problem(n=(4, 4, 4), n_packages=100)
    pr = B._Problem(prob)
    st = B.Stats()
    fake = C.c_void_p(0x1000)
    assert lib.run_photons(None, fake, C.byref(pr.optics), 1, pr.sources, pr.n_det, pr.detectors, C.byref(pr.opts),
                           fake, fake, C.byref(st), None) == B.EINVAL
    assert lib.run_photons(C.byref(pr.grid), None, C.byref(pr.optics), 1, pr.sources, pr.n_det, pr.detectors,
                           C.byref(pr.opts), fake, fake, C.byref(st), None) == B.EINVAL
    assert lib.run_photons(C.byref(pr.grid), fake, C.byref(pr.optics), 1, pr.sources, pr.n_det, pr.detectors,
                           None, fake, fake, C.byref(st), None) == B.EINVAL
    assert lib.run_photons(C.byref(pr.grid), fake, C.byref(pr.optics), 1, pr.sources, pr.n_det, pr.detectors,
                           C.byref(pr.opts), None, fake, C.byref(st), None) == B.EINVAL  # images with peel-off
    assert lib.backward_density(C.byref(pr.grid), fake, C.byref(pr.optics), 1, pr.sources, pr.n_det, pr.detectors,
                                C.byref(pr.opts), fake, None, C.byref(st), None) == B.EINVAL  # no gradient buffer
    g = B.make_grid(prob)
    assert lib.trace_path(C.byref(g), fake, 1.0, 0, -1, fake, fake, fake, 0, None, None, None, None,
                          None) == B.EINVAL
    assert lib.trace_path(C.byref(g), fake, -1.0, 0, 10, fake, fake, fake, 0, None, None, None, None,
                          None) == B.EINVAL
    assert lib.trace_path(C.byref(g), fake, 1.0, 0, 10, fake, fake, fake, 0, fake, None, None, None,
                          None) == B.EINVAL  # segment lists go together
    dets = B.make_detectors(prob["detectors"])
    assert lib.peel_off(C.byref(g), fake, 1.0, 1.0, 0, 10, fake, None, fake, 1, dets, fake, None) == B.EINVAL
    assert lib.peel_off(C.byref(g), fake, 1.0, 0.5, 0, 10, fake, None, fake, 0, dets, fake, None) == B.EINVAL
    assert lib.mcrt_last_error().decode()


@pytest.mark.parametrize("case", ["rho_dtype64", "rho_dtype32", "rho_size", "images_size", "images_dtype",
                                  "absorbed_size", "adj_size", "grad_size", "grad_albedo_size", "trace_tau",
                                  "peel_images"])
def test_binding_rejects_mismatched_tensors(lib, B, W, case):
    # the binding checks every tensor's element type and count against the
    # problem before any pointer reaches the library (host-only: the check
    # fails before the device test, so CPU tensors show it)
    import torch
    prob = W.small_problem(n=(4, 3, 2), n_packages=10, detectors=[W.frame(10.0, 0.0, 5, 4, 1.0, 1.0)])
    f64 = torch.float64
    rho = torch.ones(24, dtype=f64)
    images = torch.zeros(B.image_shape(prob), dtype=f64)
    absorbed = torch.zeros((1, 24), dtype=f64)
    with pytest.raises(ValueError) as ei:
        if case == "rho_dtype64":  # FP64 path with float densities
            B.run_photons(prob, rho.float(), images, absorbed)
        elif case == "rho_dtype32":  # FP32 path with double densities
            B.run_photons(dict(prob, precision=1), rho, images, absorbed)
        elif case == "rho_size":
            B.run_photons(prob, torch.ones(23, dtype=f64), images, absorbed)
        elif case == "images_size":
            B.run_photons(prob, rho, torch.zeros(19, dtype=f64), absorbed)
        elif case == "images_dtype":
            B.run_photons(prob, rho, images.float(), absorbed)
        elif case == "absorbed_size":
            B.run_photons(prob, rho, images, torch.zeros(23, dtype=f64))
        elif case == "adj_size":
            B.backward_density(prob, rho, torch.zeros(21, dtype=f64), torch.zeros(24, dtype=f64))
        elif case == "grad_size":
            B.backward_density(prob, rho, images, torch.zeros(12, dtype=f64))
        elif case == "grad_albedo_size":
            B.backward(prob, rho, images, grad_albedo=torch.zeros(2, dtype=f64))
        elif case == "trace_tau":
            o = torch.zeros((5, 3), dtype=f64)
            B.trace_path(prob, rho, 1.0, 0, o, o, torch.zeros(4, dtype=f64))
        elif case == "peel_images":
            pos = torch.zeros((5, 3), dtype=f64)
            B.peel_off(prob, rho, 1.0, 0.5, 0, pos, None, torch.zeros(5, dtype=f64), prob["detectors"],
                       torch.zeros(21, dtype=f64))
    assert "device tensor" not in str(ei.value), ei.value


def test_noalloc_trace_rejects_grids_beyond_its_scratch(lib, B):
    # a grid whose bricked densities exceed the scratch array is rejected
    # before any device work (host-only)
    g = B.make_grid({"box": (-1, 1, -1, 1, -1, 1), "n": (512, 512, 512)})
    fake = C.c_void_p(0x1000)
    for prec, ok_rays in ((0, 0), (1, 0)):
        rc = lib.trace_path_noalloc(C.byref(g), fake, 1.0, prec, 10, fake, fake, fake, 0, None, None, None, None,
                                    None)
        assert rc == B.EINVAL
        assert b"scratch" in lib.mcrt_last_error()
    rc = lib.trace_path_noalloc(C.byref(g), fake, -1.0, 0, 10, fake, fake, fake, 0, None, None, None, None, None)
    assert rc == B.EINVAL


def test_probes_library_exports_its_header(B):
    # the memory-system probes' header and library: every declared function
    # is exported, and invalid arguments are rejected before any launch
    hdr = os.path.join(ROOT, "include", "mcrt_probes.h")
    text = re.sub(r"/\*.*?\*/", "", open(hdr).read(), flags=re.S)
    names = re.findall(r"^\s*int\s+(\w+)\s*\(", text, flags=re.M)
    assert names == ["mcrt_probe"]
    if not os.path.exists(B.PROBES_PATH):
        pytest.skip("libmcrt_probes.so is not built")
    out = subprocess.run(["nm", "-D", "--defined-only", B.PROBES_PATH], check=True, capture_output=True,
                         text=True).stdout
    assert "mcrt_probe" in {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    lib = C.CDLL(B.PROBES_PATH)
    lib.mcrt_probe.argtypes = [C.c_int, C.c_void_p, C.c_uint64, C.c_uint64, C.c_int, C.POINTER(C.c_double),
                               C.c_void_p]
    ms = C.c_double(0)
    fake = C.c_void_p(0x1000)
    assert lib.mcrt_probe(9, fake, 1 << 20, 1 << 14, 1, C.byref(ms), None) == -1  # unknown kind
    assert lib.mcrt_probe(1, fake, 3 << 20, 1 << 14, 1, C.byref(ms), None) == -1  # not a power of two
    assert lib.mcrt_probe(2, fake, 1 << 20, 100, 1, C.byref(ms), None) == -1  # not whole workgroups
    assert lib.mcrt_probe(0, None, 1 << 20, 1, 1, C.byref(ms), None) == -1
