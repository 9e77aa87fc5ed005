import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HELPERS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "helpers")
if HELPERS not in sys.path:
    sys.path.insert(0, HELPERS)  # parity (element-wise checks), emu (the CPU harness)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def pytest_collection_modifyitems(config, items):
    # GPU tests are skipped (not failed) on a machine without a GPU when they
    # are collected together with CPU tests; `-m gpu` on a machine with an MI355X runs them.
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


@pytest.fixture(scope="session")
def orc():
    import oracle
    return oracle


@pytest.fixture(scope="session")
def W():
    from paper_1410_1629_amd import workloads
    return workloads


@pytest.fixture(scope="session")
def E(tmp_path_factory):
    """The CPU harness of the library's lane code (built once per session)."""
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "helpers"))
    import emu
    return emu.Emu(emu.build(str(tmp_path_factory.mktemp("emu"))))
