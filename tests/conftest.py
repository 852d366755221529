import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; fails loudly if it is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")
    from paper_2512_17132_amd import fdtd
    fdtd.load()
    return fdtd


@pytest.fixture
def progress(request):
    """Prints a line to the terminal at once, past pytest's output capture: a
    long test reports its stages while it runs."""
    capman = request.config.pluginmanager.getplugin("capturemanager")

    def say(msg):
        if capman is not None:
            with capman.global_and_fixture_disabled():
                print(msg, flush=True)
        else:
            print(msg, flush=True)
    return say
