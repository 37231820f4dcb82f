import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


_CAPTURE = None


def pytest_configure(config):
    global _CAPTURE
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU oracle case")
    _CAPTURE = config.pluginmanager.getplugin("capturemanager")


def say(msg):
    """A progress line that reaches the terminal even under pytest's output capture, so that a
    long GPU case shows that it is alive."""
    if _CAPTURE is not None:
        with _CAPTURE.global_and_fixture_disabled():
            print(msg, flush=True)
    else:
        print(msg, flush=True)


@pytest.fixture(scope="session")
def gpu_lib():
    """The built HIP library through its Python binding; fails loudly if missing."""
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")
    from paper_2601_16949_amd import rttda

    rttda.load()  # raises if the shared library is not built
    return rttda
