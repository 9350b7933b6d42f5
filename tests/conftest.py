import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def gpu_device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    return torch.device("cuda:0")


@pytest.fixture
def progress(request):
    """Writes a line to the terminal right away, past pytest's output capture:
    long tests report each step of their work (an oracle iteration, a root), so
    a run of many minutes is never silent."""
    capman = request.config.pluginmanager.getplugin("capturemanager")

    def say(msg):
        if capman is not None:
            with capman.global_and_fixture_disabled():
                sys.stdout.write("\n" + msg + "\n")
                sys.stdout.flush()
        else:
            print(msg, flush=True)
    return say
