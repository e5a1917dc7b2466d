import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")


def pytest_collection_modifyitems(session, config, items):
    """When GPU tests will run, let PyTorch bring up the device before the
    library does: tests that hand torch streams to the library need torch's
    HIP runtime initialised first, whatever order the files run in."""
    if any(item.get_closest_marker("gpu") for item in items):
        try:
            import torch
            torch.cuda.is_available()
        except ImportError:
            pass
