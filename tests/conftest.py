import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def lib():
    """The HIP library through its C-ABI binding (GPU tests only)."""
    from paper_2009_02845_amd import binding
    return binding.load()


# import torch while collecting, outside any per-test time limit (the first
# import on a fresh machine can take a minute or more)
try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    pass
