import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def oracle():
    from oracle import ref
    ref.lib()
    return ref


@pytest.fixture(scope="session")
def ref3():
    from oracle import ref3 as mod
    mod.lib()
    return mod


@pytest.fixture(scope="session")
def lbvp():
    """The HIP library's Python binding (imported lazily so that collecting the
    CPU tests does not need the built library)."""
    from paper_1901_08766_amd import lbvp as mod
    return mod


@pytest.fixture(scope="session")
def lbvp3():
    """The binding of the D3Q19 entry points (imported lazily, as ``lbvp``)."""
    from paper_1901_08766_amd import lbvp3 as mod
    return mod
