import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def ensure_built():
    """Load libspin1.so; compile it only when nothing is built yet."""
    from paper_2310_03636_amd import spin1
    if not os.path.exists(spin1.LIB_PATH):
        from paper_2310_03636_amd import build_lib
        build_lib.build()
    spin1.load()
    return spin1


@pytest.fixture(scope="session")
def abi():
    """The binding with the library loaded (no device work)."""
    return ensure_built()


@pytest.fixture(scope="session")
def lib():
    """The HIP library through its Python binding; GPU tests only."""
    if not gpu_available():
        pytest.skip("no GPU")
    return ensure_built()
