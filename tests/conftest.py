"""Shared pytest configuration.

Markers:
  gpu -- needs an MI355X (gfx950) and the built HIP library; everything else
         runs on the CPU.
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def ora():
    """The CPU oracle (built with gcc if its shared library is missing)."""
    import oracle
    if not os.path.exists(oracle._LIB):
        oracle.build(force=False)
    return oracle
