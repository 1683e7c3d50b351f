"""Shared pytest configuration.

Tests marked ``gpu`` need an MI355X (gfx950) and the built HIP library; all
other tests run on the CPU. The CPU oracle is built on first use.
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def ref():
    import oracle
    # Build on first use, and again when the C source is newer than the
    # library (a stale oracle would check the GPU against old arithmetic).
    src = [oracle.SOURCE, os.path.join(os.path.dirname(oracle.SOURCE), "plas_oracle.h")]
    if not os.path.exists(oracle.LIBRARY) or \
            os.path.getmtime(oracle.LIBRARY) < max(os.path.getmtime(p) for p in src):
        oracle.build()
    return oracle
