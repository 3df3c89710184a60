"""Test configuration: markers, import path and the oracle build.

`gpu` tests need an MI355X and the HIP engine (libggns.so); everything else runs
on the CPU against the FP64 oracle.
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the HIP engine")
    # the oracle is compiled before any test runs (and so before any GPU
    # call of this process) when its library is missing or stale
    import oracle.oracle as O
    if O.stale():
        O.build(force=True)


@pytest.fixture(scope="session")
def orc():
    import oracle.oracle as O
    O.lib()
    return O
