import functools
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@functools.lru_cache(maxsize=None)
def workload(name, geometry="ff"):
    from workloads import make_workload
    return make_workload(name, geometry)


@functools.lru_cache(maxsize=None)
def built(name, geometry="ff"):
    """(workload, A, S) from the oracle, cached per test session."""
    from oracle import cpm
    w = workload(name, geometry)
    A, S = cpm.build(w)
    return w, A, S
