import functools
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device); parity tests through the C-ABI")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@functools.lru_cache(maxsize=None)
def cached_config(cfg, **kw):
    import pbgen
    return pbgen.make_config(cfg, **kw)


@functools.lru_cache(maxsize=None)
def cached_problem(**kw):
    import pbgen
    return pbgen.make_problem(**kw)
